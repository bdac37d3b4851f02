"""Renders in flight together on separate HIP streams (default priority), as
a server would run them: a Kerr disk image, a q-metric celestial-sphere
image and a small batch, each with its own workspace and outputs, enqueued
round-robin on three streams and repeated.  The library keeps no state
between calls outside the caller's workspace, so every output equals the
same configuration rendered alone, bit for bit."""
import sys

import numpy as np
import pytest

from paper_2202_00086_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("fate", "r_hit", "g", "intensity", "deflection", "theta_f", "phi_f", "max_rel_h", "n_steps", "n_evals")


@pytest.fixture(scope="module")
def K():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2202_00086_amd import kerrtrace
    return kerrtrace


def _host(out):
    return {k: out[k].cpu().numpy().copy() for k in KEYS if k in out}


def _renderers(K):
    images, integ = W.heterogeneous_batch(n_images=6, seed=11, side_unit=8, side_steps=5, square=False)
    return [K.Renderer(device="cuda:0", **dict(W.kerr_disk(a=0.7, incl_deg=75.0, n=96, r_in=W.isco(0.7)),
                                               src_on=1, r_src=1000.0)),
            K.Renderer(device="cuda:0", **W.qmetric_lensing(q=0.3, n=64)),
            K.BatchRenderer(images, device="cuda:0", **integ)]


def test_concurrent_streams_equal_sequential_renders(K):
    import torch
    print("[gpu-case] three renderers, alone and then on three streams", flush=True)
    sys.stdout.flush()
    rs = _renderers(K)
    alone = []
    for r in rs:
        r.render()
        torch.cuda.synchronize()
        alone.append(_host(r.out))
    streams = [torch.cuda.Stream() for _ in rs]
    for rep in range(3):
        for r in rs:
            for key in KEYS:
                if key in r.out:
                    r.out[key].fill_(0)
        torch.cuda.synchronize()
        for r, s in zip(rs, streams):
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                r.render()
        torch.cuda.synchronize()
        for k, r in enumerate(rs):
            got = _host(r.out)
            for key, v in alone[k].items():
                np.testing.assert_array_equal(got[key].view(np.uint8), v.view(np.uint8),
                                              err_msg=f"renderer {k} {key} repeat {rep}")
