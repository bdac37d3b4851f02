"""A render captured in a HIP graph (torch.cuda.CUDAGraph) replays to the
same outputs as eager renders.  kt_render enqueues kernels only: no
allocation, no memset, no host synchronisation, so a fitting or animation
loop can capture it.  Each replay is followed by eager work and a
synchronisation, and every replay is checked against the eager result."""
import sys

import numpy as np
import pytest

from paper_2202_00086_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("fate", "r_hit", "g", "intensity", "deflection", "max_rel_h", "n_steps", "n_evals")


def _announce(*what):
    print("[gpu-case]", *what, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def K():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2202_00086_amd import kerrtrace
    return kerrtrace


def _host(out):
    return {k: out[k].cpu().numpy().copy() for k in KEYS if k in out}


@pytest.mark.parametrize("case", ["single", "batch"])
def test_captured_render_replays_equal_eager(K, case):
    import torch
    if case == "single":
        params = dict(W.kerr_disk(a=0.9, incl_deg=60.0, n=40, r_in=W.isco(0.9)), src_on=1, r_src=1000.0)
        r = K.Renderer(device="cuda:0", **params)
    else:
        images, integ = W.heterogeneous_batch(n_images=5, seed=3, side_unit=8, side_steps=4, square=False)
        r = K.BatchRenderer(images, device="cuda:0", **integ)
    _announce("graph capture", case)
    r.render()
    torch.cuda.synchronize()
    eager = _host(r.out)
    stats_eager = K.read_stats(r.out)
    for key in KEYS:
        if key in r.out:
            r.out[key].fill_(0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        r.render()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        r.render()
    scratch = torch.zeros(1 << 20, device="cuda:0")
    for rep in range(3):
        for key in KEYS:
            if key in r.out:
                r.out[key].fill_(0)
        g.replay()
        scratch.add_(1.0)  # eager work between replays
        torch.cuda.synchronize()
        got = _host(r.out)
        for key, v in eager.items():
            np.testing.assert_array_equal(got[key].view(np.uint8), v.view(np.uint8), err_msg=f"replay {rep} {key}")
        st = K.read_stats(r.out)
        assert st.evals == stats_eager.evals and list(st.fate_count) == list(stats_eager.fate_count)
        assert st.trace_ms > 0.0  # the clock stamps replay with the graph
