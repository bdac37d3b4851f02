"""The appendix's q-metric on the GPU against the oracle's q-metric, element
by element: fates, celestial-sphere codes and crossing directions, the
constraint, the initial states; every adaptive scheme; launch-shape
bit-identity; and q = 0 against the Kerr kernel at a = 0."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2202_00086_amd import workloads as W
from tests import parity as P

pytestmark = pytest.mark.gpu


def _announce(*what):
    print("[gpu-case]", *what, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def K():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2202_00086_amd import kerrtrace
    return kerrtrace


def gpu_render(K, params, launch=None):
    import torch
    r = K.Renderer(device="cuda:0", launch=launch, **params)
    out = r.render()
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items() if k != "stats"}
    res["stats"] = K.read_stats(out)
    return res


def _dirs(th, ph):
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)


def _compare(K, g, o, nx, ny, dir_tol=1e-9):
    P.check_fates(g["fate"], o["fate"], nx, ny, min_allowed=2)
    gs, os_ = g["sky"].reshape(ny, nx), o["sky"].reshape(ny, nx)
    bad = (gs != os_) & ~P.boundary_mask(os_)
    assert not bad.any(), np.argwhere(bad)[:10]
    esc = (g["fate"] == K.ESCAPED) & (o["fate"] == O.ESCAPED)
    d = np.linalg.norm(_dirs(g["theta_f"][esc], g["phi_f"][esc]) - _dirs(o["theta_f"][esc], o["phi_f"][esc]), axis=1)
    assert d.max() < dir_tol, d.max()
    m = P.value_mask(g, o, nx, ny)
    P.check_max_h(g, o, "max_rel_h", m, budget=1e-10)
    return d.max()


@pytest.mark.parametrize("q", [-0.3, 0.5, 1.0])
def test_qmetric_lensing_parity(K, q):
    nx, ny = 48, 40
    params = dict(W.qmetric_lensing(q=q, n=nx), ny=ny)
    _announce("q-metric lensing", q)
    g = gpu_render(K, params)
    o = O.trace_pixels(O.Setup(**params))
    assert (o["fate"] == O.CAPTURED).sum() > 20
    dmax = _compare(K, g, o, nx, ny)
    print(f"[q-metric {q}] max direction difference {dmax:.2e}; fates {np.bincount(g['fate']).tolist()}", flush=True)


@pytest.mark.parametrize("method", [2, 3, 4, 5])
def test_qmetric_other_schemes(K, method):
    nx, ny = 32, 32
    params = dict(W.qmetric_lensing(q=0.5, n=nx, rtol=1e-11), method=method)
    _announce("q-metric scheme", method)
    g = gpu_render(K, params)
    o = O.trace_pixels(O.Setup(**params))
    P.check_fates(g["fate"], o["fate"], nx, ny, min_allowed=2)
    esc = (g["fate"] == K.ESCAPED) & (o["fate"] == O.ESCAPED)
    d = np.linalg.norm(_dirs(g["theta_f"][esc], g["phi_f"][esc]) - _dirs(o["theta_f"][esc], o["phi_f"][esc]), axis=1)
    assert d.max() < 1e-7, d.max()


def test_qmetric_initial_states(K):
    import torch
    params = dict(W.qmetric_lensing(q=0.7, n=16), incl=1.2, r_obs=60.0, r_escape=66.0)
    state, invalid = K.init_rays(**params)
    torch.cuda.synchronize()
    st = state.cpu().numpy()
    s = O.Setup(**params)
    for p in range(0, 256, 7):
        x, y = O.pixel_xy(s, p % 16, p // 16)
        want, _ = O.camera_ray_k(O.QMETRIC, 1.0, 0.0, 0.7, 60.0, 1.2, x, y)
        np.testing.assert_allclose(st[:, p], want, rtol=4e-15, atol=1e-15)


def test_qmetric_launch_shapes_and_q_zero(K):
    params = W.qmetric_lensing(q=0.5, n=24)
    _announce("q-metric launch shapes")
    ref = gpu_render(K, params)
    # the last shape runs the 3-wave build of the kernels
    for ln in [K.kt_launch(1, 64, 1, 1), K.kt_launch(0, 128, 0, 32), K.kt_launch(1, 256, 3, 4)]:
        g = gpu_render(K, params, launch=ln)
        for key in ("fate", "sky", "theta_f", "phi_f", "max_rel_h", "n_steps"):
            np.testing.assert_array_equal(g[key].view(np.uint8), ref[key].view(np.uint8), err_msg=key)
    # q = 0 is Schwarzschild: the same fates and crossing points as the Kerr kernel at a = 0
    g0 = gpu_render(K, W.qmetric_lensing(q=0.0, n=24))
    k0 = gpu_render(K, W.lensing(a=0.0, n=24))
    np.testing.assert_array_equal(g0["fate"], k0["fate"])
    esc = g0["fate"] == K.ESCAPED
    d = np.linalg.norm(_dirs(g0["theta_f"][esc], g0["phi_f"][esc]) - _dirs(k0["theta_f"][esc], k0["phi_f"][esc]), axis=1)
    assert d.max() < 1e-9, d.max()
