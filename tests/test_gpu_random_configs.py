"""Seeded random camera configurations (valid inputs only) on the GPU
against the oracle, element by element: spins of either sign, inclinations
near the poles and in between, observer distances, fields of view, ragged
resolutions, tolerances, the adaptive schemes (eight more configurations
with rational Bulirsch-Stoer), Keplerian and constant-l0 disks with
power-law or tapered emissivity, and the point source."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2202_00086_amd import workloads as W
from tests import parity as P

pytestmark = pytest.mark.gpu


def _config(rng, retrograde=False, method=None):
    a = float(rng.uniform(-0.998, -0.05)) if retrograde else float(rng.uniform(0.0, 0.998))
    band = int(rng.integers(3))
    incl = float((rng.uniform(0.05, 0.3), rng.uniform(0.3, 2.84), rng.uniform(2.84, 3.09))[band])
    r_obs = float(10 ** rng.uniform(1.5, 3.0))
    fov = float(rng.uniform(4.0, 25.0))
    nx, ny = (int(v) for v in rng.integers(3, 41, size=2))
    method = int(rng.choice([1, 2, 3, 4])) if method is None else method
    rtol = float(rng.choice([1e-10, 1e-11, 1e-12]))
    p = dict(M=1.0, a=a, r_obs=r_obs, incl=incl, fov_x=fov, fov_y=fov * float(rng.uniform(0.5, 1.5)), nx=nx,
             ny=ny, method=method, rtol=rtol, atol=rtol, h_init=1.0, cap_buffer=0.01, r_escape=0.0,
             max_steps=1_000_000)
    if rng.uniform() < 0.6:
        r_in = W.isco(a) * float(rng.uniform(1.0, 1.5))
        p.update(disk_on=1, r_in=r_in, r_out=r_in + float(rng.uniform(5.0, 25.0)), emis_q=2.0,
                 emis_model=int(rng.integers(2)))
        if rng.uniform() < 0.4:
            p.update(rotation=1, l0=float(rng.uniform(2.0, 3.5)) if a < 0.9 else float(rng.uniform(1.7, 2.2)))
    if rng.uniform() < 0.3:
        p.update(src_on=1, r_src=r_obs)
    return p


# 40 with spin along +z, then 8 with negative spin (the hole counter-rotates
# with respect to the disk and the camera's phi direction)
CONFIGS = ([_config(np.random.default_rng(7000 + k)) for k in range(40)] +
           [_config(np.random.default_rng(7500 + k), retrograde=True) for k in range(8)])
N_CASES = len(CONFIGS)
# rational Bulirsch-Stoer (method 5) on eight more, two of them retrograde
RAT_CONFIGS = [_config(np.random.default_rng(7800 + k), retrograde=k >= 6, method=5) for k in range(8)]
ALL_CONFIGS = CONFIGS + RAT_CONFIGS


@pytest.fixture(scope="module")
def K():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2202_00086_amd import kerrtrace
    return kerrtrace


@pytest.mark.parametrize("k", range(len(ALL_CONFIGS)))
def test_random_configuration(K, k):
    import torch
    p = ALL_CONFIGS[k]
    nx, ny = p["nx"], p["ny"]
    print(f"[gpu-case] random config {k}: {p}", flush=True)
    sys.stdout.flush()
    r = K.Renderer(device="cuda:0", **p)
    out = r.render()
    torch.cuda.synchronize()
    g = {key: v.cpu().numpy() for key, v in out.items() if key != "stats"}
    st = K.read_stats(out)
    o = O.trace_pixels(O.Setup(**p))
    P.check_fates(g["fate"], o["fate"], nx, ny, min_allowed=2)
    m = P.value_mask(g, o, nx, ny)
    assert st.rays == nx * ny and sum(st.fate_count) == nx * ny
    np.testing.assert_array_equal(g["fate"] == K.INVALID, o["fate"] == O.INVALID)
    if p.get("disk_on"):
        d = m & (o["fate"] == O.DISK)
        for key in ("r_hit", "g", "intensity"):
            P.check_values(g, o, key, d, rtol=1e-8)
    if p.get("src_on"):
        e = m & np.isfinite(o["deflection"])
        if p["method"] in (K.BS, K.BS_RAT):
            # the step sequence carries rounding far (see the scheme tests):
            # the tolerance follows from the oracle's own one-ulp sensitivity
            s = O.Setup(**p)
            xy = np.array([O.pixel_xy(s, q % nx, q // nx) for q in range(nx * ny)])
            sens = P.ulp_sensitivity(lambda x, y: O.trace_xy(s, x, y), xy[:, 0].copy(), xy[:, 1].copy(),
                                     "deflection")
            P.check_values_rounding(g, o, "deflection", e, sens, rtol=1e-8)
        else:
            P.check_values(g, o, "deflection", e, rtol=1e-8)
    # the constraint: same size on both sides where the rays agree
    h_g, h_o = g["max_rel_h"][m], o["max_rel_h"][m]
    ok = np.isfinite(h_g) & np.isfinite(h_o)
    if ok.any():
        assert np.nanmax(h_g[ok]) < 10 * max(np.nanmax(h_o[ok]), 1e-14)


def test_random_configurations_as_one_batch(K):
    """The same configurations (with one shared integrator, DP45 at 1e-12) as
    one batch: every image equals its own single render bit for bit."""
    import torch
    integ = dict(method=1, rtol=1e-12, atol=1e-12, h_init=1.0, cap_buffer=0.01, r_escape=0.0,
                 max_steps=1_000_000)
    images = [{key: v for key, v in c.items() if key in W.IMAGE_KEYS} for c in CONFIGS]
    print(f"[gpu-case] random batch of {len(images)} images", flush=True)
    sys.stdout.flush()
    br = K.BatchRenderer(images, device="cuda:0", **integ)
    br.render()
    torch.cuda.synchronize()
    for k, im in enumerate(images):
        r = K.Renderer(device="cuda:0", **W.image_params(im, integ))
        out = r.render()
        torch.cuda.synchronize()
        f, n = br.first[k], br.sizes[k]
        for key in ("fate", "r_hit", "g", "intensity", "deflection", "max_rel_h", "n_steps"):
            if key in out and key in br.out:
                np.testing.assert_array_equal(br.out[key][f:f + n].cpu().numpy().view(np.uint8),
                                              out[key].cpu().numpy().view(np.uint8), err_msg=f"image {k} {key}")


MIXED = [k for k in range(N_CASES) if CONFIGS[k]["method"] == 1][:8]


@pytest.mark.parametrize("k", MIXED)
def test_random_configuration_mixed(K, k):
    """The DP45 configurations in mixed precision (budget 1e-10, r_switch
    drawn so that some rays use the FP32 part): rays kept from the mixed
    pass end within the budget, and rays re-run in FP64 equal the FP64 render
    bit for bit."""
    import torch
    p = CONFIGS[k]
    rng = np.random.default_rng(9000 + k)
    r_switch = float(p["r_obs"] * rng.uniform(0.2, 0.9))
    print(f"[gpu-case] random mixed config {k}: r_switch {r_switch:.1f}", flush=True)
    sys.stdout.flush()
    ref = K.Renderer(device="cuda:0", **p).render()
    mix = K.Renderer(device="cuda:0", **dict(p, precision=K.MIXED, h_budget=1e-10, r_switch=r_switch)).render()
    torch.cuda.synchronize()
    f = {key: v.cpu().numpy() for key, v in ref.items() if key != "stats"}
    m = {key: v.cpu().numpy() for key, v in mix.items() if key != "stats"}
    # rays kept from the mixed pass are within the budget; the others were
    # re-run in FP64 (whose own |H|_rel may exceed it at loose rtol)
    re = m["used_fp64"].astype(bool)
    kept = ~re & (m["fate"] != K.INVALID)
    if kept.any():
        assert np.nanmax(m["max_rel_h"][kept]) <= 1e-10
    for key in ("fate", "r_hit", "g", "intensity", "max_rel_h", "n_steps"):
        np.testing.assert_array_equal(m[key][re].view(np.uint8), f[key][re].view(np.uint8), err_msg=key)


def _qconfig(rng):
    q = float(rng.uniform(-0.45, 1.5))
    return dict(M=1.0, a=0.0, metric=1, q=q, r_obs=float(10 ** rng.uniform(1.7, 2.7)),
                incl=float(rng.uniform(0.2, 2.9)), fov_x=float(rng.uniform(6.0, 20.0)),
                fov_y=float(rng.uniform(6.0, 20.0)), nx=int(rng.integers(5, 33)), ny=int(rng.integers(5, 33)),
                method=int(rng.choice([1, 2, 3, 4])), rtol=1e-12, atol=1e-12, h_init=1.0, cap_buffer=0.01,
                r_escape=0.0, max_steps=1_000_000, sky_on=1, grid_deg=6.0, line_deg=0.25)


QCONFIGS = [_qconfig(np.random.default_rng(8000 + k)) for k in range(8)]


@pytest.mark.parametrize("k", range(len(QCONFIGS)))
def test_random_qmetric_configuration(K, k):
    """Random q-metric images on the coloured sphere: fates by the boundary
    rule, escape directions to 1e-9 where the sky codes are away from code
    boundaries."""
    import torch
    p = QCONFIGS[k]
    nx, ny = p["nx"], p["ny"]
    print(f"[gpu-case] random q-metric config {k}: {p}", flush=True)
    sys.stdout.flush()
    out = K.Renderer(device="cuda:0", **p).render()
    torch.cuda.synchronize()
    g = {key: v.cpu().numpy() for key, v in out.items() if key != "stats"}
    o = O.trace_pixels(O.Setup(**p))
    P.check_fates(g["fate"], o["fate"], nx, ny, min_allowed=2)
    esc = (g["fate"] == K.ESCAPED) & (o["fate"] == O.ESCAPED) & ~P.boundary_mask(o["fate"].reshape(ny, nx)).ravel()

    def dirs(th, ph):
        return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)
    if esc.any():
        d = np.linalg.norm(dirs(g["theta_f"][esc], g["phi_f"][esc]) - dirs(o["theta_f"][esc], o["phi_f"][esc]),
                           axis=1)
        tol = 1e-9 if p["method"] != K.BS else 1e-7
        assert d.max() < tol, (d.max(), p["method"])
