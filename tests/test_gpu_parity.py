"""GPU library vs CPU oracle, element by element, through the C ABI.

Every test prints the case it runs (and flushes) before touching the GPU.
Sizes are small enough for the oracle to finish in seconds while spanning
many waves and a ragged tail; the full-size image is checked on a sampled
set of pixels the oracle traces one by one.
"""
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


def gpu_render(K, params, launch=None, want=None):
    import torch
    r = K.Renderer(device="cuda:0", launch=launch, **params) if want is None else \
        K.Renderer(device="cuda:0", launch=launch, want=want, **params)
    out = r.render()
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items() if k != "stats"}
    res["stats"] = K.read_stats(out)
    return res


def ora_render(params, pix=None):
    return O.trace_pixels(O.Setup(**params), pix)


# ---------------------------------------------------------------------------

def test_init_rays_match_oracle(K):
    import torch
    for params in [W.kerr_ring(0.9, n=64), W.schwarzschild_disk(n=37), W.schwarzschild_shadow_64(),
                   dict(W.kerr_ring(0.998, n=16), r_obs=40.0, fov_x=45.0, fov_y=45.0)]:
        _announce("init_rays", params["a"], params["nx"], params["r_obs"])
        state, invalid = K.init_rays(**params)
        torch.cuda.synchronize()
        st = state.cpu().numpy()
        inv = invalid.cpu().numpy()
        s = O.Setup(**params)
        for p in range(params["nx"] * params["ny"]):
            x, y = O.pixel_xy(s, p % params["nx"], p // params["nx"])
            want, bad = O.camera_ray(params["M"], params["a"], params["r_obs"], params["incl"], x, y)
            assert bool(inv[p]) == bad
            if not bad:
                # r, theta, phi exact; momenta and E, L within a few ulp (the
                # library folds the camera metric into per-image constants)
                np.testing.assert_array_equal(st[:3, p], want[:3])
                np.testing.assert_allclose(st[3:, p], want[3:], rtol=4e-15, atol=4e-16 * np.abs(want[3:]).max())


def test_schwarzschild_shadow_64(K):
    """a = 0, 64x64, fixed-step RK4 in s: identical fates (872 captured) and
    max |H| agreement with the oracle."""
    params = W.schwarzschild_shadow_64()
    _announce("schwarzschild_shadow_64")
    g = gpu_render(K, params)
    o = ora_render(params)
    np.testing.assert_array_equal(g["fate"], o["fate"])
    assert (g["fate"] == K.CAPTURED).sum() == 872
    np.testing.assert_array_equal(g["n_steps"], o["n_steps"])
    mask = np.ones(64 * 64, bool)
    P.check_max_h(g, o, "max_abs_h", mask)
    P.check_max_h(g, o, "max_rel_h", mask)
    assert g["stats"].rays == 4096
    assert list(g["stats"].fate_count[:6]) == list(np.bincount(g["fate"], minlength=6)[:6])
    assert g["stats"].evals == g["n_evals"].sum()


@pytest.mark.parametrize("a", [0.5, 0.9, 0.998])
def test_kerr_ring_128(K, a):
    """Kerr shadow + deflection diagnostics, i = 60 deg, +-12M at 128x128."""
    params = W.kerr_ring(a, n=128)
    _announce("kerr_ring_128", a)
    g = gpu_render(K, params)
    o = ora_render(params)
    P.check_fates(g["fate"], o["fate"], 128, 128)
    m = P.value_mask(g, o, 128, 128)
    assert m.sum() > 0.9 * 128 * 128
    P.check_values(g, o, "deflection", m, rtol=1e-8)
    P.check_values(g, o, "psi", m & (o["psi"] > 1e-6), rtol=1e-7)
    # scale-free residual on every ray against the target's budget; the
    # absolute one only on escaped rays: for captured rays p_r ~ 1/Delta and
    # |H| at the last step depends on how far inside r_+ + 0.01 it lands
    P.check_max_h(g, o, "max_rel_h", m, budget=1e-10)
    P.check_max_h(g, o, "max_abs_h", m & (o["fate"] == O.ESCAPED), budget=1e-10)
    # ring flags follow the same rule as the oracle's post-pass
    np.testing.assert_array_equal(g["ring"], O.ring_flags(128, 128, g["deflection"]))
    steps_rel = np.abs(g["n_steps"][m].astype(float) - o["n_steps"][m]) / o["n_steps"][m]
    assert np.median(steps_rel) == 0.0 and steps_rel.max() < 0.02


@pytest.mark.parametrize("case", ["schw_80", "kerr_60"])
def test_disk_images(K, case):
    """Thin Keplerian disk: hit radius, redshift and intensity."""
    if case == "schw_80":
        params = W.schwarzschild_disk(n=160)
    else:
        params = W.kerr_disk(a=0.9, incl_deg=60.0, n=128, r_in=2.320883)
    _announce("disk", case)
    g = gpu_render(K, params)
    o = ora_render(params)
    n = params["nx"]
    P.check_fates(g["fate"], o["fate"], n, n)
    m = P.value_mask(g, o, n, n)
    disk = m & (o["fate"] == O.DISK)
    assert disk.sum() > 0.1 * n * n
    for key in ("r_hit", "g", "intensity", "theta_f", "phi_f"):
        P.check_values(g, o, key, disk, rtol=1e-8)
    np.testing.assert_array_equal(g["n_cross"][m], o["n_cross"][m])
    nd = ~np.isin(g["fate"], [O.DISK])
    assert np.isnan(g["r_hit"][nd]).all() and (g["intensity"][nd] == 0).all()
    # image order histogram of the disk pixels (primary, secondary, ...)
    hg = np.bincount(g["n_cross"][g["fate"] == O.DISK], minlength=3)[:3]
    ho = np.bincount(o["n_cross"][o["fate"] == O.DISK], minlength=3)[:3]
    assert np.abs(hg - ho).max() <= max(2, int(1e-3 * n * n)), (hg, ho)


def test_ragged_and_tiny_images(K):
    for nx, ny in [(1, 1), (37, 23), (65, 3), (3, 129)]:
        params = dict(W.kerr_ring(0.7, n=8), nx=nx, ny=ny)
        _announce("ragged", nx, ny)
        g = gpu_render(K, params)
        o = ora_render(params)
        P.check_fates(g["fate"], o["fate"], nx, ny, min_allowed=1)
        m = P.value_mask(g, o, nx, ny)
        P.check_values(g, o, "deflection", m, rtol=1e-8)


def test_launch_shapes_are_bit_identical(K):
    """Per-ray arithmetic does not depend on which lane or wave runs the ray:
    persistent / one-ray-per-lane / queue batch 1 / small blocks, both
    dispatch orders and both builds of the kernels (2 and 3 waves per SIMD)
    give bit-identical outputs (the default is ring-first order; every pixel
    must still be traced exactly once)."""
    params = dict(W.kerr_ring(0.9, n=96), disk_on=1, r_in=2.320883, r_out=30.0)
    _announce("launch shapes")
    base = gpu_render(K, params)
    # the last three ask for 3 waves per SIMD: the 3-wave build of the kernels
    shapes = [K.kt_launch(0, 256, 0, 32), K.kt_launch(1, 64, 1, 1), K.kt_launch(1, 128, 2, 7),
              K.kt_launch(1, 256, 1, 4096), K.kt_launch(1, 256, 0, 32, K.ORDER_ROWS),
              K.kt_launch(0, 64, 0, 32, K.ORDER_ROWS), K.kt_launch(1, 256, 3, 4), K.kt_launch(1, 128, 6, 1),
              K.kt_launch(1, 256, 3, 16, K.ORDER_ROWS)]
    for ln in shapes:
        _announce("launch", ln.persistent, ln.block, ln.blocks_per_cu, ln.batch, ln.order)
        g = gpu_render(K, params, launch=ln)
        for key, v in base.items():
            if key == "stats":
                assert g[key].evals == v.evals
                continue
            np.testing.assert_array_equal(g[key].view(np.uint8), v.view(np.uint8), err_msg=key)


def test_small_render_ticket_fetches(K):
    """A 512x512 disk image has 2 rays per lane of the default grid, so each
    wave's first fetch of 64 ids covers half of it.  The default launch,
    ticket batches 1 and 16 after that fetch, and one ray per lane without
    refill give the same outputs bit for bit, and every pixel is traced once."""
    params = W.differentiable_disk(n=512)
    want = ("fate", "r_hit", "g", "intensity", "n_cross", "n_steps", "n_evals", "max_rel_h")
    _announce("ticket fetches at 512x512")
    base = gpu_render(K, params, want=want)
    assert base["stats"].rays == 512 * 512 and sum(base["stats"].fate_count) == 512 * 512
    assert base["stats"].evals == int(base["n_evals"].astype(np.int64).sum())
    for ln in (K.kt_launch(1, 256, 0, 1), K.kt_launch(1, 256, 0, 16), K.kt_launch(0, 256, 0, 4)):
        _announce("launch", ln.persistent, ln.block, ln.blocks_per_cu, ln.batch)
        g = gpu_render(K, params, launch=ln, want=want)
        assert g["stats"].evals == base["stats"].evals
        for key, v in base.items():
            if key != "stats":
                np.testing.assert_array_equal(g[key].view(np.uint8), v.view(np.uint8), err_msg=key)


@pytest.mark.parametrize("a", [0.0, 0.9])
def test_higher_order_disk_images(K, a):
    """Disk images of order 2 and more (rays that cross the equatorial plane
    twice outside the disk before they hit it, winding round the photon
    sphere), which the value checks elsewhere leave out: the 80-degree disk
    from 6M to 30M around a Schwarzschild and an a = 0.9 Kerr hole, over
    +-7M at 4096x4096 (0.0034M pixels: the order-2 ring is a few pixels
    wide).  600 sampled order >= 2 pixels with their
    neighbourhoods against the oracle: fates under the boundary rule, and
    r_hit, g and I, where fate and order agree and no boundary is near,
    under the rounding rule (each pixel within max(1e-8, 10 S, 2 s_p), s_p
    the oracle's own one-ulp sensitivity there and S its 99.9th
    percentile)."""
    n = 4096
    params = dict(W.schwarzschild_disk(n=n), a=a, fov_x=7.0, fov_y=7.0)
    _announce("higher-order disk images", n, "+-7M, a =", a)
    img = gpu_render(K, params, want=("fate", "n_cross", "r_hit", "g", "intensity"))
    cand = np.flatnonzero((img["fate"] == O.DISK) & (img["n_cross"] >= 2))
    assert cand.size > 1000
    rng = np.random.default_rng(4096)
    sample = np.sort(rng.choice(cand, 600, replace=False)).astype(np.int64)
    s = O.Setup(**params)
    o, stats, ok = P.sampled_parity(img, n, n, sample, lambda pix: O.trace_pixels(s, pix), max_order=255)
    assert ok.sum() > 100, stats
    pix = sample[ok]
    xy = np.array([O.pixel_xy(s, int(p % n), int(p // n)) for p in pix])
    res = {}
    for key in ("r_hit", "g", "intensity"):
        sens = P.ulp_sensitivity(lambda x, y: O.trace_xy(s, x, y), xy[:, 0].copy(), xy[:, 1].copy(), key)
        res[key] = P.check_values_rounding({key: img[key][pix]}, {key: o[key][ok]}, key,
                                           np.ones(pix.size, bool), sens)
    print(f"[higher-order images] {stats}; max rel err and the oracle's p99.9 one-ulp sensitivity {res}",
          flush=True)


def test_launch_statistics_trace_time(K):
    """kt_stats.trace_ms, two readings of the device's wall clock enqueued
    just before the first trace launch and just after the last, lies within
    the render's HIP-event time (which also holds the dispatch sort and the
    post-passes) and covers most of it; a mixed render's covers both passes."""
    import torch
    for prec in (K.FP64, K.MIXED):
        params = dict(W.kerr_ring(0.9, n=512), precision=prec)
        _announce("trace time statistic", prec)
        r = K.Renderer(device="cuda:0", **params)
        r.render()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        r.render()
        b.record()
        torch.cuda.synchronize()
        ev = a.elapsed_time(b)
        st = K.read_stats(r.out)
        print(f"[stats] precision {prec}: trace_ms {st.trace_ms:.3f}, HIP events {ev:.3f} ms", flush=True)
        assert 0.0 < st.trace_ms <= 1.02 * ev + 0.02
        assert st.trace_ms >= 0.8 * ev - 0.2


def test_max_steps_forces_fate(K):
    params = dict(W.kerr_ring(0.9, n=32), max_steps=10)
    _announce("max_steps=10")
    g = gpu_render(K, params)
    assert (g["fate"] == K.MAXSTEPS).all()
    assert (g["n_steps"] == 10).all()
    o = ora_render(params)
    np.testing.assert_array_equal(g["n_steps"], o["n_steps"])


def test_invalid_pixels(K):
    """Image-plane points with x^2 + y^2 >= r0^2 have no real p_r."""
    params = dict(W.kerr_ring(0.5, n=16), r_obs=20.0, fov_x=25.0, fov_y=25.0, r_escape=30.0, r_src=25.0)
    _announce("invalid pixels")
    g = gpu_render(K, params)
    o = ora_render(params)
    np.testing.assert_array_equal(g["fate"] == K.INVALID, o["fate"] == O.INVALID)
    assert (g["fate"] == K.INVALID).sum() > 0


@pytest.mark.parametrize("a", [0.9, 0.5, 0.998])
def test_full_size_kerr_ring_rows(K, a):
    """1024x1024 at each spin of the workload, in the launch configuration the
    benchmark times: every pixel of rows j = 0 mod 16 (65,536 rays) against
    the oracle, with the oracle's own 3x3 neighbourhood wherever a boundary
    can lie, under the parity rules (fate mismatches only next to a
    boundary and at most 0.1% of the sample; deflection to 1e-8, the angle to
    the source to 1e-7 where it exceeds 1e-6)."""
    params = W.kerr_ring(a, n=1024)
    _announce("kerr_ring_1024 rows j%16==0", a)
    g = gpu_render(K, params)
    sample = P.row_sample(1024, 1024, 16)
    o, st_p, ok = P.sampled_parity(g, 1024, 1024, sample, lambda pix: ora_render(params, pix),
                                   keys=("deflection", "psi"), extra_rtol={"psi": (1e-7, 1e-6)})
    print(f"[kerr_ring_1024 a={a}] {st_p}", flush=True)
    assert st_p["deflection"]["n"] > 40000
    gs = {k: g[k][sample] for k in ("max_rel_h", "max_abs_h")}
    P.check_max_h(gs, o, "max_rel_h", ok, budget=1e-10)
    st = g["stats"]
    assert st.rays == 1024 * 1024 and sum(st.fate_count) == 1024 * 1024
    assert st.evals == g["n_evals"].astype(np.int64).sum()
    assert (g["fate"] <= K.DISK).all()
    # the constraint: DP45 at rtol 1e-12 keeps |H|_rel near 1e-11; the single
    # worst ray of the image is traced by the oracle too, whose value must be
    # of the same size (the method's, not the kernel's)
    h = g["max_rel_h"]
    assert np.nanpercentile(h, 99.9) < 1e-10
    worst = int(np.nanargmax(h))
    ow = ora_render(params, np.array([worst], np.int32))
    print(f"[kerr_ring_1024 a={a}] worst |H|_rel {h[worst]:.3e} at pixel {worst}; oracle {ow['max_rel_h'][0]:.3e}",
          flush=True)
    assert h[worst] < 2e-10 and ow["max_rel_h"][0] < 2e-10
    assert 0.5 < h[worst] / ow["max_rel_h"][0] < 2.0
    if a == 0.9:
        assert h[worst] < 1e-10  # the benchmarked image meets the budget everywhere


def test_full_size_schwarzschild_disk_rows(K):
    """2048x2048 Schwarzschild disk (i = 80 deg, 6..30M, +-35M) at full size
    in the default launch: every pixel of rows j = 0 mod 16 (131,072 rays)
    against the oracle under the parity rules (hit radius, redshift and
    intensity to 1e-8 away from fate and image-order boundaries); the mixed
    form at budget 1e-10 keeps every ray within budget and its FP64 re-runs
    equal the FP64 render bit for bit."""
    n = 2048
    params = W.schwarzschild_disk(n=n)
    _announce("schwarzschild_disk_2048 rows j%16==0")
    g = gpu_render(K, params)
    sample = P.row_sample(n, n, 16)
    o, st_p, ok = P.sampled_parity(g, n, n, sample, lambda pix: ora_render(params, pix),
                                   keys=("r_hit", "g", "intensity"))
    print(f"[disk 2048] {st_p}", flush=True)
    assert st_p["r_hit"]["n"] > 20000
    P.check_max_h({"max_rel_h": g["max_rel_h"][sample]}, o, "max_rel_h", ok, budget=1e-10)
    st = g["stats"]
    assert st.rays == n * n and sum(st.fate_count) == n * n
    assert np.nanmax(g["max_rel_h"]) < 1e-10
    _announce("schwarzschild_disk_2048 mixed 1e-10")
    m = gpu_render(K, dict(params, precision=K.MIXED, h_budget=1e-10, r_switch=300.0))
    assert np.nanmax(m["max_rel_h"]) <= 1e-10
    re = m["used_fp64"].astype(bool)
    for key in ("fate", "r_hit", "g", "intensity", "max_rel_h", "n_steps"):
        np.testing.assert_array_equal(m[key][re].view(np.uint8), g[key][re].view(np.uint8), err_msg=key)
    P.check_fates(m["fate"], g["fate"], n, n)
    print(f"[disk 2048 mixed] re-run fraction {re.mean():.4f}", flush=True)


# ---------------------------------------------------------------------------
# Mixed precision: FP32 mass part of the RHS beyond r_switch, FP64 re-run of
# every ray over the |H|_rel budget.
# ---------------------------------------------------------------------------

_BITWISE_KEYS = ("fate", "max_abs_h", "max_rel_h", "psi", "deflection", "theta_f", "phi_f", "n_cross",
                 "n_steps", "r_hit", "g", "intensity", "ring")


def test_mixed_zero_budget_equals_fp64(K):
    """h_budget = 0 sends every ray that used the FP32 part back to the FP64
    pass; rays that never used it ran the FP64 code already.  So every
    output equals the plain FP64 render bit for bit."""
    params = dict(W.kerr_ring(0.9, n=96), disk_on=1, r_in=2.320883, r_out=30.0)
    _announce("mixed budget 0")
    ref = gpu_render(K, params)
    g = gpu_render(K, dict(params, precision=K.MIXED, h_budget=0.0, r_switch=300.0))
    for key in _BITWISE_KEYS:
        np.testing.assert_array_equal(g[key].view(np.uint8), ref[key].view(np.uint8), err_msg=key)
    # the same through the 3-wave build of the kernels (3 waves per SIMD)
    g3 = gpu_render(K, dict(params, precision=K.MIXED, h_budget=0.0, r_switch=300.0),
                    launch=K.kt_launch(1, 256, 3, 4))
    for key in _BITWISE_KEYS:
        np.testing.assert_array_equal(g3[key].view(np.uint8), ref[key].view(np.uint8), err_msg="w3 " + key)
    st = g["stats"]
    assert st.evals_fp32 > 0
    assert st.fallback_rays == int(g["used_fp64"].sum()) > 0
    assert st.evals > ref["stats"].evals


def test_mixed_without_fallback_error_is_bounded(K):
    """No re-run (budget = inf): the FP32 mass part's error, stated against
    the FP64 oracle.  Fates keep the FP64 parity rule; located quantities
    agree to 1e-6."""
    params = W.kerr_ring(0.9, n=64)
    _announce("mixed no fallback")
    g = gpu_render(K, dict(params, precision=K.MIXED, h_budget=1e300, r_switch=300.0))
    o = ora_render(params)
    assert g["stats"].fallback_rays == 0 and (g["used_fp64"] == 0).all()
    assert g["stats"].evals_fp32 > 0.05 * g["stats"].evals
    P.check_fates(g["fate"], o["fate"], 64, 64)
    m = P.value_mask(g, o, 64, 64)
    e = P.rel_err(g["deflection"][m], o["deflection"][m])
    e = e[np.isfinite(e)]
    print(f"[mixed no fallback] deflection rel err max {e.max():.2e} p99 {np.percentile(e, 99):.2e}; "
          f"max |H|_rel {np.nanmax(g['max_rel_h']):.2e}", flush=True)
    assert e.max() < 1e-6


def test_mixed_default_budget(K):
    """Budget 1e-10: every ray ends within the budget, and FP64 parity holds
    for every output under the FP64 rules."""
    params = W.kerr_ring(0.9, n=96)
    _announce("mixed budget 1e-10")
    g = gpu_render(K, dict(params, precision=K.MIXED, h_budget=1e-10, r_switch=300.0))
    o = ora_render(params)
    assert np.nanmax(g["max_rel_h"]) <= 1e-10
    P.check_fates(g["fate"], o["fate"], 96, 96)
    m = P.value_mask(g, o, 96, 96)
    kept = m & (g["used_fp64"] == 0)
    if kept.any():
        e = P.rel_err(g["deflection"][kept], o["deflection"][kept])
        e = e[np.isfinite(e)]
        print(f"[mixed 1e-10] fallback {g['used_fp64'].mean():.3f}; kept-mixed deflection rel err "
              f"max {e.max() if e.size else 0:.2e}", flush=True)
    P.check_values(g, o, "deflection", m & (g["used_fp64"] == 1), rtol=1e-8)


def test_polar_rays_wind_through_the_axis(K):
    """A one-column image (x = 0, so L = 0): these rays cross the polar axis
    and theta leaves [0, pi]; the kernel must switch to the range-reduced
    sin/cos for those steps."""
    for a in (0.0, 0.9):
        params = dict(W.kerr_ring(a, n=8), nx=1, ny=41, fov_x=5.0)
        _announce("polar column", a)
        g = gpu_render(K, params)
        o = ora_render(params)
        np.testing.assert_array_equal(g["fate"], o["fate"])
        m = np.isfinite(o["deflection"])
        e = P.rel_err(g["deflection"][m], o["deflection"][m])
        assert e.max() < 1e-8, e.max()
        # the rays really do leave [0, pi]
        s = O.Setup(**params)
        tr, _ = O.trace_one(s, 0.0, O.pixel_xy(s, 0, 30)[1])
        assert tr[:, 2].min() < 0.0 or tr[:, 2].max() > math.pi


@pytest.mark.parametrize("a", [1.0, -1.0])
def test_extremal_spin(K, a):
    """|a| = M, where the horizon and the co-rotating photon orbit meet at
    r = M.  One equatorial row (i = 90 deg, y = 0, 4096 pixels over +-8M):
    every pixel has the fate of the closed-form edges in b = L/E (the
    capture buffer sets the co-rotating one at b = 2M + 0.01M, the
    counter-rotating photon orbit the other at -7M) and the oracle's, and
    the pixels between b = 2M and 2M + 0.01M are captured.  Then a 96x96
    ring image at i = 60 deg against the oracle under the parity rules."""
    from tests.test_oracle_shadow import extremal_edges
    row = dict(W.kerr_ring(a, n=8), incl=math.pi / 2, fov_x=8.0, fov_y=8.0, nx=4096, ny=1)
    _announce("extremal spin row", a)
    g = gpu_render(K, row)
    o = ora_render(row)
    s = O.Setup(**row)
    b = np.empty(4096)
    for i in range(4096):
        x, y = O.pixel_xy(s, i, 0)
        assert y == 0.0
        st, _ = O.camera_ray(1.0, a, row["r_obs"], row["incl"], x, y)
        b[i] = st[6] / st[5]
    lo, hi = extremal_edges(a)
    want = np.where((b > lo) & (b < hi), O.CAPTURED, O.ESCAPED)
    np.testing.assert_array_equal(o["fate"], want)
    np.testing.assert_array_equal(g["fate"], want)
    band = (np.abs(b) > 2.0) & (np.abs(b) < 2.01)
    assert band.sum() >= 2 and (g["fate"][band] == O.CAPTURED).all()
    esc = want == O.ESCAPED
    P.check_values(g, o, "deflection", esc, rtol=1e-8)

    params = W.kerr_ring(a, n=96)
    _announce("extremal spin image", a)
    g = gpu_render(K, params)
    o = ora_render(params)
    P.check_fates(g["fate"], o["fate"], 96, 96)
    m = P.value_mask(g, o, 96, 96)
    assert m.sum() > 0.9 * 96 * 96
    P.check_values(g, o, "deflection", m, rtol=1e-8)
    P.check_values(g, o, "psi", m & (o["psi"] > 1e-6), rtol=1e-7)
    # every ray within the 1e-10 budget on both sides; the distributions are
    # compared on escaped rays only: at the capture radius of an extremal
    # hole (Delta = (r - M)^2 ~ 1e-4) the oracle's numerically inverted
    # t-phi block puts relative rounding of ~eps (r^2 + a^2)^2 / Delta into
    # its |H|_rel, above the truncation residues that the percentiles compare
    assert (g["max_rel_h"][m] <= 1e-10).all() and (o["max_rel_h"][m] <= 1e-10).all()
    P.check_max_h(g, o, "max_rel_h", m & (o["fate"] == O.ESCAPED), budget=1e-10)
    np.testing.assert_array_equal(g["ring"], O.ring_flags(96, 96, g["deflection"]))


def test_resolved_einstein_ring(K):
    """a = 0, i = 60 deg, +-60M at 256x256, so that the primary Einstein ring
    of the source behind the hole (image radius 46.188M by the orbit
    quadrature) is resolved: every pixel against the oracle under the
    parity rules (deflection to 1e-8), the ring flags equal the oracle's
    flags of its own deflection map away from the shadow edge, and every
    flag lies within one pixel of a quadrature ring radius, all around the
    primary ring."""
    from tests import schwarzschild_quad as SQ
    n, fov = 256, 60.0
    params = dict(W.kerr_ring(0.0, n=n), fov_x=fov, fov_y=fov)
    _announce("resolved ring", n, fov)
    g = gpu_render(K, params)
    o = ora_render(params)
    P.check_fates(g["fate"], o["fate"], n, n)
    m = P.value_mask(g, o, n, n)
    P.check_values(g, o, "deflection", m, rtol=1e-8)
    dx = 2 * fov / n
    x = -fov + (np.arange(n) + 0.5) * dx
    rho = np.hypot(x[None, :], x[:, None]).ravel()
    radii = np.array(SQ.einstein_ring_radii())
    ring_o = O.ring_flags(n, n, o["deflection"])
    away = rho > radii[1] + 2 * dx
    np.testing.assert_array_equal(g["ring"][away], ring_o[away])
    flagged = g["ring"].astype(bool)
    dist = np.abs(rho[:, None] - radii[None, :]).min(1)
    assert (dist[flagged] <= dx * (1 + 1e-9)).all(), dist[flagged].max() / dx
    ang = np.degrees(np.arctan2(np.repeat(x, n), np.tile(x, n)))
    prim = flagged & (np.abs(rho - radii[0]) <= dx)
    assert np.unique(((ang[prim] + 180.0) // 5).astype(int)).size == 72
    print(f"[resolved ring] {prim.sum()} primary-ring flags, {flagged.sum()} in all", flush=True)


def test_mixed_event_location_keeps_its_precision(K):
    """Mixed precision with disk crossings and the source sphere beyond
    r_switch (r_switch = 10M, disk 6..30M at i = 80 deg, source at 1000M, no
    re-run): a lane locating an event and retaking the step keeps the
    precision of the step the event lay in, so the retake reproduces it and
    no crossing is counted twice.  Image orders and fates follow the FP64
    render under the parity rules (FP32 rounding only moves rays near
    boundaries), and the deflection stays within the FP32 part's error."""
    n = 96
    params = dict(W.schwarzschild_disk(n=n), src_on=1, r_src=1000.0)
    _announce("mixed event precision", n)
    ref = gpu_render(K, params)
    g = gpu_render(K, dict(params, precision=K.MIXED, h_budget=1e300, r_switch=10.0))
    assert g["stats"].evals_fp32 > 0.05 * g["stats"].evals
    P.check_fates(g["fate"], ref["fate"], n, n)
    near = (P.boundary_mask(ref["fate"].reshape(n, n)) | P.boundary_mask(ref["n_cross"].reshape(n, n))).ravel()
    same = (g["fate"] == ref["fate"]) & ~near
    np.testing.assert_array_equal(g["n_cross"][same], ref["n_cross"][same])
    # at rtol 1e-12 the FP32 part's rounding shows in the error estimate
    # close in (r_switch = 10M), so the controller takes more steps there
    d = g["n_steps"][same].astype(np.int64) - ref["n_steps"][same]
    m = same & np.isfinite(ref["deflection"])
    e = P.rel_err(g["deflection"][m], ref["deflection"][m])
    print(f"[mixed events] FP32 share {g['stats'].evals_fp32 / g['stats'].evals:.3f}; deflection rel err "
          f"max {e.max():.2e}; extra steps median {np.median(d):.0f}, p99 {np.percentile(d, 99):.0f}",
          flush=True)
    assert e.max() < 1e-5
