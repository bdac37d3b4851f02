"""Pins of the oracle's thin-disk event location and observables (Sect. 5).

- Schwarzschild: the radius where a pixel's ray meets the equatorial plane
  for the (n_cross+1)-th time comes from the orbit quadrature;
- the redshift of a Keplerian emitter has a closed form for a = 0, and the
  observed intensity is g^3 I_em with I_em = (M/r)^2;
- flat space: the disk hit is a straight-line / plane intersection.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests import schwarzschild_quad as SQ


def c3_setup(n=2048):
    return O.Setup(a=0.0, r_obs=1000.0, incl=math.radians(80), fov_x=35.0, fov_y=35.0, nx=n, ny=n,
                   method=O.DP45, rtol=1e-12, atol=1e-12, disk_on=1, r_in=6.0, r_out=30.0, emis_q=2.0)


def test_disk_hits_vs_quadrature():
    s = c3_setup()
    rng = np.random.default_rng(11)
    # the disk's image at i = 80 deg lies within |y| < 10M: sample that band
    rows = rng.integers(731, 1317, size=500)
    cols = rng.integers(0, 2048, size=500)
    pix = np.unique(rows * 2048 + cols).astype(np.int32)
    o = O.trace_pixels(s, pix)
    checked = 0
    for k, p in enumerate(pix):
        x, y = O.pixel_xy(s, int(p % 2048), int(p // 2048))
        rho = math.hypot(x, y)
        b = SQ.impact_parameter(rho, 1000.0)
        if abs(b - SQ.B_CRIT) < 0.05:
            continue  # near-critical: many windings, chaotic
        radii = []
        for psi in SQ.equator_crossing_angles(x, y, s.incl, n=4):
            r = SQ.radius_at_swept_angle(b, 1000.0, psi)
            if r is None or r > 1100.0:
                break
            radii.append(r)
        # the expected fate: the first crossing inside [r_in, r_out]
        want_fate, want_k, want_r = None, None, None
        for kk, r in enumerate(radii):
            if 6.0 <= r <= 30.0:
                want_fate, want_k, want_r = O.DISK, kk, r
                break
        if any(min(abs(r - 6.0), abs(r - 30.0)) < 1e-6 for r in radii):
            continue
        if want_fate is None:
            assert o["fate"][k] in (O.ESCAPED, O.CAPTURED), (x, y, radii)
            assert o["n_cross"][k] == len(radii) or o["fate"][k] == O.CAPTURED
            continue
        checked += 1
        assert o["fate"][k] == O.DISK, (x, y, radii)
        assert o["n_cross"][k] == want_k
        assert o["r_hit"][k] == pytest.approx(want_r, rel=1e-9)
    assert checked > 150


def test_redshift_closed_form():
    """a = 0: g = sqrt(1 - 3M/r) / (sqrt(1 - 2M/r0) + x sin(i) sqrt(M/r^3)),
    evaluated at the oracle's own hit radius; I = g^3 (M/r)^2."""
    s = c3_setup(256)
    o = O.trace_pixels(s)
    hit = np.flatnonzero(o["fate"] == O.DISK)
    assert hit.size > 5000
    i = hit % 256
    x = -35.0 + (i + 0.5) * (70.0 / 256)
    r = o["r_hit"][hit]
    g = np.sqrt(1 - 3 / r) / (math.sqrt(1 - 2 / 1000.0) + x * math.sin(s.incl) * np.sqrt(1 / r ** 3))
    np.testing.assert_allclose(o["g"][hit], g, rtol=1e-13)
    np.testing.assert_allclose(o["intensity"][hit], g ** 3 / r ** 2, rtol=1e-13)
    # the approaching side (x < 0 with this orientation) is blueshifted
    assert o["g"][hit][x < -15].mean() > o["g"][hit][x > 15].mean()
    # non-disk rays carry no disk observables
    miss = o["fate"] != O.DISK
    assert np.isnan(o["r_hit"][miss]).all() and (o["intensity"][miss] == 0).all()


def test_kerr_redshift_closed_form():
    """Kerr: g = sqrt(-g_tt - 2 Om g_tph - Om^2 g_phph)|_(r, pi/2) / (E - Om L)
    with E, L of the pixel and Om the prograde Keplerian rate."""
    a = 0.9
    s = O.Setup(a=a, r_obs=1000.0, incl=math.radians(60), fov_x=20, fov_y=20, nx=24, ny=24,
                method=O.DP45, disk_on=1, r_in=2.320883, r_out=30.0)
    o = O.trace_pixels(s)
    hit = np.flatnonzero(o["fate"] == O.DISK)
    assert hit.size > 50
    for p in hit:
        x, y = O.pixel_xy(s, int(p % 24), int(p // 24))
        st, _ = O.camera_ray(1.0, a, 1000.0, s.incl, x, y)
        E, L = st[5], st[6]
        r = o["r_hit"][p]
        # metric at the equator, written out directly
        gtt, gtp, gpp = -(1 - 2 / r), -2 * a / r, r * r + a * a + 2 * a * a / r
        Om = 1 / (r ** 1.5 + a)
        g = math.sqrt(-gtt - 2 * Om * gtp - Om * Om * gpp) / (E - Om * L)
        assert o["g"][p] == pytest.approx(g, rel=1e-12)


def test_flat_space_disk_is_plane_intersection():
    """M = 0: the hit radius is where the straight camera ray meets z = 0."""
    r0, incl = 200.0, math.radians(70)
    s = O.Setup(M=0.0, a=0.0, r_obs=r0, incl=incl, method=O.DP45, disk_on=1, r_in=1.0,
                r_out=100.0, cap_buffer=-1.0)
    rng = np.random.default_rng(5)
    xs, ys = rng.uniform(-40, 40, 50), rng.uniform(-40, 40, 50)
    o = O.trace_xy(s, xs, ys)
    nobs = np.array([math.sin(incl), 0, math.cos(incl)])
    eth = np.array([math.cos(incl), 0, -math.sin(incl)])
    eph = np.array([0.0, 1.0, 0.0])
    for k, (x, y) in enumerate(zip(xs, ys)):
        d = -math.sqrt(1 - (x * x + y * y) / r0 ** 2) * nobs + (y / r0) * eth - (x / r0) * eph
        P0 = r0 * nobs
        t = -P0[2] / d[2]
        if t <= 0:
            assert o["fate"][k] == O.ESCAPED
            continue
        rh = np.linalg.norm((P0 + t * d)[:2])
        if 1.0 <= rh <= 100.0:
            assert o["fate"][k] == O.DISK
            assert o["r_hit"][k] == pytest.approx(rh, rel=1e-10)
        else:
            assert o["fate"][k] == O.ESCAPED
