"""Pins of the oracle's celestial sphere (Sect. 4.1) and of the disk rotation
with constant specific angular momentum (Sect. 5).

- Minkowski (M = 0): rays are straight lines from the camera, so the point
  where each meets the sphere r = r_cs is the root of a quadratic;
- Schwarzschild equatorial rays: the longitude where the ray meets the
  sphere is minus the orbit quadrature's swept angle (x > 0 gives L < 0);
- sky codes do not depend on how a direction is written (theta outside
  [0, pi] after polar crossings, phi shifted by 2 pi), and follow the
  quadrant table of the celestial-sphere figure;
- constant-l0 rotation: Omega has the Schwarzschild closed form
  l0 (1 - 2M/r) / r^2, and equals the Keplerian Omega when l0 is the
  Keplerian specific angular momentum at that radius.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests import schwarzschild_quad as SQ


def _lensing_setup(M=1.0, a=0.0, n=32, fov=20.0, r0=100.0):
    return O.Setup(M=M, a=a, r_obs=r0, incl=math.pi / 2, fov_x=fov, fov_y=fov, nx=n, ny=n,
                   method=O.DP45, rtol=1e-12, atol=1e-12, r_escape=1.1 * r0, sky_on=1)


def _canonical(theta, phi):
    n = np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)])
    return n


def test_minkowski_exit_point_is_a_straight_line():
    s = _lensing_setup(M=0.0, n=24)
    o = O.trace_pixels(s)
    r0, rcs, inc = s.r_obs, 1.1 * s.r_obs, s.incl
    er = np.array([math.sin(inc), 0.0, math.cos(inc)])
    et = np.array([math.cos(inc), 0.0, -math.sin(inc)])
    ep = np.array([0.0, 1.0, 0.0])
    worst = 0.0
    for p in range(24 * 24):
        x, y = O.pixel_xy(s, p % 24, p // 24)
        pr = -math.sqrt(1.0 - (x * x + y * y) / r0 ** 2)
        d = pr * er + (y / r0) * et + (-x / r0) * ep          # unit direction, backward in time
        lam = -r0 * pr + math.sqrt(r0 * r0 * pr * pr - r0 * r0 + rcs * rcs)
        X = r0 * er + lam * d
        want = X / np.linalg.norm(X)
        got = _canonical(o["theta_f"][p], o["phi_f"][p])
        assert o["fate"][p] == O.ESCAPED
        worst = max(worst, np.linalg.norm(got - want))
        assert o["sky"][p] == O.sky_code(math.acos(want[2]), math.atan2(want[1], want[0]), s.grid_deg,
                                         s.line_deg)
    assert worst < 1e-10, worst


@pytest.mark.parametrize("b", [6.0, 8.0, 12.0, 20.0])
def test_schwarzschild_equatorial_exit_longitude(b):
    r0 = 100.0
    s = _lensing_setup(M=1.0, n=8, r0=r0)
    x = b * math.sqrt(1.0 - 2.0 / r0)  # image radius of impact parameter b
    tr, res = O.trace_one(s, x, 0.0)
    assert res["fate"] == O.ESCAPED
    want = SQ.swept_to_radius(b, r0, 1.1 * r0)
    assert res["theta_f"] == pytest.approx(math.pi / 2, abs=1e-12)
    assert -res["phi_f"] == pytest.approx(want, rel=1e-9)
    # and it is on the sphere
    assert tr[-1, 1] > 1.1 * r0


def test_sky_code_quadrants_and_graticule():
    g, w = 6.0, 0.25
    d = math.radians
    assert O.sky_code(d(33), d(45), g, w) == O.SKY_GREEN
    assert O.sky_code(d(33), d(200), g, w) == O.SKY_RED
    assert O.sky_code(d(123), d(105), g, w) == O.SKY_BLUE
    assert O.sky_code(d(123), d(303), g, w) == O.SKY_YELLOW
    assert O.sky_code(d(60.1), d(45), g, w) == O.SKY_LINE   # a latitude line
    assert O.sky_code(d(33), d(47.9), g, w) == O.SKY_LINE   # a longitude line
    assert O.sky_code(d(33), d(47.5), g, w) == O.SKY_GREEN
    assert O.sky_code(d(33), d(45), 0.0, w) == O.SKY_GREEN  # no graticule


def test_sky_code_ignores_the_representation():
    rng = np.random.default_rng(4)
    for _ in range(2000):
        th = rng.uniform(0.0, math.pi)
        ph = rng.uniform(0.0, 2 * math.pi)
        c = O.sky_code(th, ph)
        for t2, p2 in ((th, ph + 2 * math.pi), (th, ph - 4 * math.pi), (-th, ph + math.pi),
                       (2 * math.pi - th, ph + math.pi), (th + 2 * math.pi, ph)):
            assert O.sky_code(t2, p2) == c, (th, ph, t2, p2)


def test_constant_l0_omega():
    # Schwarzschild: Omega = -l0 g_tt / g_phph = l0 (1 - 2M/r) / r^2
    for r in (4.0, 6.0, 11.5, 30.0):
        for l0 in (1.8, 2.8, 4.0):
            assert O.disk_omega(1.0, 0.0, r, 1, l0) == pytest.approx(l0 * (1 - 2 / r) / r ** 2, rel=1e-14)
    # Kerr: with l0 the Keplerian l = -u_phi/u_t at r, both models agree
    for a in (0.0, 0.5, 0.9):
        for r in (3.0, 6.0, 15.0):
            Om = O.disk_omega(1.0, a, r, 0, 0.0)
            g = O.metric_cov(1.0, a, r, math.pi / 2)
            l_k = -(g[1] + Om * g[4]) / (g[0] + Om * g[1])
            assert O.disk_omega(1.0, a, r, 1, l_k) == pytest.approx(Om, rel=1e-12)


def test_constant_l0_redshift_closed_form():
    """a = 0, l0 = 2.8: g = sqrt((1 - 2/r) - Omega^2 r^2) / (E - Omega L) at
    the oracle's own hit radius."""
    s = O.Setup(a=0.0, r_obs=1000.0, incl=math.radians(85), fov_x=24.0, fov_y=12.0, nx=96, ny=48,
                method=O.DP45, rtol=1e-12, atol=1e-12, disk_on=1, r_in=6.0, r_out=20.0, emis_q=2.0,
                rotation=1, l0=2.8)
    o = O.trace_pixels(s)
    hit = np.flatnonzero(o["fate"] == O.DISK)
    assert hit.size > 300
    for p in hit[::7]:
        x, y = O.pixel_xy(s, int(p % 96), int(p // 96))
        st, _ = O.camera_ray(1.0, 0.0, 1000.0, s.incl, x, y)
        E, L = st[5], st[6]
        r = o["r_hit"][p]
        Om = 2.8 * (1 - 2 / r) / r ** 2
        g = math.sqrt((1 - 2 / r) - Om * Om * r * r) / (E - Om * L)
        assert o["g"][p] == pytest.approx(g, rel=1e-12)
        assert o["intensity"][p] == pytest.approx(g ** 3 / r ** 2, rel=1e-12)
