"""Pins of the oracle's ray fates (captured vs escaped).

- Schwarzschild: the shadow edge seen from r0 is the circle
  x^2 + y^2 = 27 M^2 (1 - 2M/r0) (Synge), which is why the numerical shadow
  comes out "a little smaller" than the r0 -> infinity curve (Sect. 3.2);
- Kerr: per pixel, the exact fate from the roots of Carter's radial
  potential R(r) (no ODE), and the finite-distance form of the analytic
  critical curve eq:anal / eq:xie (Sect. 3.2), which reduces to eq:anal as
  r0 -> infinity;
- extremal Kerr (|a| = M), equatorial rays: the radial potential factors,
  so the fate edges along the equator are closed forms that include the
  capture buffer (b = 2M + delta_r on the co-rotating side, -7M on the
  counter-rotating one);
- image symmetries.
"""
import math

import numpy as np
import pytest

import oracle as O


def c1_setup():
    return O.Setup(a=0.0, r_obs=1000.0, incl=math.pi / 2, fov_x=10.0, fov_y=10.0, nx=64, ny=64,
                   method=O.RK4_S, h_fixed=1.0 / 128, cap_buffer=0.01, r_escape=1100.0)


def test_schwarzschild_shadow_synge_64():
    """64x64, +-10M, r0 = 1000M, fixed-step RK4: per-pixel fate equals the
    closed-form criterion; 872 pixels are captured."""
    s = c1_setup()
    o = O.trace_pixels(s)
    i, j = np.meshgrid(np.arange(64), np.arange(64))
    x = -10 + (i.ravel() + 0.5) * (20 / 64)
    y = -10 + (j.ravel() + 0.5) * (20 / 64)
    captured = x * x + y * y < 27.0 * (1 - 2.0 / 1000.0)
    np.testing.assert_array_equal(o["fate"], np.where(captured, O.CAPTURED, O.ESCAPED))
    assert captured.sum() == 872
    # symmetries of a = 0, i = 90 deg
    f = o["fate"].reshape(64, 64)
    np.testing.assert_array_equal(f, f[:, ::-1])
    np.testing.assert_array_equal(f, f[::-1, :])


def _quartic_fate(M, a, r0, incl, x, y):
    """Exact fate from R(r) = E^2 r^4 + (a^2E^2 - L^2 - Q) r^2 + 2M(Q + (L-aE)^2) r - a^2 Q.
    The ingoing ray turns at the largest root of R in (r_+, r0), if any.
    Returns (fate, margin): margin is small when the ray is near-critical."""
    st, _ = O.camera_ray(M, a, r0, incl, x, y)
    E, L, pth = st[5], st[6], st[4]
    Q = pth ** 2 + math.cos(incl) ** 2 * (L * L / math.sin(incl) ** 2 - a * a * E * E)
    coef = [E * E, 0.0, a * a * E * E - L * L - Q, 2 * M * (Q + (L - a * E) ** 2), -a * a * Q]
    roots = np.roots(coef)
    rp = M + math.sqrt(M * M - a * a)
    real = sorted(r.real for r in roots if abs(r.imag) < 1e-9 * max(1, abs(r)) and rp < r.real < r0)
    # near-critical: two roots close together, or a complex pair close to the real axis
    margin = 1e9
    for r in roots:
        if r.real > rp and abs(r.imag) >= 1e-9 * max(1, abs(r)):
            margin = min(margin, abs(r.imag))
    if len(real) >= 2:
        margin = min(margin, real[-1] - real[-2])
    return (O.ESCAPED if real else O.CAPTURED), margin


@pytest.mark.parametrize("a", [0.5, 0.9, 0.998])
def test_kerr_fates_vs_radial_potential(a):
    """Kerr, i = 60 deg, r0 = 1000M, +-12M at 40x40 DP45: every pixel that is
    not near-critical has the fate the radial potential predicts."""
    s = O.Setup(a=a, r_obs=1000.0, incl=math.radians(60), fov_x=12.0, fov_y=12.0, nx=40, ny=40,
                method=O.DP45, rtol=1e-12, atol=1e-12)
    o = O.trace_pixels(s)
    checked = 0
    for p in range(40 * 40):
        x, y = O.pixel_xy(s, p % 40, p // 40)
        fate, margin = _quartic_fate(1.0, a, 1000.0, s.incl, x, y)
        if margin < 1e-3:
            continue
        checked += 1
        assert o["fate"][p] == fate, (p, x, y, margin)
    assert checked >= 0.98 * 1600
    assert (o["fate"] == O.CAPTURED).sum() > 50


def _xi_eta(M, a, r):
    """Spherical photon orbits, eq:xie."""
    xi = -(r ** 3 - 3 * M * r * r + a * a * r + a * a * M) / (a * (r - M))
    eta = -(r ** 3) * (r ** 3 - 6 * M * r * r + 9 * M * M * r - 4 * a * a * M) / (a * a * (r - M) ** 2)
    return xi, eta


def _critical_curve(M, a, r0, incl, rs):
    """Image-plane critical curve for an observer at finite r0: the photon with
    (L/E, Q/E^2) = (xi, eta) mapped through the camera relations."""
    g = O.metric_cov(M, a, r0, incl)
    At = math.sqrt(g[4] / (g[1] ** 2 - g[0] * g[4]))
    pts = []
    for r in rs:
        xi, eta = _xi_eta(M, a, r)
        w = eta - math.cos(incl) ** 2 * (xi * xi / math.sin(incl) ** 2 - a * a)
        if w < 0:
            continue
        x = -xi * r0 * math.sqrt(g[4]) / (At * (g[4] + xi * g[1]))
        E = 1 / At + x * g[1] / (r0 * math.sqrt(g[4]))
        y = r0 * E * math.sqrt(w) / math.sqrt(g[3])
        pts.append((x, y))
    return np.array(pts)


def test_critical_curve_reduces_to_eq_anal():
    """r0 -> infinity: the finite-distance curve tends to eq:anal."""
    M, a, incl = 1.0, 0.98, math.pi / 2
    rs = np.linspace(1.3, 3.9, 40)
    far = _critical_curve(M, a, 1e12, incl, rs)
    anal = []
    for r in rs:
        xi, eta = _xi_eta(M, a, r)
        w = eta - math.cos(incl) ** 2 * (xi * xi / math.sin(incl) ** 2 - a * a)
        if w >= 0:
            anal.append((-xi / math.sin(incl), math.sqrt(w)))
    np.testing.assert_allclose(far, np.array(anal), rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("a,incl_deg,r0", [(0.98, 90.0, 1000.0), (0.9, 60.0, 1000.0),
                                          (0.5, 60.0, 1000.0)])
def test_shadow_edge_matches_critical_curve(a, incl_deg, r0):
    """Points of the finite-r0 critical curve, pulled 1e-4 inward (toward an
    interior point) are captured; pushed 1e-4 outward, they escape."""
    incl = math.radians(incl_deg)
    rp = O.horizon(1.0, a)
    rs = np.linspace(rp + 0.05, 4.5, 400)
    pts = _critical_curve(1.0, a, r0, incl, rs)
    pts = pts[:: max(1, len(pts) // 12)]
    centre = np.array([0.5 * (pts[:, 0].min() + pts[:, 0].max()), 0.0])
    s = O.Setup(a=a, r_obs=r0, incl=incl, method=O.DP45, rtol=1e-12, atol=1e-12)
    xs, ys, want = [], [], []
    for x, y in pts:
        for sgn in (1.0, -1.0):
            p = np.array([x, sgn * y])
            for f, fate in [(1 - 1e-4, O.CAPTURED), (1 + 1e-4, O.ESCAPED)]:
                q = centre + f * (p - centre)
                xs.append(q[0])
                ys.append(q[1])
                want.append(fate)
    o = O.trace_xy(s, np.array(xs), np.array(ys))
    np.testing.assert_array_equal(o["fate"], np.array(want))


def test_finite_distance_shadow_is_smaller():
    """The paper's remark that the numerical shadow is a little smaller than
    eq:anal: the finite-r0 extents lie inside the r0 -> infinity ones."""
    rs = np.linspace(1.25, 3.95, 2000)
    fin = _critical_curve(1.0, 0.98, 1000.0, math.pi / 2, rs)
    inf = _critical_curve(1.0, 0.98, 1e12, math.pi / 2, rs)
    assert fin[:, 1].max() < inf[:, 1].max()
    assert fin[:, 0].max() - fin[:, 0].min() < inf[:, 0].max() - inf[:, 0].min()
    assert fin[:, 1].max() / inf[:, 1].max() == pytest.approx(math.sqrt(1 - 2 / 1000.0), rel=2e-4)


def test_kerr_equatorial_symmetry():
    """Kerr seen from i = 90 deg: the image is symmetric under y -> -y."""
    s = O.Setup(a=0.9, r_obs=1000.0, incl=math.pi / 2, fov_x=8.0, fov_y=8.0, nx=16, ny=16,
                method=O.DP45)
    o = O.trace_pixels(s)
    f = o["fate"].reshape(16, 16)
    np.testing.assert_array_equal(f, f[::-1, :])
    # and not under x -> -x (frame dragging): the shadow is shifted
    fs = (f == O.CAPTURED)
    assert (fs != fs[:, ::-1]).any()


def extremal_edges(a, M=1.0, cap_buffer=0.01):
    """Fate edges in b = L/E for equatorial rays of extremal Kerr (a = +-M).

    With Q = 0 and a = M the radial potential is
    R(r) = (r^2 + M^2 - M b)^2 - (r - M)^2 (b - M)^2 (E = 1), whose factor
    r^2 + M^2 - M b - (r - M)(b - M) = r (r - b + M) gives the outermost
    turning point r_t = b - M of a co-rotating ray with b > 2M.  The photon
    orbit of that side sits on the horizon (r = M, b = 2M), so what decides
    capture there is the buffer: the ray is stopped once r < r_+ + delta_r =
    M + delta_r, i.e. for b < 2M + delta_r.  The counter-rotating photon
    orbit is at r = 4M with b = -7M, outside the buffer.  For a = -M the
    picture is mirrored in b.  Returns (b_lo, b_hi): captured iff
    b_lo < b < b_hi."""
    lo, hi = -7.0 * M, 2.0 * M + cap_buffer
    return (lo, hi) if a > 0 else (-hi, -lo)


def _x_for_b(a, r0, incl, b):
    """The image-plane x (at y = 0) whose ray has L/E = b: bisection on the
    oracle's camera relations, which are monotonic in x."""
    def b_of(x):
        st, _ = O.camera_ray(1.0, a, r0, incl, x, 0.0)
        return st[6] / st[5]
    lo, hi = -20.0, 20.0
    rising = b_of(hi) > b_of(lo)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if (b_of(mid) > b) == rising:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("a", [1.0, -1.0])
def test_extremal_kerr_equatorial_edges(a):
    """|a| = M, i = 90 deg, y = 0, r0 = 1000M, DP45: rays aimed 0.002M to
    0.02M on either side of each closed-form edge get the predicted fate.
    Without the buffer the co-rotating edge would sit at b = 2M, so the rays
    at 2M + 0.005M and 2M + 0.008M would escape; a wrong horizon, spin sign
    or Delta moves the edges by more than these offsets."""
    r0, incl = 1000.0, math.pi / 2
    lo, hi = extremal_edges(a)
    bs, want = [], []
    for e in (lo, hi):
        for d in (-0.02, -0.005, -0.002, 0.002, 0.005, 0.02):
            bs.append(e + d)
            want.append(O.CAPTURED if lo < e + d < hi else O.ESCAPED)
    xs = np.array([_x_for_b(a, r0, incl, b) for b in bs])
    for x, b in zip(xs, bs):
        st, _ = O.camera_ray(1.0, a, r0, incl, x, 0.0)
        assert st[6] / st[5] == pytest.approx(b, abs=1e-12)
    s = O.Setup(a=a, r_obs=r0, incl=incl, method=O.DP45, rtol=1e-12, atol=1e-12)
    o = O.trace_xy(s, xs, np.zeros_like(xs))
    np.testing.assert_array_equal(o["fate"], np.array(want))
