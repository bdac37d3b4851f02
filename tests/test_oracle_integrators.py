"""Pins of the oracle's integrators and of the invariants along its rays.

- convergence order on y'' = -y (exact solution sin t): DP5 is 5th order,
  RK4 4th order;
- Dormand-Prince at rtol 1e-12 keeps the constraint at the level the paper
  reports for it (better than a part in 1e-10, Sect. 3.1) on the two caption
  rays, and E, L_z (never evolved), and Carter's constant along the ray;
- flat space (M = 0): BL coordinates become oblate spheroidal coordinates and
  rays are straight lines.
"""
import math

import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("method,order", [(O.DP45, 5), (O.RK4_S, 4)])
def test_convergence_order(method, order):
    T = 10.0
    errs = []
    for n in (40, 80, 160):
        y, v = O.harmonic_fixed(method, T, n)
        errs.append(math.hypot(y - math.sin(T), v - math.cos(T)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    for r in rates:
        assert abs(r - order) < 0.25, rates


def _carter_q(a, th, pth, E, L):
    c, s = math.cos(th), math.sin(th)
    return pth * pth + c * c * (L * L / (s * s) - a * a * E * E)


def _radial_roots(a, E, L, Q):
    """Real roots of Carter's radial potential
    R(r) = E^2 r^4 + (a^2E^2 - L^2 - Q) r^2 + 2(Q + (L - aE)^2) r - a^2 Q  (M = 1)."""
    r = np.roots([E * E, 0.0, a * a * E * E - L * L - Q, 2 * (Q + (L - a * E) ** 2), -a * a * Q])
    return np.sort(r[np.abs(r.imag) < 1e-12].real)


@pytest.mark.parametrize("x,y", [(-2.0, 1.87), (-1.25, 3.75)])
def test_caption_rays_constraint_and_invariants(x, y):
    """The two rays of the Sect. 3.1 captions (a = 0.98, r0 = 100).  Their fate
    follows from the radial potential alone: (-2, 1.87) has no turning point
    outside r_+ and falls in; (-1.25, 3.75) turns at the largest root of R and
    escapes.  (The captions attach the opposite fates to these ICs.)  DP45 at
    rtol 1e-12 keeps |H| far below the paper's 1e-10 statement; E, L are
    constants; Carter's Q is conserved."""
    s = O.Setup(a=0.98, r_obs=100.0, incl=math.pi / 2, method=O.DP45, rtol=1e-12, atol=1e-12,
                r_escape=1000.0)
    traj, res = O.trace_one(s, x, y)
    st, _ = O.camera_ray(1.0, 0.98, 100.0, math.pi / 2, x, y)
    E, L = st[5], st[6]
    roots = _radial_roots(0.98, E, L, st[4] ** 2)
    turning = roots[(roots > O.horizon(1.0, 0.98)) & (roots < 100.0)]
    if turning.size:
        assert res["fate"] == O.ESCAPED
        assert traj[:, 1].min() == pytest.approx(turning.max(), rel=1e-6)
    else:
        assert res["fate"] == O.CAPTURED
    assert (x, y, res["fate"]) in [(-2.0, 1.87, O.CAPTURED), (-1.25, 3.75, O.ESCAPED)]
    Hs = np.array([O.hamiltonian(1.0, 0.98, t[1:], E, L) for t in traj])
    Hrel = np.array([O.hamiltonian_rel(1.0, 0.98, t[1:], E, L) for t in traj])
    assert np.abs(Hs).max() == pytest.approx(res["max_abs_h"], rel=1e-12)
    assert Hrel.max() == pytest.approx(res["max_rel_h"], rel=1e-12)
    assert Hrel.max() < 1e-10
    Q0 = _carter_q(0.98, traj[0, 2], traj[0, 5], E, L)
    Q = np.array([_carter_q(0.98, t[2], t[5], E, L) for t in traj])
    assert np.abs(Q - Q0).max() < 1e-8 * max(1.0, abs(Q0))
    assert res["n_evals"] >= 6 * res["n_steps"]


def test_fixed_rk4_in_s_invariants():
    """RK4 at a fixed step in s (d lambda = Delta/r ds): ray is the same
    Hamiltonian flow, so H and Q stay near their initial values."""
    s = O.Setup(a=0.0, r_obs=1000.0, incl=math.pi / 2, method=O.RK4_S, h_fixed=1 / 128,
                r_escape=1100.0)
    for x, y, fate in [(3.0, 4.5, O.ESCAPED), (2.0, 2.0, O.CAPTURED)]:
        traj, res = O.trace_one(s, x, y)
        assert res["fate"] == fate
        assert res["max_abs_h"] < 1e-6
        st, _ = O.camera_ray(1.0, 0.0, 1000.0, math.pi / 2, x, y)
        Q0 = _carter_q(0.0, math.pi / 2, st[4], st[5], st[6])
        Qf = _carter_q(0.0, traj[-1, 2], traj[-1, 5], st[5], st[6])
        assert Qf == pytest.approx(Q0, rel=1e-5)


@pytest.mark.parametrize("a", [0.0, 0.6])
def test_flat_space_straight_lines(a):
    """M = 0: x = sqrt(r^2+a^2) sin cos phi, y = ... sin sin phi, z = r cos is
    Cartesian; every recorded position lies on the initial straight line."""
    s = O.Setup(M=0.0, a=a, r_obs=50.0, incl=1.1, method=O.DP45, rtol=1e-12, atol=1e-12,
                r_escape=60.0, cap_buffer=-1e9)
    for x, y in [(3.0, -4.0), (-0.5, 2.0), (7.0, 7.0)]:
        traj, res = O.trace_one(s, x, y)
        assert res["fate"] == O.ESCAPED
        r, th, ph = traj[:, 1], traj[:, 2], traj[:, 3]
        rho = np.sqrt(r * r + a * a)
        P = np.stack([rho * np.sin(th) * np.cos(ph), rho * np.sin(th) * np.sin(ph), r * np.cos(th)], 1)
        d = P[1] - P[0]
        d /= np.linalg.norm(d)
        off = (P - P[0]) - np.outer((P - P[0]) @ d, d)
        assert np.linalg.norm(off, axis=1).max() < 1e-9
        if a == 0.0:
            # spherical frame: the line's distance from the origin is |(x, y)|
            closest = np.linalg.norm(P[0] - (P[0] @ d) * d)
            assert closest == pytest.approx(math.hypot(x, y), rel=1e-9)


def test_step_control_and_counts():
    s = O.Setup(a=0.9, r_obs=1000.0, incl=math.radians(60), fov_x=12, fov_y=12, nx=8, ny=8,
                method=O.DP45)
    o = O.trace_pixels(s)
    assert (o["n_evals"] >= 6 * o["n_steps"] + 1).all()
    assert set(np.unique(o["fate"])) <= {O.ESCAPED, O.CAPTURED}
    # tighter tolerance takes more steps
    s2 = O.Setup(**{**s.__dict__, "rtol": 1e-10, "atol": 1e-10})
    o2 = O.trace_pixels(s2)
    assert o2["n_steps"].sum() < o["n_steps"].sum()


def test_max_steps_forces_fate():
    s = O.Setup(a=0.5, r_obs=1000.0, incl=1.0, fov_x=10, fov_y=10, nx=4, ny=4, max_steps=10)
    o = O.trace_pixels(s)
    assert (o["fate"] == O.MAXSTEPS).all()
    assert (o["n_steps"] == 10).all()


def test_rk4_s_parametrisation_flat():
    """The fixed-step integrator runs in s with d(lambda)/ds = Delta/r; in flat
    space (M = a = 0) that is r, lambda is Euclidean length and
    r(s) = b cosh(s - asinh(sqrt(r0^2 - b^2)/b)) for impact parameter b."""
    r0 = 100.0
    s = O.Setup(M=0.0, a=0.0, r_obs=r0, incl=1.0, method=O.RK4_S, h_fixed=1.0 / 256,
                r_escape=150.0, cap_buffer=-1e9)
    x, y = 3.0, 4.0
    b = math.hypot(x, y)
    traj, res = O.trace_one(s, x, y)
    assert res["fate"] == O.ESCAPED
    sv, r = traj[:, 0], traj[:, 1]
    want = b * np.cosh(sv - math.asinh(math.sqrt(r0 * r0 - b * b) / b))
    np.testing.assert_allclose(r, want, rtol=1e-8)
    np.testing.assert_allclose(np.diff(sv), 1.0 / 256, rtol=1e-9)
