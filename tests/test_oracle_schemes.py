"""Pins of the comparison integrators of Sect. 3.1 in the oracle:
Runge-Kutta-Fehlberg 4(5), Cash-Karp 5(4) and Bulirsch-Stoer.

- the Butcher tableaus satisfy the Runge-Kutta order conditions (all rooted
  trees up to order 5) for the order each weight row claims, and their rows
  sum to the published nodes;
- fixed-step convergence rates on a linear (y'' = -y) and a nonlinear
  (y' = y^2, exact 1/(1 - t)) problem: 4 (RKF45 propagates the 4th-order
  solution), 5 (Cash-Karp propagates the 5th), 10 (Bulirsch-Stoer with five
  extrapolation columns);
- each step's error estimate is the local error of the less accurate of its
  two solutions to leading order;
- along Kerr rays every scheme keeps E, L, Carter's Q and H, and reproduces
  the fates the radial potential predicts.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests.test_oracle_integrators import _carter_q
from tests.test_oracle_shadow import _quartic_fate

NODES = {O.RKF45: [0, 1 / 4, 3 / 8, 12 / 13, 1, 1 / 2], O.CK45: [0, 1 / 5, 3 / 10, 3 / 5, 1, 7 / 8]}


def _order_conditions(A, b):
    """Residuals of the 17 rooted-tree conditions up to order 5, grouped by
    order: {order: [sum - 1/gamma, ...]}."""
    c = A.sum(1)
    Ac = A @ c
    return {
        1: [b.sum() - 1],
        2: [b @ c - 1 / 2],
        3: [b @ c ** 2 - 1 / 3, b @ Ac - 1 / 6],
        4: [b @ c ** 3 - 1 / 4, b @ (c * Ac) - 1 / 8, b @ (A @ c ** 2) - 1 / 12, b @ (A @ Ac) - 1 / 24],
        5: [b @ c ** 4 - 1 / 5, b @ (c ** 2 * Ac) - 1 / 10, b @ (c * (A @ c ** 2)) - 1 / 15,
            b @ (c * (A @ Ac)) - 1 / 30, b @ Ac ** 2 - 1 / 20, b @ (A @ c ** 3) - 1 / 20,
            b @ (A @ (c * Ac)) - 1 / 40, b @ (A @ (A @ c ** 2)) - 1 / 60, b @ (A @ (A @ Ac)) - 1 / 120],
    }


@pytest.mark.parametrize("method, p_prop, p_emb", [(O.RKF45, 4, 5), (O.CK45, 5, 4)])
def test_tableau_order_conditions(method, p_prop, p_emb):
    A, bp, be = O.tableau(method)
    assert np.allclose(np.triu(A), 0.0)  # explicit
    np.testing.assert_allclose(A.sum(1), NODES[method], atol=1e-15)
    for b, p in ((bp, p_prop), (be, p_emb)):
        res = _order_conditions(A, b)
        for order in range(1, p + 1):
            assert np.max(np.abs(res[order])) < 1e-14, (order, res[order])
        if p < 5:  # and not one order more
            assert np.max(np.abs(res[p + 1])) > 1e-6


def _rates(method, problem, T, ns):
    exact = np.array([math.sin(T), math.cos(T)]) if problem == 0 else np.array([1.0 / (1.0 - T)])
    y0 = [0.0, 1.0] if problem == 0 else [1.0]
    errs = [np.abs(O.fixed_steps(method, problem, T, n, y0) - exact).max() for n in ns]
    return [math.log(errs[i] / errs[i + 1]) / math.log(ns[i + 1] / ns[i]) for i in range(len(ns) - 1)], errs


@pytest.mark.parametrize("method, order, ns", [(O.RKF45, 4, (16, 32, 64)), (O.CK45, 5, (8, 16, 32)),
                                               (O.BS, 10, (1, 2, 3, 4)), (O.BS_RAT, 10, (1, 2, 3, 4))])
def test_fixed_step_convergence(method, order, ns):
    r, e = _rates(method, 0, 2.0, ns)
    assert all(abs(x - order) < 0.3 for x in r), (r, e)


@pytest.mark.parametrize("method, order, ns, tol", [(O.RKF45, 4, (32, 64, 128), 0.4),
                                                    (O.CK45, 5, (16, 32, 64), 0.4),
                                                    (O.BS, 10, (5, 6, 7, 8), 0.6),
                                                    (O.BS_RAT, 10, (3, 4, 5, 6), 0.9)])
def test_fixed_step_convergence_nonlinear(method, order, ns, tol):
    """y' = y^2 to t = 1/2 (y = 2); Bulirsch-Stoer approaches its order from
    below here (9.5 ... 9.8 before rounding takes over)."""
    r, e = _rates(method, 1, 0.5, ns)
    assert all(abs(x - order) < tol for x in r), (r, e)


@pytest.mark.parametrize("method, hs", [(O.RKF45, (0.2, 0.1, 0.05)), (O.CK45, (0.2, 0.1, 0.05)),
                                        (O.DP45, (0.2, 0.1, 0.05)), (O.BS, (1.5, 1.0, 0.5)),
                                        (O.BS_RAT, (1.5, 1.0, 0.5))])
def test_error_estimate_is_the_local_error(method, hs):
    """e = y_prop - y_emb; the lower-order solution's true local error equals
    +-e to leading order, so the mismatch relative to |e| falls with h."""
    y0 = np.array([0.3, 0.8])
    rel = []
    for h in hs:
        yn, e, _ = O.one_step(method, 0, h, y0)
        # exact flow of y'' = -y: rotation
        c, s = math.cos(h), math.sin(h)
        exact = np.array([c * y0[0] + s * y0[1], -s * y0[0] + c * y0[1]])
        err_prop = yn - exact
        err_emb = (yn - e) - exact
        low = err_prop if np.linalg.norm(err_prop) > np.linalg.norm(err_emb) else -err_emb
        rel.append(np.linalg.norm(low - e) / np.linalg.norm(e))
    assert rel[-1] < 0.15 and rel[-1] < rel[0], rel


def test_evaluations_per_step():
    for m, n in [(O.DP45, 6), (O.RKF45, 6), (O.CK45, 6), (O.BS, O.BS_COLUMNS ** 2 + 1),
                 (O.BS_RAT, O.BS_COLUMNS ** 2 + 1), (O.RK4_S, 4)]:
        assert O.one_step(m, 0, 0.1, [0.0, 1.0])[2] == n


@pytest.mark.parametrize("method", [O.RKF45, O.CK45, O.BS, O.BS_RAT])
@pytest.mark.parametrize("x,y", [(-2.0, 1.87), (-1.25, 3.75)])
def test_caption_rays_invariants(method, x, y):
    """The caption rays (a = 0.98, r0 = 100) with each scheme at rtol 1e-12:
    the same fates as DP45, |H|_rel and Carter's Q kept."""
    s = O.Setup(a=0.98, r_obs=100.0, incl=math.pi / 2, method=method, rtol=1e-12, atol=1e-12,
                r_escape=1000.0)
    traj, res = O.trace_one(s, x, y)
    st, _ = O.camera_ray(1.0, 0.98, 100.0, math.pi / 2, x, y)
    E, L = st[5], st[6]
    assert res["fate"] == {(-2.0, 1.87): O.CAPTURED, (-1.25, 3.75): O.ESCAPED}[(x, y)]
    Hrel = np.array([O.hamiltonian_rel(1.0, 0.98, t[1:], E, L) for t in traj])
    assert Hrel.max() == pytest.approx(res["max_rel_h"], rel=1e-12)
    assert Hrel.max() < 1e-9
    Q0 = _carter_q(0.98, traj[0, 2], traj[0, 5], E, L)
    Q = np.array([_carter_q(0.98, t[2], t[5], E, L) for t in traj])
    assert np.abs(Q - Q0).max() < 1e-7 * max(1.0, abs(Q0))
    per = O.BS_COLUMNS ** 2 + 1 if method in (O.BS, O.BS_RAT) else 6
    assert res["n_evals"] >= per * res["n_steps"]


@pytest.mark.parametrize("method", [O.RKF45, O.CK45, O.BS, O.BS_RAT])
def test_kerr_fates_vs_radial_potential(method):
    """a = 0.9, i = 60 deg, r0 = 1000M, +-12M at 24x24: every pixel that is
    not near-critical has the fate the radial potential predicts."""
    a = 0.9
    s = O.Setup(a=a, r_obs=1000.0, incl=math.radians(60), fov_x=12.0, fov_y=12.0, nx=24, ny=24,
                method=method, rtol=1e-11, atol=1e-11)
    o = O.trace_pixels(s)
    checked = 0
    for p in range(24 * 24):
        x, y = O.pixel_xy(s, p % 24, p // 24)
        fate, margin = _quartic_fate(1.0, a, 1000.0, s.incl, x, y)
        if margin < 1e-3:
            continue
        checked += 1
        assert o["fate"][p] == fate, (p, x, y, margin)
    assert checked >= 0.97 * 576


def test_bulirsch_stoer_step_sequence_carries_rounding():
    """Why Bulirsch-Stoer's swept angle is compared under a rounding-derived
    tolerance: in the oracle itself a one-ulp nudge of the pixel coordinate
    moves the deflection by ~1e-6 for some rays, where Dormand-Prince moves
    it by ~1e-13.  The step sequences part at a step whose start states still
    agree to rounding level: there the error estimate (T_KK - T_K,K-1, a
    difference of two values that agree to the tolerance) is rounding noise
    that decides the next step size."""
    from paper_2202_00086_amd import workloads as W
    from tests import parity as P
    base = dict(W.kerr_ring(0.9, n=64, rtol=1e-11), ny=48)
    rows = np.arange(12 * 64, 20 * 64)
    sens = {}
    for method in (O.DP45, O.BS):
        s = O.Setup(**dict(base, method=method))
        xy = np.array([O.pixel_xy(s, p % 64, p // 64) for p in rows])
        sv = P.ulp_sensitivity(lambda x, y: O.trace_xy(s, x, y), xy[:, 0].copy(), xy[:, 1].copy(), "deflection")
        sens[method] = sv[np.isfinite(sv)]
    assert sens[O.DP45].max() < 1e-12
    assert sens[O.BS].max() > 1e-7
    # the most sensitive Bulirsch-Stoer ray: where its two step sequences part
    s = O.Setup(**dict(base, method=O.BS))
    xy = np.array([O.pixel_xy(s, p % 64, p // 64) for p in rows])
    sv = P.ulp_sensitivity(lambda x, y: O.trace_xy(s, x, y), xy[:, 0].copy(), xy[:, 1].copy(), "deflection")
    k = int(np.nanargmax(np.where(np.isfinite(sv), sv, 0.0)))
    x, y = xy[k]
    t1, _ = O.trace_one(s, x, y)
    found = False
    for yy in (np.nextafter(y, np.inf), np.nextafter(y, -np.inf)):
        for xx in (x, np.nextafter(x, np.inf), np.nextafter(x, -np.inf)):
            t2, _ = O.trace_one(s, xx, yy)
            n = min(len(t1), len(t2))
            h1, h2 = np.diff(t1[:n, 0]), np.diff(t2[:n, 0])
            part = np.flatnonzero(np.abs(h1 - h2) > 1e-6 * np.abs(h1))
            if part.size:
                j = int(part[0])
                # the start states of the parting step agree to rounding level
                assert np.all(np.abs(t1[j, 1:] - t2[j, 1:]) <= 1e-12 * (np.abs(t1[j, 1:]) + 1.0))
                found = True
    assert found



# ---------------------------------------------------------------------------
# The extrapolation step itself (Sect. 3.1's Bulirsch-Stoer: Richardson
# extrapolation of modified-midpoint chains to zero substep).  Data that is
# exactly a polynomial, or a rational function, of x = (1/n)^2 of the degree
# the tableau spans is extrapolated exactly by the matching form.
# ---------------------------------------------------------------------------

def _x(K):
    return np.array([1.0 / (2 * (k + 1)) ** 2 for k in range(K)])


def test_polynomial_extrapolation_is_exact_on_polynomials():
    rng = np.random.default_rng(5)
    for K in (2, 3, 5):
        c = rng.uniform(-3, 3, K)           # degree K - 1 in x
        x = _x(K)
        f = sum(c[i] * x ** i for i in range(K))
        row = O.bs_extrapolate(f)
        assert row[-1] == pytest.approx(c[0], abs=2e-13)
        assert row[0] == f[-1]


@pytest.mark.parametrize("K, num, den", [(3, (1.0, 2.0), (1.0, 3.0)),
                                         (5, (2.0, -1.5, 0.7), (1.0, 4.0, -2.5)),
                                         (5, (0.5, 3.0, 1.0), (1.0, -0.8, 6.0))])
def test_rational_extrapolation_is_exact_on_rational_functions(K, num, den):
    """K points span a rational function of numerator and denominator degree
    (K - 1)/2 each; its value at x = 0 is recovered exactly, where the
    polynomial form is off."""
    x = _x(K)
    f = np.polyval(num[::-1], x) / np.polyval(den[::-1], x)
    want = num[0] / den[0]
    assert O.bs_extrapolate(f, rational=True)[-1] == pytest.approx(want, abs=1e-12)
    assert abs(O.bs_extrapolate(f)[-1] - want) > 1e-9


def test_rational_extrapolation_degenerate_denominators():
    """Equal chain ends (a vanishing inner denominator) extrapolate to that
    value; the two forms agree on constants."""
    for f in (np.full(5, 2.5), np.zeros(5)):
        assert O.bs_extrapolate(f, rational=True)[-1] == f[0]
        assert O.bs_extrapolate(f)[-1] == f[0]


def test_rational_and_polynomial_schemes_differ_but_agree_to_tolerance():
    """On a caption ray the two extrapolations take different step sequences
    and meet the celestial sphere (its crossing located) at the same place
    to within the scheme's global error."""
    res = {}
    for m in (O.BS, O.BS_RAT):
        s = O.Setup(a=0.98, r_obs=100.0, incl=math.pi / 2, method=m, rtol=1e-12, atol=1e-12, r_escape=1000.0,
                    sky_on=1)
        traj, r = O.trace_one(s, -1.25, 3.75)
        res[m] = (traj, r)
    assert res[O.BS][1]["n_steps"] != res[O.BS_RAT][1]["n_steps"] or \
        not np.array_equal(res[O.BS][0][:, 0], res[O.BS_RAT][0][:, 0])
    assert res[O.BS][1]["fate"] == res[O.BS_RAT][1]["fate"] == O.ESCAPED
    for k in ("theta_f", "phi_f"):
        assert res[O.BS][1][k] == pytest.approx(res[O.BS_RAT][1][k], rel=1e-7)
