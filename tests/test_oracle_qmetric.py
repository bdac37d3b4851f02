"""Pins of the oracle's q-metric (the appendix's static axisymmetric vacuum
with quadrupole parameter q, taken with signature (-,+,+,+)).

- q = 0 is Schwarzschild: components, derivatives and Hamilton's equations
  equal the Kerr ones at a = 0;
- the analytic r- and theta-derivatives match central differences;
- it is a vacuum solution: the Ricci tensor assembled numerically from the
  oracle's components and first derivatives vanishes (checked first on Kerr,
  and shown to fail for a slightly wrong metric);
- the equatorial light ring sits at r = m(3 + 2q); rays just inside the
  critical impact parameter m(3+2q) ((3+2q)/(1+2q))^((1+2q)/2) are captured,
  rays just outside escape;
- far from the source the deflection is 4 m (1 + q) / b: the mass is m(1+q);
- H stays zero along rays.
"""
import math

import numpy as np
import pytest

import oracle as O

M = 1.0


def _full(kind, a, q, r, th, g5=None, m=M):
    g = O.metric_cov_k(kind, m, a, q, r, th) if g5 is None else g5
    G = np.zeros((4, 4))
    G[0, 0], G[0, 3], G[3, 0], G[1, 1], G[2, 2], G[3, 3] = g[0], g[1], g[1], g[2], g[3], g[4]
    return G


def _christoffel(kind, a, q, r, th, metric=None, m=M):
    """Gamma^a_bc from the components and their analytic first derivatives
    (coordinates t, r, theta, phi); `metric` overrides with a callable
    returning (g5, dr5, dth5)."""
    if metric is None:
        g5 = O.metric_cov_k(kind, m, a, q, r, th)
        dr5, dth5 = O.metric_derivs_k(kind, m, a, q, r, th)
    else:
        g5, dr5, dth5 = metric(r, th)
    G = _full(0, 0, 0, 0, 0, g5)
    dG = np.zeros((4, 4, 4))  # dG[c, a, b] = d_c g_ab
    dG[1] = _full(0, 0, 0, 0, 0, dr5)
    dG[2] = _full(0, 0, 0, 0, 0, dth5)
    Gi = np.linalg.inv(G)
    Gam = np.zeros((4, 4, 4))
    for a_ in range(4):
        for b in range(4):
            for c in range(4):
                Gam[a_, b, c] = 0.5 * sum(Gi[a_, d] * (dG[b, d, c] + dG[c, d, b] - dG[d, b, c]) for d in range(4))
    return Gam


def _ricci(kind, a, q, r, th, metric=None, m=M):
    h = 1e-5
    Gam = _christoffel(kind, a, q, r, th, metric, m)
    dGam = np.zeros((4, 4, 4, 4))  # dGam[e, a, b, c] = d_e Gamma^a_bc
    dGam[1] = (_christoffel(kind, a, q, r + h * r, th, metric, m)
               - _christoffel(kind, a, q, r - h * r, th, metric, m)) / (2 * h * r)
    dGam[2] = (_christoffel(kind, a, q, r, th + h, metric, m) - _christoffel(kind, a, q, r, th - h, metric, m)) / (2 * h)
    R = np.zeros((4, 4))
    scale = 0.0
    for b in range(4):
        for d in range(4):
            t1 = sum(dGam[a_, a_, b, d] for a_ in range(4))
            t2 = sum(dGam[d, a_, a_, b] for a_ in range(4))
            t3 = sum(Gam[a_, a_, e] * Gam[e, b, d] for a_ in range(4) for e in range(4))
            t4 = sum(Gam[a_, d, e] * Gam[e, a_, b] for a_ in range(4) for e in range(4))
            R[b, d] = t1 - t2 + t3 - t4
            scale = max(scale, abs(t1), abs(t2), abs(t3), abs(t4))
    return R, scale


@pytest.mark.parametrize("r, th", [(3.0, 0.7), (6.5, 1.3), (20.0, 0.4)])
def test_q_zero_is_schwarzschild(r, th):
    np.testing.assert_allclose(O.metric_cov_k(O.QMETRIC, M, 0.0, 0.0, r, th),
                               O.metric_cov_k(O.KERR, M, 0.0, 0.0, r, th), rtol=1e-15, atol=1e-300)
    for x, y in zip(O.metric_derivs_k(O.QMETRIC, M, 0.0, 0.0, r, th), O.metric_derivs_k(O.KERR, M, 0.0, 0.0, r, th)):
        np.testing.assert_allclose(x, y, rtol=1e-13, atol=1e-14)
    z = [r, th, 0.3, -0.7, 2.1]
    np.testing.assert_allclose(O.rhs_k(O.QMETRIC, M, 0.0, 0.0, z, 1.0, 3.0), O.rhs_k(O.KERR, M, 0.0, 0.0, z, 1.0, 3.0),
                               rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("q", [-0.3, 0.5, 1.2])
def test_derivatives_match_differences(q):
    for r, th in [(2.7, 0.5), (5.0, 1.1), (17.0, 1.5)]:
        dr, dth = O.metric_derivs_k(O.QMETRIC, M, 0.0, q, r, th)
        h = 1e-5
        fr = (O.metric_cov_k(O.QMETRIC, M, 0.0, q, r + h, th) - O.metric_cov_k(O.QMETRIC, M, 0.0, q, r - h, th)) / (2 * h)
        ft = (O.metric_cov_k(O.QMETRIC, M, 0.0, q, r, th + h) - O.metric_cov_k(O.QMETRIC, M, 0.0, q, r, th - h)) / (2 * h)
        np.testing.assert_allclose(dr, fr, rtol=1e-6, atol=1e-9)
        np.testing.assert_allclose(dth, ft, rtol=1e-6, atol=1e-9)


def test_ricci_check_works_on_kerr_and_sees_a_wrong_metric():
    R, scale = _ricci(O.KERR, 0.9, 0.0, 4.0, 1.0)
    assert np.abs(R).max() < 1e-7 * scale

    def wrong(r, th):  # Schwarzschild with g_rr off by a factor (1 + 0.05 M / r)
        g = O.metric_cov_k(O.KERR, M, 0.0, 0.0, r, th)
        dr, dth = O.metric_derivs_k(O.KERR, M, 0.0, 0.0, r, th)
        k = 1 + 0.05 / r
        dr = dr.copy()
        dr[2] = dr[2] * k + g[2] * (-0.05 / r ** 2)
        g = g.copy()
        g[2] *= k
        return g, dr, dth
    R, scale = _ricci(0, 0, 0, 4.0, 1.0, metric=wrong)
    assert np.abs(R).max() > 1e-4 * scale


@pytest.mark.parametrize("m, q", [(1.0, -0.3), (1.0, 0.5), (1.0, 1.2), (1.7, 0.5)])
def test_q_metric_is_ricci_flat(m, q):
    for r, th in [(3.5 * m, 0.6), (6.0 * m, 1.2), (15.0 * m, 1.5)]:
        R, scale = _ricci(O.QMETRIC, 0.0, q, r, th, m=m)
        assert np.abs(R).max() < 1e-7 * scale, (q, r, th, np.abs(R).max(), scale)


def _equatorial_setup(q, r0=1000.0):
    return O.Setup(M=M, metric=O.QMETRIC, q=q, r_obs=r0, incl=math.pi / 2, method=O.DP45, rtol=1e-12,
                   atol=1e-12, r_escape=1.1 * r0)


@pytest.mark.parametrize("q", [-0.2, 0.0, 0.4, 1.0])
def test_light_ring_and_critical_impact_parameter(q):
    r0 = 1000.0
    s = _equatorial_setup(q, r0)
    bc = M * (3 + 2 * q) * ((3 + 2 * q) / (1 + 2 * q)) ** ((1 + 2 * q) / 2)
    f0 = 1 - 2 * M / r0
    xc = bc * f0 ** ((1 + 2 * q) / 2)  # image-plane radius of impact parameter bc for a static observer
    _, out_in = O.trace_one(s, xc * (1 - 2e-4), 0.0)
    tr, out_out = O.trace_one(s, xc * (1 + 2e-4), 0.0)
    assert out_in["fate"] == O.CAPTURED
    assert out_out["fate"] == O.ESCAPED
    # the escaping ray turns just outside the light ring m (3 + 2q)
    assert tr[:, 1].min() == pytest.approx(M * (3 + 2 * q), rel=0.03)


@pytest.mark.parametrize("q", [-0.3, 0.0, 0.6])
def test_weak_field_deflection_measures_the_mass(q):
    r0 = 1e5
    b = 2000.0
    # the sky sphere makes the escape point the exact crossing of r = 1.1 r0
    s = O.Setup(M=M, metric=O.QMETRIC, q=q, r_obs=r0, incl=math.pi / 2, method=O.DP45, rtol=1e-12, atol=1e-12,
                r_escape=1.1 * r0, sky_on=1)
    f0 = 1 - 2 * M / r0
    x = b * f0 ** ((1 + 2 * q) / 2)
    tr, out = O.trace_one(s, x, 0.0)
    assert out["fate"] == O.ESCAPED
    # swept longitude from r0 inwards and back out to 1.1 r0, minus the
    # straight-line value for the same end radii
    dphi = -out["phi_f"]
    straight = math.pi - math.asin(b / r0) - math.asin(b / (1.1 * r0))
    alpha = dphi - straight
    want = 4 * M * (1 + q) / b
    assert alpha == pytest.approx(want, rel=5e-3)


@pytest.mark.parametrize("q", [-0.3, 0.7])
def test_constraint_kept_along_rays(q):
    s = O.Setup(M=M, metric=O.QMETRIC, q=q, r_obs=100.0, incl=1.1, fov_x=12.0, fov_y=12.0, nx=12, ny=12,
                method=O.DP45, rtol=1e-12, atol=1e-12, r_escape=110.0)
    o = O.trace_pixels(s)
    assert (o["fate"] == O.CAPTURED).any() and (o["fate"] == O.ESCAPED).any()
    assert np.nanmax(o["max_rel_h"]) < 1e-10
    x, y = O.pixel_xy(s, 3, 8)
    tr, res = O.trace_one(s, x, y)
    st, _ = O.camera_ray_k(O.QMETRIC, M, 0.0, q, 100.0, 1.1, x, y)
    Hs = [abs(O.hamiltonian_k(O.QMETRIC, M, 0.0, q, t[1:], st[5], st[6])) for t in tr]
    assert max(Hs) == pytest.approx(res["max_abs_h"], rel=1e-12)
    assert O.hamiltonian_rel_k(O.QMETRIC, M, 0.0, q, tr[0, 1:], st[5], st[6]) < 1e-15
