"""Pins of the oracle's spacetime, Hamiltonian and equations of motion.

Each check compares the oracle with something it does not compute itself:
textbook identities of the Kerr metric, a numerical 4x4 inverse, a
complex-step derivative of H built on that inverse, Carter's separated form
and the Schwarzschild limit; and the rounding of its relative residual
next to a horizon against a 50-digit evaluation.
"""
import math

import numpy as np
import pytest

import oracle as O

RNG = np.random.default_rng(7)


def _random_states(n, a_max=0.999):
    """Random (M, a, r, theta, p_r, p_theta, E, L) outside the horizon."""
    out = []
    while len(out) < n:
        M = RNG.uniform(0.5, 2.0)
        a = RNG.uniform(-a_max, a_max) * M
        rp = M + math.sqrt(M * M - a * a)
        r = rp * (1.05 + 30.0 * RNG.random() ** 2)
        th = RNG.uniform(0.05, math.pi - 0.05)
        out.append((M, a, r, th, RNG.normal(), RNG.normal() * r, RNG.uniform(0.2, 2.0),
                    RNG.normal() * 5.0))
    return out


def _g_cov_numpy(M, a, r, th):
    """4x4 covariant metric (t, r, theta, phi) of the Kerr line element; works
    for complex r, theta (used for complex-step derivatives)."""
    s, c = np.sin(th), np.cos(th)
    Sig = r * r + a * a * c * c
    Del = r * r - 2 * M * r + a * a
    g = np.zeros((4, 4), dtype=np.result_type(r, th, complex))
    g[0, 0] = -(1 - 2 * M * r / Sig)
    g[0, 3] = g[3, 0] = -2 * M * r * a * s * s / Sig
    g[1, 1] = Sig / Del
    g[2, 2] = Sig
    g[3, 3] = s * s * (r * r + a * a + 2 * M * r * a * a * s * s / Sig)
    return g


def test_schwarzschild_limit():
    """a = 0: g = diag(-(1-2M/r), 1/(1-2M/r), r^2, r^2 sin^2)."""
    M, r, th = 1.3, 7.1, 0.9
    g = O.metric_cov(M, 0.0, r, th)
    f = 1 - 2 * M / r
    np.testing.assert_allclose(g, [-f, 0.0, 1 / f, r * r, r * r * math.sin(th) ** 2], rtol=1e-15)


@pytest.mark.parametrize("k", range(40))
def test_kerr_metric_identities(k):
    """Textbook Kerr identities: g_tphi^2 - g_tt g_phph = Delta sin^2 theta and
    det g = -Sigma^2 sin^2 theta."""
    M, a, r, th, *_ = _random_states(1)[0]
    g = O.metric_cov(M, a, r, th)
    s, c = math.sin(th), math.cos(th)
    Sig = r * r + a * a * c * c
    Del = r * r - 2 * M * r + a * a
    lhs = g[1] ** 2 - g[0] * g[4]
    assert lhs == pytest.approx(Del * s * s, rel=1e-12)
    det = (g[0] * g[4] - g[1] ** 2) * g[2] * g[3]
    assert det == pytest.approx(-Sig * Sig * s * s, rel=1e-12)


def test_horizon():
    for M, a in [(1.0, 0.0), (1.0, 0.9), (2.0, 1.5), (1.0, 0.998)]:
        rp = O.horizon(M, a)
        assert rp * rp - 2 * M * rp + a * a == pytest.approx(0.0, abs=1e-13 * M * M)
    assert O.horizon(1.0, 0.0) == 2.0


@pytest.mark.parametrize("state", _random_states(60))
def test_inverse_metric_and_rhs_vs_complex_step(state):
    """The oracle's contravariant metric equals a numerical 4x4 inverse of the
    covariant metric, and its Hamilton equations equal dH/dp (exact, linear)
    and -dH/dx by complex-step differentiation of H = 1/2 p g^-1 p."""
    M, a, r, th, pr, pth, E, L = state
    gi, dgr, dgth = O.metric_inv(M, a, r, th)
    ginv = np.linalg.inv(_g_cov_numpy(M, a, r, th).real)
    np.testing.assert_allclose(gi, [ginv[0, 0], ginv[0, 3], ginv[1, 1], ginv[2, 2], ginv[3, 3]],
                               rtol=1e-12, atol=1e-14 * np.abs(ginv).max())

    p = np.array([-E, pr, pth, L])

    def H(rr, tt):
        return 0.5 * p @ np.linalg.inv(_g_cov_numpy(M, a, rr, tt)) @ p

    eps = 1e-30
    dHdr = H(r + 1j * eps * r, th).imag / (eps * r)
    dHdth = H(r, th + 1j * eps).imag / eps
    xdot = ginv @ p  # dx^mu/dlambda = g^{mu nu} p_nu
    got = O.rhs(M, a, [r, th, 0.3, pr, pth], E, L)
    scale = np.abs(got).max() + 1.0
    want = [xdot[1], xdot[2], xdot[3], -dHdr, -dHdth, xdot[0]]
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-12 * scale)
    # the Hamiltonian itself
    assert O.hamiltonian(M, a, [r, th, 0.3, pr, pth], E, L) == pytest.approx(H(r, th).real,
                                                                            rel=1e-11, abs=1e-12 * scale)


@pytest.mark.parametrize("state", _random_states(30))
def test_carter_separated_form(state):
    """2 Sigma H = Delta p_r^2 + p_th^2 + (L/sin - a E sin)^2 - ((r^2+a^2)E - aL)^2/Delta
    (Carter 1968), and the relative residual uses the magnitudes of those terms."""
    M, a, r, th, pr, pth, E, L = state
    s, c = math.sin(th), math.cos(th)
    Sig = r * r + a * a * c * c
    Del = r * r - 2 * M * r + a * a
    terms = [Del * pr * pr, pth * pth, (L / s - a * E * s) ** 2, -((r * r + a * a) * E - a * L) ** 2 / Del]
    z = [r, th, 0.0, pr, pth]
    H = O.hamiltonian(M, a, z, E, L)
    D = sum(abs(t) for t in terms)
    assert 2 * Sig * H == pytest.approx(sum(terms), abs=1e-12 * D)
    assert O.hamiltonian_rel(M, a, z, E, L) == pytest.approx(abs(2 * Sig * H) / D, rel=1e-9, abs=1e-15)


def test_rhs_phi_independent():
    """Axisymmetry: nothing depends on phi."""
    z1 = [5.0, 1.1, 0.0, 0.3, 2.0]
    z2 = [5.0, 1.1, 2.7, 0.3, 2.0]
    np.testing.assert_array_equal(O.rhs(1.0, 0.7, z1, 0.9, 2.1), O.rhs(1.0, 0.7, z2, 0.9, 2.1))


@pytest.mark.parametrize("a,r", [(1.0, 1.0105), (1.0, 1.05), (0.998, 1.075), (0.9, 1.45)])
def test_relative_residual_rounding_near_the_horizon(a, r):
    """The oracle's |H|_rel of exactly null states (p_r from H = 0 in 50-digit
    arithmetic, then rounded to double) against a 50-digit evaluation of the
    same rounded state: the oracle's own rounding stays within
    2 eps (r^2 + a^2)^2 / Delta.  The t-phi block of its metric inverse
    divides by g_t_phi^2 - g_tt g_phi_phi = Delta sin^2 theta, formed from
    terms of size (r^2 + a^2)^2; next to an extremal horizon, where
    Delta = (r - M)^2 is ~1e-4 at the capture radius, that rounding reaches
    ~1e-12, above the truncation residues of an rtol 1e-12 integration."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    rng = np.random.default_rng(11)
    M = 1.0
    bound = 2.0 * np.finfo(float).eps * (r * r + a * a) ** 2 / (r * r - 2 * M * r + a * a)
    errs = []
    for _ in range(100):
        th, b, pth = float(rng.uniform(0.3, 2.8)), float(rng.uniform(-6.5, 1.9)), float(rng.uniform(-1.0, 1.0))
        R, TH, A = mp.mpf(r), mp.mpf(th), mp.mpf(a)
        Del = R * R - 2 * R + A * A
        T = b / mp.sin(TH) - A * mp.sin(TH)
        W = R * R + A * A - A * b
        pr2 = (W * W / Del - pth * pth - T * T) / Del
        if pr2 <= 0:
            continue
        z = np.array([r, th, 0.0, -float(mp.sqrt(pr2)), pth])
        PR, PTH = mp.mpf(z[3]), mp.mpf(pth)
        K = Del * PR * PR + PTH * PTH + T * T - W * W / Del
        D = Del * PR * PR + PTH * PTH + T * T + W * W / Del
        exact = float(abs(K) / D)
        errs.append(abs(O.hamiltonian_rel(M, a, z, 1.0, b) - exact))
    errs = np.array(errs)
    assert errs.size > 50
    assert errs.max() <= bound, (errs.max(), bound)
    if a == 1.0 and r < 1.02:
        # the effect is real at the extremal capture radius, not a loose bound
        assert np.median(errs) > 1e-13
