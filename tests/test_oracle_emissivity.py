"""Pins of the oracle's tapered disk emissivity, used for the differentiable
disk image: I_em = (M/r)^2 (1 - sqrt(r_in/r)) times the smoothstep
3s^2 - 2s^3, s = (r_out - r)/(2M), over the last 2M before r_out.

The form is a modelling choice (the paper's Page-Thorne model is not given);
what is pinned are the properties it is chosen for: it vanishes at r_in and
at r_out, it and its radial derivative are continuous where the taper
starts and at r_out (so the image is continuous in r_in and r_out and the
finite differences of the adjoint's check see no jumps), and it is the
untapered profile inside r_out - 2M.
"""
import math

import pytest

import oracle as O

M, RIN, ROUT = 1.0, 2.5, 30.0


def em(r, rin=RIN, rout=ROUT):
    return O.emissivity(M, r, rin, rout, 2.0, 1)


def d_dr(r, h=1e-6):
    return (em(r + h) - em(r - h)) / (2 * h)


def test_vanishes_at_both_edges():
    assert em(RIN) == 0.0
    assert abs(em(ROUT)) < 1e-18
    assert em(0.5 * (RIN + ROUT)) > 0.0


def test_continuous_with_continuous_slope_where_the_taper_starts():
    r1 = ROUT - 2 * M
    for h in (1e-5, 1e-7):
        assert em(r1 + h) == pytest.approx(em(r1 - h), rel=10 * h)
    left, right = d_dr(r1 - 1e-6, 1e-8), d_dr(r1 + 1e-6, 1e-8)
    assert right == pytest.approx(left, rel=1e-4)


def test_slope_vanishes_linearly_at_the_outer_edge():
    d1, d2 = d_dr(ROUT - 1e-3, 1e-7), d_dr(ROUT - 1e-4, 1e-7)
    assert d1 < 0.0 and d2 < 0.0
    assert d2 / d1 == pytest.approx(0.1, rel=2e-3)


def test_untapered_inside():
    for r in (3.0, 7.3, 20.0, ROUT - 2 * M - 1e-9):
        base = (M / r) ** 2
        assert em(r) / base + math.sqrt(RIN / r) == pytest.approx(1.0, rel=1e-14)


def test_inner_edge_is_a_simple_zero():
    # 1 - sqrt(r_in/r) ~ (r - r_in)/(2 r_in): the slope at r_in is (M/r_in)^2 / (2 r_in)
    assert d_dr(RIN + 1e-6, 1e-8) == pytest.approx((M / RIN) ** 2 / (2 * RIN), rel=1e-4)


def test_power_law_model_is_unchanged():
    assert O.emissivity(M, 7.0, RIN, ROUT, 2.0, 0) == pytest.approx((1 / 7.0) ** 2, rel=1e-15)
    assert O.emissivity(M, 7.0, RIN, ROUT, 3.0, 0) == pytest.approx((1 / 7.0) ** 3, rel=1e-15)
