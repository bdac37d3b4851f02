"""Pins of the oracle's camera: the initial momenta printed in the paper's
figure captions (Sect. 3.1), the null condition and the image-plane grid."""
import math
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig34_initial_momenta.txt")


def _golden_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([float(v) for v in line.split()])
    return rows


@pytest.mark.parametrize("row", _golden_rows())
def test_caption_initial_momenta(row):
    """a = 0.98, r0 = 100, theta0 = pi/2: the oracle's p_t, p_r, p_theta, p_phi
    reproduce the captions' printed values."""
    x, y, pt, pr, pth, pph, tol_pr = row
    st, bad = O.camera_ray(1.0, 0.98, 100.0, math.pi / 2, x, y)
    assert not bad
    assert st[0] == 100.0 and st[1] == math.pi / 2 and st[2] == 0.0
    assert -st[5] == pytest.approx(pt, abs=5e-7)
    assert st[3] == pytest.approx(pr, abs=tol_pr)
    assert st[4] == pytest.approx(pth, abs=5e-7)
    assert st[6] == pytest.approx(pph, abs=5e-7)


@pytest.mark.parametrize("a,incl,r0", [(0.0, 1.0, 1000.0), (0.9, math.radians(60), 1000.0),
                                      (0.998, math.radians(5), 100.0), (0.5, math.radians(85), 1e4)])
def test_initial_state_is_null(a, incl, r0):
    """H(lambda = 0) vanishes to rounding for every pixel of a 32x32 grid."""
    rng = np.random.default_rng(3)
    for x, y in rng.uniform(-35, 35, size=(200, 2)):
        st, bad = O.camera_ray(1.0, a, r0, incl, x, y)
        assert not bad
        H = O.hamiltonian(1.0, a, st[:5], st[5], st[6])
        assert abs(H) <= 1e-15 * max(1.0, st[3] ** 2)
        assert O.hamiltonian_rel(1.0, a, st[:5], st[5], st[6]) <= 1e-15


def test_observer_frame_energy_is_one():
    """The ZAMO tetrad of eq:matrix measures P^t = 1 and |P|^2 = 0 (eq:const):
    recompute the frame components directly from the metric at the camera."""
    M, a, r0, incl = 1.0, 0.9, 50.0, 1.0
    g = O.metric_cov(M, a, r0, incl)
    for x, y in [(3.0, -2.0), (-7.5, 0.25), (0.1, 9.0)]:
        st, _ = O.camera_ray(M, a, r0, incl, x, y)
        E, L, pr, pth = st[5], st[6], st[3], st[4]
        At = math.sqrt(g[4] / (g[1] ** 2 - g[0] * g[4]))
        Pt = At * (E + g[1] / g[4] * L)         # eta^{t mu} Lambda_mu^nu p_nu with p_t = -E
        Pr, Pth, Pph = pr / math.sqrt(g[2]), pth / math.sqrt(g[3]), L / math.sqrt(g[4])
        assert Pt == pytest.approx(1.0, rel=1e-14)
        assert -Pt ** 2 + Pr ** 2 + Pth ** 2 + Pph ** 2 == pytest.approx(0.0, abs=1e-14)
        # eq:pimf: x = -r0 P^phi / P^t, y = r0 P^theta / P^t
        assert -r0 * Pph / Pt == pytest.approx(x, rel=1e-13)
        assert r0 * Pth / Pt == pytest.approx(y, rel=1e-13)
        assert pr < 0  # ingoing


def test_invalid_outside_image_disk():
    st, bad = O.camera_ray(1.0, 0.5, 10.0, 1.0, 8.0, 6.0)  # x^2 + y^2 = r0^2
    assert bad


def test_pixel_centres():
    s = O.Setup(fov_x=12.0, fov_y=6.0, nx=4, ny=3)
    xs = [O.pixel_xy(s, i, 0)[0] for i in range(4)]
    ys = [O.pixel_xy(s, 0, j)[1] for j in range(3)]
    np.testing.assert_allclose(xs, [-9.0, -3.0, 3.0, 9.0])
    np.testing.assert_allclose(ys, [-4.0, 0.0, 4.0])
