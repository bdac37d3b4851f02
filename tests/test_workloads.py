"""Seeded workload generators: reproducible, in range, and the ISCO input
pinned to the circular-orbit energy it is the minimum of."""
import math

import numpy as np
import pytest

from paper_2202_00086_amd import workloads as W


def _circular_energy(r, a):
    """Specific energy of a circular equatorial orbit moving in +phi (M = 1),
    Bardeen, Press & Teukolsky (1972)."""
    return (1.0 - 2.0 / r + a / r ** 1.5) / math.sqrt(1.0 - 3.0 / r + 2.0 * a / r ** 1.5)


@pytest.mark.parametrize("a, r", [(0.0, 6.0), (1.0, 1.0), (-1.0, 9.0)])
def test_isco_special_values(a, r):
    assert W.isco(a) == pytest.approx(r, rel=1e-12)


@pytest.mark.parametrize("a", [-0.9, -0.3, 0.1, 0.5, 0.9, 0.998])
def test_isco_is_the_minimum_of_the_circular_orbit_energy(a):
    r = W.isco(a)
    e = [_circular_energy(r * f, a) for f in (0.999, 1.0, 1.001)]
    assert e[1] < e[0] and e[1] < e[2]
    h = 1e-5 * r
    de = (_circular_energy(r + h, a) - _circular_energy(r - h, a)) / (2 * h)
    assert abs(de) < 1e-7


def test_isco_scales_with_mass():
    assert W.isco(1.8, M=2.0) == pytest.approx(2.0 * W.isco(0.9), rel=1e-14)


def test_heterogeneous_batch_is_seeded_and_in_range():
    im1, integ = W.heterogeneous_batch()
    im2, _ = W.heterogeneous_batch()
    assert im1 == im2 and len(im1) == 256
    sides = np.array([[i["nx"], i["ny"]] for i in im1])
    assert sides.min() == 64 and sides.max() == 1024 and (sides % 64 == 0).all()
    # one square side per image, drawn before a, i and r_obs
    assert (sides[:, 0] == sides[:, 1]).all()
    assert int((sides[:, 0] * sides[:, 1]).sum()) == 105_156_608
    a = np.array([i["a"] for i in im1])
    incl = np.degrees([i["incl"] for i in im1])
    r = np.array([i["r_obs"] for i in im1])
    assert (a >= 0).all() and (a < 0.998).all()
    assert (incl >= 5).all() and (incl < 85).all()
    assert (r >= 100).all() and (r < 1e4).all()
    for i in im1:
        assert i["r_in"] == W.isco(i["a"]) and i["r_out"] == 30.0 and i["disk_on"] == 1
    assert integ["r_escape"] == 0.0
    assert set(im1[0]) <= set(W.IMAGE_KEYS)
    p = W.image_params(im1[3], integ)
    assert p["r_escape"] == 1.1 * im1[3]["r_obs"] and p["nx"] == im1[3]["nx"]
    assert W.heterogeneous_batch(seed=1)[0] != im1


def test_heterogeneous_batch_draw_order():
    """Side, then a, inclination and r_obs, per image, from one generator."""
    rng = np.random.default_rng(20220201)
    ref = []
    for _ in range(3):
        side = 64 * (1 + int(rng.integers(0, 16)))
        ref.append((side, float(rng.uniform(0.0, 0.998)), math.radians(float(rng.uniform(5.0, 85.0))),
                    float(10.0 ** rng.uniform(2.0, 4.0))))
    im, _ = W.heterogeneous_batch(n_images=3)
    assert [(i["nx"], i["a"], i["incl"], i["r_obs"]) for i in im] == ref
    ragged, _ = W.heterogeneous_batch(n_images=40, seed=7, side_unit=8, side_steps=8, square=False)
    assert any(i["nx"] != i["ny"] for i in ragged)
