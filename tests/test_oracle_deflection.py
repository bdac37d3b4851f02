"""Pins of the oracle's deflection diagnostics for a point source behind
the hole (the Einstein-ring geometry of Sect. 4.3).

- Schwarzschild: the swept angle from the observer to the outbound crossing
  of r_src equals the orbit quadrature, and the angle to the source (at the
  antipode of the observer) is |Psi - pi| folded into [0, pi];
- ring flags: brute force on synthetic deflection maps.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests import schwarzschild_quad as SQ


@pytest.mark.parametrize("b", [6.0, 8.0, 12.0, 20.0])
def test_swept_angle_vs_quadrature(b):
    r0 = 1000.0
    rho = b * math.sqrt(1 - 2 / r0)
    s = O.Setup(a=0.0, r_obs=r0, incl=math.radians(60), method=O.DP45, rtol=1e-12, atol=1e-12,
                src_on=1, r_src=r0)
    ang = np.linspace(0.1, 2 * math.pi, 5, endpoint=False)
    o = O.trace_xy(s, rho * np.cos(ang), rho * np.sin(ang))
    want = SQ.swept_to_radius(b, r0, r0)
    assert (o["fate"] == O.ESCAPED).all()
    np.testing.assert_allclose(o["deflection"], want, rtol=1e-9)
    folded = np.abs(((want - math.pi) + math.pi) % (2 * math.pi) - math.pi)
    np.testing.assert_allclose(o["psi"], folded, atol=1e-8)


def test_captured_rays_have_no_deflection():
    s = O.Setup(a=0.0, r_obs=1000.0, incl=1.0, method=O.DP45, src_on=1, r_src=1000.0)
    o = O.trace_xy(s, np.array([1.0, -2.0]), np.array([0.5, 1.0]))
    assert (o["fate"] == O.CAPTURED).all()
    assert np.isnan(o["deflection"]).all() and np.isnan(o["psi"]).all()


def _ring_brute(nx, ny, d):
    d = d.reshape(ny, nx)
    out = np.zeros((ny, nx), np.uint8)
    for j in range(ny):
        for i in range(nx):
            for jj, ii in ((j, i + 1), (j + 1, i)):
                if jj < ny and ii < nx and np.isfinite(d[j, i]) and np.isfinite(d[jj, ii]):
                    lo, hi = sorted((d[j, i], d[jj, ii]))
                    # an odd multiple of pi in (lo, hi]
                    k = math.ceil((lo / math.pi - 1) / 2)
                    while (2 * k + 1) * math.pi <= lo:
                        k += 1
                    if (2 * k + 1) * math.pi <= hi:
                        out[j, i] = 1
    return out.ravel()


def test_ring_flags_bruteforce():
    rng = np.random.default_rng(1)
    nx, ny = 23, 17
    d = rng.uniform(0, 12, nx * ny)
    d[rng.random(nx * ny) < 0.1] = np.nan
    np.testing.assert_array_equal(O.ring_flags(nx, ny, d), _ring_brute(nx, ny, d))


def _ring_radii(r0=1000.0):
    return SQ.einstein_ring_radii(r0)


def test_einstein_ring_radii_by_quadrature():
    """The primary ring at image radius 46.188M lies outside the +-12M field
    of the 1024^2 Kerr ring image (it needs the +-60M one); the 3 pi and 5 pi rings
    hug the shadow edge sqrt(27) sqrt(1 - 2/r0)."""
    r1, r3, r5 = _ring_radii()
    edge = math.sqrt(27.0) * math.sqrt(1.0 - 2.0 / 1000.0)
    assert abs(r1 - 46.18763) < 1e-4
    assert abs(r3 - 5.19741) < 1e-4
    assert edge < r5 < r3 < r1
    assert r5 - edge < 2e-5
    # weak field: the point-lens Einstein radius sqrt(4 M D_l D_ls / D_s) =
    # sqrt(2000) is the first-order value; the exact orbit bends more, so the
    # ring is wider by a few per cent
    assert 1.0 < r1 / math.sqrt(2000.0) < 1.05


def test_oracle_resolved_ring_lies_on_the_quadrature_radius():
    """a = 0, i = 60 deg, +-60M at 96x96: every ring-flagged pixel lies within
    one pixel of a quadrature ring radius, and the primary ring is flagged
    all around."""
    n, fov = 96, 60.0
    s = O.Setup(a=0.0, r_obs=1000.0, incl=math.radians(60), fov_x=fov, fov_y=fov, nx=n, ny=n, method=O.DP45,
                rtol=1e-12, atol=1e-12, r_escape=1100.0, src_on=1, r_src=1000.0)
    o = O.trace_pixels(s)
    ring = O.ring_flags(n, n, o["deflection"])
    dx = 2 * fov / n
    x = -fov + (np.arange(n) + 0.5) * dx
    rho = np.hypot(x[None, :], x[:, None]).ravel()
    radii = np.array(_ring_radii())
    dist = np.abs(rho[:, None] - radii[None, :]).min(1)
    flagged = ring.astype(bool)
    assert flagged.sum() > 100
    assert (dist[flagged] <= dx * (1 + 1e-9)).all(), dist[flagged].max() / dx
    # all around the primary ring: every 10-degree sector holds a flag
    ang = np.degrees(np.arctan2(x[:, None] + 0 * x[None, :], x[None, :] + 0 * x[:, None])).ravel()
    prim = flagged & (np.abs(rho - radii[0]) <= dx)
    sectors = np.unique(((ang[prim] + 180.0) // 10).astype(int))
    assert sectors.size == 36
