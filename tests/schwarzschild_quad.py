"""Semi-analytic Schwarzschild photon orbits, used to pin the oracle.

A photon of impact parameter b moves in a plane; with u = 1/r its orbit obeys
(du/dphi)^2 = F(u) = 2M u^3 - u^2 + 1/b^2 = 2M (u - u1)(u - u2)(u - u3),
u1 < 0 < u2 <= u3 when b > 3 sqrt(3) M (u2 is the turning point).  The swept
angle from u_a to the turning point is a quadrature made regular by the
substitution u = u2 - t^2.  Independent of the oracle: SciPy quadrature and
root finding on the textbook orbit equation.
"""
import math
import warnings

import numpy as np
from scipy import integrate, optimize

# quad reports round-off when it cannot reach 1e-14; the pins use 1e-9
warnings.filterwarnings("ignore", category=integrate.IntegrationWarning)

B_CRIT = math.sqrt(27.0)


def impact_parameter(rho, r0, M=1.0):
    """b of the pixel at image radius rho for an observer at r0 (a = 0)."""
    return rho / math.sqrt(1.0 - 2.0 * M / r0)


def _roots(b, M):
    r = np.sort(np.roots([2.0 * M, -1.0, 0.0, 1.0 / (b * b)]).real)
    return r[0], r[1], r[2]


def to_turning_point(b, ua, M=1.0):
    """Swept angle from u = ua to the turning point (b > b_crit)."""
    u1, u2, u3 = _roots(b, M)
    T = math.sqrt(max(u2 - ua, 0.0))

    def f(t):
        return 2.0 / math.sqrt(2.0 * M * (u2 - u1 - t * t) * (u3 - u2 + t * t))

    val, _ = integrate.quad(f, 0.0, T, epsabs=1e-15, epsrel=1e-14, limit=200)
    return val


def plunge_angle(b, ua, ub, M=1.0):
    """Swept angle from ua to ub > ua along an orbit without turning point."""
    val, _ = integrate.quad(lambda u: 1.0 / math.sqrt(2 * M * u ** 3 - u * u + 1 / (b * b)), ua, ub,
                            epsabs=1e-15, epsrel=1e-14, limit=200)
    return val


def swept_to_radius(b, r0, r_end, M=1.0):
    """Total swept angle from r0 (ingoing) to the outbound crossing of r_end."""
    return to_turning_point(b, 1.0 / r0, M) + to_turning_point(b, 1.0 / r_end, M)


def radius_at_swept_angle(b, r0, psi, M=1.0):
    """Radius reached after sweeping psi from r0 (ingoing start).  Returns
    None when the photon is captured or escapes before sweeping psi."""
    u0 = 1.0 / r0
    if b <= B_CRIT * M:
        u_h = 1.0 / (2.0 * M)
        if plunge_angle(b, u0, u_h, M) <= psi:
            return None
        u = optimize.brentq(lambda v: plunge_angle(b, u0, v, M) - psi, u0, u_h, xtol=1e-16, rtol=1e-15)
        return 1.0 / u
    u1, u2, u3 = _roots(b, M)
    G0 = to_turning_point(b, u0, M)
    if psi <= G0:
        u = optimize.brentq(lambda v: G0 - to_turning_point(b, v, M) - psi, u0, u2, xtol=1e-16, rtol=1e-15)
        return 1.0 / u
    rest = psi - G0
    if rest >= to_turning_point(b, 0.0, M):
        return None
    u = optimize.brentq(lambda v: to_turning_point(b, v, M) - rest, 0.0, u2, xtol=1e-16, rtol=1e-15)
    return 1.0 / u


def equator_crossing_angles(x, y, incl, n=3):
    """Swept angles at which the orbit plane of pixel (x, y) meets the
    equatorial plane, for an observer at inclination incl.  The plane is
    spanned by the observer direction and e_perp ~ y e_theta - x e_phi."""
    rho = math.hypot(x, y)
    psi0 = math.atan2(rho * math.cos(incl), y * math.sin(incl))
    if psi0 <= 0:
        psi0 += math.pi
    return [psi0 + k * math.pi for k in range(n)]


def einstein_ring_radii(r0=1000.0, M=1.0):
    """Image radii of the Einstein rings of a source at r_src = r0 directly
    behind the hole, seen from r0: Psi(b) = (2k + 1) pi (k = 0, 1, 2) by the
    orbit quadrature, b converted to the image radius rho = b sqrt(1 - 2M/r0)."""
    out = []
    for k, (lo, hi) in ((1, (6.0, 100.0)), (3, (5.1962, 6.0)), (5, (5.1961525, 5.1962))):
        b = optimize.brentq(lambda v: swept_to_radius(v * M, r0, r0, M) - k * math.pi, lo, hi, xtol=1e-14)
        out.append(b * M * math.sqrt(1.0 - 2.0 * M / r0))
    return out
