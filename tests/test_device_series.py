"""The polynomials of the trace kernel's source (sincos_shift, the stage
angles; sincos_theta, the full polar angle; exp_fast and log_join, the
q-metric's powers) against the functions they approximate, in 50-digit
arithmetic: each polynomial, with its coefficients
as the doubles the kernel holds, stays within the error bound its comment
states over its range.  A wrong sign, a dropped or mistyped coefficient, or
a polynomial for a different function fails these bounds."""
import os
import re

import mpmath as mp
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_00086_amd", "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("kt_device.h", "kt_elem.h")]

mp.mp.dps = 50


def _function_body(name):
    for path in SOURCES:
        text = open(path).read()
        m = re.search(rf"__device__ (?:__forceinline__|inline __attribute__\(\(always_inline\)\)) \w+ {name}\(",
                      text)
        if m:
            return text[m.start():text.index("\n}\n", m.start())]
    raise AssertionError(f"{name} not found in {SOURCES}")


def _horner(body, var):
    """Coefficients (highest degree first) of the Horner chain for `var`."""
    first = re.search(rf"double {var} = ([-+0-9.e]+);", body)
    rest = re.findall(rf"{var} = fma\({var}, \w+, ([-+0-9.e]+)\);", body)
    return [mp.mpf(float(first.group(1)))] + [mp.mpf(float(v)) for v in rest]


def _poly(coefs_high_first, x):
    p = coefs_high_first[0]
    for c in coefs_high_first[1:]:
        p = p * x + c
    return p


def _grid(end, n=1500):
    return [end * mp.mpf(k) / n for k in range(1, n + 1)]


def test_stage_shift_polynomials():
    body = _function_body("sincos_shift")
    ps, pc = _horner(body, "ps"), _horner(body, "pc")
    assert len(ps) == 5 and len(pc) == 6
    worst_s = worst_c = mp.mpf(0)
    for d in _grid(mp.mpf(1) / 2):
        x = d * d
        sd = d - _poly(ps, x) * x * d      # sin d as the kernel forms it
        cdm1 = -_poly(pc, x) * x           # cos d - 1
        worst_s = max(worst_s, abs(sd / mp.sin(d) - 1))
        worst_c = max(worst_c, abs(cdm1 - (mp.cos(d) - 1)))
    assert worst_s < 2.6e-17, worst_s       # relative error of sin d
    assert worst_c < 6e-18, worst_c         # absolute error of cos d


def test_polar_angle_polynomials():
    body = _function_body("sincos_theta")
    pc, ps = _horner(body, "pc"), _horner(body, "ps")
    assert len(pc) == 8 and len(ps) == 8
    worst_c = worst_s = mp.mpf(0)
    for u in _grid(mp.pi / 2):
        x = u * u
        cu = 1 + _poly(pc, x) * x          # cos u (sin theta up to sign)
        msu = _poly(ps, x) * x * u - u     # -sin u (cos theta)
        worst_c = max(worst_c, abs(cu - mp.cos(u)))
        worst_s = max(worst_s, abs(msu + mp.sin(u)))
    assert worst_c < 1.4e-17, worst_c
    assert worst_s < 4.1e-17, worst_s


@pytest.mark.parametrize("theta", [0.0, 1e-9, 0.3, 1.2, 1.5707963267948966, 2.9, 3.141592653589793 - 1e-9])
def test_polar_angle_fold_and_signs(theta):
    """The fold u = |t| - pi/2 and the sign choices of sincos_theta give sin
    and cos of theta itself (to 1e-15 absolute) at the poles, the equator
    and in between, and past the polar axis (theta < 0 or > pi)."""
    body = _function_body("sincos_theta")
    pc, ps = _horner(body, "pc"), _horner(body, "ps")
    for th in (mp.mpf(theta), -mp.mpf(theta), mp.mpf(theta) + mp.pi / 3 + mp.pi):
        t = th - 2 * mp.pi * mp.nint(th / (2 * mp.pi))
        u = abs(t) - mp.pi / 2
        x = u * u
        s = (-1 if t < 0 else 1) * abs(1 + _poly(pc, x) * x)  # copysign(cos u, t)
        c = _poly(ps, x) * x * u - u
        assert abs(s - mp.sin(th)) < 1e-15
        assert abs(c - mp.cos(th)) < 1e-15


def test_exp_polynomial():
    """exp_fast: e^t = 1 + t + t^2 G(t) on |t| <= (ln 2)/2, relative error."""
    body = _function_body("exp_fast")
    g = _horner(body, "p")
    assert len(g) == 12  # ten coefficients of G, then the two unit steps
    assert g[-2:] == [1, 1]
    T = mp.log(2) / 2
    worst = max(abs(_poly(g, t) / mp.exp(t) - 1) for t in [T * k / 1500 for k in range(-1500, 1501)])
    assert worst < 1e-17, worst


def test_log_polynomial():
    """log_join: ln m = 2 s + 2 s s^2 L(s^2) for m in [1/sqrt 2, sqrt 2),
    s = (m - 1)/(m + 1), relative error."""
    body = _function_body("log_join")
    lc = _horner(body, "p")
    assert len(lc) == 7
    smax = (mp.sqrt(2) - 1) / (mp.sqrt(2) + 1)
    worst = mp.mpf(0)
    for k in range(1, 1501):
        s = smax * k / 1500
        lm = 2 * s + 2 * s * s * s * _poly(lc, s * s)
        worst = max(worst, abs(lm / mp.log((1 + s) / (1 - s)) - 1))
    assert worst < 2e-18, worst


def test_coefficients_are_the_generators_output():
    """Every coefficient list in the kernel source is exactly what
    csrc/minimax_coefs.py prints (its Remez fits in 50-digit arithmetic,
    rounded to double)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("minimax_coefs", os.path.join(CSRC, "minimax_coefs.py"))
    mc = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mc)
    fits = mc.fit_all()

    def low_first(name, var):
        return [float(v) for v in _horner(_function_body(name), var)][::-1]

    assert low_first("sincos_shift", "ps") == fits["shift_sin"][0]
    assert low_first("sincos_shift", "pc") == fits["shift_cos"][0]
    assert low_first("sincos_theta", "pc") == [-v for v in fits["theta_cos"][0]]
    assert low_first("sincos_theta", "ps") == fits["theta_sin"][0]
    assert low_first("exp_fast", "p")[2:] == fits["exp_g"][0]   # after the two unit steps
    assert low_first("log_join", "p") == fits["log_l"][0]
