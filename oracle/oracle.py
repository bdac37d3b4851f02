"""ctypes front end of the CPU FP64 oracle (libkt_oracle.so).

TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the benchmark's
CPU-baseline leg may use it.  It shares no code with the GPU library; the
only thing both sides are fed from is the seeded workload description.

All arrays are host numpy arrays.  Angles are radians, lengths in units of M
(M itself is a parameter; the paper sets M = 1).
"""
import ctypes as C
import math
import os
from dataclasses import dataclass, fields

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("KT_ORACLE_LIB") or os.path.join(HERE, "libkt_oracle.so")

ESCAPED, CAPTURED, DISK, MAXSTEPS, STEPFAIL, INVALID = range(6)
RK4_S, DP45, RKF45, CK45, BS, BS_RAT = 0, 1, 2, 3, 4, 5
SKY_NONE, SKY_GREEN, SKY_RED, SKY_BLUE, SKY_YELLOW, SKY_LINE = range(6)
KERR, QMETRIC = 0, 1
BS_COLUMNS = 5


class _Setup(C.Structure):
    _fields_ = [
        ("M", C.c_double), ("a", C.c_double), ("metric", C.c_int32), ("q", C.c_double),
        ("r_obs", C.c_double), ("incl", C.c_double), ("fov_x", C.c_double), ("fov_y", C.c_double),
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("method", C.c_int32),
        ("h_fixed", C.c_double), ("rtol", C.c_double), ("atol", C.c_double), ("h_init", C.c_double),
        ("cap_buffer", C.c_double), ("r_escape", C.c_double),
        ("max_steps", C.c_int64),
        ("disk_on", C.c_int32), ("r_in", C.c_double), ("r_out", C.c_double), ("emis_q", C.c_double),
        ("rotation", C.c_int32), ("l0", C.c_double), ("emis_model", C.c_int32),
        ("src_on", C.c_int32), ("r_src", C.c_double),
        ("sky_on", C.c_int32), ("grid_deg", C.c_double), ("line_deg", C.c_double),
    ]


class _Out(C.Structure):
    _fields_ = [
        ("fate", C.c_void_p),
        ("r_hit", C.c_void_p), ("g", C.c_void_p), ("intensity", C.c_void_p),
        ("max_abs_h", C.c_void_p), ("max_rel_h", C.c_void_p),
        ("psi", C.c_void_p), ("deflection", C.c_void_p),
        ("theta_f", C.c_void_p), ("phi_f", C.c_void_p),
        ("n_cross", C.c_void_p),
        ("n_steps", C.c_void_p), ("n_evals", C.c_void_p),
        ("sky", C.c_void_p),
    ]


_F64_OUT = ("r_hit", "g", "intensity", "max_abs_h", "max_rel_h", "psi", "deflection",
            "theta_f", "phi_f")


@dataclass
class Setup:
    """Oracle problem description (one image)."""
    M: float = 1.0
    a: float = 0.0
    metric: int = 0                # 0 Kerr, 1 q-metric
    q: float = 0.0
    r_obs: float = 1000.0
    incl: float = math.pi / 2
    fov_x: float = 10.0
    fov_y: float = 10.0
    nx: int = 64
    ny: int = 64
    method: int = DP45
    h_fixed: float = 1.0 / 128
    rtol: float = 1e-12
    atol: float = 1e-12
    h_init: float = 1.0
    cap_buffer: float = 0.01
    r_escape: float = 0.0          # 0 means 1.1 * r_obs
    max_steps: int = 1_000_000
    disk_on: int = 0
    r_in: float = 6.0
    r_out: float = 30.0
    emis_q: float = 2.0
    rotation: int = 0              # 0 Keplerian, 1 constant l0
    l0: float = 0.0
    emis_model: int = 0            # 0 (M/r)^emis_q, 1 tapered (M/r)^2 (1 - sqrt(r_in/r))
    src_on: int = 0
    r_src: float = 1000.0
    sky_on: int = 0
    grid_deg: float = 6.0
    line_deg: float = 0.25

    def _c(self):
        s = _Setup()
        for f in fields(self):
            setattr(s, f.name, getattr(self, f.name))
        if s.r_escape <= 0.0:
            s.r_escape = 1.1 * self.r_obs
        return s


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH} (run oracle/build.py)")
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.ko_metric_cov.argtypes = [C.c_double] * 4 + [dp]
        L.ko_metric_inv.argtypes = [C.c_double] * 4 + [dp, dp, dp]
        L.ko_hamiltonian.argtypes = [C.c_double, C.c_double, dp, C.c_double, C.c_double]
        L.ko_hamiltonian.restype = C.c_double
        L.ko_hamiltonian_rel.argtypes = [C.c_double, C.c_double, dp, C.c_double, C.c_double]
        L.ko_hamiltonian_rel.restype = C.c_double
        L.ko_rhs.argtypes = [C.c_double, C.c_double, dp, C.c_double, C.c_double, dp]
        L.ko_camera_ray.argtypes = [C.c_double] * 6 + [dp]
        L.ko_camera_ray.restype = C.c_int
        L.ko_pixel_xy.argtypes = [C.POINTER(_Setup), C.c_int32, C.c_int32, dp, dp]
        L.ko_trace_xy.argtypes = [C.POINTER(_Setup), dp, dp, C.c_int64, C.POINTER(_Out), C.c_int]
        L.ko_trace_pixels.argtypes = [C.POINTER(_Setup), C.c_void_p, C.c_int64, C.POINTER(_Out),
                                      C.c_int]
        L.ko_trace_one.argtypes = [C.POINTER(_Setup), C.c_double, C.c_double, dp, C.c_int64,
                                   C.POINTER(_Out)]
        L.ko_trace_one.restype = C.c_int64
        L.ko_ring_flags.argtypes = [C.c_int32, C.c_int32, dp, C.c_void_p]
        L.ko_horizon.argtypes = [C.c_double, C.c_double]
        L.ko_horizon.restype = C.c_double
        L.ko_harmonic_fixed.argtypes = [C.c_int32, C.c_double, C.c_int64, dp]
        L.ko_fixed_steps.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_int64, dp, dp]
        L.ko_one_step.argtypes = [C.c_int32, C.c_int32, C.c_double, dp, dp, dp]
        L.ko_one_step.restype = C.c_int
        L.ko_tableau.argtypes = [C.c_int32, dp, dp, dp]
        L.ko_bs_extrapolate.argtypes = [C.c_int32, C.c_int32, dp, dp]
        L.ko_sky_code.argtypes = [C.c_double] * 4
        L.ko_sky_code.restype = C.c_int
        L.ko_disk_omega.argtypes = [C.c_double] * 3 + [C.c_int32, C.c_double]
        L.ko_disk_omega.restype = C.c_double
        L.ko_metric_cov_k.argtypes = [C.c_int32] + [C.c_double] * 5 + [dp]
        L.ko_metric_derivs_k.argtypes = [C.c_int32] + [C.c_double] * 5 + [dp, dp]
        L.ko_hamiltonian_k.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, dp, C.c_double, C.c_double]
        L.ko_hamiltonian_k.restype = C.c_double
        L.ko_hamiltonian_rel_k.argtypes = L.ko_hamiltonian_k.argtypes
        L.ko_hamiltonian_rel_k.restype = C.c_double
        L.ko_rhs_k.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, dp, C.c_double, C.c_double, dp]
        L.ko_camera_ray_k.argtypes = [C.c_int32] + [C.c_double] * 7 + [dp]
        L.ko_camera_ray_k.restype = C.c_int
        L.ko_emissivity.argtypes = [C.c_double] * 5 + [C.c_int32]
        L.ko_emissivity.restype = C.c_double
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def metric_cov(M, a, r, th):
    g = np.zeros(5)
    lib().ko_metric_cov(M, a, r, th, _dptr(g))
    return g


def metric_inv(M, a, r, th):
    gi, dr, dth = np.zeros(5), np.zeros(5), np.zeros(5)
    lib().ko_metric_inv(M, a, r, th, _dptr(gi), _dptr(dr), _dptr(dth))
    return gi, dr, dth


def hamiltonian(M, a, state, E, L):
    z = np.ascontiguousarray(state, dtype=np.float64)
    return lib().ko_hamiltonian(M, a, _dptr(z), E, L)


def hamiltonian_rel(M, a, state, E, L):
    z = np.ascontiguousarray(state, dtype=np.float64)
    return lib().ko_hamiltonian_rel(M, a, _dptr(z), E, L)


def rhs(M, a, state, E, L):
    """d/dlambda (r, theta, phi, p_r, p_theta) and dt/dlambda (6 values)."""
    z = np.ascontiguousarray(state, dtype=np.float64)
    out = np.zeros(6)
    lib().ko_rhs(M, a, _dptr(z), E, L, _dptr(out))
    return out


def camera_ray(M, a, r_obs, incl, x, y):
    """(state[7] = r, theta, phi, p_r, p_theta, E, L ; invalid flag)."""
    out = np.zeros(7)
    bad = lib().ko_camera_ray(M, a, r_obs, incl, x, y, _dptr(out))
    return out, bool(bad)


def horizon(M, a):
    return lib().ko_horizon(M, a)


def pixel_xy(setup, i, j):
    x, y = C.c_double(), C.c_double()
    s = setup._c()
    lib().ko_pixel_xy(C.byref(s), i, j, C.byref(x), C.byref(y))
    return x.value, y.value


def _alloc(n):
    o = {"fate": np.zeros(n, np.uint8), "n_cross": np.zeros(n, np.uint8), "sky": np.zeros(n, np.uint8),
         "n_steps": np.zeros(n, np.int32), "n_evals": np.zeros(n, np.int32)}
    for k in _F64_OUT:
        o[k] = np.zeros(n, np.float64)
    c = _Out()
    for k, v in o.items():
        setattr(c, k, v.ctypes.data)
    return o, c


def trace_pixels(setup, pix=None, threads=0):
    """Trace pixels pix (row-major j*nx+i; None = whole image).  Returns a
    dict of numpy arrays indexed like pix."""
    s = setup._c()
    if pix is None:
        n = setup.nx * setup.ny
        pptr = None
    else:
        pix = np.ascontiguousarray(pix, dtype=np.int32)
        n = pix.size
        pptr = pix.ctypes.data
    o, c = _alloc(n)
    lib().ko_trace_pixels(C.byref(s), pptr, n, C.byref(c), threads)
    return o


def trace_xy(setup, x, y, threads=0):
    s = setup._c()
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    o, c = _alloc(x.size)
    lib().ko_trace_xy(C.byref(s), _dptr(x), _dptr(y), x.size, C.byref(c), threads)
    return o


def trace_one(setup, x, y, max_points=200_000):
    """Trace one ray; returns (trajectory[k, 6] = lambda, r, theta, phi, p_r,
    p_theta per accepted state, result dict)."""
    s = setup._c()
    traj = np.zeros((max_points, 6))
    o, c = _alloc(1)
    n = lib().ko_trace_one(C.byref(s), x, y, _dptr(traj), max_points, C.byref(c))
    return traj[:n], {k: v[0] for k, v in o.items()}


def ring_flags(nx, ny, deflection):
    d = np.ascontiguousarray(deflection, dtype=np.float64)
    ring = np.zeros(nx * ny, np.uint8)
    lib().ko_ring_flags(nx, ny, _dptr(d), ring.ctypes.data)
    return ring


def sky_code(theta, phi, grid_deg=6.0, line_deg=0.25):
    return lib().ko_sky_code(theta, phi, grid_deg, line_deg)


def metric_cov_k(kind, M, a, q, r, th):
    g = np.zeros(5)
    lib().ko_metric_cov_k(kind, M, a, q, r, th, _dptr(g))
    return g


def metric_derivs_k(kind, M, a, q, r, th):
    dr, dth = np.zeros(5), np.zeros(5)
    lib().ko_metric_derivs_k(kind, M, a, q, r, th, _dptr(dr), _dptr(dth))
    return dr, dth


def hamiltonian_k(kind, M, a, q, state, E, L):
    z = np.ascontiguousarray(state, dtype=np.float64)
    return lib().ko_hamiltonian_k(kind, M, a, q, _dptr(z), E, L)


def hamiltonian_rel_k(kind, M, a, q, state, E, L):
    z = np.ascontiguousarray(state, dtype=np.float64)
    return lib().ko_hamiltonian_rel_k(kind, M, a, q, _dptr(z), E, L)


def rhs_k(kind, M, a, q, state, E, L):
    z = np.ascontiguousarray(state, dtype=np.float64)
    out = np.zeros(6)
    lib().ko_rhs_k(kind, M, a, q, _dptr(z), E, L, _dptr(out))
    return out


def camera_ray_k(kind, M, a, q, r_obs, incl, x, y):
    out = np.zeros(7)
    bad = lib().ko_camera_ray_k(kind, M, a, q, r_obs, incl, x, y, _dptr(out))
    return out, bool(bad)


def emissivity(M, r, r_in, r_out, emis_q=2.0, model=0):
    return lib().ko_emissivity(M, r, r_in, r_out, emis_q, model)


def disk_omega(M, a, r, rotation=0, l0=0.0):
    return lib().ko_disk_omega(M, a, r, rotation, l0)


def harmonic_fixed(method, T, n):
    out = np.zeros(2)
    lib().ko_harmonic_fixed(method, T, n, _dptr(out))
    return out


def fixed_steps(method, problem, T, n, y0):
    """n fixed steps on test problem 0 (y'' = -y as (y, y')) or 1 (y' = y^2)."""
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    out = np.zeros(y0.size)
    lib().ko_fixed_steps(method, problem, T, n, _dptr(y0), _dptr(out))
    return out


def one_step(method, problem, h, y0):
    """(y_new, error estimate, evaluations) of one step on a test problem."""
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    yn, e = np.zeros(y0.size), np.zeros(y0.size)
    nev = lib().ko_one_step(method, problem, h, _dptr(y0), _dptr(yn), _dptr(e))
    return yn, e, nev


def tableau(method):
    """(A[6, 6], b_propagated[6], b_embedded[6]) of RKF45 or CK45."""
    A, bp, be = np.zeros(36), np.zeros(6), np.zeros(6)
    lib().ko_tableau(method, _dptr(A), _dptr(bp), _dptr(be))
    return A.reshape(6, 6), bp, be


def bs_extrapolate(values, rational=False):
    """Last tableau row of the Bulirsch-Stoer extrapolation of chain ends
    values[k] (n_k = 2 (k + 1) substeps) to zero substep; row[-1] is the
    extrapolated value."""
    f = np.ascontiguousarray(values, dtype=np.float64)
    row = np.zeros(f.size)
    lib().ko_bs_extrapolate(1 if rational else 0, f.size, _dptr(f), _dptr(row))
    return row
