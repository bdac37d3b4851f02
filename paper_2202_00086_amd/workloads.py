"""Seeded synthetic workloads: camera configurations around an analytic metric.

This module only describes inputs (plain parameter dicts); it holds none of
the ray tracer's arithmetic.  Both the GPU binding (kerrtrace.Renderer) and
the CPU oracle (oracle.Setup) accept these keyword names.

  schwarzschild_shadow_64   a = 0, 64x64, r_obs = 1000M, i = 90 deg, +-10M,
                            fixed-step RK4 in s (h_s = 1/128), capture r < 2.01M,
                            escape r > 1100M.
  kerr_ring_1024(a)         a in {0.5, 0.9, 0.998}, 1024x1024, i = 60 deg,
                            r_obs = 1000M, +-12M, DP45 rtol = atol = 1e-12,
                            point source at r_src = 1000M behind the hole.
  schwarzschild_disk_2048   a = 0, 2048x2048, i = 80 deg, r_obs = 1000M,
                            +-35M, thin Keplerian disk 6M..30M, I_em ~ r^-2.
"""
import math


def schwarzschild_shadow_64():
    return dict(M=1.0, a=0.0, r_obs=1000.0, incl=math.pi / 2, fov_x=10.0, fov_y=10.0, nx=64, ny=64,
                method=0, h_fixed=1.0 / 128, cap_buffer=0.01, r_escape=1100.0, max_steps=1_000_000)


def kerr_ring(a=0.9, n=1024, rtol=1e-12):
    return dict(M=1.0, a=a, r_obs=1000.0, incl=math.radians(60.0), fov_x=12.0, fov_y=12.0, nx=n,
                ny=n, method=1, rtol=rtol, atol=rtol, h_init=1.0, cap_buffer=0.01, r_escape=1100.0,
                max_steps=1_000_000, src_on=1, r_src=1000.0)


def schwarzschild_disk(n=2048, rtol=1e-12):
    return dict(M=1.0, a=0.0, r_obs=1000.0, incl=math.radians(80.0), fov_x=35.0, fov_y=35.0, nx=n,
                ny=n, method=1, rtol=rtol, atol=rtol, h_init=1.0, cap_buffer=0.01, r_escape=1100.0,
                max_steps=1_000_000, disk_on=1, r_in=6.0, r_out=30.0, emis_q=2.0)


def kerr_disk(a=0.9, incl_deg=60.0, n=256, r_in=None, r_obs=1000.0, fov=35.0, rtol=1e-12):
    """Kerr thin disk, r_in defaults to 1.01 r_+ ... set explicitly by callers."""
    return dict(M=1.0, a=a, r_obs=r_obs, incl=math.radians(incl_deg), fov_x=fov, fov_y=fov, nx=n,
                ny=n, method=1, rtol=rtol, atol=rtol, h_init=1.0, cap_buffer=0.01, r_escape=1.1 * r_obs,
                max_steps=1_000_000, disk_on=1, r_in=r_in if r_in is not None else 6.0, r_out=30.0,
                emis_q=2.0)


def oracle_setup(params):
    """oracle.Setup keyword arguments from a workload dict."""
    return {k: v for k, v in params.items()}
