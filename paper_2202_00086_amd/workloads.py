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
  hamiltonian_norm_map      a = 0.98, 625x625, r_obs = 100M, i = 90 deg, +-8M
                            (the integrator comparison grid).
  lensing(a)                celestial-sphere lensing, r_obs = 100M, i = 90 deg.
  thin_disk_l0(a)           the Sect. 5 disk images with constant-l0 rotation.
  qmetric_lensing(q)        the appendix's q-metric in the lensing setup.
  differentiable_disk       a = 0.7, i = 45 deg, 512x512 disk with the tapered
                            emissivity; disk_fit_target is its fit target.
  heterogeneous_batch       256 seeded square Kerr disk images: sides 64..1024
                            in steps of 64, a ~ U[0, 0.998], i ~ U[5, 85] deg,
                            r_obs log-uniform in [100, 1e4]M, +-35M, disk
                            from the prograde ISCO to 30M, I_em ~ r^-2.
"""
import math

import numpy as np


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


def hamiltonian_norm_map(n=625, method=1, rtol=1e-12):
    """The integrator comparison of Sect. 3.1: a dense n x n grid over
    -8M <= x, y <= 8M seen from r0 = 100M; spin 0.98 and inclination 90 deg
    as for the two rays of that section's figures."""
    return dict(M=1.0, a=0.98, r_obs=100.0, incl=math.pi / 2, fov_x=8.0, fov_y=8.0, nx=n, ny=n,
                method=method, rtol=rtol, atol=rtol, h_init=1.0, cap_buffer=0.01, r_escape=110.0,
                max_steps=1_000_000)


def lensing(a=0.98, n=512, M=1.0, fov=20.0, rtol=1e-12):
    """Gravitational lensing of the coloured celestial sphere (Sect. 4.1-4.2):
    observer in the equatorial plane at r0 = 100M, phi0 = 0; sphere at
    r_cs = 1.1 r0; graticule every 6 deg (lines 0.25 deg wide on either
    side).  M = 0 (a = 0) is the flat reference image."""
    return dict(M=M, a=a, r_obs=100.0, incl=math.pi / 2, fov_x=fov, fov_y=fov, nx=n, ny=n, method=1,
                rtol=rtol, atol=rtol, h_init=1.0, cap_buffer=0.01, r_escape=110.0, max_steps=1_000_000,
                sky_on=1, grid_deg=6.0, line_deg=0.25)


def qmetric_lensing(q=0.5, n=512, fov=20.0, rtol=1e-12):
    """The q-metric (mass parameter M = 1, quadrupole q) seen like the Kerr
    lensing images: observer at r0 = 100M in the equatorial plane, the
    coloured sphere at 1.1 r0, capture at r < 2M + 0.01M."""
    return dict(lensing(a=0.0, n=n, fov=fov, rtol=rtol), metric=1, q=q)


def thin_disk_l0(a=0.5, nx=2048, ny=1024, rtol=1e-12):
    """The thin-disk images of Sect. 5: r0 = 1000M, i = 85 deg, x in [-24, 24],
    y in [-12, 12], disk from the ISCO to 20M rotating with constant specific
    angular momentum l0 = 2.8 (a = 0, 0.5) or 1.8 (a = 0.95); I_em ~ r^-2
    stands in for the Page-Thorne model."""
    return dict(M=1.0, a=a, r_obs=1000.0, incl=math.radians(85.0), fov_x=24.0, fov_y=12.0, nx=nx, ny=ny,
                method=1, rtol=rtol, atol=rtol, h_init=1.0, cap_buffer=0.01, r_escape=1100.0,
                max_steps=1_000_000, disk_on=1, r_in=isco(a), r_out=20.0, emis_q=2.0, rotation=1,
                l0=1.8 if a > 0.9 else 2.8)


def differentiable_disk(a=0.7, incl_deg=45.0, r_in=None, n=512, rtol=1e-12):
    """The differentiable disk image: Kerr thin disk seen from r0 = 1000M,
    +-35M, r_out = 30M, Keplerian rotation, the tapered emissivity
    (M/r)^2 (1 - sqrt(r_in/r)) that makes the image continuous in r_in, DP45
    in FP64.  r_in defaults to the ISCO; the gradient's parameters are
    (a, incl, r_in)."""
    return dict(M=1.0, a=a, r_obs=1000.0, incl=math.radians(incl_deg), fov_x=35.0, fov_y=35.0, nx=n, ny=n,
                method=1, rtol=rtol, atol=rtol, h_init=1.0, cap_buffer=0.01, r_escape=1100.0,
                max_steps=1_000_000, disk_on=1, r_in=isco(a) if r_in is None else r_in, r_out=30.0,
                emis_q=2.0, emis_model=1)


def disk_fit_target(n=512):
    """The target of the fit: the same image at a = 0.6, i = 50 deg,
    r_in = 1.1 ISCO(0.6)."""
    return differentiable_disk(a=0.6, incl_deg=50.0, r_in=1.1 * isco(0.6), n=n)


def isco(a, M=1.0):
    """Radius of the innermost stable circular orbit of Kerr for orbits
    moving in +phi (prograde for a > 0, retrograde for a < 0), from the
    closed form of Bardeen, Press & Teukolsky (1972).  A workload input: the
    disk's inner edge."""
    chi = abs(a) / M
    z1 = 1.0 + (1.0 - chi * chi) ** (1.0 / 3.0) * ((1.0 + chi) ** (1.0 / 3.0) + (1.0 - chi) ** (1.0 / 3.0))
    z2 = math.sqrt(3.0 * chi * chi + z1 * z1)
    root = math.sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2))
    return M * (3.0 + z2 - root if a >= 0.0 else 3.0 + z2 + root)


# keys that describe one image; everything else is the shared integrator
IMAGE_KEYS = ("M", "a", "metric", "q", "r_obs", "incl", "fov_x", "fov_y", "nx", "ny", "disk_on", "r_in", "r_out",
              "emis_q", "rotation", "l0", "emis_model", "src_on", "r_src", "sky_on", "grid_deg", "line_deg")


def heterogeneous_batch(n_images=256, seed=20220201, side_unit=64, side_steps=16, fov=35.0, rtol=1e-12,
                        square=True):
    """(images, integ): `images` is a list of per-image dicts (IMAGE_KEYS),
    `integ` the shared integrator dict.  Per image, in this order: the side
    side_unit * (1 + k) with k uniform in [0, side_steps) (square images; with
    square=False nx and ny are drawn one after the other, for ragged test
    batches), a, the inclination and r_obs.  The 256-image default draws
    105,156,608 rays.  The escape radius is 1.1 r_obs of each image
    (r_escape = 0 in `integ`)."""
    rng = np.random.default_rng(seed)
    images = []
    for _ in range(n_images):
        nx = int(side_unit * (1 + rng.integers(0, side_steps)))
        ny = nx if square else int(side_unit * (1 + rng.integers(0, side_steps)))
        a = float(rng.uniform(0.0, 0.998))
        incl = math.radians(float(rng.uniform(5.0, 85.0)))
        r_obs = float(10.0 ** rng.uniform(2.0, 4.0))
        images.append(dict(M=1.0, a=a, r_obs=r_obs, incl=incl, fov_x=fov, fov_y=fov, nx=nx, ny=ny,
                           disk_on=1, r_in=isco(a), r_out=30.0, emis_q=2.0))
    integ = dict(method=1, rtol=rtol, atol=rtol, h_init=1.0, cap_buffer=0.01, r_escape=0.0,
                 max_steps=1_000_000)
    return images, integ


def image_params(image, integ):
    """Single-image parameters of one batch entry (escape at 1.1 r_obs when
    the shared r_escape is 0)."""
    p = dict(integ, **image)
    if p.get("r_escape", 0.0) == 0.0:
        p["r_escape"] = 1.1 * image["r_obs"]
    return p
