"""Comparison rules between the GPU library and the CPU oracle.

Fates: mismatches may only sit within one pixel (8-neighbourhood) of a fate
boundary of the oracle image, and there may be at most `frac` of them (near
the critical curve rays orbit the photon ring and tiny rounding differences
flip them).

Values (FP64): relative error <= rtol on pixels with the same fate and the
same image order (n_cross), image order <= 1, and no fate or n_cross
boundary within one pixel (8-neighbourhood).

max |H|: agree to 1% or within `abs_floor` (H is a cancellation residue).
"""
import numpy as np


def boundary_mask(img):
    """True where any 8-neighbour differs from the pixel (2-D int image)."""
    img = np.asarray(img)
    ny, nx = img.shape
    pad = np.pad(img, 1, mode="edge")
    m = np.zeros(img.shape, bool)
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            if dj or di:
                m |= pad[1 + dj:1 + dj + ny, 1 + di:1 + di + nx] != img
    return m


def check_fates(gpu_fate, ora_fate, nx, ny, frac=1e-3, min_allowed=0):
    g = np.asarray(gpu_fate).reshape(ny, nx)
    o = np.asarray(ora_fate).reshape(ny, nx)
    mism = g != o
    near = boundary_mask(o)
    bad = mism & ~near
    assert not bad.any(), f"fate mismatches away from a boundary at {np.argwhere(bad)[:10].tolist()}"
    allowed = max(min_allowed, int(frac * nx * ny))
    assert mism.sum() <= allowed, f"{mism.sum()} fate mismatches > {allowed}"
    return mism.sum()


def value_mask(gpu, ora, nx, ny):
    """Pixels where FP64 observables must agree."""
    gf = np.asarray(gpu["fate"]).reshape(ny, nx)
    of = np.asarray(ora["fate"]).reshape(ny, nx)
    m = gf == of
    near = boundary_mask(of)
    if "n_cross" in gpu and "n_cross" in ora:
        gc = np.asarray(gpu["n_cross"]).reshape(ny, nx)
        oc = np.asarray(ora["n_cross"]).reshape(ny, nx)
        m &= (gc == oc) & (oc <= 1)
        near |= boundary_mask(oc)
    return (m & ~near).ravel()


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def check_values(gpu, ora, key, mask, rtol=1e-8):
    a = np.asarray(gpu[key])[mask]
    b = np.asarray(ora[key])[mask]
    fa, fb = np.isfinite(a), np.isfinite(b)
    assert (fa == fb).all(), f"{key}: finiteness differs at {np.flatnonzero(fa != fb)[:10]}"
    if fa.any():
        e = rel_err(a[fa], b[fa])
        assert e.max() <= rtol, f"{key}: max rel err {e.max():.3e} > {rtol:.1e} (idx {np.argmax(e)})"
        return e.max()
    return 0.0


def check_max_h(gpu, ora, key, mask, abs_floor=1e-13, rel=1e-2, budget=0.0):
    """Per pixel: both maxima within `budget`, or agreement to
    abs_floor + rel * max.  With adaptive steps the two sides' step sequences
    part at rounding level, so the truncation residues that set max |H| agree
    only statistically: the percentiles of the two distributions must then
    agree to 25%."""
    a = np.asarray(gpu[key])[mask]
    b = np.asarray(ora[key])[mask]
    d = np.abs(a - b)
    lim = abs_floor + rel * np.maximum(np.abs(a), np.abs(b))
    bad = (d > lim) & ~((a <= budget) & (b <= budget))
    assert not bad.any(), f"{key}: {bad.sum()} pixels disagree, worst {a[bad][:3]} vs {b[bad][:3]}"
    if budget > 0.0 and a.size:
        for q in (50, 90, 99):
            pa, pb = np.percentile(a, q), np.percentile(b, q)
            assert abs(pa - pb) <= 0.25 * max(pa, pb) + abs_floor, (key, q, pa, pb)
