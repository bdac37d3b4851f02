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


def neighbours(pix, nx, ny):
    """(pix[k], 8) ids of the 8-neighbours of each pixel, -1 outside the image."""
    pix = np.asarray(pix, np.int64)
    j, i = np.divmod(pix, nx)
    out = []
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            if dj or di:
                jj, ii = j + dj, i + di
                ok = (jj >= 0) & (jj < ny) & (ii >= 0) & (ii < nx)
                out.append(np.where(ok, jj * nx + ii, -1))
    return np.stack(out, 1)


def sampled_parity(gpu, nx, ny, sample, trace, keys=(), rtol=1e-8, frac=1e-3, extra_rtol=None, max_order=1):
    """The parity rules on a sample of a full-size image.

    gpu: dict of full-image numpy arrays (fate, n_cross and the keys);
    sample: pixel ids; trace(pix) -> oracle dict for those pixels.  The
    oracle traces the sample, then the 8-neighbours of every sampled pixel
    whose GPU 3x3 neighbourhood holds a fate or image-order boundary or
    whose fates differ, so that the oracle's own neighbourhood decides
    "within one pixel of a boundary" wherever one can lie.  Elsewhere the
    GPU's uniform neighbourhood stands in for the oracle's, which can only
    add pixels to the value check (a stricter test).

    Returns (oracle sample dict, stats, mask of the sampled pixels whose
    values were compared).  Asserts: fate mismatches only next
    to an oracle boundary and at most frac of the sample; the keys within
    rtol (extra_rtol: {key: (rtol, min |value|)} overrides) where fate and
    image order agree, image order <= max_order and no oracle boundary is
    near."""
    sample = np.asarray(sample, np.int64)
    g_f = np.asarray(gpu["fate"]).ravel()
    has_nc = "n_cross" in gpu
    g_c = np.asarray(gpu["n_cross"]).ravel() if has_nc else np.zeros_like(g_f)
    o = trace(sample.astype(np.int32))
    o_c_s = o["n_cross"] if has_nc else np.zeros_like(o["fate"])
    nb = neighbours(sample, nx, ny)
    nbs = np.where(nb >= 0, nb, sample[:, None])  # clamp: outside counts as the pixel itself
    g_near = ((g_f[nbs] != g_f[sample][:, None]) | (g_c[nbs] != g_c[sample][:, None])).any(1)
    mism = g_f[sample] != o["fate"]
    need = g_near | mism
    # neighbour values: the oracle's where traced (the sample, then the
    # needed neighbours), else the GPU's
    img_f = g_f.astype(np.int16)
    img_c = g_c.astype(np.int16)
    img_f[sample] = o["fate"]
    img_c[sample] = o_c_s
    traced = np.zeros(g_f.size, bool)
    traced[sample] = True
    extra = np.unique(nb[need].ravel())
    extra = extra[extra >= 0]
    extra = extra[~traced[extra]]
    if extra.size:
        oe = trace(extra.astype(np.int32))
        img_f[extra] = oe["fate"]
        img_c[extra] = oe["n_cross"] if has_nc else 0
    nf = img_f[nbs]
    ncv = img_c[nbs]
    o_near = ((nf != o["fate"][:, None]) | (ncv != o_c_s[:, None])).any(1)
    bad = mism & ~o_near
    assert not bad.any(), f"fate mismatches away from an oracle boundary at pixels {sample[bad][:10].tolist()}"
    allowed = int(frac * sample.size)
    assert mism.sum() <= allowed, f"{mism.sum()} fate mismatches > {allowed} ({frac:.1e} of {sample.size})"
    ok = ~mism & ~o_near
    if has_nc:
        ok &= (g_c[sample] == o_c_s) & (o_c_s <= max_order)
    stats = {"sample": int(sample.size), "oracle_rays": int(sample.size + extra.size),
             "fate_mismatches": int(mism.sum()), "compared": int(ok.sum())}
    for key in keys:
        tol, floor = (extra_rtol or {}).get(key, (rtol, 0.0))
        a = np.asarray(gpu[key]).ravel()[sample][ok]
        b = o[key][ok]
        fa, fb = np.isfinite(a), np.isfinite(b)
        assert (fa == fb).all(), f"{key}: finiteness differs at pixels {sample[ok][fa != fb][:10].tolist()}"
        m = fa & (np.abs(b) > floor)
        e = rel_err(a[m], b[m])
        stats[key] = {"n": int(m.sum()), "max_rel_err": float(e.max()) if e.size else 0.0}
        assert not e.size or e.max() <= tol, \
            f"{key}: max rel err {e.max():.3e} > {tol:.1e} at pixel {sample[ok][m][np.argmax(e)]}"
    return o, stats, ok


def row_sample(nx, ny, every=16):
    """Pixel ids of rows j = 0 mod every."""
    return (np.arange(0, ny, every)[:, None] * nx + np.arange(nx)[None, :]).ravel()


def ulp_sensitivity(trace_xy, x, y, key):
    """Per-pixel relative change of the oracle's `key` when the pixel's
    image-plane coordinate moves by one ulp (x and y, up and down): how far
    the method itself carries rounding-level differences.  Pixels whose fate
    changes under a nudge get inf.  trace_xy(x, y) -> oracle dict."""
    base = trace_xy(x, y)
    sens = np.zeros(x.size)
    for xx, yy in ((np.nextafter(x, np.inf), y), (np.nextafter(x, -np.inf), y),
                   (x, np.nextafter(y, np.inf)), (x, np.nextafter(y, -np.inf))):
        o = trace_xy(xx, yy)
        d = np.where(o["fate"] != base["fate"], np.inf, rel_err(o[key], base[key]))
        sens = np.fmax(sens, np.where(np.isfinite(base[key]) | ~np.isfinite(d), d, 0.0))
    return sens


def check_values_rounding(gpu, ora, key, mask, sens, rtol=1e-8):
    """Values against the oracle where the method carries rounding-level
    differences far (Bulirsch-Stoer's step control: its error estimate is a
    difference of two extrapolated values that agree to the tolerance, so
    rounding changes it at the 1e-5 level and with it the step sequence).
    The tolerance follows from the oracle's own behaviour, sens being its
    per-pixel one-ulp sensitivity (four nudges: a sample, which can miss a
    pixel's sensitivity): each pixel within max(rtol, 10 S, 2 sens), S the
    99.9th percentile of the image's sensitivities, and at most 3x the
    oracle's own count of pixels above rtol (plus two) above rtol.  For
    schemes whose sensitivity is at rounding level this is the plain rtol
    check.  Returns (max error, S)."""
    a = np.asarray(gpu[key])[mask]
    b = np.asarray(ora[key])[mask]
    s = np.asarray(sens)[mask]
    fa, fb = np.isfinite(a), np.isfinite(b)
    assert (fa == fb).all(), f"{key}: finiteness differs at {np.flatnonzero(fa != fb)[:10]}"
    keep = fa & np.isfinite(s)
    e = rel_err(a[keep], b[keep])
    s = s[keep]
    if not e.size:
        return 0.0, 0.0
    S = float(np.quantile(s, 0.999))
    tol = np.maximum(max(rtol, 10.0 * S), 2.0 * s)
    bad = e > tol
    assert not bad.any(), (f"{key}: {bad.sum()} pixels beyond their rounding tolerance, worst rel err "
                           f"{e[bad].max():.3e} (own sensitivity {s[bad][np.argmax(e[bad])]:.2e}, image p99.9 {S:.2e})")
    n_over, n_own = int((e > rtol).sum()), int((s > rtol).sum())
    assert n_over <= 3 * n_own + 2, f"{key}: {n_over} pixels above {rtol:.0e}, oracle's own {n_own}"
    return float(e.max()), S
