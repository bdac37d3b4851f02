"""The discrete adjoint of the disk image against central finite differences
(h = 1e-6) of the CPU oracle's forward image, pixel by pixel, and through
torch.autograd for an L2 image loss."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2202_00086_amd import workloads as W
from tests import parity as P

pytestmark = pytest.mark.gpu

H = 1e-6
KEYS = ("a", "incl", "r_in")


def _announce(*what):
    print("[gpu-case]", *what, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _oracle_fd(params, nx, ny):
    """Base oracle image and per-pixel central differences of I in a, incl,
    r_in, with the pixels whose fate or image order changes under the
    perturbations marked."""
    base = O.trace_pixels(O.Setup(**params))
    fd, stable = {}, np.ones(nx * ny, bool)
    for k in KEYS:
        up = O.trace_pixels(O.Setup(**dict(params, **{k: params[k] + H})))
        dn = O.trace_pixels(O.Setup(**dict(params, **{k: params[k] - H})))
        fd[k] = (up["intensity"] - dn["intensity"]) / (2 * H)
        for o in (up, dn):
            stable &= (o["fate"] == base["fate"]) & (o["n_cross"] == base["n_cross"])
    return base, fd, stable


def test_adjoint_matches_oracle_finite_differences(torch_mod):
    from paper_2202_00086_amd import autograd as AG
    nx = ny = 40
    params = W.differentiable_disk(n=nx)
    _announce("adjoint per-pixel", nx)
    out, grads, stats, _ = AG.adjoint_maps(**params)
    torch_mod.cuda.synchronize()
    st = stats.cpu().numpy()
    g = {k: v.cpu().numpy() for k, v in zip(KEYS, grads)}
    fate = out["fate"].cpu().numpy()
    print(f"[adjoint] stats ok/failed/overflow/mismatch = {st.tolist()}", flush=True)
    assert st[1] == 0 and st[2] == 0 and st[3] == 0
    assert st[0] == int((fate == O.DISK).sum())
    base, fd, stable = _oracle_fd(params, nx, ny)
    gpu = {"fate": fate, "n_cross": out["n_cross"].cpu().numpy()}
    m = P.value_mask(gpu, base, nx, ny) & (base["fate"] == O.DISK) & stable
    assert m.sum() > 150
    worst = {}
    for k in KEYS:
        a, b = g[k][m], fd[k][m]
        scale = np.abs(b).max()
        err = np.abs(a - b) / (np.abs(b) + 1e-3 * scale)
        worst[k] = float(err.max())
        assert err.max() < 1e-4, (k, err.max(), np.argmax(err))
    print(f"[adjoint] {m.sum()} pixels; worst relative difference to FD {worst}", flush=True)
    # zero away from the disk
    off = fate != O.DISK
    for k in KEYS:
        assert (g[k][off] == 0.0).all()


def test_autograd_loss_gradient_matches_finite_differences(torch_mod):
    """L = sum over primary/secondary disk pixels of (I - T)^2, T the image
    at (0.6, 50 deg, 1.1 ISCO(0.6)); the mask comes from the base render."""
    torch = torch_mod
    from paper_2202_00086_amd import autograd as AG
    nx = 32
    params = W.differentiable_disk(n=nx)
    target = W.disk_fit_target(n=nx)
    _announce("adjoint autograd loss", nx)
    from paper_2202_00086_amd import kerrtrace as K
    T = K.Renderer(device="cuda:0", want=("fate", "r_hit", "g", "intensity"), **target).render()["intensity"]
    a = torch.tensor(params["a"], dtype=torch.float64, requires_grad=True)
    i = torch.tensor(params["incl"], dtype=torch.float64, requires_grad=True)
    rin = torch.tensor(params["r_in"], dtype=torch.float64, requires_grad=True)
    fixed = {k: v for k, v in params.items() if k not in ("a", "incl", "r_in")}
    I, fate, ncross = AG.disk_image(a, i, rin, **fixed)
    base, _, stable = _oracle_fd(params, nx, nx)
    gpu = {"fate": fate.cpu().numpy(), "n_cross": ncross.cpu().numpy()}
    mask_np = P.value_mask(gpu, base, nx, nx) & (base["fate"] == O.DISK) & stable
    mask = torch.from_numpy(mask_np).to("cuda:0")
    loss = ((I - T) ** 2 * mask).sum()
    loss.backward()
    got = np.array([a.grad.item(), i.grad.item(), rin.grad.item()])
    Tn = T.cpu().numpy()

    def oracle_loss(**kw):
        o = O.trace_pixels(O.Setup(**dict(params, **kw)))
        return float((((o["intensity"] - Tn) ** 2)[mask_np]).sum())
    want = np.array([(oracle_loss(**{k: params[k] + H}) - oracle_loss(**{k: params[k] - H})) / (2 * H)
                     for k in KEYS])
    print(f"[adjoint] loss {loss.item():.6e}; grad {got}; FD {want}", flush=True)
    np.testing.assert_allclose(got, want, rtol=1e-4, atol=1e-9 * np.abs(want).max())


def test_adjoint_work_list_order_and_cotangent_mask(torch_mod):
    """The work list (differentiated rays, sorted by forward step count when
    n_steps is given) changes only which lane runs a ray: with split sweeps
    off, gradients are bit-identical with and without step counts.  Disk
    pixels with a zero cotangent are skipped (zero gradient, not counted),
    with split sweeps too."""
    import ctypes as C
    torch = torch_mod
    from paper_2202_00086_amd import kerrtrace as K
    params = W.differentiable_disk(n=48)
    _announce("adjoint work list", 48)
    r = K.Renderer(device="cuda:0", want=("fate", "r_hit", "g", "intensity", "n_cross", "n_steps"),
                   stats=False, **params)
    out = r.render()
    n = r.n
    cot = torch.ones(n, dtype=torch.float64, device="cuda:0")
    cot[::3] = 0.0
    nbytes = K.kt_adjoint_workspace_bytes(r.cam, r.integ)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    sequential = K.make_structs(**dict(params, split_above=-1))[4]
    res = []
    for steps, integ in ((out["n_steps"].data_ptr(), sequential), (None, sequential),
                         (out["n_steps"].data_ptr(), r.integ)):
        grads = [torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0") for _ in range(3)]
        stats = torch.zeros(4, dtype=torch.int64, device="cuda:0")
        rc = K.kt_adjoint(r.cam, r.st, r.disk, integ, out["fate"].data_ptr(), out["r_hit"].data_ptr(),
                          cot.data_ptr(), grads[0].data_ptr(), grads[1].data_ptr(), grads[2].data_ptr(),
                          stats.data_ptr(), ws.data_ptr(), nbytes, stream, steps)
        assert rc == K.KT_OK, K.kt_last_error()
        torch.cuda.synchronize()
        res.append(([g.cpu().numpy() for g in grads], stats.cpu().numpy()))
    assert _split_rays(ws) > 0  # the last call split some sweeps
    fate = out["fate"].cpu().numpy()
    c = cot.cpu().numpy()
    want = int(((fate == K.DISK) & (c != 0.0)).sum())
    for grads, st in res:
        assert st.tolist() == [want, 0, 0, 0]
        for g in grads:
            assert np.isfinite(g).all()
            assert (g[(fate != K.DISK) | (c == 0.0)] == 0.0).all()
            assert (g[(fate == K.DISK) & (c != 0.0)] != 0.0).mean() > 0.9
    for g1, g2 in zip(res[0][0], res[1][0]):
        np.testing.assert_array_equal(g1.view(np.uint8), g2.view(np.uint8))
    for g1, g3 in zip(res[0][0], res[2][0]):
        _assert_split_close(g3, g1)


def _split_rays(ws):
    """How many work-list entries the last kt_adjoint call on this workspace
    took for split sweeps: the library keeps that count in the workspace's
    first bytes (a uint32 at byte 16, after the work-list ticket)."""
    return int(ws[16:20].cpu().numpy().view(np.uint32)[0])


# Split sweeps apply the same step maps as the sequential sweep, associated
# differently; the per-pixel gradients agree to rounding amplified by the
# length of the sweep.
SPLIT_RTOL = 1e-9


def _assert_split_close(split, seq):
    scale = np.abs(seq).max()
    err = np.abs(split - seq) / (np.abs(seq) + 1e-6 * scale)
    assert err.max() <= SPLIT_RTOL, (err.max(), int(np.argmax(err)))
    return float(err.max())


def test_full_size_adjoint_sampled(torch_mod):
    """512x512 (the size the benchmark differentiates): every disk ray is
    differentiated without failure, and a fixed sample of stable disk pixels
    matches central differences of the oracle traced pixel by pixel."""
    from paper_2202_00086_amd import autograd as AG
    n = 512
    params = W.differentiable_disk(n=n)
    _announce("adjoint full size sampled", n)
    out, grads, stats, _ = AG.adjoint_maps(**params)
    torch_mod.cuda.synchronize()
    st = stats.cpu().numpy()
    fate = out["fate"].cpu().numpy()
    ncross = out["n_cross"].cpu().numpy()
    print(f"[adjoint 512] stats ok/failed/overflow/mismatch = {st.tolist()}", flush=True)
    assert st.tolist() == [int((fate == O.DISK).sum()), 0, 0, 0]
    g = {k: v.cpu().numpy() for k, v in zip(KEYS, grads)}
    near = (P.boundary_mask(fate.reshape(n, n)) | P.boundary_mask(ncross.reshape(n, n))).ravel()
    cand = np.flatnonzero((fate == O.DISK) & (ncross <= 1) & ~near)
    rng = np.random.default_rng(512)
    pix = np.sort(rng.choice(cand, size=60, replace=False)).astype(np.int32)
    base = O.trace_pixels(O.Setup(**params), pix)
    assert (base["fate"] == O.DISK).all()
    stable = np.ones(pix.size, bool)
    fd = {}
    for k in KEYS:
        up = O.trace_pixels(O.Setup(**dict(params, **{k: params[k] + H})), pix)
        dn = O.trace_pixels(O.Setup(**dict(params, **{k: params[k] - H})), pix)
        fd[k] = (up["intensity"] - dn["intensity"]) / (2 * H)
        for o in (up, dn):
            stable &= (o["fate"] == base["fate"]) & (o["n_cross"] == base["n_cross"])
    assert stable.sum() >= 50
    for k in KEYS:
        a, b = g[k][pix][stable], fd[k][stable]
        err = np.abs(a - b) / (np.abs(b) + 1e-3 * np.abs(b).max())
        print(f"[adjoint 512] {k}: worst relative difference to FD {err.max():.2e}", flush=True)
        assert err.max() < 1e-4, (k, err.max())


def test_full_size_split_sweeps_match_sequential(torch_mod):
    """512x512 with the L2 loss's kind of cotangent (every disk ray of order
    <= 1): the default adjoint splits the longest rays' sweeps (a few
    thousand of them), and every pixel's gradient equals that of the
    sequential sweeps to SPLIT_RTOL; both count the same rays."""
    torch = torch_mod
    from paper_2202_00086_amd import kerrtrace as K
    params = W.differentiable_disk(n=512)
    _announce("adjoint 512 split against sequential")
    r = K.Renderer(device="cuda:0", want=("fate", "r_hit", "g", "intensity", "n_cross", "n_steps"),
                   stats=False, **params)
    out = r.render()
    cot = ((out["fate"] == K.DISK) & (out["n_cross"] <= 1)).to(torch.float64).contiguous()
    nbytes = K.kt_adjoint_workspace_bytes(r.cam, r.integ)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    split_maps, split_sum, split_st = _adjoint_call(K, torch, r, out, cot, ws, nbytes)
    n_split = _split_rays(ws)
    seq = K.make_structs(**dict(params, split_above=-1))[4]
    seq_maps, seq_sum, seq_st = _adjoint_call(K, torch, r, out, cot, ws, nbytes, integ=seq)
    print(f"[adjoint 512] {n_split} rays split; stats {split_st.tolist()}", flush=True)
    assert n_split > 1000
    assert split_st.tolist() == seq_st.tolist() and split_st[1:].tolist() == [0, 0, 0]
    errs = [_assert_split_close(a, b) for a, b in zip(split_maps, seq_maps)]
    np.testing.assert_allclose(split_sum, seq_sum, rtol=1e-11)
    print(f"[adjoint 512] split vs sequential: worst per-pixel relative difference {max(errs):.2e}", flush=True)


def _random_disk(seed):
    """Seeds 31-34: prograde spin, Keplerian or constant-l0 rotation; 35 and 36:
    retrograde spin (the disk counter-rotates with the hole), Keplerian."""
    rng = np.random.default_rng(seed)
    retro = seed >= 35
    a = float(rng.uniform(-0.95, -0.1)) if retro else float(rng.uniform(0.1, 0.95))
    p = W.differentiable_disk(a=a, incl_deg=float(rng.uniform(20.0, 80.0)),
                              r_in=W.isco(a) * float(rng.uniform(1.0, 1.3)), n=24)
    p["r_out"] = float(rng.uniform(18.0, 30.0))
    if not retro and rng.uniform() < 0.5:
        p.update(rotation=1, l0=float(rng.uniform(2.2, 3.2)) if a < 0.8 else float(rng.uniform(1.8, 2.3)))
    return p


@pytest.mark.parametrize("seed", [31, 32, 33, 34, 35, 36])
def test_random_disk_adjoint_matches_finite_differences(torch_mod, seed):
    """Seeded disks (spin of either sign, inclination, inner and outer
    radius, Keplerian or constant-l0 rotation) at 24x24: per-pixel gradients
    against central differences of the oracle."""
    from paper_2202_00086_amd import autograd as AG
    params = _random_disk(seed)
    _announce("adjoint random disk", seed, {k: params[k] for k in ("a", "incl", "r_in", "r_out")},
              params.get("rotation", 0))
    out, grads, stats, _ = AG.adjoint_maps(**params)
    torch_mod.cuda.synchronize()
    st = stats.cpu().numpy()
    fate = out["fate"].cpu().numpy()
    assert st.tolist() == [int((fate == O.DISK).sum()), 0, 0, 0]
    g = {k: v.cpu().numpy() for k, v in zip(KEYS, grads)}
    base, fd, stable = _oracle_fd(params, 24, 24)
    gpu = {"fate": fate, "n_cross": out["n_cross"].cpu().numpy()}
    m = P.value_mask(gpu, base, 24, 24) & (base["fate"] == O.DISK) & stable
    # constant-l0 orbits that are not timelike have g = NaN and I = 0
    m &= np.isfinite(base["g"])
    assert m.sum() > 20
    for k in KEYS:
        a, b = g[k][m], fd[k][m]
        err = np.abs(a - b) / (np.abs(b) + 1e-3 * np.abs(b).max())
        assert err.max() < 1e-4, (k, err.max())


def _adjoint_call(K, torch, r, out, cot, ws, nbytes, integ=None, steps=True, r_hit=None):
    import ctypes as C
    n = r.n
    grads = [torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0") for _ in range(3)]
    gsum = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda:0")
    stats = torch.zeros(4, dtype=torch.int64, device="cuda:0")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = K.kt_adjoint(r.cam, r.st, r.disk, integ or r.integ, out["fate"].data_ptr(),
                      (r_hit if r_hit is not None else out["r_hit"]).data_ptr(), cot.data_ptr(),
                      grads[0].data_ptr(), grads[1].data_ptr(), grads[2].data_ptr(), stats.data_ptr(),
                      ws.data_ptr(), nbytes, stream, out["n_steps"].data_ptr() if steps else None,
                      gsum.data_ptr())
    assert rc == K.KT_OK, K.kt_last_error()
    torch.cuda.synchronize()
    return [g.cpu().numpy() for g in grads], gsum.cpu().numpy(), stats.cpu().numpy()


def test_adjoint_image_sums_and_checkpoint_interval(torch_mod):
    """grad_sum: the library's own sums of the three gradient maps, equal to
    an exactly rounded sum of the maps to 1e-13 and bit-identical whatever
    lanes ran the rays (with and without step counts when sweeps are not
    split).  The checkpoint interval (1 = every step stored, 2, 8, 64 =
    default, 256 accepted steps) changes only what is recomputed: the maps
    are bit-identical, with split sweeps too (split rays store every step
    whatever the interval)."""
    import ctypes as C
    import math as _m
    torch = torch_mod
    from paper_2202_00086_amd import kerrtrace as K
    params = W.differentiable_disk(n=40)
    _announce("adjoint sums and checkpoint intervals", 40)
    r = K.Renderer(device="cuda:0", want=("fate", "r_hit", "g", "intensity", "n_cross", "n_steps"),
                   stats=False, **params)
    out = r.render()
    cot = torch.linspace(-1.0, 2.0, r.n, dtype=torch.float64, device="cuda:0")
    res = {}
    for every in (1, 2, 8, 0, 256):
        for split in (-1, 0):
            integ = K.make_structs(**dict(params, checkpoint_every=every, split_above=split))[4]
            nbytes = K.kt_adjoint_workspace_bytes(r.cam, integ)
            assert nbytes > 0
            ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
            for steps in (True, False):
                res[(every, split, steps)] = _adjoint_call(K, torch, r, out, cot, ws, nbytes, integ, steps)
                if split == 0 and steps:
                    assert _split_rays(ws) > 0
    for group in ((-1, True), (-1, False), (0, False), (0, True)):
        base_maps, base_sum, base_st = res[(0,) + group]
        assert base_st[1:].tolist() == [0, 0, 0] and base_st[0] > 300
        for k in range(3):
            want = _m.fsum(base_maps[k].tolist())
            tot = _m.fsum(abs(v) for v in base_maps[k].tolist())
            assert abs(base_sum[k] - want) <= 1e-13 * tot, (group, k, base_sum[k], want)
    # bit-identical: every interval, and sequential sweeps with or without step counts
    seq_maps, seq_sum, seq_st = res[(0, -1, True)]
    split_maps, split_sum, _ = res[(0, 0, True)]
    for key, (maps, sums, st) in res.items():
        assert st.tolist() == seq_st.tolist(), key
        want_maps, want_sum = (split_maps, split_sum) if key[1:] == (0, True) else (seq_maps, seq_sum)
        np.testing.assert_array_equal(sums.view(np.uint8), want_sum.view(np.uint8), err_msg=str(key))
        for a, b in zip(maps, want_maps):
            np.testing.assert_array_equal(a.view(np.uint8), b.view(np.uint8), err_msg=str(key))
    # split against sequential: close, per pixel and in the sums
    errs = [_assert_split_close(a, b) for a, b in zip(split_maps, seq_maps)]
    np.testing.assert_allclose(split_sum, seq_sum, rtol=1e-11)
    print(f"[adjoint] split vs sequential sweeps: worst per-pixel relative difference {max(errs):.2e}", flush=True)
    bad = K.make_structs(**dict(params, checkpoint_every=48))[4]
    assert K.kt_adjoint_workspace_bytes(r.cam, bad) == 0


def test_adjoint_mismatch_is_counted_and_autograd_raises(torch_mod):
    """A forward hit radius that the re-integration does not reproduce (one
    pixel's r_hit nudged by an ulp-sized amount) is counted as a mismatch,
    gets a zero gradient and drops out of grad_sum; DiskImage.backward
    raises instead of returning such a gradient."""
    torch = torch_mod
    from paper_2202_00086_amd import autograd as AG
    from paper_2202_00086_amd import kerrtrace as K
    params = W.differentiable_disk(n=24)
    _announce("adjoint mismatch", 24)
    r = K.Renderer(device="cuda:0", want=("fate", "r_hit", "g", "intensity", "n_cross", "n_steps"),
                   stats=False, **params)
    out = r.render()
    torch.cuda.synchronize()
    cot = torch.ones(r.n, dtype=torch.float64, device="cuda:0")
    nbytes = K.kt_adjoint_workspace_bytes(r.cam, r.integ)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    maps, sums, st = _adjoint_call(K, torch, r, out, cot, ws, nbytes)
    disk = np.flatnonzero(out["fate"].cpu().numpy() == K.DISK)
    k = int(disk[disk.size // 2])
    r_hit = out["r_hit"].clone()
    r_hit[k] = r_hit[k] * (1.0 + 1e-13)
    maps2, sums2, st2 = _adjoint_call(K, torch, r, out, cot, ws, nbytes, r_hit=r_hit)
    assert st2.tolist() == [st[0] - 1, 0, 0, 1]
    for a, b in zip(maps, maps2):
        assert b[k] == 0.0
        keep = np.ones(r.n, bool)
        keep[k] = False
        np.testing.assert_array_equal(a[keep], b[keep])
    with pytest.raises(K.KtError, match="not reproducing"):
        AG.check_adjoint_stats(torch.tensor(st2))
    AG.check_adjoint_stats(torch.tensor(st))
    # through autograd: nudge the renderer's stored r_hit before backward
    a = torch.tensor(params["a"], dtype=torch.float64, requires_grad=True)
    i = torch.tensor(params["incl"], dtype=torch.float64, requires_grad=True)
    rin = torch.tensor(params["r_in"], dtype=torch.float64, requires_grad=True)
    fixed = {kk: v for kk, v in params.items() if kk not in ("a", "incl", "r_in")}
    I, fate, _ = AG.disk_image(a, i, rin, **fixed)
    I.grad_fn.renderer.out["r_hit"][k] *= 1.0 + 1e-13
    with pytest.raises(K.KtError, match="not reproducing"):
        I.sum().backward()
