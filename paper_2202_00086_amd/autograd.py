"""The disk image as a differentiable function of (a, inclination, r_in).

DiskImage.forward renders the observed intensity with kt_render (DP45,
FP64, disk on); backward calls kt_adjoint with the incoming gradient as the
per-pixel cotangent and returns the three image sums the library computes
(grad_sum).  Both directions, the reduction included, run in the library's
HIP kernels; this module only marshals tensors.  A backward pass in which
any differentiated ray failed, overflowed the checkpoint store or did not
reproduce the forward's hit radius raises KtError instead of returning a
gradient with those rays missing.
"""
import ctypes as C

import torch

from . import kerrtrace as K

_WANT = ("fate", "r_hit", "g", "intensity", "n_cross", "n_steps")


class DiskImage(torch.autograd.Function):
    """I(a, incl, r_in) for fixed camera and integrator parameters.

    Returns (intensity[n], fate[n], n_cross[n]); only the intensity is
    differentiable.  a, incl and r_in are 0-dimensional float64 tensors."""

    @staticmethod
    def forward(ctx, a, incl, r_in, params, device):
        p = dict(params, a=float(a), incl=float(incl), r_in=float(r_in), disk_on=1)
        r = K.Renderer(device=device, want=_WANT, stats=False, **p)
        out = r.render()
        ctx.renderer = r
        ctx.device = torch.device(device)
        ctx.mark_non_differentiable(out["fate"], out["n_cross"])
        return out["intensity"], out["fate"], out["n_cross"]

    @staticmethod
    def backward(ctx, g_int, g_fate, g_ncross):
        r = ctx.renderer
        dev = ctx.device
        n = r.n
        cot = torch.zeros(n, dtype=torch.float64, device=dev) if g_int is None else \
            g_int.to(dtype=torch.float64).contiguous()
        grad_sum = torch.empty(3, dtype=torch.float64, device=dev)
        stats = torch.zeros(4, dtype=torch.int64, device=dev)
        nbytes = K.kt_adjoint_workspace_bytes(r.cam, r.integ)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        stream = torch.cuda.current_stream(dev)
        rc = K.kt_adjoint(r.cam, r.st, r.disk, r.integ, r.out["fate"].data_ptr(), r.out["r_hit"].data_ptr(),
                          cot.data_ptr(), None, None, None, stats.data_ptr(), ws.data_ptr(), nbytes,
                          C.c_void_p(stream.cuda_stream), r.out["n_steps"].data_ptr(), grad_sum.data_ptr())
        if rc != K.KT_OK:
            raise K.KtError(rc, K.kt_last_error())
        check_adjoint_stats(stats)
        ctx.renderer.adjoint_stats = stats
        return grad_sum[0], grad_sum[1], grad_sum[2], None, None


def check_adjoint_stats(stats):
    """Raise KtError when kt_adjoint left any differentiated ray out
    (stats = [differentiated, failed, overflow, mismatch]; synchronises)."""
    ok, failed, overflow, mismatch = (int(v) for v in stats.cpu().tolist())
    if failed or overflow or mismatch:
        raise K.KtError(K.KT_EINVAL, f"adjoint left rays out of the gradient: {failed} failed, {overflow} beyond "
                                     f"the checkpoint capacity, {mismatch} not reproducing the forward hit "
                                     f"radius (of {ok + failed + overflow + mismatch})")


def disk_image(a, incl, r_in, device="cuda:0", **params):
    """(intensity, fate, n_cross) of the disk image; differentiable in the
    three tensor arguments."""
    return DiskImage.apply(a, incl, r_in, params, device)


def adjoint_maps(device="cuda:0", cot=None, **params):
    """Per-pixel gradients dI/d(a, incl, r_in) (times cot, default 1) of one
    render, with the adjoint's statistics and image sums: (render outputs,
    (ga, gi, gr), stats[ok, failed, overflow, mismatch], grad_sum[3])."""
    r = K.Renderer(device=device, want=_WANT, stats=False, **params)
    out = r.render()
    n = r.n
    dev = torch.device(device)
    cot = torch.ones(n, dtype=torch.float64, device=dev) if cot is None else cot
    grads = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3)]
    grad_sum = torch.empty(3, dtype=torch.float64, device=dev)
    stats = torch.zeros(4, dtype=torch.int64, device=dev)
    nbytes = K.kt_adjoint_workspace_bytes(r.cam, r.integ)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    rc = K.kt_adjoint(r.cam, r.st, r.disk, r.integ, out["fate"].data_ptr(), out["r_hit"].data_ptr(),
                      cot.data_ptr(), grads[0].data_ptr(), grads[1].data_ptr(), grads[2].data_ptr(),
                      stats.data_ptr(), ws.data_ptr(), nbytes, C.c_void_p(stream.cuda_stream),
                      out["n_steps"].data_ptr(), grad_sum.data_ptr())
    if rc != K.KT_OK:
        raise K.KtError(rc, K.kt_last_error())
    return out, tuple(grads), stats, grad_sum
