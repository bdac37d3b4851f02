"""Benchmark: rays/s and RK stage-evals/s of one 1024x1024 Kerr image on one
MI355X.

Workload (the headline configuration): Kerr a = 0.9, M = 1, observer at
r = 1000M, inclination 60 deg, image plane +-12M at 1024x1024, Dormand-Prince
5(4) at rtol = atol = 1e-12 in FP64, point source at r_src = 1000M behind the
hole (deflection angle and ring mask), capture at r < r_+ + 0.01M, escape at
r > 1100M.  Inputs are synthetic camera parameters; nothing is read from
disk.

One step = one kt_render call: the persistent trace kernel plus its small
post-passes (redshift, ring flags, stats).  W untimed warmup steps, then K
timed steps between two device synchronisations; HIP events on the stream
the kernels run on give the per-launch duration used for the roofline.

Prints ONE JSON line.  --gpus above 1 is refused: the library runs on one GPU.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rays/s & RK stage-evals/s, 1024² Kerr a=0.9; mixed vs FP64 at |H|≤1e-10"

# Algorithmic FP64 work per unit, counted mechanically: a counting scalar
# runs a plain Carter-form reference of each unit (tests/flopcount/, checked
# against the oracle by tests/test_flop_count.py, which also pins these
# numbers).  +, -, x, / and sqrt count 1, sin and cos 1 each, pow and atan2 2.
#   rhs      Hamilton's equations in Carter's form              per evaluation
#   diag     H and |H|_rel from the evaluation's intermediates   per accepted step
#   stages   Dormand-Prince stage states 2..7 (26 coefficients)  per attempted step
#   error    the embedded error estimate (6 weights)             per attempted step
#   control  RMS error norm and the new step size                per attempted step
#   arc      swept angle between accepted positions (source on)  per accepted step
#   q_rhs, q_diag   the same two units for the appendix's q-metric
FLOP_UNITS = {"rhs": 53, "diag": 5, "stages": 230, "error": 60, "control": 30, "arc": 26, "q_rhs": 75,
              "q_diag": 8}
# the earlier hand count and the survey's estimate, printed for comparison
FLOP_PER_EVAL_HAND_COUNT = 58 + (290 + 37 + 7 + 22) / 6.0
FLOP_PER_EVAL_SURVEY_ESTIMATE = 150.0


def flop_per_launch(evals, attempts6, accepted, src_on, qmetric=False):
    """Algorithmic FLOP of a Dormand-Prince launch: evals RHS evaluations,
    attempts6 the evaluations spent in step attempts (evals minus each ray's
    first, FSAL seed, evaluation; six per attempt, trial steps of event
    location included) and `accepted` accepted steps.  With the source on,
    every accepted step is priced with an arc (a slight overcount: the few
    steps after the source sphere take none)."""
    u = FLOP_UNITS
    attempts = attempts6 / 6.0
    rhs, diag = (u["q_rhs"], u["q_diag"]) if qmetric else (u["rhs"], u["diag"])
    return (evals * rhs + attempts * (u["stages"] + u["error"] + u["control"])
            + accepted * (diag + (u["arc"] if src_on else 0)))


PEAK_FP64_VECTOR = 78.6e12  # MI355X FP64 vector, FLOP/s
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "trace_kernel_kerr_ring_1024_a0.9_counters.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2202_00086_amd", "csrc", f)
                  for f in ("kt_device.h", "kt_elem.h", "kt_ray.h", "kt_internal.h", "kt_trace.hip", "kt_trace_w3.hip")]


def kernel_source_hash():
    """sha256 of the trace kernel's sources with comments and blank space
    removed, so that a counter summary stays valid across comment edits."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        text = open(f).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def traffic_from_profile():
    """HBM bytes per trace launch from the committed counter summary, if it
    was taken on the current kernel source."""
    if not os.path.exists(PROFILE_COUNTERS):
        return None
    vals = {}
    for line in open(PROFILE_COUNTERS):
        if ":" in line and line.strip().startswith("-"):
            k, v = line.strip().lstrip("- ").split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def progress(msg):
    """One line on stderr per finished piece of work, so a long run shows
    where it is."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _threads():
    try:
        n_avail = len(os.sched_getaffinity(0))
    except AttributeError:
        n_avail = os.cpu_count() or 1
    return min(n_avail, int(os.environ.get("OMP_NUM_THREADS", n_avail))), n_avail


def host_cpu():
    """What the host reports about its CPU (a virtual machine may name only
    the family)."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ":" in ln:
                    k, v = (x.strip() for x in ln.split(":", 1))
                    if k in ("model name", "cpu family", "model", "stepping", "cpu MHz") and k not in info:
                        info[k] = v
                    if k == "flags" and "flags" not in info:
                        info["flags"] = " ".join(f for f in v.split() if f.startswith(("avx", "fma")))
    except OSError:
        pass
    return info


def oracle_image(params, pix=None, threads=0):
    import oracle as O
    t0 = time.perf_counter()
    o = O.trace_pixels(O.Setup(**params), pix, threads=threads)
    return o, time.perf_counter() - t0


def cpu_baseline(params, gpu_out=None, single_rows_every=64):
    """The oracle, as it stands, on the host cores: (i) the whole image on
    every core it may use (the `value`), with the parity of the GPU image
    against it; (ii) one thread on rows j = 0 mod single_rows_every, with
    the whole image's time extrapolated from it."""
    import numpy as np

    threads, n_avail = _threads()
    nx, ny = params["nx"], params["ny"]
    o, dt = oracle_image(params, threads=threads)
    res = {"value": nx * ny / dt, "unit": "rays/s", "cores": threads, "kind": "oracle",
           "sample": f"the whole {nx}x{ny} image ({nx * ny} rays) in {dt:.1f} s wall on {threads} threads "
                     f"(plain C FP64 oracle, -O2, OpenMP dynamic 64)",
           "stage_evals_per_s": float(o["n_evals"].astype(np.int64).sum()) / dt,
           "cpus_visible": n_avail, "cpu": host_cpu()}
    pix = (np.arange(0, ny, single_rows_every)[:, None] * nx + np.arange(nx)[None, :]).ravel().astype(np.int32)
    o1, dt1 = oracle_image(params, pix, threads=1)
    res["single_thread"] = {"rays_per_s": pix.size / dt1, "sample": f"rows j = 0 mod {single_rows_every} "
                            f"({pix.size} rays) in {dt1:.1f} s on 1 thread",
                            "whole_image_s_extrapolated": dt1 * nx * ny / pix.size}
    if gpu_out is not None:
        res["gpu_parity_whole_image"] = image_parity(gpu_out, o, nx, ny, ("deflection", "psi"))
    return res, o


def image_parity(gpu_out, o, nx, ny, keys):
    """The parity rules of the test suite on a whole image: fate mismatches
    (and how many sit next to an oracle boundary), and the largest relative
    error of each key where fates and image order agree, order <= 1 and no
    boundary is within one pixel."""
    import numpy as np

    from tests import parity as P
    g = {k: v.cpu().numpy() for k, v in gpu_out.items() if k != "stats"}
    mism = g["fate"] != o["fate"]
    near = P.boundary_mask(o["fate"].reshape(ny, nx)).ravel()
    m = P.value_mask(g, o, nx, ny)
    res = {"rays": nx * ny, "fate_mismatches": int(mism.sum()),
           "fate_mismatches_away_from_boundary": int((mism & ~near).sum()), "values_compared": int(m.sum())}
    for k in keys:
        a, b = g[k][m], o[k][m]
        ok = np.isfinite(a) & np.isfinite(b) & (np.abs(b) > 1e-6)
        e = P.rel_err(a[ok], b[ok])
        res[k] = {"max_rel_err": float(e.max()) if e.size else 0.0, "p99": float(np.percentile(e, 99)) if e.size else 0.0}
    return res


def error_vs_oracle(out, o, nx, ny, keys):
    """Max and p99 relative error per output of a (mixed) render against the
    FP64 oracle's image, on pixels where the parity rules compare values."""
    return image_parity(out, o, nx, ny, keys)


def run_form(K, torch, params, steps, warmup, launch=None):
    r = K.Renderer(device="cuda:0", launch=launch, **params)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        r.render(stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        r.render(stream)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [a.elapsed_time(b) for a, b in ev]
    st = K.read_stats(r.out)
    n = r.n
    res = {"wall_s": wall, "ms_per_step": 1e3 * wall / steps,
           "launch_ms": sum(launch_ms) / len(launch_ms), "launch_ms_min": min(launch_ms),
           "rays": n, "evals": int(st.evals), "evals_fp32": int(st.evals_fp32),
           "fallback_rays": int(st.fallback_rays), "fates": [int(c) for c in st.fate_count[:6]],
           "trace_ms_last": float(st.trace_ms), "out": r.out}
    res.update(h_stats(torch, r.out["max_rel_h"]))
    if "n_steps" in r.out:
        res["steps_accepted"] = int(r.out["n_steps"].to(torch.int64).sum().item())
    return res


def h_stats(torch, h):
    """Max, p99.9 and the count over 1e-10 of max |H|_rel (NaN rays skipped)."""
    h = h[~torch.isnan(h)]
    return {"max_rel_h": float(h.max().item()),
            "p999_rel_h": float(torch.quantile(h[::max(1, h.numel() // 4000000)].float(), 0.999).item()),
            "rays_over_1e-10": int((h > 1e-10).sum().item())}


def launch_flop(st, steps_accepted, src_on, qmetric=False):
    """Algorithmic FLOP of one render from its statistics (every ray but the
    invalid ones spends one evaluation seeding its first step)."""
    valid = int(st.rays) - int(st.fate_count[5])
    return flop_per_launch(int(st.evals), int(st.evals) - valid, steps_accepted, src_on, qmetric)


def error_vs(torch, test, ref, keys=("deflection", "psi")):
    """Max and p99 relative error of `test` against `ref` per output, over rays
    with the same fate and a finite reference value; plus the fate agreement."""
    res = {"fate_agreement": float((test["fate"] == ref["fate"]).double().mean().item())}
    same = test["fate"] == ref["fate"]
    for k in keys:
        a, b = test[k], ref[k]
        m = same & torch.isfinite(b) & (b.abs() > 1e-6)
        e = ((a[m] - b[m]).abs() / b[m].abs()).double()
        if e.numel():
            res[k] = {"max": float(e.max().item()), "p99": float(torch.quantile(e[::max(1, e.numel() // 100000)], 0.99).item())}
    return res


BATCH_WANT = ("fate", "r_hit", "g", "intensity", "max_rel_h", "used_fp64", "n_cross", "n_steps")


def _time(torch, fn, steps):
    """Wall time per call of fn() over `steps` calls between two syncs."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


SCHEME_WANT = ("fate", "max_abs_h", "max_rel_h", "n_evals")


def run_scheme_forms(K, torch, W, steps):
    """The four adaptive schemes the paper compares (Sect. 3.1) on the same
    persistent kernel: on the paper's Hamiltonian-norm grid (625^2, +-8M,
    r0 = 100M, a = 0.98) and on the headline 1024^2 workload, all at
    rtol = atol = 1e-12.  Per scheme: time, rays/s, evaluations per ray and
    the constraint statistics."""
    res = {"tolerance": 1e-12}
    for wname, make in (("hamiltonian_norm_map_625", lambda m: W.hamiltonian_norm_map(625, method=m)),
                        ("kerr_ring_1024_a0.9", lambda m: dict(W.kerr_ring(0.9, n=1024, rtol=1e-12), method=m))):
        row = {}
        for m in (K.DP45, K.RKF45, K.CK45, K.BS, K.BS_RAT):
            r = K.Renderer(device="cuda:0", want=SCHEME_WANT, **make(m))
            r.render()
            t = _time(torch, r.render, steps)
            st = K.read_stats(r.out)
            ok = r.out["fate"] <= K.DISK
            ha = r.out["max_abs_h"][ok]
            hr = r.out["max_rel_h"][ok]
            row[K.METHOD_NAMES[m]] = {
                "ms_per_image": 1e3 * t, "rays_per_s": r.n / t, "stage_evals_per_s": st.evals / t,
                "evals_per_ray": st.evals / r.n, "mean_abs_h": float(ha.mean().item()),
                "max_abs_h": float(ha.max().item()), "mean_rel_h": float(hr.mean().item()),
                "max_rel_h": float(hr.max().item()),
                "p999_rel_h": float(torch.quantile(hr.float()[::max(1, hr.numel() // 200000)], 0.999).item()),
                "fates": [int(c) for c in st.fate_count[:6]]}
        res[wname] = row
    return res


def run_f4_forms(K, torch, W, steps):
    """The Sect. 4-5 and appendix images on the same persistent kernel: the
    coloured celestial sphere around Kerr a = 0.98 and in flat space, the
    q-metric (q = 0.5) in the same setup, and the constant-l0 thin disk at
    a = 0.95.  Per image: time, rays/s, stage-evals/s, evaluations per ray,
    max |H|_rel and the fate histogram."""
    res = {}
    for name, p in (("resolved_ring_1024_a0_fov60", dict(W.kerr_ring(0.0, n=1024), fov_x=60.0, fov_y=60.0)),
                    ("lensing_1024_a0.98", W.lensing(a=0.98, n=1024)),
                    ("lensing_1024_flat", W.lensing(a=0.0, n=1024, M=0.0)),
                    ("qmetric_lensing_1024_q0.5", W.qmetric_lensing(q=0.5, n=1024)),
                    ("thin_disk_l0_2048x1024_a0.95", W.thin_disk_l0(a=0.95))):
        r = K.Renderer(device="cuda:0", **p)
        r.render()
        t = _time(torch, r.render, steps)
        st = K.read_stats(r.out)
        hr = r.out["max_rel_h"][r.out["fate"] <= K.DISK]
        hr = hr[~torch.isnan(hr)]
        steps_acc = int(r.out["n_steps"].to(torch.int64).sum().item())
        flop = launch_flop(st, steps_acc, bool(p.get("src_on")), qmetric=p.get("metric", 0) == 1)
        res[name] = {"ms_per_image": 1e3 * t, "rays_per_s": r.n / t, "stage_evals_per_s": st.evals / t,
                     "evals_per_ray": st.evals / r.n, "alu_frac": flop / t / PEAK_FP64_VECTOR,
                     "flop_per_eval": flop / st.evals,
                     "max_rel_h": float(hr.max().item()) if hr.numel() else None,
                     "fates": [int(c) for c in st.fate_count[:6]]}
        if "ring" in r.out and name.startswith("resolved_ring"):
            res[name].update(ring_report(torch, r.out, p))
        del r
    return res


def ring_report(torch, out, p):
    """Ring flags of the resolved-ring image against the Schwarzschild orbit
    quadrature's ring radii: how many flags, and the largest distance (in
    pixels) of a flag from the nearest ring radius."""
    import numpy as np

    from tests import schwarzschild_quad as SQ
    n, fov = p["nx"], p["fov_x"]
    dx = 2 * fov / n
    x = -fov + (np.arange(n) + 0.5) * dx
    rho = np.hypot(x[None, :], x[:, None]).ravel()
    radii = np.array(SQ.einstein_ring_radii(p["r_obs"]))
    ring = out["ring"].cpu().numpy().astype(bool)
    dist = np.abs(rho[ring][:, None] - radii[None, :]).min(1) / dx
    prim = int((np.abs(rho[ring] - radii[0]) <= dx).sum())
    return {"ring_radii_quadrature": radii.tolist(), "ring_flags": int(ring.sum()), "primary_ring_flags": prim,
            "max_flag_distance_px": float(dist.max()) if dist.size else None}


def run_adjoint_form(K, torch, W, steps, default_only=False):
    """The differentiable disk image (512^2, a = 0.7, i = 45 deg, r_in =
    ISCO, tapered emissivity): forward render and the discrete adjoint of the
    L2 loss against the image at (0.6, 50 deg, 1.1 ISCO(0.6)), both timed.
    default_only: the default adjoint alone (with step counts, split sweeps),
    so that a profile of the run covers that configuration only."""
    import ctypes as C
    import numpy as np
    params = W.differentiable_disk(n=512)
    want = ("fate", "r_hit", "g", "intensity", "n_cross", "n_steps")
    T = K.Renderer(device="cuda:0", want=want, stats=False, **W.disk_fit_target(n=512)).render()["intensity"]
    r = K.Renderer(device="cuda:0", want=want, stats=False, **params)
    r.render()
    t_fwd = _time(torch, r.render, steps)
    out = r.out
    mask = (out["fate"] == K.DISK) & (out["n_cross"] <= 1)
    cot = (2.0 * (out["intensity"] - T) * mask).contiguous()
    grads = [torch.empty(r.n, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    grad_sum = torch.empty(3, dtype=torch.float64, device="cuda:0")
    stats = torch.zeros(4, dtype=torch.int64, device="cuda:0")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def variant(**kw):
        """A kt_adjoint call with these integrator fields, on a workspace of its own."""
        integ = K.make_structs(**dict(params, **kw))[4]
        nb = K.kt_adjoint_workspace_bytes(r.cam, integ)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda:0")

        def call(sorted_list=True):
            rc = K.kt_adjoint(r.cam, r.st, r.disk, integ, out["fate"].data_ptr(), out["r_hit"].data_ptr(),
                              cot.data_ptr(), grads[0].data_ptr(), grads[1].data_ptr(), grads[2].data_ptr(),
                              stats.data_ptr(), ws.data_ptr(), nb, stream,
                              out["n_steps"].data_ptr() if sorted_list else None, grad_sum.data_ptr())
            if rc != K.KT_OK:
                raise K.KtError(rc, K.kt_last_error())
        return call, ws, nb

    def timed(call, **kw):
        call(**kw)
        t = _time(torch, lambda: call(**kw), steps)
        return t, grad_sum.cpu().tolist(), [int(v) for v in stats.cpu().tolist()]

    # the default: checkpoints every 64 steps, long rays' sweeps split
    adjoint, ws, nbytes = variant()
    if default_only:
        t_adj, g_default, st = timed(adjoint)
        return {"forward_ms": 1e3 * t_fwd, "adjoint_ms": 1e3 * t_adj, "adjoint_over_forward": t_adj / t_fwd,
                "split_rays": int(ws[16:20].cpu().numpy().view(np.uint32)[0]),
                "grad": dict(zip(("a", "incl", "r_in"), g_default)),
                "rays_differentiated": st[0], "failed": st[1], "overflow": st[2], "mismatch": st[3]}
    t_unsorted, g_unsorted, _ = timed(adjoint, sorted_list=False)
    t_adj, g_default, st = timed(adjoint)
    n_split = int(ws[16:20].cpu().numpy().view(np.uint32)[0])  # the library's count of split rays
    seq, ws_seq, _ = variant(split_above=-1)
    t_seq, g_seq, st_seq = timed(seq)
    del ws_seq
    # every accepted step stored (checkpoint_every 1): no recomputation in
    # the backward sweep, a larger workspace
    every, ws1, nbytes1 = variant(checkpoint_every=1)
    t_adj1, g_every, _ = timed(every)
    del ws1
    every_seq, ws1s, _ = variant(checkpoint_every=1, split_above=-1)
    t_adj1_seq, _, _ = timed(every_seq)
    del ws1s
    rel = max(abs(a - b) / abs(b) for a, b in zip(g_default, g_seq))
    return {"workload": "Kerr a=0.7 disk, 512x512, i=45 deg, r_obs=1000M, +-35M, r_in=ISCO(0.7), r_out=30M, "
                        "tapered emissivity, DP45 rtol=atol=1e-12; L2 loss vs (a=0.6, i=50 deg, r_in=1.1 ISCO)",
            "forward_ms": 1e3 * t_fwd, "adjoint_ms": 1e3 * t_adj, "adjoint_over_forward": t_adj / t_fwd,
            "split_rays": n_split,
            "adjoint_ms_sequential_sweeps": 1e3 * t_seq,
            "adjoint_ms_without_step_counts": 1e3 * t_unsorted,
            "adjoint_ms_every_step_stored": 1e3 * t_adj1,
            "adjoint_ms_every_step_stored_sequential_sweeps": 1e3 * t_adj1_seq,
            "every_step_grad_identical": g_every == g_default,
            "split_vs_sequential_grad_rel_diff": rel,
            "sequential_grad_identical_without_step_counts": g_unsorted == g_seq,
            "workspace_bytes": {"checkpoint_every_64": nbytes, "every_step": nbytes1},
            "loss": float((((out["intensity"] - T) ** 2) * mask).sum().item()),
            "grad": dict(zip(("a", "incl", "r_in"), g_default)),
            "rays_differentiated": st[0], "failed": st[1], "overflow": st[2], "mismatch": st[3],
            "sequential_stats_equal": st_seq == st,
            "differentiated_rays_per_s": st[0] / t_adj}


def run_batch_forms(K, torch, W, steps):
    """The 256-image heterogeneous Kerr disk workload: one autotuned
    persistent FP64 launch, the same images as 256 separate FP64 launches,
    and the mixed-precision batch with FP64 fallback."""
    images, integ = W.heterogeneous_batch()
    n = sum(i["nx"] * i["ny"] for i in images)
    # autotune on a probe of every 8th image
    probe = K.BatchRenderer(images[::8], device="cuda:0", want=BATCH_WANT, stats=False, **integ)
    best, times = probe.autotune(repeats=1)
    del probe
    res = {"workload": "256 seeded Kerr thin-disk images, sides 64..1024, a~U[0,0.998], "
                       "i~U[5,85] deg, r_obs log-uniform [100,1e4]M, +-35M, r_in=ISCO(a), r_out=30M, "
                       "DP45 rtol=atol=1e-12",
           "rays": n, "autotuned_launch": {"block": best.block, "blocks_per_cu": best.blocks_per_cu,
                                           "batch": best.batch},
           "autotune_probe": "every 8th image (32 images), 30 built-in shapes, 1 repeat"}
    br = K.BatchRenderer(images, device="cuda:0", want=BATCH_WANT, launch=best, **integ)
    br.render()
    t = _time(torch, br.render, steps)
    st = K.read_stats(br.out)
    flop = launch_flop(st, int(br.out["n_steps"].to(torch.int64).sum().item()), src_on=False)
    res["batch_fp64"] = {"rays_per_s": n / t, "stage_evals_per_s": st.evals / t, "ms_per_step": 1e3 * t,
                         "alu_frac": flop / t / PEAK_FP64_VECTOR, "flop_per_eval": flop / st.evals}
    res["batch_fp64"].update(h_stats(torch, br.out["max_rel_h"]))
    ref = {k: v for k, v in br.out.items()}
    singles = [K.Renderer(device="cuda:0", want=BATCH_WANT, stats=False, **W.image_params(im, integ))
               for im in images]
    def per_image():
        for r in singles:
            r.render()
    per_image()
    t = _time(torch, per_image, max(1, steps // 2))
    res["per_image_fp64"] = {"rays_per_s": n / t, "ms_per_step": 1e3 * t,
                             "launches": len(images), "launch": "default (persistent, block 256, batch 4, ring-first order)"}
    res["per_image_fp64"].update(h_stats(torch, torch.cat([r.out["max_rel_h"] for r in singles])))
    del singles
    bm = K.BatchRenderer(images, device="cuda:0", want=BATCH_WANT, launch=best,
                         **dict(integ, precision=K.MIXED, h_budget=1e-10, r_switch=300.0))
    bm.render()
    t = _time(torch, bm.render, steps)
    sm = K.read_stats(bm.out)
    h = bm.out["max_rel_h"]
    used64 = bm.out["used_fp64"].bool()
    res["batch_mixed_budget1e-10"] = {
        "rays_per_s": n / t, "stage_evals_per_s": sm.evals / t, "ms_per_step": 1e3 * t,
        "r_switch": 300.0, "h_budget": 1e-10, "fallback_fraction": sm.fallback_rays / n,
        "fp32_eval_fraction": sm.evals_fp32 / max(1, sm.evals),
        # rays over the budget after the re-run: all are FP64 results (re-run,
        # or never in FP32), the method's own level at rtol 1e-12
        "over_budget_after_rerun": int(((h > 1e-10) & ~torch.isnan(h)).sum().item()),
        "over_budget_rerun_rays": int(((h > 1e-10) & used64).sum().item()),
        "error_vs_fp64": error_vs(torch, bm.out, ref, keys=("r_hit", "g", "intensity"))}
    res["batch_mixed_budget1e-10"].update(h_stats(torch, h))
    # the workload's own comparison: the mixed batched launch against
    # per-image FP64 launches, and against the FP64 batched launch
    res["mixed_batch_over_per_image_fp64"] = (n / t) / res["per_image_fp64"]["rays_per_s"]
    res["mixed_batch_over_fp64_batch"] = (n / t) / res["batch_fp64"]["rays_per_s"]
    return res


# FP64 at the loosest tolerance whose p99.9 |H|_rel stays within 1e-10 on the
# headline image (the equal-accuracy FP64 line; `--only mixed` sweeps it),
# and the r_switch the mixed form runs with.
RTOL_EQUAL_ACCURACY = 6e-12
MIXED_R_SWITCH = 300.0


def form_entry(f, extra=None):
    e = {"rays_per_s": f["rays"] / (f["ms_per_step"] / 1e3), "stage_evals_per_s": f["evals"] / (f["ms_per_step"] / 1e3),
         "ms_per_step": f["ms_per_step"], "max_rel_h": f["max_rel_h"], "p999_rel_h": f["p999_rel_h"],
         "rays_over_1e-10": f["rays_over_1e-10"]}
    if f["evals_fp32"] or f["fallback_rays"]:
        e.update(fallback_fraction=f["fallback_rays"] / f["rays"], fp32_eval_fraction=f["evals_fp32"] / max(1, f["evals"]))
    e.update(extra or {})
    return e


def run_mixed_sweep(K, torch, W, steps):
    """The precision forms on the headline image: FP64 over a grid of
    tolerances between 1e-12 and 1e-11 (the loosest whose p99.9 |H|_rel is
    within 1e-10 is the equal-accuracy FP64 line), and the mixed form over
    r_switch in {20, 50, 100, 300}M at budget 1e-10 and without re-run, plus
    one looser budget.  Each form states its error per output against the
    FP64 oracle's whole image under the parity rules' value mask."""
    import numpy as np
    params = W.kerr_ring(0.9, n=1024, rtol=1e-12)
    nx = ny = 1024
    o_full, _ = oracle_image(params, threads=_threads()[0])

    def vs_oracle(out):
        return error_vs_oracle(out, o_full, nx, ny, ("deflection", "psi"))

    res = {"rtol_grid": {}, "mixed": {}}
    best = None
    for rtol in np.geomspace(1e-12, 1e-11, 8):
        f = run_form(K, torch, dict(params, rtol=float(rtol), atol=float(rtol)), steps, 1)
        res["rtol_grid"][f"{rtol:.3e}"] = form_entry(f, {"error_vs_fp64_oracle": vs_oracle(f["out"])})
        progress(f"fp64 rtol {rtol:.3e}: p99.9 |H|_rel {f['p999_rel_h']:.3g}")
        if f["p999_rel_h"] <= 1e-10:
            best = float(rtol)
    res["rtol_equal_accuracy"] = best
    for r_switch in (20.0, 50.0, 100.0, 300.0):
        for budget, tag in ((1e-10, "budget1e-10"), (1e300, "no_rerun")):
            f = run_form(K, torch, dict(params, precision=K.MIXED, h_budget=budget, r_switch=r_switch), steps, 1)
            res["mixed"][f"r_switch{r_switch:g}_{tag}"] = form_entry(f, {"error_vs_fp64_oracle": vs_oracle(f["out"])})
            progress(f"mixed r_switch {r_switch:g} {tag}: {f['ms_per_step']:.3f} ms")
    for budget in (1e-9,):
        f = run_form(K, torch, dict(params, precision=K.MIXED, h_budget=budget, r_switch=MIXED_R_SWITCH), steps, 1)
        res["mixed"][f"r_switch{MIXED_R_SWITCH:g}_budget{budget:g}"] = form_entry(
            f, {"error_vs_fp64_oracle": vs_oracle(f["out"])})
    return res


def run_cpu_legs(K, torch, W, steps):
    """The oracle on the host cores beyond the default line: the 2048^2
    Schwarzschild disk in full, and a fixed 1% sample of every image of the
    256-image batch (extrapolated to the whole batch)."""
    import numpy as np
    threads, _ = _threads()
    res = {"threads": threads, "cpu": host_cpu()}
    pd = W.schwarzschild_disk(n=2048)
    _, dt = oracle_image(pd, threads=threads)
    res["schwarzschild_disk_2048_whole"] = {"rays": 2048 * 2048, "s": dt, "rays_per_s": 2048 * 2048 / dt}
    progress(f"oracle: 2048^2 disk in {dt:.1f} s")
    images, integ = W.heterogeneous_batch()
    rng = np.random.default_rng(1)
    tot = n_all = 0
    t_all = 0.0
    for im in images:
        n = im["nx"] * im["ny"]
        pix = np.sort(rng.choice(n, size=max(1, n // 100), replace=False)).astype(np.int32)
        _, dt = oracle_image(W.image_params(im, integ), pix, threads=threads)
        t_all += dt
        tot += pix.size
        n_all += n
    res["heterogeneous_batch_1pct"] = {"rays": tot, "s": t_all, "rays_per_s": tot / t_all,
                                       "whole_batch_s_extrapolated": t_all * n_all / tot, "batch_rays": n_all}
    return res


def run_render(K, torch, W, steps, workload):
    """One workload rendered `steps` times in the default launch (for
    profiling a single kernel form)."""
    if workload == "batch":
        images, integ = W.heterogeneous_batch()
        r = K.BatchRenderer(images, device="cuda:0", want=BATCH_WANT, **integ)
    else:
        params = {"ring": W.kerr_ring(0.9, n=1024), "disk": W.schwarzschild_disk(n=2048),
                  "qmetric": W.qmetric_lensing(q=0.5, n=1024)}[workload]
        r = K.Renderer(device="cuda:0", **params)
    t = _time(torch, r.render, steps)
    st = K.read_stats(r.out)
    return {"workload": workload, "rays": r.n, "ms_per_render": 1e3 * t, "evals": int(st.evals)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-forms", action="store_true", help="skip the extra forms")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (three times), "
                         "to calibrate HBM byte counters")
    ap.add_argument("--only", choices=("batch", "adjoint", "images", "integrators", "mixed", "cpu", "render"),
                    default=None, help="run one extra form alone and print its JSON (for profiling); no headline line")
    ap.add_argument("--workload", choices=("ring", "disk", "qmetric", "batch"), default="ring",
                    help="with --only render: the workload rendered --steps times")
    ap.add_argument("--adjoint-default-only", action="store_true",
                    help="with --only adjoint: the default adjoint configuration alone (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: this build measures one GPU (rays are "
              "independent, so more GPUs would each trace a share of the pixels)", file=sys.stderr)
        sys.exit(2)
    if args.only:
        import torch

        from paper_2202_00086_amd import kerrtrace as K
        from paper_2202_00086_amd import workloads as W
        if args.only == "render":
            print(json.dumps({"render": run_render(K, torch, W, max(1, args.steps), args.workload)}), flush=True)
            return
        if args.only == "adjoint":
            res = run_adjoint_form(K, torch, W, max(1, args.steps), args.adjoint_default_only)
            print(json.dumps({"adjoint": res}), flush=True)
            return
        run = {"batch": run_batch_forms, "images": run_f4_forms,
               "integrators": run_scheme_forms, "mixed": run_mixed_sweep, "cpu": run_cpu_legs}[args.only]
        print(json.dumps({args.only: run(K, torch, W, max(1, args.steps))}), flush=True)
        return
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "copies": 3}), flush=True)
        return

    import torch

    from paper_2202_00086_amd import kerrtrace as K
    from paper_2202_00086_amd import workloads as W

    params = W.kerr_ring(0.9, n=1024, rtol=1e-12)
    main_form = run_form(K, torch, params, args.steps, args.warmup)
    progress(f"headline form: {main_form['ms_per_step']:.3f} ms per render")
    secs = main_form["ms_per_step"] / 1e3
    rays_per_s = main_form["rays"] / secs
    evals_per_s = main_form["evals"] / secs

    st = K.read_stats(main_form["out"])
    flop = launch_flop(st, main_form["steps_accepted"], src_on=True)
    launch_s = main_form["launch_ms"] / 1e3
    achieved = flop / launch_s
    traffic = traffic_from_profile()
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VECTOR / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR, "traffic": traffic,
                "flop_per_launch": flop, "flop_per_eval": flop / main_form["evals"],
                "flop_basis": "counted: Carter-form reference per unit x the launch's evaluations, attempts "
                              "and accepted steps",
                "frac_other_bases": {
                    "hand_count_117.3_per_eval": main_form["evals"] * FLOP_PER_EVAL_HAND_COUNT / launch_s / PEAK_FP64_VECTOR,
                    "survey_estimate_150_per_eval": main_form["evals"] * FLOP_PER_EVAL_SURVEY_ESTIMATE / launch_s / PEAK_FP64_VECTOR},
                "evals_per_launch": main_form["evals"], "steps_accepted_per_launch": main_form["steps_accepted"],
                "launch_ms": main_form["launch_ms"],
                # the last timed render's trace launch alone, on the GPU's wall
                # clock (kt_stats.trace_ms): a cross-check of launch_ms, which
                # also holds the dispatch sort and the post-passes
                "trace_ms_device_clock": main_form["trace_ms_last"]}

    cb = o_full = None
    if not args.no_cpu:
        cb, o_full = cpu_baseline(params, main_form["out"])
        progress("cpu baseline done")

    forms = {}
    if not args.no_forms:
        k = max(3, args.steps // 4)
        nx = ny = 1024

        def vs_oracle(out):
            return error_vs_oracle(out, o_full, nx, ny, ("deflection", "psi")) if o_full is not None else None
        for rtol, name in ((1e-11, "fp64_rtol1e-11"), (RTOL_EQUAL_ACCURACY, "fp64_equal_accuracy")):
            if rtol is None:
                continue
            f = run_form(K, torch, dict(params, rtol=rtol, atol=rtol), k, 1)
            progress(f"form {name} done")
            forms[name] = form_entry(f, {"rtol": rtol, "error_vs_fp64_rtol1e-12": error_vs(torch, f["out"], main_form["out"]),
                                         "error_vs_fp64_oracle": vs_oracle(f["out"])})
        for budget, name in ((1e-10, "mixed_budget1e-10"), (1e300, "mixed_no_fallback")):
            pm = dict(params, precision=K.MIXED, h_budget=budget, r_switch=MIXED_R_SWITCH)
            f = run_form(K, torch, pm, k, 1)
            progress(f"form {name} done")
            forms[name] = form_entry(f, {"r_switch": MIXED_R_SWITCH, "h_budget": budget,
                                         "error_vs_fp64": error_vs(torch, f["out"], main_form["out"]),
                                         "error_vs_fp64_oracle": vs_oracle(f["out"])})

        # the 2048^2 Schwarzschild disk: FP64 against the mixed form, with the
        # mixed form's error per output
        pd = W.schwarzschild_disk(n=2048)
        fd = run_form(K, torch, pd, k, 1)
        forms["disk_2048_fp64"] = form_entry(fd, {"fates": fd["fates"]})
        fm = run_form(K, torch, dict(pd, precision=K.MIXED, h_budget=1e-10, r_switch=MIXED_R_SWITCH), k, 1)
        forms["disk_2048_mixed_budget1e-10"] = form_entry(fm, {
            "r_switch": MIXED_R_SWITCH, "h_budget": 1e-10,
            "error_vs_fp64": error_vs(torch, fm["out"], fd["out"], keys=("r_hit", "g", "intensity"))})
        del fd, fm
        progress("disk forms done")

    batch = schemes = adjoint = images = None
    if not args.no_forms:
        batch = run_batch_forms(K, torch, W, max(2, args.steps // 8))
        progress("batch forms done")
        schemes = run_scheme_forms(K, torch, W, max(2, args.steps // 8))
        progress("integrator forms done")
        adjoint = run_adjoint_form(K, torch, W, max(2, args.steps // 8))
        progress("adjoint form done")
        images = run_f4_forms(K, torch, W, max(2, args.steps // 8))
        progress("image forms done")

    out = {"metric": METRIC, "value": rays_per_s, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": main_form["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "Kerr a=0.9, 1024x1024, i=60 deg, r_obs=1000M, +-12M, DP45 "
                                  "rtol=atol=1e-12, FP64, point source r_src=1000M",
                      "rays": main_form["rays"], "precision": "fp64", "integrator": "dp45"},
           "stage_evals_per_s": evals_per_s, "evals_per_ray": main_form["evals"] / main_form["rays"],
           "max_rel_h": main_form["max_rel_h"], "p999_rel_h": main_form["p999_rel_h"],
           "rays_over_1e-10": main_form["rays_over_1e-10"],
           "fates": main_form["fates"], "roofline": roofline,
           "form_note": "value is the FP64 form at rtol 1e-12; the other FP64 tolerances and the mixed-precision "
                        "forms are in 'forms'",
           "kernel_source_sha256": kernel_source_hash(),
           "paper_context": {"value": 1e3, "unit": "rays/s", "kind": "order of magnitude, not a target",
                             "note": "the paper states that its serial Fortran code traces 1024^2 geodesics in "
                                     "a time of the same order as GRay's, O(10^3) s, on an unnamed CPU, and that "
                                     "Odyssey (CUDA) is about two orders of magnitude faster; it prints no exact "
                                     "timing"}}
    if forms:
        out["forms"] = forms
    if batch:
        out["batch"] = batch
    if schemes:
        out["integrators"] = schemes
    if adjoint:
        out["adjoint"] = adjoint
    if images:
        out["images"] = images
    if cb is not None:
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
