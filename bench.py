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

# Algorithmic FP64 work, counted on the formulas the method evaluates
# (+, -, x, /, sqrt = 1; FMA = 2; sincos, atan2, pow = 2), independent of how
# the kernel computes them (e.g. three reciprocals count 3 even though the
# kernel derives them from one):
#   Hamiltonian RHS in Carter form                              58 per evaluation
#   per Dormand-Prince step (six evaluations): stage sums and
#   error estimate 290, error norm and step-size control 37,
#   constraint diagnostics 7                                   334 per step
#   swept angle between successive positions (source on)        22 per step
RHS_FLOP = 58
STEP_FLOP = 290 + 37 + 7
ARC_FLOP = 22
PEAK_FP64_VECTOR = 78.6e12  # MI355X FP64 vector, FLOP/s
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "trace_kernel_kerr_ring_1024_a0.9_counters.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2202_00086_amd", "csrc", f)
                  for f in ("kt_device.h", "kt_elem.h", "kt_ray.h", "kt_internal.h", "kt_trace.hip")]


def flop_per_eval(src_on):
    return RHS_FLOP + (STEP_FLOP + (ARC_FLOP if src_on else 0)) / 6.0


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


def cpu_baseline(params, rows_every=16):
    """The oracle, as it stands, on rows j = 0 mod rows_every of the image."""
    import numpy as np

    import oracle as O
    try:
        n_avail = len(os.sched_getaffinity(0))
    except AttributeError:
        n_avail = os.cpu_count() or 1
    threads = min(n_avail, int(os.environ.get("OMP_NUM_THREADS", n_avail)))
    nx, ny = params["nx"], params["ny"]
    pix = (np.arange(0, ny, rows_every)[:, None] * nx + np.arange(nx)[None, :]).ravel().astype(np.int32)
    t0 = time.perf_counter()
    o = O.trace_pixels(O.Setup(**params), pix, threads=threads)
    dt = time.perf_counter() - t0
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": pix.size / dt, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "cpu_model": model, "cpus_visible": n_avail,
            "sample": f"rows j = 0 mod {rows_every} of the same image ({pix.size} rays, "
                      f"{dt:.1f} s wall on {threads} threads; plain C FP64 oracle, -O2, OpenMP)",
            "stage_evals_per_s": float(o["n_evals"].astype(np.int64).sum()) / dt}


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
    return {"wall_s": wall, "ms_per_step": 1e3 * wall / steps,
            "launch_ms": sum(launch_ms) / len(launch_ms), "launch_ms_min": min(launch_ms),
            "rays": n, "evals": int(st.evals), "evals_fp32": int(st.evals_fp32),
            "fallback_rays": int(st.fallback_rays), "fates": [int(c) for c in st.fate_count[:6]],
            "max_rel_h": float(r.out["max_rel_h"].max().item()),
            "p999_rel_h": float(torch.quantile(r.out["max_rel_h"].float()[::16], 0.999).item()),
            "out": r.out}


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


BATCH_WANT = ("fate", "r_hit", "g", "intensity", "max_rel_h", "used_fp64", "n_cross")


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
        for m in (K.DP45, K.RKF45, K.CK45, K.BS):
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
    for name, p in (("lensing_1024_a0.98", W.lensing(a=0.98, n=1024)),
                    ("lensing_1024_flat", W.lensing(a=0.0, n=1024, M=0.0)),
                    ("qmetric_lensing_1024_q0.5", W.qmetric_lensing(q=0.5, n=1024)),
                    ("thin_disk_l0_2048x1024_a0.95", W.thin_disk_l0(a=0.95))):
        r = K.Renderer(device="cuda:0", **p)
        r.render()
        t = _time(torch, r.render, steps)
        st = K.read_stats(r.out)
        hr = r.out["max_rel_h"][r.out["fate"] <= K.DISK]
        hr = hr[~torch.isnan(hr)]
        kerr_dp45 = p.get("metric", 0) == 0
        res[name] = {"ms_per_image": 1e3 * t, "rays_per_s": r.n / t, "stage_evals_per_s": st.evals / t,
                     "evals_per_ray": st.evals / r.n,
                     "alu_frac": st.evals / t * flop_per_eval(src_on=False) / PEAK_FP64_VECTOR if kerr_dp45 else None,
                     "max_rel_h": float(hr.max().item()) if hr.numel() else None,
                     "fates": [int(c) for c in st.fate_count[:6]]}
        del r
    return res


def run_adjoint_form(K, torch, W, steps):
    """The differentiable disk image (512^2, a = 0.7, i = 45 deg, r_in =
    ISCO, tapered emissivity): forward render and the discrete adjoint of the
    L2 loss against the image at (0.6, 50 deg, 1.1 ISCO(0.6)), both timed."""
    import ctypes as C
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
    nbytes = K.kt_adjoint_workspace_bytes(r.cam, r.integ)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def adjoint(sorted_list=True):
        rc = K.kt_adjoint(r.cam, r.st, r.disk, r.integ, out["fate"].data_ptr(), out["r_hit"].data_ptr(),
                          cot.data_ptr(), grads[0].data_ptr(), grads[1].data_ptr(), grads[2].data_ptr(),
                          stats.data_ptr(), ws.data_ptr(), nbytes, stream,
                          out["n_steps"].data_ptr() if sorted_list else None, grad_sum.data_ptr())
        if rc != K.KT_OK:
            raise K.KtError(rc, K.kt_last_error())
    adjoint(False)
    t_unsorted = _time(torch, lambda: adjoint(False), steps)
    adjoint()
    t_adj = _time(torch, adjoint, steps)
    st = [int(v) for v in stats.cpu().tolist()]
    return {"workload": "Kerr a=0.7 disk, 512x512, i=45 deg, r_obs=1000M, +-35M, r_in=ISCO(0.7), r_out=30M, "
                        "tapered emissivity, DP45 rtol=atol=1e-12; L2 loss vs (a=0.6, i=50 deg, r_in=1.1 ISCO)",
            "forward_ms": 1e3 * t_fwd, "adjoint_ms": 1e3 * t_adj, "adjoint_over_forward": t_adj / t_fwd,
            "adjoint_ms_without_step_counts": 1e3 * t_unsorted,
            "loss": float((((out["intensity"] - T) ** 2) * mask).sum().item()),
            "grad": dict(zip(("a", "incl", "r_in"), grad_sum.cpu().tolist())),
            "rays_differentiated": st[0], "failed": st[1], "overflow": st[2], "mismatch": st[3],
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
           "autotune_probe": "every 8th image (32 images), 20 built-in shapes, 1 repeat"}
    br = K.BatchRenderer(images, device="cuda:0", want=BATCH_WANT, launch=best, **integ)
    br.render()
    t = _time(torch, br.render, steps)
    st = K.read_stats(br.out)
    res["batch_fp64"] = {"rays_per_s": n / t, "stage_evals_per_s": st.evals / t, "ms_per_step": 1e3 * t,
                         "alu_frac": st.evals / t * flop_per_eval(src_on=False) / PEAK_FP64_VECTOR}
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
    del singles
    bm = K.BatchRenderer(images, device="cuda:0", want=BATCH_WANT, launch=best,
                         **dict(integ, precision=K.MIXED, h_budget=1e-10, r_switch=300.0))
    bm.render()
    t = _time(torch, bm.render, steps)
    sm = K.read_stats(bm.out)
    h = bm.out["max_rel_h"]
    res["batch_mixed_budget1e-10"] = {
        "rays_per_s": n / t, "stage_evals_per_s": sm.evals / t, "ms_per_step": 1e3 * t,
        "r_switch": 300.0, "h_budget": 1e-10, "fallback_fraction": sm.fallback_rays / n,
        "fp32_eval_fraction": sm.evals_fp32 / max(1, sm.evals),
        "max_rel_h": float(h[~torch.isnan(h)].max().item()),
        "error_vs_fp64": error_vs(torch, bm.out, ref, keys=("r_hit", "g", "intensity"))}
    # the workload's own comparison: the mixed batched launch against
    # per-image FP64 launches, and against the FP64 batched launch
    res["mixed_batch_over_per_image_fp64"] = (n / t) / res["per_image_fp64"]["rays_per_s"]
    res["mixed_batch_over_fp64_batch"] = (n / t) / res["batch_fp64"]["rays_per_s"]
    return res


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
    ap.add_argument("--only", choices=("batch", "adjoint", "images", "integrators"), default=None,
                    help="run one extra form alone and print its JSON (for profiling); no headline line")
    args = ap.parse_args()
    if args.only:
        import torch

        from paper_2202_00086_amd import kerrtrace as K
        from paper_2202_00086_amd import workloads as W
        run = {"batch": run_batch_forms, "adjoint": run_adjoint_form, "images": run_f4_forms,
               "integrators": run_scheme_forms}[args.only]
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
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: the ray tracer runs on one GPU "
              "(rays are independent; see the sharding notes in the design document)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2202_00086_amd import kerrtrace as K
    from paper_2202_00086_amd import workloads as W

    params = W.kerr_ring(0.9, n=1024, rtol=1e-12)
    main_form = run_form(K, torch, params, args.steps, args.warmup)
    secs = main_form["ms_per_step"] / 1e3
    rays_per_s = main_form["rays"] / secs
    evals_per_s = main_form["evals"] / secs

    fpe = flop_per_eval(src_on=True)
    flop = main_form["evals"] * fpe
    achieved = flop / (main_form["launch_ms"] / 1e3)
    traffic = traffic_from_profile()
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VECTOR / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR, "traffic": traffic,
                "flop_per_eval": fpe, "evals_per_launch": main_form["evals"],
                "launch_ms": main_form["launch_ms"]}

    forms = {}
    if not args.no_forms:
        k = max(3, args.steps // 4)
        p11 = W.kerr_ring(0.9, n=1024, rtol=1e-11)
        f = run_form(K, torch, p11, k, 1)
        forms["fp64_rtol1e-11"] = {"rays_per_s": f["rays"] / (f["ms_per_step"] / 1e3),
                                   "stage_evals_per_s": f["evals"] / (f["ms_per_step"] / 1e3),
                                   "ms_per_step": f["ms_per_step"], "max_rel_h": f["max_rel_h"],
                                   "p999_rel_h": f["p999_rel_h"],
                                   "error_vs_fp64_rtol1e-12": error_vs(torch, f["out"], main_form["out"])}
        for budget, name in ((1e-10, "mixed_budget1e-10"), (1e300, "mixed_no_fallback")):
            pm = dict(params, precision=K.MIXED, h_budget=budget, r_switch=300.0)
            f = run_form(K, torch, pm, k, 1)
            forms[name] = {"rays_per_s": f["rays"] / (f["ms_per_step"] / 1e3),
                           "stage_evals_per_s": f["evals"] / (f["ms_per_step"] / 1e3),
                           "ms_per_step": f["ms_per_step"], "r_switch": 300.0, "h_budget": budget,
                           "fallback_fraction": f["fallback_rays"] / f["rays"],
                           "fp32_eval_fraction": f["evals_fp32"] / max(1, f["evals"]),
                           "max_rel_h": f["max_rel_h"], "p999_rel_h": f["p999_rel_h"],
                           "error_vs_fp64": error_vs(torch, f["out"], main_form["out"])}

        # the 2048^2 Schwarzschild disk: FP64 against the mixed form, with the
        # mixed form's error per output
        pd = W.schwarzschild_disk(n=2048)
        fd = run_form(K, torch, pd, k, 1)
        forms["disk_2048_fp64"] = {"rays_per_s": fd["rays"] / (fd["ms_per_step"] / 1e3),
                                   "stage_evals_per_s": fd["evals"] / (fd["ms_per_step"] / 1e3),
                                   "ms_per_step": fd["ms_per_step"], "max_rel_h": fd["max_rel_h"],
                                   "fates": fd["fates"]}
        fm = run_form(K, torch, dict(pd, precision=K.MIXED, h_budget=1e-10, r_switch=300.0), k, 1)
        forms["disk_2048_mixed_budget1e-10"] = {
            "rays_per_s": fm["rays"] / (fm["ms_per_step"] / 1e3),
            "stage_evals_per_s": fm["evals"] / (fm["ms_per_step"] / 1e3),
            "ms_per_step": fm["ms_per_step"], "r_switch": 300.0, "h_budget": 1e-10,
            "fallback_fraction": fm["fallback_rays"] / fm["rays"],
            "fp32_eval_fraction": fm["evals_fp32"] / max(1, fm["evals"]), "max_rel_h": fm["max_rel_h"],
            "error_vs_fp64": error_vs(torch, fm["out"], fd["out"], keys=("r_hit", "g", "intensity"))}
        del fd, fm

    batch = schemes = adjoint = images = None
    if not args.no_forms:
        batch = run_batch_forms(K, torch, W, max(2, args.steps // 8))
        schemes = run_scheme_forms(K, torch, W, max(2, args.steps // 8))
        adjoint = run_adjoint_form(K, torch, W, max(2, args.steps // 8))
        images = run_f4_forms(K, torch, W, max(2, args.steps // 8))

    out = {"metric": METRIC, "value": rays_per_s, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": main_form["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "Kerr a=0.9, 1024x1024, i=60 deg, r_obs=1000M, +-12M, DP45 "
                                  "rtol=atol=1e-12, FP64, point source r_src=1000M",
                      "rays": main_form["rays"], "precision": "fp64", "integrator": "dp45"},
           "stage_evals_per_s": evals_per_s, "evals_per_ray": main_form["evals"] / main_form["rays"],
           "max_rel_h": main_form["max_rel_h"], "p999_rel_h": main_form["p999_rel_h"],
           "fates": main_form["fates"], "roofline": roofline,
           "form_note": "value is the FP64 form that meets max |H|_rel <= 1e-10; the FP64 "
                        "rtol 1e-11 and mixed-precision forms are in 'forms'",
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
    if not args.no_cpu:
        cb = cpu_baseline(params)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
