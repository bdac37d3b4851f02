"""Python binding of libkerrtrace.so (the C ABI in include/kerrtrace.h).

The functions kt_render, kt_render_ex, kt_render_noalloc, kt_render_batch, kt_autotune_batch,
kt_adjoint, kt_workspace_bytes, kt_adjoint_workspace_bytes,
kt_workspace_bytes_batch, kt_init_rays, kt_last_error and kt_version mirror
the C entry points one to one and only marshal arguments: every step of the ray tracing runs in the HIP kernels of
the library.  PyTorch supplies device memory and the HIP stream.

render() is a convenience wrapper that allocates the output tensors and the
workspace on the current device and calls kt_render_ex on torch's current
stream.  There is no fallback: if the library is missing, importing this
module raises.
"""
import ctypes as C
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# KERRTRACE_LIB selects another build of the same library (e.g. a variant
# compiled with different occupancy) for side-by-side timing.
LIB_PATH = os.environ.get("KERRTRACE_LIB") or os.path.join(HERE, "libkerrtrace.so")

KT_OK, KT_EINVAL, KT_EDEVICE, KT_ENOMEM = 0, -1, -2, -3
ESCAPED, CAPTURED, DISK, MAXSTEPS, STEPFAIL, INVALID = range(6)
RK4_S, DP45, RKF45, CK45, BS, BS_RAT = 0, 1, 2, 3, 4, 5
METHOD_NAMES = {RK4_S: "rk4_s", DP45: "dp45", RKF45: "rkf45", CK45: "ck45", BS: "bs", BS_RAT: "bs_rat"}
FP64, MIXED = 0, 1

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2202_00086_amd.build`")
_lib = C.CDLL(LIB_PATH)


class kt_camera(C.Structure):
    _fields_ = [("r_obs", C.c_double), ("incl", C.c_double), ("fov_x", C.c_double),
                ("fov_y", C.c_double), ("nx", C.c_int32), ("ny", C.c_int32)]


class kt_spacetime(C.Structure):
    _fields_ = [("M", C.c_double), ("a", C.c_double), ("metric", C.c_int32), ("q", C.c_double)]


class kt_disk(C.Structure):
    _fields_ = [("enabled", C.c_int32), ("r_in", C.c_double), ("r_out", C.c_double),
                ("emis_index", C.c_double), ("rotation", C.c_int32), ("l0", C.c_double),
                ("emissivity", C.c_int32)]


class kt_source(C.Structure):
    _fields_ = [("enabled", C.c_int32), ("r_src", C.c_double), ("sky", C.c_int32),
                ("grid_deg", C.c_double), ("line_deg", C.c_double)]


class kt_image(C.Structure):
    _fields_ = [("camera", kt_camera), ("spacetime", kt_spacetime), ("disk", kt_disk),
                ("source", kt_source)]


MAX_IMAGES = 4096


class kt_integrator(C.Structure):
    _fields_ = [("method", C.c_int32), ("precision", C.c_int32), ("h_fixed", C.c_double),
                ("rtol", C.c_double), ("atol", C.c_double), ("h_init", C.c_double),
                ("capture_buffer", C.c_double), ("r_escape", C.c_double),
                ("h_budget", C.c_double), ("r_switch", C.c_double), ("max_steps", C.c_int64),
                ("checkpoint_every", C.c_int32), ("split_above", C.c_int32)]


class kt_launch(C.Structure):
    _fields_ = [("persistent", C.c_int32), ("block", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("batch", C.c_int32), ("order", C.c_int32)]


class kt_stats(C.Structure):
    _fields_ = [("rays", C.c_uint64), ("evals", C.c_uint64), ("evals_fp32", C.c_uint64),
                ("fallback_rays", C.c_uint64), ("fate_count", C.c_uint64 * 8), ("trace_ms", C.c_double)]


OUTPUT_FIELDS = ("fate", "r_hit", "g", "intensity", "max_abs_h", "max_rel_h", "psi", "deflection",
                 "theta_f", "phi_f", "n_cross", "used_fp64", "ring", "n_steps", "n_evals", "sky")
KEPLER, L0 = 0, 1
METRIC_KERR, METRIC_Q = 0, 1
EMIS_POWER, EMIS_TAPERED = 0, 1
ORDER_RING, ORDER_ROWS = 0, 1  # dispatch order (kt_launch.order)
SKY_NONE, SKY_GREEN, SKY_RED, SKY_BLUE, SKY_YELLOW, SKY_LINE = range(6)


class kt_outputs(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in OUTPUT_FIELDS] + [("stats", C.c_void_p)]


_P = C.POINTER
_lib.kt_render.argtypes = [_P(kt_camera), _P(kt_spacetime), _P(kt_disk), _P(kt_source),
                           _P(kt_integrator), _P(kt_outputs), C.c_void_p, C.c_size_t, C.c_void_p]
_lib.kt_render.restype = C.c_int
_lib.kt_render_ex.argtypes = _lib.kt_render.argtypes + [_P(kt_launch)]
_lib.kt_render_ex.restype = C.c_int
_lib.kt_render_noalloc.argtypes = [_P(kt_camera), _P(kt_spacetime), _P(kt_disk), _P(kt_source),
                                   _P(kt_integrator), _P(kt_outputs), C.c_void_p, _P(kt_launch)]
_lib.kt_render_noalloc.restype = C.c_int
_lib.kt_render_batch.argtypes = [C.c_int32, _P(kt_image), _P(kt_integrator), _P(kt_outputs), C.c_void_p,
                                 C.c_size_t, C.c_void_p, _P(kt_launch)]
_lib.kt_render_batch.restype = C.c_int
_lib.kt_autotune_batch.argtypes = [C.c_int32, _P(kt_image), _P(kt_integrator), _P(kt_outputs), C.c_void_p,
                                   C.c_size_t, C.c_void_p, _P(kt_launch), C.c_int32, C.c_int32,
                                   _P(kt_launch), _P(C.c_float)]
_lib.kt_autotune_batch.restype = C.c_int
_lib.kt_workspace_bytes.argtypes = [_P(kt_camera), _P(kt_integrator)]
_lib.kt_workspace_bytes.restype = C.c_size_t
_lib.kt_workspace_bytes_batch.argtypes = [C.c_int32, _P(kt_image), _P(kt_integrator)]
_lib.kt_adjoint.argtypes = [_P(kt_camera), _P(kt_spacetime), _P(kt_disk), _P(kt_integrator), C.c_void_p,
                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
_lib.kt_adjoint.restype = C.c_int
_lib.kt_adjoint_workspace_bytes.argtypes = [_P(kt_camera), _P(kt_integrator)]
_lib.kt_adjoint_workspace_bytes.restype = C.c_size_t
_lib.kt_workspace_bytes_batch.restype = C.c_size_t
_lib.kt_init_rays.argtypes = [_P(kt_camera), _P(kt_spacetime), C.c_void_p, C.c_void_p, C.c_void_p]
_lib.kt_init_rays.restype = C.c_int
_lib.kt_last_error.argtypes = []
_lib.kt_last_error.restype = C.c_char_p
_lib.kt_version.argtypes = []
_lib.kt_version.restype = C.c_int

EXPORTED = ("kt_render", "kt_render_ex", "kt_render_noalloc", "kt_render_batch", "kt_autotune_batch", "kt_adjoint",
            "kt_workspace_bytes", "kt_workspace_bytes_batch", "kt_adjoint_workspace_bytes", "kt_init_rays",
            "kt_last_error", "kt_version")
AUTOTUNE_DEFAULT_COUNT = 30


class KtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"kerrtrace error {code}: {msg}")
        self.code = code


def _ref(x):
    return None if x is None else C.byref(x)


def kt_last_error():
    return _lib.kt_last_error().decode()


def kt_version():
    return _lib.kt_version()


def kt_workspace_bytes(camera, integ):
    return _lib.kt_workspace_bytes(C.byref(camera), C.byref(integ))


def kt_render(camera, spacetime, disk, source, integ, outputs, workspace_ptr, workspace_bytes, stream_ptr):
    return _lib.kt_render(C.byref(camera), C.byref(spacetime), _ref(disk), _ref(source),
                          C.byref(integ), C.byref(outputs), workspace_ptr, workspace_bytes, stream_ptr)


def kt_render_ex(camera, spacetime, disk, source, integ, outputs, workspace_ptr, workspace_bytes,
                 stream_ptr, launch=None):
    return _lib.kt_render_ex(C.byref(camera), C.byref(spacetime), _ref(disk), _ref(source),
                             C.byref(integ), C.byref(outputs), workspace_ptr, workspace_bytes,
                             stream_ptr, _ref(launch))


NOALLOC_SCRATCH_BYTES = 64 << 20  # KT_NOALLOC_SCRATCH_BYTES


def kt_render_noalloc(camera, spacetime, disk, source, integ, outputs, stream_ptr, launch=None):
    """kt_render_ex on the library's own scratch array (no workspace)."""
    return _lib.kt_render_noalloc(C.byref(camera), C.byref(spacetime), _ref(disk), _ref(source),
                                  C.byref(integ), C.byref(outputs), stream_ptr, _ref(launch))


def kt_workspace_bytes_batch(images, integ):
    """images: a ctypes array of kt_image."""
    return _lib.kt_workspace_bytes_batch(len(images), images, C.byref(integ))


def kt_render_batch(images, integ, outputs, workspace_ptr, workspace_bytes, stream_ptr, launch=None):
    """images: a ctypes array of kt_image."""
    return _lib.kt_render_batch(len(images), images, C.byref(integ), C.byref(outputs), workspace_ptr,
                                workspace_bytes, stream_ptr, _ref(launch))


def kt_autotune_batch(images, integ, outputs, workspace_ptr, workspace_bytes, stream_ptr, candidates=None,
                      repeats=2):
    """Returns (rc, best kt_launch, list of mean ms per candidate)."""
    n_c = 0 if candidates is None else len(candidates)
    arr = None if candidates is None else (kt_launch * n_c)(*candidates)
    times = (C.c_float * (n_c or AUTOTUNE_DEFAULT_COUNT))()
    best = kt_launch()
    rc = _lib.kt_autotune_batch(len(images), images, C.byref(integ), C.byref(outputs), workspace_ptr,
                                workspace_bytes, stream_ptr, arr, n_c, repeats, C.byref(best), times)
    return rc, best, list(times)


def kt_adjoint_workspace_bytes(camera, integ):
    return _lib.kt_adjoint_workspace_bytes(C.byref(camera), C.byref(integ))


def kt_adjoint(camera, spacetime, disk, integ, fate_ptr, r_hit_ptr, cot_ptr, grad_a_ptr, grad_incl_ptr,
               grad_rin_ptr, stats_ptr, workspace_ptr, workspace_bytes, stream_ptr, n_steps_ptr=None,
               grad_sum_ptr=None):
    return _lib.kt_adjoint(C.byref(camera), C.byref(spacetime), C.byref(disk), C.byref(integ), fate_ptr,
                           r_hit_ptr, n_steps_ptr, cot_ptr, grad_a_ptr, grad_incl_ptr, grad_rin_ptr,
                           grad_sum_ptr, stats_ptr, workspace_ptr, workspace_bytes, stream_ptr)


def kt_init_rays(camera, spacetime, state_ptr, invalid_ptr, stream_ptr):
    return _lib.kt_init_rays(C.byref(camera), C.byref(spacetime), state_ptr, invalid_ptr, stream_ptr)


# ---------------------------------------------------------------------------
# Convenience layer over torch tensors
# ---------------------------------------------------------------------------

def make_structs(M=1.0, a=0.0, metric=0, q=0.0, r_obs=1000.0, incl=math.pi / 2, fov_x=10.0, fov_y=10.0, nx=64,
                 ny=64, method=DP45, precision=FP64, h_fixed=1.0 / 128, rtol=1e-12, atol=1e-12,
                 h_init=1.0, cap_buffer=0.01, r_escape=0.0, h_budget=1e-10, r_switch=300.0,
                 max_steps=1_000_000, disk_on=0, r_in=6.0, r_out=30.0, emis_q=2.0, rotation=0, l0=0.0,
                 emis_model=0, src_on=0, r_src=1000.0, sky_on=0, grid_deg=6.0, line_deg=0.25,
                 checkpoint_every=0, split_above=0):
    """C structs from keyword parameters (the same names the workloads use)."""
    cam = kt_camera(r_obs, incl, fov_x, fov_y, nx, ny)
    st = kt_spacetime(M, a, int(metric), q)
    integ = kt_integrator(method, precision, h_fixed, rtol, atol, h_init, cap_buffer, r_escape,
                          h_budget, r_switch, int(max_steps), int(checkpoint_every), int(split_above))
    disk = kt_disk(int(disk_on), r_in, r_out, emis_q, int(rotation), l0, int(emis_model))
    src = kt_source(int(src_on), r_src, int(sky_on), grid_deg, line_deg)
    return cam, st, disk, src, integ


_DTYPES = {"fate": "uint8", "n_cross": "uint8", "used_fp64": "uint8", "ring": "uint8", "sky": "uint8",
           "n_steps": "int32", "n_evals": "int32"}


def alloc_outputs(n, device, want=OUTPUT_FIELDS, stats=True):
    """Device tensors for the requested outputs (fate is always allocated)."""
    import torch
    t = {}
    for f in OUTPUT_FIELDS:
        if f == "fate" or f in want:
            t[f] = torch.empty(n, dtype=getattr(torch, _DTYPES.get(f, "float64")), device=device)
    if stats:
        t["stats"] = torch.zeros(C.sizeof(kt_stats), dtype=torch.uint8, device=device)
    return t


def outputs_struct(t):
    o = kt_outputs()
    for f in OUTPUT_FIELDS:
        setattr(o, f, t[f].data_ptr() if f in t else None)
    o.stats = t["stats"].data_ptr() if "stats" in t else None
    return o


def read_stats(t):
    """kt_stats from a stats tensor (synchronises)."""
    raw = bytes(t["stats"].cpu().numpy())
    return kt_stats.from_buffer_copy(raw)


class Renderer:
    """Owns outputs and workspace for one configuration; render() enqueues one
    image on the current torch stream."""

    def __init__(self, device="cuda:0", want=OUTPUT_FIELDS, stats=True, launch=None, **params):
        import torch
        self.device = torch.device(device)
        self.params = params
        self.cam, self.st, self.disk, self.src, self.integ = make_structs(**params)
        self.n = self.cam.nx * self.cam.ny
        self.want = tuple(want)
        if "ring" in self.want and not self.src.enabled:
            self.want = tuple(w for w in self.want if w != "ring")
        if "sky" in self.want:
            self.want = tuple(dict.fromkeys(self.want + ("theta_f", "phi_f")))
        self.out = alloc_outputs(self.n, self.device, self.want, stats)
        self.ws_bytes = kt_workspace_bytes(self.cam, self.integ)
        if self.ws_bytes == 0:
            raise KtError(KT_EINVAL, "kt_workspace_bytes returned 0")
        # torch's caching allocator returns 256-byte-aligned blocks
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.c_out = outputs_struct(self.out)
        self.launch = launch

    def render(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        rc = kt_render_ex(self.cam, self.st, self.disk, self.src, self.integ, self.c_out,
                          self.ws.data_ptr(), self.ws_bytes, C.c_void_p(stream.cuda_stream),
                          self.launch)
        if rc != KT_OK:
            raise KtError(rc, kt_last_error())
        return self.out

    def autotune(self, candidates=None, repeats=2, stream=None):
        """Pick the fastest launch shape for this image (kt_autotune_batch on
        a one-image table, Kerr spacetimes), keep it for later renders and
        return (best, times_ms)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        table = image_table([split_params(self.params)[0]])
        rc, best, times = kt_autotune_batch(table, self.integ, self.c_out, self.ws.data_ptr(), self.ws_bytes,
                                            C.c_void_p(stream.cuda_stream), candidates, repeats)
        if rc != KT_OK:
            raise KtError(rc, kt_last_error())
        self.launch = best
        return best, times


_IMAGE_KEYS = ("M", "a", "metric", "q", "r_obs", "incl", "fov_x", "fov_y", "nx", "ny", "disk_on", "r_in", "r_out",
               "emis_q", "rotation", "l0", "emis_model", "src_on", "r_src", "sky_on", "grid_deg", "line_deg")


def split_params(params):
    """(per-image keyword parameters, integrator keyword parameters)."""
    img = {k: v for k, v in params.items() if k in _IMAGE_KEYS}
    integ = {k: v for k, v in params.items() if k not in _IMAGE_KEYS}
    return img, integ


def image_table(images):
    """ctypes array of kt_image from a list of per-image keyword dicts."""
    arr = (kt_image * len(images))()
    for k, im in enumerate(images):
        cam, st, disk, src, _ = make_structs(**im)
        arr[k] = kt_image(cam, st, disk, src)
    return arr


class BatchRenderer:
    """Owns outputs and workspace for a batch of images; render() enqueues
    all of them as one launch on the current torch stream.  `images` is a
    list of per-image keyword dicts (camera, spacetime, disk, source keys);
    `integ` holds the shared integrator keywords.  Outputs are concatenated;
    views(name) splits one of them per image."""

    def __init__(self, images, device="cuda:0", want=OUTPUT_FIELDS, stats=True, launch=None, **integ):
        import torch
        self.device = torch.device(device)
        self.images = [dict(im) for im in images]
        self.table = image_table(self.images)
        *_, self.integ = make_structs(**integ)
        self.sizes = [im.camera.nx * im.camera.ny for im in self.table]
        self.first = [sum(self.sizes[:k]) for k in range(len(self.sizes))]
        self.n = sum(self.sizes)
        self.want = tuple(want)
        if "ring" in self.want and not all(im.source.enabled for im in self.table):
            self.want = tuple(w for w in self.want if w != "ring")
        if "sky" in self.want:
            self.want = tuple(dict.fromkeys(self.want + ("theta_f", "phi_f")))
        self.out = alloc_outputs(self.n, self.device, self.want, stats)
        self.ws_bytes = kt_workspace_bytes_batch(self.table, self.integ)
        if self.ws_bytes == 0:
            raise KtError(KT_EINVAL, "kt_workspace_bytes_batch returned 0")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.c_out = outputs_struct(self.out)
        self.launch = launch

    def render(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        rc = kt_render_batch(self.table, self.integ, self.c_out, self.ws.data_ptr(), self.ws_bytes,
                             C.c_void_p(stream.cuda_stream), self.launch)
        if rc != KT_OK:
            raise KtError(rc, kt_last_error())
        return self.out

    def autotune(self, candidates=None, repeats=2, stream=None):
        """Pick the fastest launch shape on this batch (kt_autotune_batch),
        keep it for later renders and return (best, times_ms)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        rc, best, times = kt_autotune_batch(self.table, self.integ, self.c_out, self.ws.data_ptr(),
                                            self.ws_bytes, C.c_void_p(stream.cuda_stream), candidates,
                                            repeats)
        if rc != KT_OK:
            raise KtError(rc, kt_last_error())
        self.launch = best
        return best, times

    def views(self, name):
        t = self.out[name]
        return [t[f:f + n] for f, n in zip(self.first, self.sizes)]


def render(device="cuda:0", want=OUTPUT_FIELDS, launch=None, **params):
    """Render one image; returns a dict of device tensors (not synchronised)."""
    return Renderer(device=device, want=want, launch=launch, **params).render()


def init_rays(device="cuda:0", **params):
    """Initial state of every pixel: (state[7, n] float64, invalid[n] uint8)."""
    import torch
    cam, st, *_ = make_structs(**params)
    n = cam.nx * cam.ny
    state = torch.empty(7 * n, dtype=torch.float64, device=device)
    invalid = torch.empty(n, dtype=torch.uint8, device=device)
    stream = torch.cuda.current_stream(torch.device(device))
    rc = kt_init_rays(cam, st, state.data_ptr(), invalid.data_ptr(), C.c_void_p(stream.cuda_stream))
    if rc != KT_OK:
        raise KtError(rc, kt_last_error())
    return state.view(7, n), invalid
