"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, and rejects bad arguments before touching the device."""
import ctypes as C
import math
import os
import re

import pytest

# The rejection tests below hand the library placeholder device pointers that
# validation must refuse before any launch; they run only where no GPU is
# visible so that a validation bug can never reach a kernel.
def _gpu_visible():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


no_gpu_only = pytest.mark.skipif(_gpu_visible(), reason="placeholder pointers: CPU-only check")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kerrtrace.h")


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char \*)\s*(kt_\w+)\s*\(", text, re.M)))


def test_header_declares_expected_entry_points():
    assert _declared_functions() == sorted(
        ["kt_render", "kt_render_ex", "kt_render_noalloc", "kt_render_batch", "kt_autotune_batch", "kt_adjoint",
         "kt_workspace_bytes", "kt_workspace_bytes_batch", "kt_adjoint_workspace_bytes", "kt_init_rays",
         "kt_last_error", "kt_version"])


def test_library_exports_every_declared_symbol():
    from paper_2202_00086_amd import kerrtrace as K
    lib = C.CDLL(K.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert set(K.EXPORTED) == set(_declared_functions())
    assert K.kt_version() == 203


def test_struct_layouts_match_header():
    """ctypes mirrors of the header structs have the C sizes."""
    from paper_2202_00086_amd import kerrtrace as K
    assert C.sizeof(K.kt_camera) == 4 * 8 + 2 * 4
    assert C.sizeof(K.kt_spacetime) == 32
    assert C.sizeof(K.kt_disk) == 56
    assert C.sizeof(K.kt_source) == 40
    assert C.sizeof(K.kt_integrator) == 8 + 8 * 8 + 8 + 8  # checkpoint_every and split_above
    assert K.kt_integrator.split_above.offset == 84
    assert C.sizeof(K.kt_launch) == 20
    assert C.sizeof(K.kt_stats) == 13 * 8
    assert C.sizeof(K.kt_outputs) == 17 * 8
    assert C.sizeof(K.kt_image) == 40 + 32 + 56 + 40


def _args(**kw):
    from paper_2202_00086_amd import kerrtrace as K
    cam, st, disk, src, integ = K.make_structs(**kw)
    return K, cam, st, disk, src, integ


BAD = [
    dict(a=1.2),
    dict(M=0.0, a=0.1),
    dict(M=-1.0),
    dict(r_obs=1.5, a=0.0),
    dict(r_obs=1e300),                               # r_obs^2 overflows: camera constants not finite
    dict(nx=0),
    dict(ny=-3),
    dict(nx=65536, ny=32768),                        # 2^31 rays: beyond the int32 ray ids
    dict(fov_x=0.0),
    dict(incl=0.0),
    dict(incl=math.pi),
    dict(rtol=0.0),
    dict(rtol=float("nan")),
    dict(a=float("inf")),
    dict(method=7),
    dict(precision=5),
    dict(max_steps=0),
    dict(h_init=-1.0),
    dict(disk_on=1, r_in=1.0, r_out=30.0),          # r_in inside the horizon
    dict(disk_on=1, r_in=10.0, r_out=5.0),
    dict(r_escape=500.0),                            # inside the observer
    dict(src_on=1, r_src=1.0),
    dict(disk_on=1, rotation=2),
    dict(disk_on=1, emis_model=3),
    dict(disk_on=1, rotation=1, l0=float("nan")),
    dict(sky_on=1, grid_deg=-6.0),
    dict(metric=2),
    dict(metric=1, q=-1.0),
    dict(metric=1, q=float("nan")),
    dict(metric=1, q=0.5, a=0.3),
    dict(metric=1, q=0.5, disk_on=1, r_in=6.0),
    dict(metric=1, q=0.5, method=0),
    dict(metric=1, q=0.5, precision=1),
    dict(sky_on=1, line_deg=float("inf")),
    dict(checkpoint_every=48),                       # not a power of two
    dict(checkpoint_every=3),                        # not a power of two
    dict(checkpoint_every=-1),                       # negative
    dict(checkpoint_every=2048),                     # above 1024
    dict(split_above=-2),                            # below -1
]


@no_gpu_only
@pytest.mark.parametrize("kw", BAD)
def test_validation_rejects(kw):
    K, cam, st, disk, src, integ = _args(**kw)
    out = K.kt_outputs()
    out.fate = 0x1000  # never dereferenced: validation fails first
    rc = K.kt_render(cam, st, disk, src, integ, out, C.c_void_p(0x100000), 1 << 30, None)
    assert rc == K.KT_EINVAL
    assert K.kt_last_error() != ""


@no_gpu_only
def test_null_fate_and_workspace_rejected():
    K, cam, st, disk, src, integ = _args()
    out = K.kt_outputs()
    assert K.kt_render(cam, st, disk, src, integ, out, C.c_void_p(0x100000), 1 << 30, None) == K.KT_EINVAL
    out.fate = 0x1000
    assert K.kt_render(cam, st, disk, src, integ, out, None, 1 << 30, None) == K.KT_EINVAL
    # misaligned workspace
    assert K.kt_render(cam, st, disk, src, integ, out, C.c_void_p(0x100008), 1 << 30, None) == K.KT_EINVAL


@no_gpu_only
def test_workspace_too_small_is_enomem():
    K, cam, st, disk, src, integ = _args(nx=100, ny=100)
    need = K.kt_workspace_bytes(cam, integ)
    assert need >= 100 * 100 * 8
    out = K.kt_outputs()
    out.fate = 0x1000
    rc = K.kt_render(cam, st, disk, src, integ, out, C.c_void_p(0x100000), need - 1, None)
    assert rc == K.KT_ENOMEM
    assert "workspace" in K.kt_last_error()


@no_gpu_only
def test_ring_needs_source_and_deflection():
    K, cam, st, disk, src, integ = _args()
    out = K.kt_outputs()
    out.fate = 0x1000
    out.ring = 0x2000
    assert K.kt_render(cam, st, disk, src, integ, out, C.c_void_p(0x100000), 1 << 30, None) == K.KT_EINVAL


@no_gpu_only
def test_sky_needs_final_angles():
    K, cam, st, disk, src, integ = _args(sky_on=1)
    out = K.kt_outputs()
    out.fate = 0x1000
    out.sky = 0x2000
    assert K.kt_render(cam, st, disk, src, integ, out, C.c_void_p(0x100000), 1 << 30, None) == K.KT_EINVAL
    assert "theta_f" in K.kt_last_error()


@no_gpu_only
def test_launch_shape_validated():
    K, cam, st, disk, src, integ = _args()
    out = K.kt_outputs()
    out.fate = 0x1000
    for ln in [K.kt_launch(1, 96, 0, 32), K.kt_launch(1, 256, 0, 0), K.kt_launch(1, 256, -1, 32),
               K.kt_launch(1, 256, 0, 32, 2)]:
        rc = K.kt_render_ex(cam, st, disk, src, integ, out, C.c_void_p(0x100000), 1 << 30, None, ln)
        assert rc == K.KT_EINVAL


def test_workspace_bytes_zero_on_bad_camera():
    K, cam, st, disk, src, integ = _args(nx=0)
    assert K.kt_workspace_bytes(cam, integ) == 0
    K, cam, st, disk, src, integ = _args(nx=65536, ny=32768)  # 2^31 rays
    assert K.kt_workspace_bytes(cam, integ) == 0
    assert K.kt_adjoint_workspace_bytes(cam, integ) == 0
    K, cam, st, disk, src, integ = _args(checkpoint_every=96)
    assert K.kt_adjoint_workspace_bytes(cam, integ) == 0
    for every in (1, 2, 8, 64, 1024):
        K, cam, st, disk, src, integ = _args(checkpoint_every=every)
        assert K.kt_adjoint_workspace_bytes(cam, integ) > 0
    K, cam, st, disk, src, integ = _args(split_above=-2)
    assert K.kt_adjoint_workspace_bytes(cam, integ) == 0
    # the split buffers: a store of 32 steps (6 doubles each) per lane of the grid,
    # 4 (store / 64 + records) segment items (8 doubles and a 4-byte owner each)
    # and 8192 records of 112 bytes
    sizes = {}
    for split in (-1, 0, 700):
        K, cam, st, disk, src, integ = _args(nx=512, ny=512, split_above=split)
        sizes[split] = K.kt_adjoint_workspace_bytes(cam, integ)
    assert sizes[0] == sizes[700] > sizes[-1]
    lanes = 65536
    items = 4 * (32 * lanes // 64 + 8192)
    extra = 32 * lanes * 48 + items * (64 + 4) + 8192 * 112
    assert 0 <= sizes[0] - sizes[-1] - extra < 4 * 256


def _batch(images, **integ_kw):
    from paper_2202_00086_amd import kerrtrace as K
    table = K.image_table(images)
    *_, integ = K.make_structs(**integ_kw)
    return K, table, integ


GOOD_IMAGE = dict(a=0.5, nx=8, ny=6, incl=1.0)


@no_gpu_only
@pytest.mark.parametrize("k, kw", [(0, dict(a=1.2)), (1, dict(nx=0)), (2, dict(disk_on=1, r_in=1.0)),
                                   (1, dict(src_on=1, r_src=1.0)), (2, dict(incl=0.0))])
def test_batch_validation_names_the_image(k, kw):
    images = [dict(GOOD_IMAGE) for _ in range(3)]
    images[k].update(kw)
    K, table, integ = _batch(images)
    out = K.kt_outputs()
    out.fate = 0x1000
    rc = K.kt_render_batch(table, integ, out, C.c_void_p(0x100000), 1 << 30, None)
    assert rc == K.KT_EINVAL
    assert K.kt_last_error().startswith(f"image {k}:"), K.kt_last_error()


@no_gpu_only
def test_batch_rejects_bad_counts_and_shared_arguments():
    from paper_2202_00086_amd import kerrtrace as K
    K_, table, integ = _batch([GOOD_IMAGE])
    out = K.kt_outputs()
    out.fate = 0x1000
    ws = C.c_void_p(0x100000)
    lib = K._lib
    assert lib.kt_render_batch(0, table, C.byref(integ), C.byref(out), ws, 1 << 30, None, None) == K.KT_EINVAL
    assert lib.kt_render_batch(K.MAX_IMAGES + 1, table, C.byref(integ), C.byref(out), ws, 1 << 30, None,
                               None) == K.KT_EINVAL
    assert lib.kt_render_batch(1, None, C.byref(integ), C.byref(out), ws, 1 << 30, None, None) == K.KT_EINVAL
    _, table, bad_integ = _batch([GOOD_IMAGE], rtol=0.0)
    assert K.kt_render_batch(table, bad_integ, out, ws, 1 << 30, None) == K.KT_EINVAL
    # ring with an image whose source is off
    _, table, integ = _batch([dict(GOOD_IMAGE, src_on=1), GOOD_IMAGE])
    out.ring = 0x2000
    out.deflection = 0x3000
    assert K.kt_render_batch(table, integ, out, ws, 1 << 30, None) == K.KT_EINVAL
    assert "image 1" in K.kt_last_error()


@no_gpu_only
def test_batch_total_rays_limit():
    """Every image is valid, their total is not: the render refuses it and
    the workspace size is 0."""
    K, table, integ = _batch([dict(GOOD_IMAGE, nx=40000, ny=40000), dict(GOOD_IMAGE, nx=40000, ny=20000)])
    out = K.kt_outputs()
    out.fate = 0x1000
    assert K.kt_workspace_bytes_batch(table, integ) == 0
    assert K.kt_render_batch(table, integ, out, C.c_void_p(0x100000), 1 << 40, None) == K.KT_EINVAL
    assert "2^31" in K.kt_last_error()


@no_gpu_only
def test_batch_workspace_size():
    """The batch workspace holds the image table on top of the per-ray
    buffers, and a smaller one is refused."""
    images = [dict(GOOD_IMAGE, nx=10 + k, ny=7) for k in range(5)]
    K, table, integ = _batch(images)
    need = K.kt_workspace_bytes_batch(table, integ)
    n = sum((10 + k) * 7 for k in range(5))
    cam, _, _, _, integ1 = K.make_structs(nx=n, ny=1)
    assert need > K.kt_workspace_bytes(cam, integ1)
    out = K.kt_outputs()
    out.fate = 0x1000
    assert K.kt_render_batch(table, integ, out, C.c_void_p(0x100000), need - 1, None) == K.KT_ENOMEM
    # mixed precision needs the fallback list and flags too
    _, table, integ_m = _batch(images, precision=K.MIXED)
    assert K.kt_workspace_bytes_batch(table, integ_m) >= need + 5 * n
    assert K.kt_workspace_bytes_batch((K.kt_image * 0)(), integ) == 0


@no_gpu_only
def test_autotune_validation():
    from paper_2202_00086_amd import kerrtrace as K
    _, table, integ = _batch([GOOD_IMAGE])
    out = K.kt_outputs()
    out.fate = 0x1000
    ws = C.c_void_p(0x100000)
    lib = K._lib
    best = K.kt_launch()
    one = (K.kt_launch * 1)(K.kt_launch(1, 256, 0, 32))
    bad = (K.kt_launch * 1)(K.kt_launch(1, 96, 0, 32))

    def call(cands, n, repeats, best_ref):
        return lib.kt_autotune_batch(1, table, C.byref(integ), C.byref(out), ws, 1 << 30, None, cands, n,
                                     repeats, best_ref, None)
    assert call(None, 0, 0, C.byref(best)) == K.KT_EINVAL          # repeats
    assert call(None, 0, 101, C.byref(best)) == K.KT_EINVAL
    assert call(None, 3, 2, C.byref(best)) == K.KT_EINVAL          # NULL list with a count
    assert call(one, 0, 2, C.byref(best)) == K.KT_EINVAL           # list without a count
    assert call(one, 1, 2, None) == K.KT_EINVAL                    # no place for the result
    assert call(bad, 1, 2, C.byref(best)) == K.KT_EINVAL           # shape out of range
    assert "candidate" in K.kt_last_error()
    bad_order = (K.kt_launch * 1)(K.kt_launch(1, 256, 0, 32, 7))
    assert call(bad_order, 1, 2, C.byref(best)) == K.KT_EINVAL     # unknown dispatch order
    assert "order 7" in K.kt_last_error()


@no_gpu_only
def test_adjoint_validation():
    from paper_2202_00086_amd import kerrtrace as K
    from paper_2202_00086_amd import workloads as W
    p = W.differentiable_disk(n=16)
    cam, st, disk, src, integ = K.make_structs(**p)
    ws = C.c_void_p(0x100000)
    need = K.kt_adjoint_workspace_bytes(cam, integ)
    assert need > 256 * 64 * 6 * 8

    def call(cam=cam, st=st, disk=disk, integ=integ, fate=0x1000, cot=0x2000, nbytes=1 << 40):
        return K.kt_adjoint(cam, st, disk, integ, fate, None, cot, None, None, None, None, ws, nbytes, None)
    _, _, _, _, rk = K.make_structs(**dict(p, method=K.RKF45))
    assert call(integ=rk) == K.KT_EINVAL and "KT_DP45" in K.kt_last_error()
    _, _, _, _, mx = K.make_structs(**dict(p, precision=K.MIXED))
    assert call(integ=mx) == K.KT_EINVAL
    _, _, nodisk, _, _ = K.make_structs(**dict(p, disk_on=0))
    assert call(disk=nodisk) == K.KT_EINVAL
    assert call(fate=None) == K.KT_EINVAL
    assert call(cot=None) == K.KT_EINVAL
    assert call(nbytes=need - 1) == K.KT_ENOMEM
    _, bad_st, _, _, _ = K.make_structs(**dict(p, a=1.5))
    assert call(st=bad_st) == K.KT_EINVAL
    assert K.kt_adjoint(cam, st, disk, integ, 0x1000, None, 0x2000, None, None, None, None, None, need,
                        None) == K.KT_EINVAL


@no_gpu_only
def test_qmetric_not_in_batches_or_the_adjoint():
    from paper_2202_00086_amd import kerrtrace as K
    from paper_2202_00086_amd import workloads as W
    _, table, integ = _batch([dict(GOOD_IMAGE), dict(GOOD_IMAGE, metric=1, q=0.4)])
    out = K.kt_outputs()
    out.fate = 0x1000
    assert K.kt_render_batch(table, integ, out, C.c_void_p(0x100000), 1 << 30, None) == K.KT_EINVAL
    assert "image 1" in K.kt_last_error()
    cam, st, disk, src, integ = K.make_structs(**dict(W.differentiable_disk(n=16), metric=1, q=0.4, a=0.0))
    assert K.kt_adjoint(cam, st, disk, integ, 0x1000, None, 0x2000, None, None, None, None, C.c_void_p(0x100000),
                        1 << 40, None) == K.KT_EINVAL


def test_plain_c_program_uses_the_header_and_library(tmp_path):
    """A C99 program compiled with gcc against include/kerrtrace.h links the
    library and reads its version (no GPU needed for that call)."""
    import subprocess
    from paper_2202_00086_amd import kerrtrace as K
    from tests.c_abi import build_demo
    exe = build_demo(str(tmp_path))
    r = subprocess.run([exe, "--version"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    assert int(r.stdout.strip()) == K.kt_version()
