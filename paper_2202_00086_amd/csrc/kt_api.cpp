// kt_api.cpp -- host runtime and C ABI of the Kerr ray tracer: argument
// validation, per-image camera constants, workspace layout and the launch
// sequence on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "kerrtrace.h"
#include "kt_internal.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

bool finite_all(std::initializer_list<double> v) {
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

// Compute units of the current device (cached per device id).
int device_cus() {
    static std::mutex mu;
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lk(mu);
    if (cache[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        cache[dev] = n;
    }
    return cache[dev];
}

double horizon(double M, double a) { return M + std::sqrt(M * M - a * a); }

int validate_common(const kt_camera* cam, const kt_spacetime* st) {
    if (!cam || !st) return fail(KT_EINVAL, "camera and spacetime must not be NULL");
    if (!finite_all({cam->r_obs, cam->incl, cam->fov_x, cam->fov_y, st->M, st->a}))
        return fail(KT_EINVAL, "non-finite camera or spacetime parameter");
    if (!(st->M > 0.0)) return fail(KT_EINVAL, "M must be > 0 (got %g)", st->M);
    if (st->a * st->a > st->M * st->M) return fail(KT_EINVAL, "|a| must be <= M (a=%g, M=%g)", st->a, st->M);
    if (!(cam->incl > 0.0 && cam->incl < M_PI))
        return fail(KT_EINVAL, "incl must lie in (0, pi) (got %g)", cam->incl);
    if (!(cam->fov_x > 0.0 && cam->fov_y > 0.0)) return fail(KT_EINVAL, "fov_x and fov_y must be > 0");
    if (cam->nx < 1 || cam->ny < 1) return fail(KT_EINVAL, "nx and ny must be >= 1");
    if (static_cast<int64_t>(cam->nx) * cam->ny >= (int64_t{1} << 31))
        return fail(KT_EINVAL, "nx*ny must be < 2^31");
    return KT_OK;
}

// Per-image camera constants at (r_obs, incl) from the Kerr metric
// (eq:Kerr) and the observer tetrad (eq:matrix, second eq:momentums).
void camera_constants(const kt_camera* cam, const kt_spacetime* st, kt::Params& p) {
    const double M = st->M, a = st->a, r0 = cam->r_obs;
    const double s = std::sin(cam->incl), c = std::cos(cam->incl);
    const double Sig = r0 * r0 + a * a * c * c;
    const double Del = r0 * r0 - 2.0 * M * r0 + a * a;
    const double g_tph = -2.0 * M * a * r0 * s * s / Sig;
    const double g_phph = s * s * (r0 * r0 + a * a + 2.0 * M * a * a * r0 * s * s / Sig);
    // g_tph^2 - g_tt g_phph = Delta sin^2 for Kerr, so A_t = sqrt(g_phph / (Delta sin^2))
    const double At = std::sqrt(g_phph / (Del * s * s));
    p.E0 = 1.0 / At;
    p.cE = g_tph / (r0 * std::sqrt(g_phph));
    p.cL = -std::sqrt(g_phph) / r0;
    p.cth = std::sqrt(Sig) / r0;
    p.g_rr = Sig / Del;
    p.r0 = r0;
    p.incl = cam->incl;
    p.inv_r0 = 1.0 / r0;
    p.fov_x = cam->fov_x;
    p.fov_y = cam->fov_y;
    p.dx = 2.0 * cam->fov_x / cam->nx;
    p.dy = 2.0 * cam->fov_y / cam->ny;
    p.nx = cam->nx;
    p.ny = cam->ny;
    p.n_rays = cam->nx * cam->ny;
    p.M = M;
    p.a = a;
    p.a2 = a * a;
    p.two_a2 = 2.0 * a * a;
}

size_t ws_bytes(const kt_camera* cam, const kt_integrator* integ) {
    size_t n = static_cast<size_t>(cam->nx) * static_cast<size_t>(cam->ny);
    size_t b = kt::ws_fb_list_offset(n);
    if (integ->precision == KT_MIXED) b = kt::ws_need_offset(n) + n;
    return (b + 255) & ~static_cast<size_t>(255);
}

}  // namespace

extern "C" {

const char* kt_last_error(void) { return g_err; }

int kt_version(void) { return KT_VERSION_NUMBER; }

size_t kt_workspace_bytes(const kt_camera* camera, const kt_integrator* integ) {
    if (!camera || !integ || camera->nx < 1 || camera->ny < 1) return 0;
    return ws_bytes(camera, integ);
}

int kt_init_rays(const kt_camera* camera, const kt_spacetime* spacetime, double* state,
                 uint8_t* invalid, void* hip_stream) {
    g_err[0] = 0;
    int rc = validate_common(camera, spacetime);
    if (rc) return rc;
    if (!state || !invalid) return fail(KT_EINVAL, "state and invalid must not be NULL");
    if (!(camera->r_obs > horizon(spacetime->M, spacetime->a)))
        return fail(KT_EINVAL, "r_obs must lie outside the horizon");
    kt::Params p;
    std::memset(&p, 0, sizeof p);
    camera_constants(camera, spacetime, p);
    if (kt::launch_init_rays(p, state, invalid, hip_stream))
        return fail(KT_EDEVICE, "init kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
    return KT_OK;
}

int kt_render_ex(const kt_camera* camera, const kt_spacetime* spacetime, const kt_disk* disk,
                 const kt_source* source, const kt_integrator* integ, const kt_outputs* out,
                 void* workspace, size_t workspace_bytes, void* hip_stream, const kt_launch* launch) {
    g_err[0] = 0;
    int rc = validate_common(camera, spacetime);
    if (rc) return rc;
    if (!integ || !out) return fail(KT_EINVAL, "integ and out must not be NULL");
    if (!out->fate) return fail(KT_EINVAL, "out->fate must not be NULL");
    const double M = spacetime->M, a = spacetime->a;
    const double r_plus = horizon(M, a);
    if (integ->method != KT_RK4_S && integ->method != KT_DP45)
        return fail(KT_EINVAL, "unknown integrator method %d", integ->method);
    if (integ->precision != KT_FP64 && integ->precision != KT_MIXED)
        return fail(KT_EINVAL, "unknown precision %d", integ->precision);
    if (integ->precision == KT_MIXED) {
        if (integ->method != KT_DP45) return fail(KT_EINVAL, "KT_MIXED needs method KT_DP45");
        if (!(integ->h_budget >= 0.0) || !(integ->r_switch > 0.0))
            return fail(KT_EINVAL, "KT_MIXED needs h_budget >= 0 and r_switch > 0");
    }
    if (!finite_all({integ->h_fixed, integ->rtol, integ->atol, integ->h_init, integ->capture_buffer,
                     integ->r_escape, integ->h_budget, integ->r_switch}))
        return fail(KT_EINVAL, "non-finite integrator parameter");
    if (integ->method == KT_RK4_S && !(integ->h_fixed > 0.0))
        return fail(KT_EINVAL, "h_fixed must be > 0");
    if (integ->method == KT_DP45 && !(integ->rtol > 0.0 && integ->atol > 0.0 && integ->h_init > 0.0))
        return fail(KT_EINVAL, "rtol, atol and h_init must be > 0");
    if (!(integ->capture_buffer >= 0.0)) return fail(KT_EINVAL, "capture_buffer must be >= 0");
    if (integ->max_steps < 1 || integ->max_steps > 100000000)
        return fail(KT_EINVAL, "max_steps must lie in [1, 1e8]");
    const double r_cap = r_plus + integ->capture_buffer;
    if (!(camera->r_obs > r_cap)) return fail(KT_EINVAL, "r_obs must exceed r_+ + capture_buffer");
    const double r_esc = integ->r_escape == 0.0 ? 1.1 * camera->r_obs : integ->r_escape;
    if (!(r_esc > camera->r_obs)) return fail(KT_EINVAL, "r_escape must exceed r_obs");

    const bool disk_on = disk && disk->enabled;
    if (disk_on) {
        if (!finite_all({disk->r_in, disk->r_out, disk->emis_index}))
            return fail(KT_EINVAL, "non-finite disk parameter");
        if (!(disk->r_in > r_plus && disk->r_out > disk->r_in))
            return fail(KT_EINVAL, "disk needs r_+ < r_in < r_out");
    }
    const bool src_on = source && source->enabled;
    if (src_on) {
        if (!std::isfinite(source->r_src) || !(source->r_src > r_cap))
            return fail(KT_EINVAL, "r_src must be finite and outside r_+ + capture_buffer");
    }
    if (out->ring && !(src_on && out->deflection))
        return fail(KT_EINVAL, "ring needs an enabled source and a deflection output");

    kt_launch ln{1, 256, 0, 32};
    if (launch) ln = *launch;
    if (ln.block != 64 && ln.block != 128 && ln.block != 256)
        return fail(KT_EINVAL, "launch block must be 64, 128 or 256");
    if (ln.batch < 1 || ln.batch > 4096) return fail(KT_EINVAL, "launch batch must lie in [1, 4096]");
    if (ln.blocks_per_cu < 0 || ln.blocks_per_cu > 64)
        return fail(KT_EINVAL, "launch blocks_per_cu must lie in [0, 64]");

    const size_t need = ws_bytes(camera, integ);
    if (!workspace) return fail(KT_EINVAL, "workspace must not be NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(KT_EINVAL, "workspace must be 256-byte aligned");
    if (workspace_bytes < need)
        return fail(KT_ENOMEM, "workspace too small: %zu < %zu bytes", workspace_bytes, need);

    kt::Params p;
    std::memset(&p, 0, sizeof p);
    camera_constants(camera, spacetime, p);
    p.r_cap = r_cap;
    p.r_esc = r_esc;
    p.method = integ->method;
    p.precision = integ->precision;
    p.h_fixed = integ->h_fixed;
    p.rtol = integ->rtol;
    p.atol = integ->atol;
    p.h_init = integ->h_init;
    p.max_steps = integ->max_steps;
    p.max_evals = 16 * integ->max_steps;
    p.h_budget = integ->h_budget;
    p.r_switch = integ->r_switch;
    p.disk_on = disk_on ? 1 : 0;
    if (disk_on) {
        p.r_in = disk->r_in;
        p.r_out = disk->r_out;
        p.emis_q = disk->emis_index;
    }
    p.src_on = src_on ? 1 : 0;
    if (src_on) {
        p.r_src = source->r_src;
        p.src_tol = 1e-12 * source->r_src;
        // the source sits at (theta, phi) = (pi - incl, pi)
        const double ts = M_PI - camera->incl;
        p.src_n[0] = std::sin(ts) * std::cos(M_PI);
        p.src_n[1] = std::sin(ts) * std::sin(M_PI);
        p.src_n[2] = std::cos(ts);
    }
    p.out.fate = out->fate;
    p.out.r_hit = out->r_hit;
    p.out.g = out->g;
    p.out.intensity = out->intensity;
    p.out.max_abs_h = out->max_abs_h;
    p.out.max_rel_h = out->max_rel_h;
    p.out.psi = out->psi;
    p.out.deflection = out->deflection;
    p.out.theta_f = out->theta_f;
    p.out.phi_f = out->phi_f;
    p.out.n_cross = out->n_cross;
    p.out.used_fp64 = out->used_fp64;
    p.out.ring = out->ring;
    p.out.n_steps = out->n_steps;
    p.out.n_evals = out->n_evals;
    p.out.stats = out->stats;
    char* ws = static_cast<char*>(workspace);
    p.ticket = reinterpret_cast<uint32_t*>(ws + kt::WS_TICKET);
    p.acc = reinterpret_cast<unsigned long long*>(ws + kt::WS_ACC);
    p.fb_count = reinterpret_cast<uint32_t*>(ws + kt::WS_FB_COUNT);
    p.rc_buf = reinterpret_cast<double*>(ws + kt::WS_RC);
    p.ws_params = reinterpret_cast<kt::Params*>(ws + kt::WS_PARAMS);
    p.need_fb = reinterpret_cast<uint8_t*>(ws + kt::ws_need_offset(static_cast<size_t>(p.n_rays)));
    p.fb_list = reinterpret_cast<uint32_t*>(ws + kt::ws_fb_list_offset(static_cast<size_t>(p.n_rays)));
    p.persistent = ln.persistent ? 1 : 0;
    p.batch = ln.batch;
    p.from_list = 0;

    if (kt::launch_ws_init(p, hip_stream))
        return fail(KT_EDEVICE, "workspace init launch failed: %s", hipGetErrorString(hipGetLastError()));
    int grid;
    if (p.persistent) {
        const int per_cu = ln.blocks_per_cu > 0 ? ln.blocks_per_cu : kt::trace_max_blocks_per_cu(p, ln.block);
        grid = device_cus() * per_cu;
        const int64_t needed = (static_cast<int64_t>(p.n_rays) + ln.block - 1) / ln.block;
        if (grid > needed) grid = static_cast<int>(needed);
    } else {
        grid = static_cast<int>((static_cast<int64_t>(p.n_rays) + ln.block - 1) / ln.block);
    }
    if (grid < 1) grid = 1;
    if (kt::launch_trace(p, grid, ln.block, hip_stream))
        return fail(KT_EDEVICE, "trace kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
    if (p.precision == KT_MIXED) {
        // re-run every ray over the |H|_rel budget in FP64, from a compacted
        // list whose length stays on the device
        if (kt::launch_fallback_list(p, hip_stream))
            return fail(KT_EDEVICE, "fallback list launch failed: %s", hipGetErrorString(hipGetLastError()));
        int grid2 = ln.persistent ? grid
                                  : static_cast<int>((static_cast<int64_t>(p.n_rays) + ln.block - 1) / ln.block);
        if (grid2 < 1) grid2 = 1;
        if (kt::launch_trace_fallback(p, grid2, ln.block, hip_stream))
            return fail(KT_EDEVICE, "fallback trace launch failed: %s", hipGetErrorString(hipGetLastError()));
    }
    if ((out->r_hit || out->g || out->intensity) && kt::launch_disk_obs(p, hip_stream))
        return fail(KT_EDEVICE, "disk observables launch failed: %s", hipGetErrorString(hipGetLastError()));
    if (out->ring && kt::launch_ring(p, hip_stream))
        return fail(KT_EDEVICE, "ring kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
    if (out->stats && kt::launch_stats(p, hip_stream))
        return fail(KT_EDEVICE, "stats kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
    return KT_OK;
}

int kt_render(const kt_camera* camera, const kt_spacetime* spacetime, const kt_disk* disk,
              const kt_source* source, const kt_integrator* integ, const kt_outputs* out,
              void* workspace, size_t workspace_bytes, void* hip_stream) {
    return kt_render_ex(camera, spacetime, disk, source, integ, out, workspace, workspace_bytes,
                        hip_stream, nullptr);
}

}  // extern "C"
