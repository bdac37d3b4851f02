// host_abi_driver.cpp -- test-only: the library's host runtime (kt_api.cpp)
// linked with the host stand-ins of stub_launch.cpp, driven through the C
// ABI with host buffers of exactly the sizes the library asks for, under
// AddressSanitizer and UndefinedBehaviorSanitizer.  Valid calls must return
// KT_OK (their stand-in kernels touch every byte the real ones would);
// invalid ones must return their error code.  Prints "ok N" at the end.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "kerrtrace.h"

namespace {

int g_calls = 0;

void* alloc_exact(size_t n) {
    void* p = nullptr;
    if (posix_memalign(&p, 256, n ? n : 1) != 0) std::abort();
    return p;
}

void expect(int got, int want, const char* what) {
    ++g_calls;
    if (got != want) {
        std::fprintf(stderr, "FAIL %s: got %d want %d (%s)\n", what, got, want, kt_last_error());
        std::exit(1);
    }
}

struct Outs {
    std::vector<void*> bufs;
    kt_outputs o;
    Outs(size_t n, bool all) {
        std::memset(&o, 0, sizeof o);
        o.fate = static_cast<uint8_t*>(take(n));
        if (all) {
            for (double** d : {&o.r_hit, &o.g, &o.intensity, &o.max_abs_h, &o.max_rel_h, &o.psi, &o.deflection,
                               &o.theta_f, &o.phi_f})
                *d = static_cast<double*>(take(8 * n));
            for (uint8_t** b : {&o.n_cross, &o.used_fp64}) *b = static_cast<uint8_t*>(take(n));
            o.n_steps = static_cast<int32_t*>(take(4 * n));
            o.n_evals = static_cast<int32_t*>(take(4 * n));
            o.stats = static_cast<kt_stats*>(take(sizeof(kt_stats)));
        }
    }
    void* take(size_t b) {
        bufs.push_back(alloc_exact(b));
        return bufs.back();
    }
    ~Outs() {
        for (void* p : bufs) std::free(p);
    }
};

kt_integrator integ_of(int method, int precision) {
    kt_integrator it;
    std::memset(&it, 0, sizeof it);
    it.method = method;
    it.precision = precision;
    it.h_fixed = 1.0 / 128;
    it.rtol = it.atol = 1e-12;
    it.h_init = 1.0;
    it.capture_buffer = 0.01;
    it.h_budget = 1e-10;
    it.r_switch = 300.0;
    it.max_steps = 1000000;
    return it;
}

void render_case(int nx, int ny, int method, int precision, bool disk_on, bool src_on, bool sky_on,
                 const kt_launch* ln, bool all) {
    kt_camera cam = {1000.0, 1.0, 12.0, 9.0, nx, ny};
    kt_spacetime st = {1.0, 0.9, KT_METRIC_KERR, 0.0};
    kt_disk disk = {disk_on ? 1 : 0, 2.4, 30.0, 2.0, KT_ROT_KEPLER, 0.0, KT_EMIS_POWER};
    kt_source src = {src_on ? 1 : 0, 1000.0, sky_on ? 1 : 0, 6.0, 0.25};
    kt_integrator it = integ_of(method, precision);
    const size_t n = static_cast<size_t>(nx) * ny;
    Outs out(n, all);
    if (src_on && all) out.o.ring = static_cast<uint8_t*>(out.take(n));
    if (sky_on && all) out.o.sky = static_cast<uint8_t*>(out.take(n));
    const size_t wsb = kt_workspace_bytes(&cam, &it);
    void* ws = alloc_exact(wsb);
    expect(kt_render_ex(&cam, &st, &disk, &src, &it, &out.o, ws, wsb, nullptr, ln), KT_OK, "render");
    expect(kt_render_ex(&cam, &st, &disk, &src, &it, &out.o, ws, wsb - 1, nullptr, ln), KT_ENOMEM, "small ws");
    std::free(ws);
}

void batch_case(bool mixed, bool src_on) {
    std::vector<kt_image> ims;
    const int sizes[][2] = {{1, 1}, {7, 3}, {64, 64}, {5, 40}, {33, 17}};
    for (int k = 0; k < 5; ++k) {
        kt_image im;
        std::memset(&im, 0, sizeof im);
        im.camera = {100.0 + 300.0 * k, 0.3 + 0.5 * k, 35.0, 35.0, sizes[k][0], sizes[k][1]};
        im.spacetime = {1.0, 0.2 * k, KT_METRIC_KERR, 0.0};
        im.disk = {1, 6.0, 30.0, 2.0, KT_ROT_KEPLER, 0.0, KT_EMIS_POWER};
        im.source = {src_on ? 1 : 0, im.camera.r_obs, 0, 0.0, 0.0};
        ims.push_back(im);
    }
    kt_integrator it = integ_of(KT_DP45, mixed ? KT_MIXED : KT_FP64);
    size_t n = 0;
    for (auto& im : ims) n += static_cast<size_t>(im.camera.nx) * im.camera.ny;
    Outs out(n, true);
    if (src_on) out.o.ring = static_cast<uint8_t*>(out.take(n));
    const size_t wsb = kt_workspace_bytes_batch(5, ims.data(), &it);
    void* ws = alloc_exact(wsb);
    kt_launch ln = {1, 128, 2, 16, KT_ORDER_RING};
    expect(kt_render_batch(5, ims.data(), &it, &out.o, ws, wsb, nullptr, nullptr), KT_OK, "batch");
    expect(kt_render_batch(5, ims.data(), &it, &out.o, ws, wsb, nullptr, &ln), KT_OK, "batch launch");
    expect(kt_render_batch(5, ims.data(), &it, &out.o, ws, wsb - 1, nullptr, nullptr), KT_ENOMEM, "batch small ws");
    ims[3].camera.r_obs = 1.5;  // inside the horizon: named in the error
    expect(kt_render_batch(5, ims.data(), &it, &out.o, ws, wsb, nullptr, nullptr), KT_EINVAL, "batch bad image");
    if (!std::strstr(kt_last_error(), "image 3")) {
        std::fprintf(stderr, "FAIL batch message: %s\n", kt_last_error());
        std::exit(1);
    }
    std::free(ws);
}

void adjoint_case(int nx, int ny, int every, bool maps, bool sums, bool stats, int split = 0) {
    kt_camera cam = {1000.0, 0.8, 35.0, 35.0, nx, ny};
    kt_spacetime st = {1.0, 0.7, KT_METRIC_KERR, 0.0};
    kt_disk disk = {1, 3.4, 30.0, 2.0, KT_ROT_KEPLER, 0.0, KT_EMIS_TAPERED};
    kt_integrator it = integ_of(KT_DP45, KT_FP64);
    it.checkpoint_every = every;
    it.split_above = split;
    const size_t n = static_cast<size_t>(nx) * ny;
    std::vector<void*> b;
    auto take = [&](size_t bytes) { b.push_back(alloc_exact(bytes)); return b.back(); };
    auto* fate = static_cast<uint8_t*>(take(n));
    auto* r_hit = static_cast<double*>(take(8 * n));
    auto* steps = static_cast<int32_t*>(take(4 * n));
    auto* cot = static_cast<double*>(take(8 * n));
    double* g[3] = {nullptr, nullptr, nullptr};
    if (maps)
        for (auto& p : g) p = static_cast<double*>(take(8 * n));
    double* gs = sums ? static_cast<double*>(take(24)) : nullptr;
    uint64_t* sp = stats ? static_cast<uint64_t*>(take(32)) : nullptr;
    const size_t wsb = kt_adjoint_workspace_bytes(&cam, &it);
    void* ws = alloc_exact(wsb);
    expect(kt_adjoint(&cam, &st, &disk, &it, fate, r_hit, steps, cot, g[0], g[1], g[2], gs, sp, ws, wsb, nullptr),
           KT_OK, "adjoint");
    expect(kt_adjoint(&cam, &st, &disk, &it, fate, nullptr, nullptr, cot, g[0], g[1], g[2], gs, sp, ws, wsb - 1,
                      nullptr),
           KT_ENOMEM, "adjoint small ws");
    std::free(ws);
    for (void* p : b) std::free(p);
}

}  // namespace

int main() {
    const kt_launch shapes[] = {{1, 256, 0, 4, KT_ORDER_RING}, {1, 64, 1, 1, KT_ORDER_ROWS},
                                {0, 128, 0, 32, KT_ORDER_RING}, {1, 128, 3, 4096, KT_ORDER_ROWS}};
    const int dims[][2] = {{1, 1}, {3, 7}, {64, 64}, {1000, 3}, {257, 129}};
    for (auto& d : dims)
        for (auto& ln : shapes) {
            render_case(d[0], d[1], KT_DP45, KT_FP64, false, true, false, &ln, true);
            render_case(d[0], d[1], KT_DP45, KT_MIXED, true, false, false, &ln, true);
        }
    for (int m = KT_RK4_S; m <= KT_BS_RAT; ++m) render_case(33, 20, m, KT_FP64, true, true, true, nullptr, true);
    render_case(16, 16, KT_DP45, KT_FP64, false, false, false, nullptr, false);  // fate only
    batch_case(false, false);
    batch_case(true, true);
    for (int every : {0, 8, 1024}) {
        adjoint_case(40, 24, every, true, true, true);
        adjoint_case(1, 1, every, false, true, false);
        adjoint_case(300, 301, every, false, false, true);
    }
    // split backward sweeps off, and at a fixed threshold
    adjoint_case(40, 24, 1, true, true, true, -1);
    adjoint_case(300, 301, 0, true, false, true, 500);

    // init_rays
    {
        kt_camera cam = {50.0, 1.0, 60.0, 60.0, 9, 4};
        kt_spacetime st = {1.0, 0.5, KT_METRIC_KERR, 0.0};
        auto* state = static_cast<double*>(alloc_exact(7 * 8 * 36));
        auto* inv = static_cast<uint8_t*>(alloc_exact(36));
        expect(kt_init_rays(&cam, &st, state, inv, nullptr), KT_OK, "init_rays");
        expect(kt_init_rays(&cam, &st, nullptr, inv, nullptr), KT_EINVAL, "init_rays null");
        std::free(state);
        std::free(inv);
    }

    // invalid arguments: every one is refused before any device work
    {
        kt_camera cam = {1000.0, 1.0, 12.0, 12.0, 8, 8};
        kt_spacetime st = {1.0, 0.9, KT_METRIC_KERR, 0.0};
        kt_integrator it = integ_of(KT_DP45, KT_FP64);
        Outs out(64, false);
        const size_t wsb = kt_workspace_bytes(&cam, &it);
        void* ws = alloc_exact(wsb);
        expect(kt_render(&cam, &st, nullptr, nullptr, &it, &out.o, ws, wsb, nullptr), KT_OK, "plain render");
        expect(kt_render(nullptr, &st, nullptr, nullptr, &it, &out.o, ws, wsb, nullptr), KT_EINVAL, "null camera");
        expect(kt_render(&cam, &st, nullptr, nullptr, &it, nullptr, ws, wsb, nullptr), KT_EINVAL, "null out");
        expect(kt_render(&cam, &st, nullptr, nullptr, &it, &out.o, nullptr, wsb, nullptr), KT_EINVAL, "null ws");
        expect(kt_render(&cam, &st, nullptr, nullptr, &it, &out.o, static_cast<char*>(ws) + 8, wsb, nullptr),
               KT_EINVAL, "misaligned ws");
        kt_spacetime bad = st;
        bad.a = std::nan("");
        expect(kt_render(&cam, &bad, nullptr, nullptr, &it, &out.o, ws, wsb, nullptr), KT_EINVAL, "nan spin");
        kt_integrator bi = it;
        bi.checkpoint_every = 12;
        expect(kt_render(&cam, &st, nullptr, nullptr, &bi, &out.o, ws, wsb, nullptr), KT_EINVAL, "checkpoint_every");
        kt_camera huge = {1000.0, 1.0, 12.0, 12.0, 65536, 32768};
        if (kt_workspace_bytes(&huge, &it) != 0 || kt_adjoint_workspace_bytes(&huge, &it) != 0) {
            std::fprintf(stderr, "FAIL: workspace bytes of 2^31 rays\n");
            return 1;
        }
        expect(kt_render_batch(0, nullptr, &it, &out.o, ws, wsb, nullptr, nullptr), KT_EINVAL, "empty batch");
        kt_launch best;
        std::memset(&best, 0, sizeof best);
        std::free(ws);
    }
    std::printf("ok %d\n", g_calls);
    return 0;
}
