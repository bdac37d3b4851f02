// stub_launch.cpp -- test-only host stand-ins for the library's kernel
// launchers, so that the host runtime (argument checks, workspace layout,
// parameter packing) runs without a GPU under AddressSanitizer and
// UndefinedBehaviorSanitizer.  The driver hands the library host buffers of
// exactly the sizes it asked for; every stand-in touches all the memory its
// kernel would read or write, so a layout that reaches past a buffer is an
// AddressSanitizer report.
#include <cstdint>
#include <cstdlib>
#include <cstring>

#include "kt_internal.h"

namespace {

volatile unsigned char g_sink;

void write_bytes(void* p, size_t n) {
    if (p && n) std::memset(p, 0x5a, n);
}
void read_bytes(const void* p, size_t n) {
    if (!p || !n) return;
    const unsigned char* c = static_cast<const unsigned char*>(p);
    unsigned char acc = 0;
    for (size_t i = 0; i < n; i += 61) acc ^= c[i];
    acc ^= c[n - 1];
    g_sink = acc;
}

void touch_outputs(const kt::Params& p) {
    const size_t n = static_cast<size_t>(p.n_rays);
    const kt::Outputs& o = p.out;
    write_bytes(o.fate, n);
    for (double* d : {o.r_hit, o.g, o.intensity, o.max_abs_h, o.max_rel_h, o.psi, o.deflection, o.theta_f, o.phi_f})
        write_bytes(d, 8 * n);
    for (uint8_t* b : {o.n_cross, o.used_fp64, o.ring, o.sky}) write_bytes(b, n);
    write_bytes(o.n_steps, 4 * n);
    write_bytes(o.n_evals, 4 * n);
}

}  // namespace

namespace kt {

int launch_ws_init(const Params& p, void*) {
    write_bytes(p.ticket, 4);
    write_bytes(p.fb_count, 4);
    write_bytes(p.acc, 16 * 8);
    std::memcpy(p.ws_params, &p, sizeof p);
    if (p.perm) write_bytes(p.order_hist, 4 * (SORT_BINS + 1));
    return 0;
}

int launch_upload_images(const Image* host, int32_t n, Image* dev, void*) {
    std::memcpy(dev, host, sizeof(Image) * static_cast<size_t>(n));
    return 0;
}

int launch_order(const Params& p, void*) {
    const size_t n = static_cast<size_t>(p.n_rays);
    write_bytes(p.order_hist, 4 * (SORT_BINS + 1));
    write_bytes(p.order_bins, 2 * n);
    write_bytes(p.perm, 4 * n);
    read_bytes(p.images, sizeof(Image) * static_cast<size_t>(p.n_images));
    return 0;
}

int launch_trace(const Params& p, int grid, int block, void*) {
    if (grid < 1 || (block != 64 && block != 128 && block != 256)) return -1;
    const size_t n = static_cast<size_t>(p.n_rays);
    read_bytes(p.ws_params, sizeof(Params));
    read_bytes(p.images, sizeof(Image) * static_cast<size_t>(p.n_images));
    if (p.perm) read_bytes(p.perm, 4 * n);
    write_bytes(p.ticket, 4);
    write_bytes(p.acc, 16 * 8);
    write_bytes(p.rc_buf, 8 * n);
    if (p.precision == KT_MIXED) write_bytes(p.need_fb, n);
    touch_outputs(p);
    return 0;
}

int launch_fallback_list(const Params& p, void*) {
    const size_t n = static_cast<size_t>(p.n_rays);
    read_bytes(p.need_fb, n);
    write_bytes(p.fb_list, 4 * n);
    write_bytes(p.fb_count, 4);
    write_bytes(p.ticket, 4);
    return 0;
}

int launch_trace_fallback(const Params& p, int grid, int block, void* s) {
    read_bytes(p.fb_list, 4 * static_cast<size_t>(p.n_rays));
    return launch_trace(p, grid, block, s);
}

int launch_reset_ticket(const Params& p, void*) {
    write_bytes(p.ticket, 4);
    return 0;
}

int launch_ring(const Params& p, void*) {
    const size_t n = static_cast<size_t>(p.n_rays);
    read_bytes(p.out.deflection, 8 * n);
    write_bytes(p.out.ring, n);
    return 0;
}

int launch_sky(const Params& p, void*) {
    const size_t n = static_cast<size_t>(p.n_rays);
    read_bytes(p.out.theta_f, 8 * n);
    read_bytes(p.out.phi_f, 8 * n);
    write_bytes(p.out.sky, n);
    return 0;
}

int launch_disk_obs(const Params& p, void*) {
    const size_t n = static_cast<size_t>(p.n_rays);
    read_bytes(p.rc_buf, 8 * n);
    read_bytes(p.out.fate, n);
    write_bytes(p.out.r_hit, 8 * n);
    write_bytes(p.out.g, 8 * n);
    write_bytes(p.out.intensity, 8 * n);
    return 0;
}

int launch_stats(const Params& p, void*) {
    read_bytes(p.out.fate, static_cast<size_t>(p.n_rays));
    write_bytes(p.acc, 16 * 8);
    read_bytes(p.fb_count, 4);
    write_bytes(p.out.stats, sizeof(kt_stats));
    return 0;
}

int launch_stamp(const Params& p, int slot, void*) {
    if (slot < 0 || slot >= 16) std::abort();
    write_bytes(p.acc + slot, 8);
    return 0;
}

int launch_init_rays(const Params& p, double* state, uint8_t* invalid, void*) {
    const size_t n = static_cast<size_t>(p.n_rays);
    write_bytes(state, 7 * 8 * n);
    write_bytes(invalid, n);
    return 0;
}

int trace_max_blocks_per_cu(const Params&, int block) { return 512 / block; }

int launch_adjoint(const AdjParams& p, void*) {
    const size_t n = static_cast<size_t>(p.n_rays);
    const size_t lanes = static_cast<size_t>(p.n_lanes);
    write_bytes(p.ticket, 4);
    write_bytes(p.stats, 4 * 8);
    write_bytes(p.hist, 4 * (SORT_BINS + 1));
    write_bytes(p.keys, 2 * n);
    write_bytes(p.list, 4 * n);
    read_bytes(p.fate, n);
    read_bytes(p.cot, 8 * n);
    read_bytes(p.r_hit, 8 * n);
    read_bytes(p.n_steps, 4 * n);
    write_bytes(p.ckpt, static_cast<size_t>(p.max_ckpt) * 6 * lanes * 8);
    write_bytes(p.seg, (size_t{1} << p.ck_shift) * 6 * lanes * 8);
    write_bytes(p.grad_a, 8 * n);
    write_bytes(p.grad_incl, 8 * n);
    write_bytes(p.grad_rin, 8 * n);
    if (p.max_long > 0) {  // split backward sweeps
        write_bytes(p.counters, 3 * 4);
        write_bytes(p.longs, static_cast<size_t>(p.max_long) * sizeof(AdjLong));
        write_bytes(p.owner, 4 * static_cast<size_t>(p.item_cap));
        write_bytes(p.items, 8 * 8 * static_cast<size_t>(p.item_cap));
        write_bytes(p.long_store, 6 * 8 * static_cast<size_t>(p.long_cap));
    }
    if (p.grad_sum) {
        write_bytes(p.partials, 3 * ADJ_RED_BLOCKS * 8);
        write_bytes(p.grad_sum, 3 * 8);
    }
    return 0;
}

}  // namespace kt

// the 3-wave build of the trace kernels touches the same memory
namespace kt_w3 {
int launch_trace(const kt::Params& p, int grid, int block, void* s) { return kt::launch_trace(p, grid, block, s); }
int launch_trace_fallback(const kt::Params& p, int grid, int block, void* s) {
    return kt::launch_trace_fallback(p, grid, block, s);
}
int trace_max_blocks_per_cu(const kt::Params&, int block) { return 768 / block; }
}  // namespace kt_w3
