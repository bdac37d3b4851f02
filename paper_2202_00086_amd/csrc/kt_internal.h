// kt_internal.h -- parameter blocks shared by the host runtime and the kernels.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "kerrtrace.h"
#include "kt_adjoint_math.h"

namespace kt {

constexpr int ACC_EVALS = 0, ACC_EVALS_FP32 = 1;  // acc[8..15]: fate histogram
constexpr int ACC_T0 = 2, ACC_T1 = 3;  // wall clock ticks just before and just after the trace launches

struct Outputs {
    uint8_t* fate;
    double *r_hit, *g, *intensity, *max_abs_h, *max_rel_h, *psi, *deflection, *theta_f, *phi_f;
    uint8_t *n_cross, *used_fp64, *ring;
    int32_t *n_steps, *n_evals;
    uint8_t* sky;
    kt_stats* stats;
};

// Everything that belongs to one image: spacetime, camera constants, disk,
// source, and where its rays sit in the batch.
struct Image {
    // spacetime (eq:Kerr; or the q-metric, metric = KT_METRIC_Q) and the end radii
    double M, a, a2, two_a2;
    int32_t metric;
    double q;
    double r_cap, r_esc;
    // camera and per-image camera constants (Sect. 2.3)
    double r0, incl, fov_x, fov_y, dx, dy;
    double E0;      // 1 / A_t
    double cE;      // g_tphi / (r0 sqrt(g_phph)):  E = E0 + x cE
    double cL;      // -sqrt(g_phph) / r0:          L = x cL
    double cth;     // sqrt(g_thth) / r0:           p_theta = y cth
    double g_rr;    // g_rr at the camera:          p_r = -sqrt(g_rr (1 - (y/r0)^2 - (x/r0)^2))
    int32_t nx, ny;
    int64_t first;  // ray id of pixel 0 (outputs of this image start here)
    // disk (Sect. 5)
    int32_t disk_on, rotation, emis_model;
    double r_in, r_out, emis_q, l0;
    // source for the deflection diagnostics
    int32_t src_on;
    double r_src, src_tol;
    double src_n[3];  // unit vector towards the source
    // celestial sphere at r_esc (Sect. 4.1)
    int32_t sky_on;
    double esc_tol, grid_deg, line_deg;
    // dispatch order: pixels go out by the bin of |rho - rho_ring|, rho the
    // image-plane radius, bin = that distance times order_scale
    double rho_ring, order_scale;
};

// Everything a render needs, copied into the workspace by ws_init.
struct Params {
    // integrator (shared by all images)
    int32_t method, precision;
    double h_fixed, rtol, atol, h_init;
    int64_t max_steps, max_evals;
    double h_budget, r_switch;
    // images: a single render uses a one-entry table (img0)
    int64_t n_rays;
    int32_t n_images;
    const Image* images;  // device table
    Image img0;
    // outputs and workspace
    Outputs out;
    uint32_t* ticket;
    unsigned long long* acc;
    uint32_t* fb_list;
    uint32_t* fb_count;
    double* rc_buf;
    uint8_t* need_fb;   // KT_MIXED: 1 where the ray must be re-run in FP64
    Params* ws_params;  // where ws_init leaves the device copy of this struct
    uint32_t* perm;     // dispatch order: ray id of each slot, or NULL for slot = ray id
    uint32_t* order_hist;  // uint32[SORT_BINS + 1] counts, then offsets and the total
    uint16_t* order_bins;  // uint16[n_rays] bin of each ray
    // launch
    int32_t persistent, batch;
    int32_t from_list;  // take ray ids from fb_list[0 .. *fb_count)
    double wall_khz;    // the device's wall clock rate, kHz (0: unknown)
};

// Bins of the device counting sorts (dispatch order, adjoint work list), and
// the key of an id the sort leaves out.
constexpr int SORT_BINS = 1024;
constexpr uint16_t SORT_SKIP = 0xffff;

// Workspace layout (byte offsets from the start of the caller's buffer).
constexpr size_t WS_TICKET = 0;       // uint32 ray ticket
constexpr size_t WS_ACC = 64;         // uint64[16]
constexpr size_t WS_FB_COUNT = 192;   // uint32 fallback list length
constexpr size_t WS_PARAMS = 256;     // device copy of Params
constexpr size_t WS_PARAMS_MAX = 1792;
static_assert(sizeof(Params) <= WS_PARAMS_MAX, "Params must fit its workspace slot");

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct WsLayout {
    size_t images;   // Image[n_images] (batch renders)
    size_t rc;       // double[n_rays] disk crossing radius per ray
    size_t fb_list;  // uint32[n_rays] (KT_MIXED)
    size_t need;     // uint8[n_rays] (KT_MIXED)
    size_t perm;     // uint32[n_rays] dispatch order
    size_t hist;     // uint32[SORT_BINS + 1]
    size_t bins;     // uint16[n_rays]
    size_t total;
};

inline WsLayout ws_layout(size_t n_rays, size_t n_images, bool batch, bool mixed) {
    WsLayout w;
    w.images = WS_PARAMS + WS_PARAMS_MAX;
    w.rc = align256(w.images + (batch ? n_images * sizeof(Image) : 0));
    w.fb_list = align256(w.rc + 8 * n_rays);
    w.need = align256(w.fb_list + (mixed ? 4 * n_rays : 0));
    w.perm = align256(w.need + (mixed ? n_rays : 0));
    w.hist = align256(w.perm + 4 * n_rays);
    w.bins = align256(w.hist + 4 * (SORT_BINS + 1));
    w.total = align256(w.bins + 2 * n_rays);
    return w;
}

enum : int32_t { FEAT_DISK = 1, FEAT_SRC = 2, FEAT_SKY = 4 };

constexpr int32_t image_features(const Image& im) {
    return (im.disk_on ? FEAT_DISK : 0) | (im.src_on ? FEAT_SRC : 0) | (im.sky_on ? FEAT_SKY : 0);
}

// The values the trace kernel's inner loop reads every step, passed by value
// so they sit in scalar registers; everything else is read through `cold`.
// For batch renders the per-image ones become per-lane values.
struct Hot {
    double M, a, a2, two_a2;
    double rtol, atol, r_cap, r_esc, r_src, r_in, r_out;
    double h_budget, r_switch;  // KT_MIXED
    int32_t feat;               // FEAT_* bits of the image's disk, source and sky
    int32_t max_steps, max_evals;
    const Params* cold;         // the workspace copy of Params
};

// A ray whose backward sweep is split into segments (the first n_long
// entries of the work list).  The forward pass stores every accepted step
// in the split-ray store from `base`, then the cotangents of the state at
// the start of the located partial step.  Segment s covers the steps
// [ADJ_SEG s, ADJ_SEG (s + 1)); its four basis runs are segment items
// item_base + 4 s + b.
enum : int32_t { ADJ_LONG_DONE = 0, ADJ_LONG_SPLIT = 1 };
struct AdjLong {
    int32_t ray, status, n, n_seg;  // n accepted steps before the crossing
    uint32_t base, item_base, pad0, pad1;
    double zb[4];                   // cotangents of (r, theta, p_r, p_theta); that of phi is 0
    double pb[3];                   // of (E, L, a)
    double gr, E, L;                // the r_in gradient (from the seed alone) and the ray constants
};

// Everything the adjoint kernel needs (passed by value).
struct AdjParams {
    Image im;
    double dcam[5][2];  // d(E0, cE, cL, cth, g_rr) / d(a, incl)
    adj::DiskModel dm;
    double rtol, atol, h_init;
    int64_t max_attempts;
    int64_t n_rays;
    const uint8_t* fate;
    const double* r_hit;
    const double* cot;
    double *grad_a, *grad_incl, *grad_rin;  // per pixel: the caller's arrays or the workspace's
    double* grad_sum;           // the three sums (caller's device memory), or NULL
    double* partials;           // [3][ADJ_RED_BLOCKS] block sums of the reduction
    uint32_t* ticket;
    unsigned long long* stats;  // [ok, failed, overflow, mismatch]
    double* ckpt;               // [max_ckpt][6][n_lanes]
    double* seg;                // [1 << ck_shift][6][n_lanes]
    int32_t n_lanes, max_ckpt;
    int32_t ck_shift;           // checkpoints every 1 << ck_shift accepted steps
    // work list: the differentiated rays, longest forward integration first
    const int32_t* n_steps;     // the forward render's step counts (may be NULL)
    uint32_t* hist;             // [SORT_BINS + 1] bin counts, then offsets; [SORT_BINS] = list length
    uint16_t* keys;             // [n_rays] bin of each ray, SORT_SKIP if not differentiated
    uint32_t* list;             // [n_rays] ray ids
    // split backward sweeps (only with n_steps; max_long 0 switches them off)
    int32_t split_above;        // 0: threshold from the work list; > 0: this many steps
    int32_t max_long;           // records in `longs`
    uint32_t long_cap, item_cap;
    uint32_t* counters;         // [0] n_long, [1] store allocation, [2] item allocation
    double* long_store;         // [long_cap][6] every accepted step (state, size) of the split rays
    AdjLong* longs;             // [max_long]
    uint32_t* owner;            // [item_cap] record of each segment item (0xffffffff: none)
    double* items;              // [item_cap][8] one segment's sweep of one basis cotangent
};

#ifndef KT_ADJ_MAX_LANES
#define KT_ADJ_MAX_LANES 65536
#endif
constexpr int ADJ_MAX_LANES = KT_ADJ_MAX_LANES;
constexpr int ADJ_MAX_CKPT = 256;            // checkpoint slots per lane, at least
constexpr int ADJ_MIN_STEPS_COVERED = 2048;  // and at least this many accepted steps covered
constexpr int ADJ_CK_SHIFT_DEFAULT = 6;      // checkpoints every 64 accepted steps
// 0 stores every accepted step (start state and accepted size): the reverse
// sweep then reads each step instead of recomputing it
constexpr int ADJ_CK_SHIFT_MIN = 0, ADJ_CK_SHIFT_MAX = 10;
constexpr int ADJ_RED_BLOCKS = 256;      // fixed grid of the gradient reduction (deterministic)
// Split backward sweeps: segments of ADJ_SEG steps, at most ADJ_SEG_MAX of
// them per ray, at most ADJ_MAX_LONG split rays, and a store of
// ADJ_LONG_STEPS_PER_LANE accepted steps per lane of the grid.
constexpr int ADJ_SEG = 64, ADJ_SEG_MAX = 32;
constexpr int ADJ_MAX_LONG = 8192;
constexpr int ADJ_LONG_STEPS_PER_LANE = 32;
constexpr int ADJ_SPLIT_MIN = 128;        // the automatic threshold is at least this many steps

// log2 of kt_integrator.checkpoint_every (0 selects 64); -1 unless a power
// of two in [1, 1024].
inline int adj_ck_shift(int32_t every) {
    if (every == 0) return ADJ_CK_SHIFT_DEFAULT;
    for (int s = ADJ_CK_SHIFT_MIN; s <= ADJ_CK_SHIFT_MAX; ++s)
        if (every == (1 << s)) return s;
    return -1;
}

struct AdjLayout {
    size_t stats, hist, partials, ckpt, seg, keys, list, grad, longs, owner, items, long_store, total;
    int32_t n_lanes, max_ckpt, max_long;
    uint32_t long_cap, item_cap;
};

// Byte offsets in the first 256 bytes of the adjoint's workspace.
constexpr size_t ADJ_WS_TICKET = 0, ADJ_WS_COUNTERS = 16;

// split: room for split backward sweeps (kt_integrator.split_above >= 0).
inline AdjLayout adj_layout(size_t n_rays, int64_t max_steps, int ck_shift, bool split) {
    AdjLayout w;
    size_t lanes = (n_rays + 255) / 256 * 256;
    if (lanes > static_cast<size_t>(ADJ_MAX_LANES)) lanes = ADJ_MAX_LANES;
    if (lanes < 256) lanes = 256;
    int64_t ck = (max_steps >> ck_shift) + 2;
    const int64_t cap = ADJ_MAX_CKPT > (ADJ_MIN_STEPS_COVERED >> ck_shift) ? ADJ_MAX_CKPT
                                                                         : (ADJ_MIN_STEPS_COVERED >> ck_shift);
    if (ck > cap) ck = cap;
    w.n_lanes = static_cast<int32_t>(lanes);
    w.max_ckpt = static_cast<int32_t>(ck);
    w.stats = 64;
    w.hist = 256;
    w.partials = align256(w.hist + 4u * (SORT_BINS + 1));
    w.ckpt = align256(w.partials + 3u * ADJ_RED_BLOCKS * sizeof(double));
    w.seg = align256(w.ckpt + static_cast<size_t>(ck) * 6u * lanes * sizeof(double));
    w.keys = align256(w.seg + (size_t{1} << ck_shift) * 6u * lanes * sizeof(double));
    w.list = align256(w.keys + 2u * n_rays);
    w.grad = align256(w.list + 4u * n_rays);
    w.max_long = split ? static_cast<int32_t>(n_rays < size_t{ADJ_MAX_LONG} ? n_rays : size_t{ADJ_MAX_LONG}) : 0;
    w.long_cap = split ? static_cast<uint32_t>(lanes * ADJ_LONG_STEPS_PER_LANE) : 0u;
    // every split ray's segments fit: sum over rays of 4 ceil(n / ADJ_SEG)
    // <= 4 (long_cap / ADJ_SEG + max_long), since the rays' stores do not overlap
    w.item_cap = split ? 4u * (w.long_cap / ADJ_SEG + static_cast<uint32_t>(w.max_long)) : 0u;
    w.longs = align256(w.grad + 3u * sizeof(double) * n_rays);
    w.owner = align256(w.longs + static_cast<size_t>(w.max_long) * sizeof(AdjLong));
    w.items = align256(w.owner + 4u * static_cast<size_t>(w.item_cap));
    w.long_store = align256(w.items + 8u * sizeof(double) * w.item_cap);
    w.total = align256(w.long_store + 6u * sizeof(double) * w.long_cap);
    return w;
}

// Leave msg for kt_last_error() on this host thread and return code (kt_api.cpp).
int set_error(int code, const char* msg);

// The argument checks of a single-image render; fills the image's table
// entry.  Returns KT_OK or the error code (message left as for a render).
int validate_single(const kt_camera* camera, const kt_spacetime* spacetime, const kt_disk* disk,
                    const kt_source* source, const kt_integrator* integ, const kt_outputs* out, Image* im);

// Host-side launchers (kt_trace.hip, kt_adjoint.hip).
int launch_adjoint(const AdjParams& p, void* stream);
int launch_ws_init(const Params& p, void* stream);  // also copies p into the workspace
int launch_upload_images(const Image* host, int32_t n, Image* dev, void* stream);
int launch_order(const Params& p, void* stream);  // fills p.perm (ring-first dispatch)
int launch_trace(const Params& p, int grid, int block, void* stream);  // pass of p.precision
int launch_fallback_list(const Params& p, void* stream);  // compact need_fb, switch the copy to from_list
int launch_trace_fallback(const Params& p, int grid, int block, void* stream);  // FP64 re-run from the list
int launch_reset_ticket(const Params& p, void* stream);
int launch_ring(const Params& p, void* stream);
int launch_sky(const Params& p, void* stream);  // needs theta_f and phi_f outputs
int launch_disk_obs(const Params& p, void* stream);
int launch_stats(const Params& p, void* stream);
int launch_stamp(const Params& p, int slot, void* stream);  // acc[slot] = the wall clock now
int launch_init_rays(const Params& p, double* state, uint8_t* invalid, void* stream);
int trace_max_blocks_per_cu(const Params& p, int block);

}  // namespace kt

// The same trace kernels built for 3 waves per SIMD (kt_trace_w3.hip): the
// default for renders of many rays per lane, and for launch shapes of 3 or
// more waves per SIMD.  Their outputs equal the 2-wave kernels' bit for bit.
namespace kt_w3 {
int launch_trace(const kt::Params& p, int grid, int block, void* stream);
int launch_trace_fallback(const kt::Params& p, int grid, int block, void* stream);
int trace_max_blocks_per_cu(const kt::Params& p, int block);
}  // namespace kt_w3
