// kt_trace.hip -- gfx950 kernels of the Kerr backward ray tracer.
//
// trace_kernel<METHOD>: one ray per lane.  Each lane holds its ray's state
// (r, theta, phi, p_r, p_theta), its constants (E, L) and its step control in
// VGPRs and advances one integrator step per loop iteration; all busy lanes
// of a wave evaluate the six (DP45) or four (RK4) right-hand sides together.
// When a ray ends, the lane writes that ray's outputs and takes the next
// slot from its wave's queue, a contiguous range of slots that the wave
// refills in batches from a global atomic ticket (persistent mode).  A slot
// names a ray through the dispatch order (ring first: rays near the photon
// ring, which take the most steps, go out first), through the compacted list
// of the FP64 re-run pass, or directly.  A wave exits once the ticket has
// passed the last slot and all its lanes are idle.
//
// Event location (disk plane, source sphere) reuses the same loop: a lane in
// LOCATE mode takes trial steps of size h' from the step's start state, so
// trial steps run in lockstep with other lanes' ordinary steps.
#include <hip/hip_runtime.h>

#include "kt_device.h"
#include "kt_internal.h"
#include "kt_ray.h"
#include "kt_sort.h"

// The file is compiled twice.  As itself it defines every kernel of the
// render in namespace kt, with the trace kernels built for 2 waves per SIMD.
// kt_trace_w3.hip includes it again with KT_TRACE_ONLY set: only the trace
// kernels and their launchers, in namespace kt_w3, built for 3 waves per SIMD
// and compiled without machine loop-invariant code motion (see there).
#ifndef KT_WAVES_PER_EU
#define KT_WAVES_PER_EU 2
#endif
#ifndef KT_TRACE_NS
#define KT_TRACE_NS kt
#endif
#ifndef KT_TRACE_ONLY
#define KT_TRACE_ONLY 0
#endif

namespace KT_TRACE_NS {
using namespace kt;

// Great-circle angle between the directions (theta1, phi1) and
// (theta2, phi1 + dphi), given sin/cos of the thetas: atan2(|n1 x n2|, n1.n2).
__device__ __forceinline__ double arc_angle(double s1, double c1, double s2, double c2, double dphi) {
    double sd, cd;
    sincos_fast(dphi, &sd, &cd);
    // frame rotated so that phi1 = 0: n1 = (s1, 0, c1), n2 = (s2 cd, s2 sd, c2)
    const double cx = -c1 * s2 * sd;
    const double cy = fma(c1 * s2, cd, -s1 * c2);
    const double cz = s1 * s2 * sd;
    const double cr = sqrt(fma(cx, cx, fma(cy, cy, cz * cz)));
    const double dt = fma(s1 * s2, cd, c1 * c2);
    return atan2_upper(cr, dt);
}

// The same angle for the short arcs of single steps: 2 asin(|n2 - n1| / 2)
// with the small-angle series, where
// |n2 - n1|^2 = (s2 - s1)^2 + (c2 - c1)^2 + 4 s1 s2 sin^2(dphi / 2).
// Returns a negative value when the arc is outside the range of the series
// (|dphi| > 1/2 or chord/2 > 1/16); the caller then takes arc_angle.
__device__ __forceinline__ double arc_angle_short(double s1, double c1, double s2, double c2,
                                                  double dphi) {
    if (!(fabs(dphi) <= 0.5)) return -1.0;
    // sin x, |x| <= 1/4, through x^11 (truncation below 1e-17 relative)
    const double x = 0.5 * dphi, x2 = x * x;
    double p = -1.0 / 39916800.0;
    p = fma(p, x2, 1.0 / 362880.0);
    p = fma(p, x2, -1.0 / 5040.0);
    p = fma(p, x2, 1.0 / 120.0);
    p = fma(p, x2, -1.0 / 6.0);
    const double sh = fma(p * x2, x, x);
    const double ds = s2 - s1, dc = c2 - c1;
    const double q = (4.0 * s1) * s2;
    const double h = 0.5 * sqrt_fast(fma(q * sh, sh, fma(ds, ds, dc * dc)));
    return h <= 0.0625 ? 2.0 * asin_small(h) : -1.0;
}

// Celestial-sphere code of the direction (theta, phi) (Sect. 4.1).  theta is
// folded into [0, pi] (past the polar axis a ray continues on the meridian
// phi + pi) and phi into [0, 2 pi); then the graticule test (distance to the
// nearest multiple of grid_deg in either angle) and the quadrant.
__device__ __forceinline__ uint8_t sky_code(double th, double ph, double grid_deg, double line_deg) {
    constexpr double PI = 3.14159265358979323846, TWO_PI = 6.28318530717958647692;
    constexpr double DEG = 180.0 / PI;
    double t = th - TWO_PI * floor(th * (1.0 / TWO_PI));
    if (t > PI) {
        t = TWO_PI - t;
        ph += PI;
    }
    double p = ph - TWO_PI * floor(ph * (1.0 / TWO_PI));
    if (p >= TWO_PI) p -= TWO_PI;
    if (grid_deg > 0.0) {
        const double td = t * DEG, pd = p * DEG;
        const double dt = fabs(td - grid_deg * rint(td / grid_deg));
        const double dp = fabs(pd - grid_deg * rint(pd / grid_deg));
        if (dt <= line_deg || dp <= line_deg) return KT_SKY_LINE;
    }
    if (t < HALF_PI) return p < PI ? KT_SKY_GREEN : KT_SKY_RED;
    return p < PI ? KT_SKY_BLUE : KT_SKY_YELLOW;
}

// Index of the image that ray id `ray` belongs to (binary search over the
// images' first ray ids).
__device__ __forceinline__ int find_image(const Params& P, int64_t ray) {
    int lo = 0, hi = P.n_images - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P.images[mid].first <= ray)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// The per-image values the step loop needs.  For a single image they come
// from kernel arguments (wave-uniform); for a batch they are loaded per ray.
struct LaneImg {
    Spacetime st;
    double r_cap, r_esc, r_src, r_in, r_out;
    int32_t feat;  // FEAT_* bits
    int32_t k;     // image index
};

__device__ __forceinline__ LaneImg lane_img(const Image& im, int k) {
    LaneImg li;
    li.st = Spacetime{im.M, im.a, im.a2, im.two_a2};
    li.r_cap = im.r_cap;
    li.r_esc = im.r_esc;
    li.r_src = im.r_src;
    li.r_in = im.r_in;
    li.r_out = im.r_out;
    li.feat = image_features(im);
    li.k = k;
    return li;
}

// Lane flags, packed in one int.
enum : int {
    F_VALID = 1 << 0,     // pixel has a real initial p_r
    F_FRESH = 1 << 1,     // k1 = f(y0) not evaluated yet
    F_LOCATE = 1 << 2,    // taking trial steps to locate an event
    F_REJECTED = 1 << 3,  // previous attempt was rejected (no step growth)
    F_RETAKE = 1 << 4,    // re-taking an accepted step after locating an event in it
    F_SKIPDISK = 1 << 5,  // disk crossing of the re-taken step already handled
    F_SRCDONE = 1 << 6,   // source sphere crossed
    F_EVSRC = 1 << 7,     // event being located is the source sphere
    F_USED32 = 1 << 24,   // mixed pass: some step used the FP32 mass part
    F_EVESC = 1 << 25,    // event being located is the celestial sphere
    F_EV32 = 1 << 26,     // mixed pass: the step whose event is being located (and
                          // then retaken) ran with the FP32 mass part
};
constexpr int NCROSS_SHIFT = 8;   // 8 bits: equatorial crossings outside the disk
constexpr int EVIT_SHIFT = 16;    // 8 bits: trial steps of the current event

// Per-lane state that is touched at most once per step lives in LDS,
// laid out [field][thread] so a wave's accesses are consecutive words.
// C_PSI accumulates the swept angle and, once the source sphere is crossed,
// holds the deflection; C_SRCPSI holds the angle to the source.
enum : int {
    C_MAXABS = 0, C_MAXREL, C_LAM, C_PSI, C_SRCPSI, C_CS, C_CC, C_EVA, C_EVFA, C_EVB, C_EVFB, C_EVC,
    N_COLD
};
constexpr int BLOCK_MAX = 256;

template <int METHOD, class ST>
__device__ __forceinline__ void take_step(const ST& st, const RayConst& rc, const double y[5],
                                          const double k1[5], double s0, double c0, double h, double yn[5],
                                          double kn[5], double er[5], Diag* dg) {
    if constexpr (METHOD == KT_DP45) {
        dp45_step(st, rc, y, k1, s0, c0, h, yn, kn, er, dg);
    } else if constexpr (METHOD == KT_RKF45) {
        erk6_step<Fehlberg45>(st, rc, y, k1, s0, c0, h, yn, kn, er, dg);
    } else if constexpr (METHOD == KT_CK45) {
        erk6_step<CashKarp45>(st, rc, y, k1, s0, c0, h, yn, kn, er, dg);
    } else if constexpr (METHOD == KT_BS) {
        bs_step<false>(st, rc, y, k1, h, yn, kn, er, dg);
    } else if constexpr (METHOD == KT_BS_RAT) {
        bs_step<true>(st, rc, y, k1, h, yn, kn, er, dg);
    } else {
        rk4s_step(st, rc, y, k1, h, yn, kn, dg);
#pragma unroll
        for (int i = 0; i < 5; ++i) er[i] = 0.0;
    }
}

// FEAT >= 0 fixes the image's features (FEAT_* bits) at compile time, so the
// event tests of absent features vanish from the step loop; FEAT_DYN reads
// them from the launch (single images) or the lane's image (batches).
constexpr int FEAT_DYN = -1;

template <int METHOD, int PREC, bool BATCH, bool QMET = false, int FEAT = FEAT_DYN>
__global__ void __launch_bounds__(BLOCK_MAX) __attribute__((amdgpu_waves_per_eu(KT_WAVES_PER_EU)))
trace_kernel(const Hot hp) {
    static_assert(!(QMET && (BATCH || METHOD == KT_RK4_S || PREC != KT_FP64)),
                  "the q-metric runs single images with the adaptive FP64 schemes");
    static_assert(FEAT == FEAT_DYN || !BATCH, "batches read each image's features");
    constexpr int EVALS_PER_STEP = evals_per_step<METHOD>();
    constexpr bool ADAPTIVE = (METHOD != KT_RK4_S);
    constexpr bool S_TIME = (METHOD == KT_RK4_S);
    constexpr bool MIXED = (PREC == KT_MIXED) && (METHOD == KT_DP45) && !QMET;
    __shared__ double cold[N_COLD][BLOCK_MAX];
    const int tid = threadIdx.x;
#define COLD(f) cold[f][tid]
    // cold parameters are read from the workspace copy where needed
    const Params& P = *hp.cold;

    LaneImg li;
    li.st = Spacetime{hp.M, hp.a, hp.a2, hp.two_a2};
    li.r_cap = hp.r_cap;
    li.r_esc = hp.r_esc;
    li.r_src = hp.r_src;
    li.r_in = hp.r_in;
    li.r_out = hp.r_out;
    li.feat = hp.feat;
    li.k = 0;
    const uint32_t lane = __lane_id();
    const uint32_t n_total = P.from_list ? *P.fb_count : static_cast<uint32_t>(P.n_rays);

    // this wave's queue of ray ids [q_next, q_end).  A persistent wave's
    // first fetch takes 64 ids, one per lane, in one atomic; later fetches
    // take P.batch.  Taken in batch-sized pieces, the start of the launch was
    // a burst of 64 / batch serial round trips per wave on one address, and
    // the wave's first rays came from interleaved places in the dispatch
    // order instead of one run of similar cost.
    uint32_t q_next, q_end;
    bool exhausted;
    bool first_fetch = P.persistent != 0;
    if (P.persistent) {
        q_next = q_end = 0;
        exhausted = false;
    } else {
        const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
        q_next = min(wave * 64u, n_total);
        q_end = min(q_next + 64u, n_total);
        exhausted = true;
    }

    int32_t ray = -1;
    int fl = 0;
    double y[5], k1[5];
    double E = 0.0, L = 0.0, h = 0.0;
    int nsteps = 0, nevals = 0;
    unsigned long long evals_acc = 0, evals32_acc = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) y[i] = k1[i] = 0.0;

#if KT_WAVES_PER_EU == 3
    // With three waves per SIMD the issue arbiter's preference for the
    // oldest wave runs the three generations of blocks at very different
    // speeds, and the rays a slow wave holds end the launch late.  Each wave
    // steps its priority down from 3 to 0 and round again, one level per
    // loop iteration; the waves' cycles are out of phase, so the highest
    // priority moves from wave to wave and their shares of the issue slots
    // even out.
    uint32_t prio_it = 0;
#endif
    for (;;) {
#if KT_WAVES_PER_EU == 3
        switch (prio_it & 3u) {
            case 0: __builtin_amdgcn_s_setprio(3); break;
            case 1: __builtin_amdgcn_s_setprio(2); break;
            case 2: __builtin_amdgcn_s_setprio(1); break;
            default: __builtin_amdgcn_s_setprio(0); break;
        }
        ++prio_it;
#endif
        // ---- refill idle lanes from the wave queue -------------------------
        unsigned long long idle = __ballot(ray < 0);
        while (idle != 0ull) {
            if (q_next >= q_end) {
                if (exhausted) break;
                const int leader = __ffsll(idle) - 1;
                uint32_t base = 0;
                const uint32_t take = first_fetch ? 64u : static_cast<uint32_t>(P.batch);
                first_fetch = false;
                if (static_cast<int>(lane) == leader) base = atomicAdd(P.ticket, take);
                base = static_cast<uint32_t>(__shfl(static_cast<int>(base), leader));
                if (base >= n_total) {
                    exhausted = true;
                    break;
                }
                q_next = base;
                q_end = min(base + take, n_total);
            }
            const uint32_t rank = static_cast<uint32_t>(__popcll(idle & ((1ull << lane) - 1ull)));
            const uint32_t avail = q_end - q_next;
            if (ray < 0 && rank < avail) {
                const uint32_t slot = q_next + rank;
                ray = P.from_list ? static_cast<int32_t>(P.fb_list[slot])
                      : P.perm    ? static_cast<int32_t>(P.perm[slot])
                                  : static_cast<int32_t>(slot);
                if constexpr (BATCH) {
                    const int k = find_image(P, ray);
                    const Image& im = P.images[k];
                    li = lane_img(im, k);
                    fl = camera_state(im, ray - static_cast<int32_t>(im.first), y, &E, &L) ? (F_VALID | F_FRESH) : 0;
                } else {
                    fl = camera_state(P.img0, ray, y, &E, &L) ? (F_VALID | F_FRESH) : 0;
                }
                h = ADAPTIVE ? P.h_init : P.h_fixed;
                nsteps = 0;
                nevals = 0;
            }
            q_next += min(static_cast<uint32_t>(__popcll(idle)), avail);
            idle = __ballot(ray < 0);
        }
        if (__ballot(ray >= 0) == 0ull) break;
        if (ray < 0) continue;

        // ---- one step per busy lane ----------------------------------------
        // the q-metric carries (q, q(2+q)) in the spacetime's (a, a^2) slots
        const auto st = [&]() {
            if constexpr (QMET)
                return QSpacetime{li.st.M, li.st.a, li.st.a2};
            else
                return li.st;
        }();
        const RayConst rc = make_ray_const(st, E, L);
        const double NaN = __builtin_nan("");
        int fate = -1;  // >= 0 once the ray ends
        double thf = y[1], phf = y[2], r_c = NaN, psi = NaN, defl = NaN;

        if (!(fl & F_VALID)) {
            fate = KT_FATE_INVALID;
            COLD(C_MAXABS) = NaN;
            COLD(C_MAXREL) = NaN;
        } else if (fl & F_FRESH) {
            // first evaluation: k1 = f(y0) (FSAL seed) and H at lambda = 0
            Diag dg;
            rhs<true, S_TIME>(st, rc, y, k1, &dg);
            nevals = 1;
            COLD(C_MAXABS) = fabs(dg.H);
            COLD(C_MAXREL) = dg.rel();
            COLD(C_LAM) = 0.0;
            COLD(C_PSI) = 0.0;
            COLD(C_CS) = dg.s;
            COLD(C_CC) = dg.c;
            fl &= ~F_FRESH;
        } else if (!(fl & (F_LOCATE | F_RETAKE)) && (nsteps >= hp.max_steps || nevals >= hp.max_evals)) {
            fate = KT_FATE_MAXSTEPS;
        } else {
            const bool locating = (fl & F_LOCATE) != 0;
            bool use32 = false;
            if constexpr (MIXED) {
                // The FP32 mass part runs wave-uniformly.  A lane locating an
                // event, or retaking the step it lay in, must use the
                // precision of that accepted step (its trial steps are steps
                // of the same stepper, and the retake must reproduce the
                // step bit for bit).  The lowest such lane sets the wave's
                // precision and lanes that cannot use it sit this pass out;
                // with no such lane the FP32 part runs when every stepping
                // lane is beyond r_switch.
                const bool pinned = (fl & (F_LOCATE | F_RETAKE)) != 0;
                const bool ev32 = (fl & F_EV32) != 0;
                const unsigned long long pin = __ballot(pinned);
                if (pin != 0ull) {
                    const int lead = __ffsll(pin) - 1;
                    use32 = ((__ballot(pinned && ev32) >> lead) & 1ull) != 0ull;
                } else {
                    use32 = __all(y[0] >= hp.r_switch);
                }
                const bool fits = pinned ? (ev32 == use32) : (!use32 || y[0] >= hp.r_switch);
                if (!fits) continue;
            }
            const double hs = locating ? COLD(C_EVC) : h;
            double yn[5], kn[5], er[5];
            Diag dg;
            // sin/cos of theta at the step start (from the last evaluation there)
            const double s0 = COLD(C_CS), c0 = COLD(C_CC);
            if constexpr (MIXED) {
                const Spacetime32 sf{static_cast<float>(st.M), static_cast<float>(st.a), static_cast<float>(st.a2)};
                if (use32) {
                    dp45_step<true>(st, rc, y, k1, s0, c0, hs, yn, kn, er, &dg, &sf);
                    fl |= F_USED32;
                    evals32_acc += EVALS_PER_STEP;
                } else {
                    dp45_step<false>(st, rc, y, k1, s0, c0, hs, yn, kn, er, &dg);
                }
            } else {
                take_step<METHOD>(st, rc, y, k1, s0, c0, hs, yn, kn, er, &dg);
            }
            nevals += EVALS_PER_STEP;
            if (locating) {
                // Illinois regula falsi on the event function
                const bool src = (fl & F_EVSRC) != 0;
                const bool esc = (fl & F_EVESC) != 0;
                const Image& im = BATCH ? P.images[li.k] : P.img0;
                const double fc = esc ? yn[0] - li.r_esc : src ? yn[0] - li.r_src : yn[1] - HALF_PI;
                const double tol = esc ? im.esc_tol : src ? im.src_tol : 1e-14;
                const int it = ((fl >> EVIT_SHIFT) & 0xff) + 1;
                fl = (fl & ~(0xff << EVIT_SHIFT)) | (it << EVIT_SHIFT);
                if ((fabs(fc) <= tol || it >= 64) && esc) {
                    // the ray meets the celestial sphere here
                    fate = KT_FATE_ESCAPED;
                    thf = yn[1];
                    phf = yn[2];
                } else if (fabs(fc) <= tol || it >= 64) {
                    if (!src) {
                        if (yn[0] >= li.r_in && yn[0] <= li.r_out) {
                            fate = KT_FATE_DISK;
                            r_c = yn[0];
                            thf = yn[1];
                            phf = yn[2];
                        } else {
                            const int nc = min(((fl >> NCROSS_SHIFT) & 0xff) + 1, 255);
                            fl = (fl & ~(0xff << NCROSS_SHIFT)) | (nc << NCROSS_SHIFT) | F_SKIPDISK;
                        }
                    } else {
                        defl = COLD(C_PSI) + arc_angle(s0, c0, dg.s, dg.c, yn[2] - y[2]);
                        double sp, cp;
                        sincos_fast(yn[2], &sp, &cp);
                        const double* sn = im.src_n;
                        const double nx = dg.s * cp, ny = dg.s * sp, nz = dg.c;
                        const double cx = ny * sn[2] - nz * sn[1];
                        const double cy = nz * sn[0] - nx * sn[2];
                        const double cz = nx * sn[1] - ny * sn[0];
                        psi = atan2_upper(sqrt(fma(cx, cx, fma(cy, cy, cz * cz))),
                                          fma(nx, sn[0], fma(ny, sn[1], nz * sn[2])));
                        COLD(C_PSI) = defl;  // parked until the ray ends
                        COLD(C_SRCPSI) = psi;
                        fl |= F_SRCDONE;
                    }
                    // continue from the end of the accepted step: retake it (bit-identical)
                    fl = (fl & ~F_LOCATE) | F_RETAKE;
                } else {
                    double a = COLD(C_EVA), fa = COLD(C_EVFA), b = COLD(C_EVB), fb = COLD(C_EVFB);
                    if (fc * fb < 0.0) {
                        a = b;
                        fa = fb;
                    } else {
                        fa *= 0.5;
                    }
                    b = COLD(C_EVC);
                    fb = fc;
                    COLD(C_EVA) = a;
                    COLD(C_EVFA) = fa;
                    COLD(C_EVB) = b;
                    COLD(C_EVFB) = fb;
                    COLD(C_EVC) = b - fb * (b - a) / (fb - fa);
                }
            } else {
                bool finite = true;
#pragma unroll
                for (int i = 0; i < 5; ++i) finite = finite && isfinite(yn[i]);
                double h_next = h;
                bool accept = true;
                if (!finite) {
                    fate = KT_FATE_STEPFAIL;
                    accept = false;
                } else if constexpr (ADAPTIVE) {
                    // mean square of err_i / (atol + rtol max(|y_i|, |yn_i|))
                    double sc[5];
#pragma unroll
                    for (int i = 0; i < 5; ++i) sc[i] = fma(hp.rtol, fmax(fabs(y[i]), fabs(yn[i])), hp.atol);
                    const double msq = error_msq<fp64_control<METHOD>()>(er, sc);
                    if (isnan(msq)) {
                        fate = KT_FATE_STEPFAIL;
                        accept = false;
                    } else if (msq > 1.0) {
                        h *= reject_factor<METHOD>(msq);
                        fl |= F_REJECTED;
                        accept = false;
                        if (h < 1e-12 * fmax(1.0, fabs(COLD(C_LAM)))) fate = KT_FATE_STEPFAIL;
                    } else {
                        double fac = accept_factor<METHOD>(msq);
                        if (fl & F_REJECTED) fac = fmin(fac, 1.0);
                        h_next = h * fac;
                    }
                }
                if (accept) {
                    if (!(fl & F_RETAKE)) {
                        ++nsteps;
                        COLD(C_MAXABS) = fmax(COLD(C_MAXABS), fabs(dg.H));
                        // |H|_rel = Kabs / D: the quotient is taken only when
                        // it raises the running maximum (Kabs > max D)
                        const double mr = COLD(C_MAXREL);
                        if (dg.Kabs > mr * dg.D) COLD(C_MAXREL) = dg.rel();
                    }
                    fl &= ~F_RETAKE;
                    bool locate = false;
                    // thin disk: sign change of theta - pi/2 over the step
                    const int32_t feat = FEAT >= 0 ? FEAT : li.feat;
                    if ((feat & FEAT_DISK) && !(fl & F_SKIPDISK)) {
                        const double ga = y[1] - HALF_PI, gb = yn[1] - HALF_PI;
                        if (ga * gb < 0.0) {
                            fl = (fl & ~(F_EVSRC | F_EV32 | (0xff << EVIT_SHIFT))) | F_LOCATE | (use32 ? F_EV32 : 0);
                            COLD(C_EVA) = 0.0;
                            COLD(C_EVFA) = ga;
                            COLD(C_EVB) = h;
                            COLD(C_EVFB) = gb;
                            COLD(C_EVC) = h - gb * h / (gb - ga);
                            locate = true;
                        } else if (gb == 0.0) {
                            if (yn[0] >= li.r_in && yn[0] <= li.r_out) {
                                fate = KT_FATE_DISK;
                                r_c = yn[0];
                                thf = yn[1];
                                phf = yn[2];
                            } else {
                                const int nc = min(((fl >> NCROSS_SHIFT) & 0xff) + 1, 255);
                                fl = (fl & ~(0xff << NCROSS_SHIFT)) | (nc << NCROSS_SHIFT);
                            }
                        }
                    }
                    if (!locate && fate < 0) {
                        if (yn[0] < li.r_cap) {
                            fate = KT_FATE_CAPTURED;
                            thf = yn[1];
                            phf = yn[2];
                        } else {
                            if ((feat & FEAT_SRC) && !(fl & F_SRCDONE)) {
                                if (y[0] < li.r_src && yn[0] >= li.r_src) {
                                    const double fa = y[0] - li.r_src, fb = yn[0] - li.r_src;
                                    fl = (fl & ~(F_EV32 | (0xff << EVIT_SHIFT))) | F_EVSRC | F_LOCATE | (use32 ? F_EV32 : 0);
                                    COLD(C_EVA) = 0.0;
                                    COLD(C_EVFA) = fa;
                                    COLD(C_EVB) = h;
                                    COLD(C_EVFB) = fb;
                                    COLD(C_EVC) = h - fb * h / (fb - fa);
                                    locate = true;
                                } else {
                                    const double dphi = yn[2] - y[2];
                                    double arc = arc_angle_short(s0, c0, dg.s, dg.c, dphi);
                                    if (arc < 0.0) arc = arc_angle(s0, c0, dg.s, dg.c, dphi);
                                    COLD(C_PSI) += arc;
                                }
                            }
                            if (!locate) {
                                if (yn[0] > li.r_esc && (feat & FEAT_SKY)) {
                                    // locate the crossing of the celestial sphere
                                    const double fa = y[0] - li.r_esc, fb = yn[0] - li.r_esc;
                                    fl = (fl & ~(F_EVSRC | F_EV32 | (0xff << EVIT_SHIFT))) | F_EVESC | F_LOCATE | (use32 ? F_EV32 : 0);
                                    COLD(C_EVA) = 0.0;
                                    COLD(C_EVFA) = fa;
                                    COLD(C_EVB) = h;
                                    COLD(C_EVFB) = fb;
                                    COLD(C_EVC) = h - fb * h / (fb - fa);
                                } else if (yn[0] > li.r_esc) {
                                    fate = KT_FATE_ESCAPED;
                                    thf = yn[1];
                                    phf = yn[2];
                                } else {
                                    // commit the step
#pragma unroll
                                    for (int i = 0; i < 5; ++i) {
                                        y[i] = yn[i];
                                        k1[i] = kn[i];
                                    }
                                    COLD(C_LAM) += h;
                                    h = h_next;
                                    fl &= ~(F_REJECTED | F_SKIPDISK);
                                    COLD(C_CS) = dg.s;
                                    COLD(C_CC) = dg.c;
                                }
                            }
                        }
                    }
                }
            }
        }

        if (fate >= 0) {
            const Outputs& o = P.out;
            if (fl & F_SRCDONE) {
                defl = COLD(C_PSI);
                psi = COLD(C_SRCPSI);
            }
            o.fate[ray] = static_cast<uint8_t>(fate);
            P.rc_buf[ray] = r_c;
            if (o.max_abs_h) o.max_abs_h[ray] = COLD(C_MAXABS);
            if (o.max_rel_h) o.max_rel_h[ray] = COLD(C_MAXREL);
            if (o.psi) o.psi[ray] = psi;
            if (o.deflection) o.deflection[ray] = defl;
            if (o.theta_f) o.theta_f[ray] = thf;
            if (o.phi_f) o.phi_f[ray] = phf;
            if (o.n_cross) o.n_cross[ray] = static_cast<uint8_t>((fl >> NCROSS_SHIFT) & 0xff);
            if (o.used_fp64) o.used_fp64[ray] = static_cast<uint8_t>(P.from_list ? 1 : 0);
            if (o.n_steps) o.n_steps[ray] = nsteps;
            if (o.n_evals) o.n_evals[ray] = nevals;
            if constexpr (MIXED) {
                const double mr = COLD(C_MAXREL);
                P.need_fb[ray] = ((fl & F_USED32) && !(mr <= hp.h_budget)) ? 1 : 0;
            }
            evals_acc += static_cast<unsigned long long>(nevals);
            ray = -1;
        }
    }
#undef COLD

    // one atomic per wave for each evaluation counter
    for (int off = 32; off > 0; off >>= 1) evals_acc += __shfl_down(evals_acc, off);
    if (lane == 0 && evals_acc != 0ull) atomicAdd(P.acc + ACC_EVALS, evals_acc);
    if constexpr (MIXED) {
        for (int off = 32; off > 0; off >>= 1) evals32_acc += __shfl_down(evals32_acc, off);
        if (lane == 0 && evals32_acc != 0ull) atomicAdd(P.acc + ACC_EVALS_FP32, evals32_acc);
    }
}

#if !KT_TRACE_ONLY
// Compact the re-run flags into the fallback list (order does not matter:
// every ray is independent) and count them.
__global__ void fallback_list_kernel(const uint8_t* __restrict__ need, int64_t n, uint32_t* __restrict__ list,
                                     uint32_t* count) {
    __shared__ uint32_t block_base;
    __shared__ uint32_t wave_counts[BLOCK_MAX / 64];
    const int tid = threadIdx.x, wave = tid >> 6;
    const uint32_t lane = __lane_id();
    for (int64_t base = static_cast<int64_t>(blockIdx.x) * blockDim.x; base < n;
         base += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t k = base + tid;
        const bool want = k < n && need[k];
        const unsigned long long m = __ballot(want);
        const uint32_t rank = static_cast<uint32_t>(__popcll(m & ((1ull << lane) - 1ull)));
        if (lane == 0) wave_counts[wave] = static_cast<uint32_t>(__popcll(m));
        __syncthreads();
        if (tid == 0) {
            uint32_t tot = 0;
            for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) {
                const uint32_t c = wave_counts[w];
                wave_counts[w] = tot;
                tot += c;
            }
            block_base = tot ? atomicAdd(count, tot) : 0u;
        }
        __syncthreads();
        if (want) list[block_base + wave_counts[wave] + rank] = static_cast<uint32_t>(k);
        __syncthreads();
    }
}

// Switch the workspace copy of the parameters to the list-driven FP64 pass.
__global__ void to_fallback_kernel(Params* wp) {
    if (threadIdx.x == 0) {
        *wp->ticket = 0u;
        wp->from_list = 1;
        wp->precision = KT_FP64;
    }
}

// Redshift and observed intensity of every disk pixel from the crossing
// radius the trace kernel parked in rc_buf (eq:redshift read as
// g = 1 / (u^t (E - Omega L)); I_obs = g^3 I_em with I_em = (M/r)^q).
// Omega is Keplerian or from the constant specific angular momentum l0.
__global__ void disk_obs_kernel(const Params* pp) {
    const Params& p = *pp;
    const int64_t n = p.n_rays;
    const double NaN = __builtin_nan("");
    for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < n;
         k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double r_hit = NaN, g = NaN, inten = 0.0;
        if (p.out.fate[k] == KT_FATE_DISK) {
            const Image& im = p.images[find_image(p, k)];
            double z[5], E, L;
            camera_state(im, static_cast<int32_t>(k - im.first), z, &E, &L);
            const double rc = p.rc_buf[k];
            const double inv_rc = 1.0 / rc;
            const double gtt = -(1.0 - 2.0 * im.M * inv_rc);
            const double gtp = -2.0 * im.M * im.a * inv_rc;
            const double gpp = rc * rc + im.a2 + 2.0 * im.M * im.a2 * inv_rc;
            double Om;
            if (im.rotation == KT_ROT_L0) {
                Om = -(gtp + im.l0 * gtt) / (gpp + im.l0 * gtp);
            } else {
                const double sM = sqrt(im.M);
                Om = sM / fma(rc, sqrt(rc), im.a * sM);
            }
            const double norm = -gtt - 2.0 * Om * gtp - Om * Om * gpp;  // (u^t)^-2
            r_hit = rc;
            if (norm > 0.0) {
                g = sqrt(norm) / (E - Om * L);
                double em;
                if (im.emis_model == KT_EMIS_TAPERED) {
                    const double mr = im.M * inv_rc;
                    em = mr * mr * (1.0 - sqrt(im.r_in * inv_rc));
                    const double sv = (im.r_out - rc) / (2.0 * im.M);
                    if (sv < 1.0) em *= sv * sv * (3.0 - 2.0 * sv);
                } else {
                    em = pow(im.M * inv_rc, im.emis_q);
                }
                inten = g * g * g * em;
            }
        }
        if (p.out.r_hit) p.out.r_hit[k] = r_hit;
        if (p.out.g) p.out.g[k] = g;
        if (p.out.intensity) p.out.intensity[k] = inten;
    }
}

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------

__global__ void ws_init_kernel(const Params p) {
    const int t = threadIdx.x;
    if (t == 0) {
        *p.ticket = 0u;
        *p.fb_count = 0u;
        *p.ws_params = p;
    }
    if (t < 16) p.acc[t] = 0ull;
    if (p.perm)
        for (int b = t; b <= SORT_BINS; b += blockDim.x) p.order_hist[b] = 0u;
}

// ---- dispatch order ------------------------------------------------------
// Rays near the photon ring take the most steps; the persistent waves finish
// soonest when those go out first and the cheap rays fill the tail.  The
// slots are sorted by the bin of |rho - rho_ring| (a counting sort over
// SORT_BINS bins).  Every ray's arithmetic is independent of the lane and
// wave that runs it, so outputs do not change.
#ifndef KT_ORDER_GROUP_SHIFT
#define KT_ORDER_GROUP_SHIFT 5
#endif
// Rays go out in groups of consecutive ids (keyed by the group's first
// ray), so the outputs of neighbouring pixels, which share cache lines, are
// written close together in time and merge in L2 instead of reaching HBM as
// many partial-line writes.
constexpr int64_t ORDER_GROUP_MASK = (int64_t{1} << KT_ORDER_GROUP_SHIFT) - 1;

struct RingKey {
    const Params* p;  // the workspace copy
    __device__ int operator()(int64_t ray) const {
        const Params& P = *p;
        ray &= ~ORDER_GROUP_MASK;
        const Image* im = P.images;
        int64_t pix = ray;
        if (P.n_images > 1) {
            im = &P.images[find_image(P, ray)];
            pix = ray - im->first;
        }
        const int32_t j = static_cast<int32_t>(pix / im->nx);
        const int32_t i = static_cast<int32_t>(pix - static_cast<int64_t>(j) * im->nx);
        const double x = -im->fov_x + (static_cast<double>(i) + 0.5) * im->dx;
        const double y = -im->fov_y + (static_cast<double>(j) + 0.5) * im->dy;
        const double d = fabs(sqrt(fma(x, x, y * y)) - im->rho_ring) * im->order_scale;
        return d < static_cast<double>(SORT_BINS - 1) ? static_cast<int>(d) : SORT_BINS - 1;
    }
};

// Copy a chunk of the image table into device memory (the table travels in
// kernel arguments, so nothing on the host has to outlive the call).
constexpr int UPLOAD_CHUNK = 12;
struct ImageChunk {
    Image im[UPLOAD_CHUNK];
    int32_t n, base;
};
static_assert(sizeof(ImageChunk) <= 3900, "image chunk must fit the kernel-argument limit");

__global__ void upload_images_kernel(const ImageChunk c, Image* dev) {
    const int t = threadIdx.x;
    if (t < c.n) dev[c.base + t] = c.im[t];
}

__global__ void reset_ticket_kernel(uint32_t* ticket) {
    if (threadIdx.x == 0) *ticket = 0u;
}

// Odd multiples of pi that are <= v.
__device__ __forceinline__ double odd_pi_count(double v) {
    constexpr double PI = 3.14159265358979323846;
    return floor((v + PI) / (2.0 * PI));
}

// Ring flags, within each image: an odd multiple of pi between a pixel's
// deflection and its +i or +j neighbour's.
__global__ void ring_kernel(const Params* pp) {
    const Params& P = *pp;
    const double* __restrict__ defl = P.out.deflection;
    uint8_t* __restrict__ ring = P.out.ring;
    const int64_t n = P.n_rays;
    for (int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; p < n;
         p += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const Image& im = P.images[find_image(P, p)];
        const int64_t pix = p - im.first;
        const int32_t nx = im.nx;
        const int32_t j = static_cast<int32_t>(pix / nx);
        const int32_t i = static_cast<int32_t>(pix - static_cast<int64_t>(j) * nx);
        const double d = defl[p];
        uint8_t flag = 0;
        if (isfinite(d)) {
            const double k = odd_pi_count(d);
            if (i + 1 < nx && isfinite(defl[p + 1]) && odd_pi_count(defl[p + 1]) != k) flag = 1;
            if (j + 1 < im.ny && isfinite(defl[p + nx]) && odd_pi_count(defl[p + nx]) != k) flag = 1;
        }
        ring[p] = flag;
    }
}

// Celestial-sphere codes from the located crossings (theta_f, phi_f).
__global__ void sky_kernel(const Params* pp) {
    const Params& P = *pp;
    const int64_t n = P.n_rays;
    for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < n;
         k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        uint8_t code = KT_SKY_NONE;
        if (P.out.fate[k] == KT_FATE_ESCAPED) {
            const Image& im = P.images[find_image(P, k)];
            if (im.sky_on) code = sky_code(P.out.theta_f[k], P.out.phi_f[k], im.grid_deg, im.line_deg);
        }
        P.out.sky[k] = code;
    }
}

// Fate histogram into acc[8..15].
__global__ void fate_hist_kernel(const uint8_t* __restrict__ fate, int64_t n, unsigned long long* acc) {
    // per-lane counts, summed over the wave with shuffles: most fates are
    // equal, so atomics per element would serialise on one LDS word
    __shared__ unsigned int hist[8];
    if (threadIdx.x < 8) hist[threadIdx.x] = 0u;
    __syncthreads();
    unsigned int c[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    for (int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; p < n;
         p += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int f = fate[p] & 7;
#pragma unroll
        for (int k = 0; k < 8; ++k) c[k] += f == k ? 1u : 0u;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        unsigned int v = c[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += static_cast<unsigned int>(__shfl_xor(static_cast<int>(v), off));
        if (__lane_id() == 0 && v) atomicAdd(&hist[k], v);
    }
    __syncthreads();
    if (threadIdx.x < 8 && hist[threadIdx.x]) atomicAdd(acc + 8 + threadIdx.x, static_cast<unsigned long long>(hist[threadIdx.x]));
}

// One reading of the GPU's constant-rate wall clock into acc[slot].  Enqueued
// just before the first trace launch and just after the last one when a
// render asks for statistics, so the trace kernels themselves carry no timing
// code.
__global__ void stamp_kernel(unsigned long long* acc, int slot) {
    if (threadIdx.x == 0) acc[slot] = static_cast<unsigned long long>(wall_clock64());
}

__global__ void stats_kernel(const unsigned long long* acc, const uint32_t* fb_count, int64_t n_rays,
                             double wall_khz, kt_stats* out) {
    if (threadIdx.x == 0) {
        out->rays = static_cast<uint64_t>(n_rays);
        out->evals = acc[ACC_EVALS];
        out->evals_fp32 = acc[ACC_EVALS_FP32];
        out->fallback_rays = *fb_count;
        for (int k = 0; k < 8; ++k) out->fate_count[k] = acc[8 + k];
        const unsigned long long t0 = acc[ACC_T0], t1 = acc[ACC_T1];
        out->trace_ms = (wall_khz > 0.0 && t1 > t0) ? static_cast<double>(t1 - t0) / wall_khz : 0.0;
    }
}

__global__ void init_rays_kernel(const Image im, int64_t n, double* state, uint8_t* invalid) {
    for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < n;
         k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double z[5], E, L;
        const bool ok = camera_state(im, static_cast<int32_t>(k), z, &E, &L);
        for (int c = 0; c < 5; ++c) state[c * n + k] = z[c];
        state[5 * n + k] = E;
        state[6 * n + k] = L;
        invalid[k] = ok ? 0 : 1;
    }
}

#endif  // !KT_TRACE_ONLY

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

static int check_launch() { return hipGetLastError() == hipSuccess ? 0 : -1; }

#if !KT_TRACE_ONLY
static int small_grid(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 4096) g = 4096;
    return g < 1 ? 1 : static_cast<int>(g);
}

int launch_ws_init(const Params& p, void* stream) {
    hipLaunchKernelGGL(ws_init_kernel, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), p);
    return check_launch();
}

int launch_order(const Params& p, void* stream) {
    const SortBufs b{p.n_rays, p.order_hist, p.order_bins, p.perm};
    return launch_sort(b, RingKey{p.ws_params}, static_cast<hipStream_t>(stream));
}

int launch_reset_ticket(const Params& p, void* stream) {
    hipLaunchKernelGGL(reset_ticket_kernel, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream),
                       p.ticket);
    return check_launch();
}

int launch_upload_images(const Image* host, int32_t n, Image* dev, void* stream) {
    for (int32_t base = 0; base < n; base += UPLOAD_CHUNK) {
        ImageChunk c;
        c.n = n - base < UPLOAD_CHUNK ? n - base : UPLOAD_CHUNK;
        c.base = base;
        for (int t = 0; t < c.n; ++t) c.im[t] = host[base + t];
        hipLaunchKernelGGL(upload_images_kernel, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), c, dev);
        if (check_launch()) return -1;
    }
    return 0;
}

#endif  // !KT_TRACE_ONLY

static Hot make_hot(const Params& p) {
    const Image& im = p.img0;  // batch renders take the per-image values from the table
    Hot hp;
    hp.M = im.M;
    hp.a = im.a;
    hp.a2 = im.a2;
    hp.two_a2 = im.two_a2;
    if (im.metric == KT_METRIC_Q) {
        hp.a = im.q;
        hp.a2 = im.q * (2.0 + im.q);
        hp.two_a2 = 0.0;
    }
    hp.rtol = p.rtol;
    hp.atol = p.atol;
    hp.r_cap = im.r_cap;
    hp.r_esc = im.r_esc;
    hp.r_src = im.r_src;
    hp.r_in = im.r_in;
    hp.r_out = im.r_out;
    hp.h_budget = p.h_budget;
    hp.r_switch = p.r_switch;
    hp.feat = image_features(im);
    hp.max_steps = static_cast<int32_t>(p.max_steps);
    hp.max_evals = static_cast<int32_t>(p.max_evals);
    hp.cold = p.ws_params;
    return hp;
}

// The single-image Dormand-Prince FP64 kernel with the image's features
// fixed at compile time (every other form reads them at run time).
template <int FEAT>
static void launch_dp45_feat(const Hot& hp, int grid, int block, hipStream_t s) {
    hipLaunchKernelGGL((trace_kernel<KT_DP45, KT_FP64, false, false, FEAT>), dim3(grid), dim3(block), 0, s, hp);
}

template <int METHOD, int PREC>
static void launch_variant(const Params& p, const Hot& hp, int grid, int block, hipStream_t s) {
    if constexpr (PREC == KT_FP64 && METHOD != KT_RK4_S) {
        if (p.img0.metric == KT_METRIC_Q) {
            hipLaunchKernelGGL((trace_kernel<METHOD, PREC, false, true>), dim3(grid), dim3(block), 0, s, hp);
            return;
        }
    }
    if constexpr (METHOD == KT_DP45 && PREC == KT_FP64) {
        if (p.n_images == 1) {
            switch (hp.feat & 7) {
            case 0: launch_dp45_feat<0>(hp, grid, block, s); return;
            case 1: launch_dp45_feat<1>(hp, grid, block, s); return;
            case 2: launch_dp45_feat<2>(hp, grid, block, s); return;
            case 3: launch_dp45_feat<3>(hp, grid, block, s); return;
            case 4: launch_dp45_feat<4>(hp, grid, block, s); return;
            case 5: launch_dp45_feat<5>(hp, grid, block, s); return;
            case 6: launch_dp45_feat<6>(hp, grid, block, s); return;
            default: launch_dp45_feat<7>(hp, grid, block, s); return;
            }
        }
    }
    if (p.n_images > 1)
        hipLaunchKernelGGL((trace_kernel<METHOD, PREC, true>), dim3(grid), dim3(block), 0, s, hp);
    else
        hipLaunchKernelGGL((trace_kernel<METHOD, PREC, false>), dim3(grid), dim3(block), 0, s, hp);
}

int launch_trace(const Params& p, int grid, int block, void* stream) {
    const Hot hp = make_hot(p);
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (p.method) {
    case KT_DP45:
        if (p.precision == KT_MIXED)
            launch_variant<KT_DP45, KT_MIXED>(p, hp, grid, block, s);
        else
            launch_variant<KT_DP45, KT_FP64>(p, hp, grid, block, s);
        break;
    case KT_RKF45: launch_variant<KT_RKF45, KT_FP64>(p, hp, grid, block, s); break;
    case KT_CK45: launch_variant<KT_CK45, KT_FP64>(p, hp, grid, block, s); break;
    case KT_BS: launch_variant<KT_BS, KT_FP64>(p, hp, grid, block, s); break;
    case KT_BS_RAT: launch_variant<KT_BS_RAT, KT_FP64>(p, hp, grid, block, s); break;
    default: launch_variant<KT_RK4_S, KT_FP64>(p, hp, grid, block, s); break;
    }
    return check_launch();
}

#if !KT_TRACE_ONLY
int launch_fallback_list(const Params& p, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(fallback_list_kernel, dim3(small_grid(p.n_rays, 256)), dim3(256), 0, s, p.need_fb,
                       static_cast<int64_t>(p.n_rays), p.fb_list, p.fb_count);
    if (check_launch()) return -1;
    hipLaunchKernelGGL(to_fallback_kernel, dim3(1), dim3(64), 0, s, p.ws_params);
    return check_launch();
}

#endif  // !KT_TRACE_ONLY

int launch_trace_fallback(const Params& p, int grid, int block, void* stream) {
    const Hot hp = make_hot(p);
    launch_variant<KT_DP45, KT_FP64>(p, hp, grid, block, static_cast<hipStream_t>(stream));
    return check_launch();
}

template <int METHOD, int PREC>
static hipError_t occupancy_variant(const Params& p, int* nb, int block) {
    if constexpr (PREC == KT_FP64 && METHOD != KT_RK4_S) {
        if (p.img0.metric == KT_METRIC_Q)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, trace_kernel<METHOD, PREC, false, true>, block, 0);
    }
    if (p.n_images > 1)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, trace_kernel<METHOD, PREC, true>, block, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, trace_kernel<METHOD, PREC, false>, block, 0);
}

int trace_max_blocks_per_cu(const Params& p, int block) {
    int nb = 0;
    hipError_t e;
    switch (p.method) {
    case KT_DP45:
        e = p.precision == KT_MIXED ? occupancy_variant<KT_DP45, KT_MIXED>(p, &nb, block)
                                    : occupancy_variant<KT_DP45, KT_FP64>(p, &nb, block);
        break;
    case KT_RKF45: e = occupancy_variant<KT_RKF45, KT_FP64>(p, &nb, block); break;
    case KT_CK45: e = occupancy_variant<KT_CK45, KT_FP64>(p, &nb, block); break;
    case KT_BS: e = occupancy_variant<KT_BS, KT_FP64>(p, &nb, block); break;
    case KT_BS_RAT: e = occupancy_variant<KT_BS_RAT, KT_FP64>(p, &nb, block); break;
    default: e = occupancy_variant<KT_RK4_S, KT_FP64>(p, &nb, block); break;
    }
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

#if !KT_TRACE_ONLY
int launch_disk_obs(const Params& p, void* stream) {
    hipLaunchKernelGGL(disk_obs_kernel, dim3(small_grid(p.n_rays, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), p.ws_params);
    return check_launch();
}

int launch_ring(const Params& p, void* stream) {
    hipLaunchKernelGGL(ring_kernel, dim3(small_grid(p.n_rays, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), p.ws_params);
    return check_launch();
}

int launch_sky(const Params& p, void* stream) {
    hipLaunchKernelGGL(sky_kernel, dim3(small_grid(p.n_rays, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), p.ws_params);
    return check_launch();
}

int launch_stats(const Params& p, void* stream) {
    const int64_t n = p.n_rays;
    // few blocks: each ends with one 64-bit atomic per fate on the same
    // eight words, and thousands of those serialise
    const int grid = small_grid(n, 256) < 256 ? small_grid(n, 256) : 256;
    hipLaunchKernelGGL(fate_hist_kernel, dim3(grid), dim3(256), 0,
                       static_cast<hipStream_t>(stream), p.out.fate, n, p.acc);
    if (check_launch()) return -1;
    hipLaunchKernelGGL(stats_kernel, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), p.acc,
                       p.fb_count, n, p.wall_khz, p.out.stats);
    return check_launch();
}

int launch_stamp(const Params& p, int slot, void* stream) {
    hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), p.acc, slot);
    return check_launch();
}

int launch_init_rays(const Params& p, double* state, uint8_t* invalid, void* stream) {
    hipLaunchKernelGGL(init_rays_kernel, dim3(small_grid(p.n_rays, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), p.img0, static_cast<int64_t>(p.n_rays), state, invalid);
    return check_launch();
}

#endif  // !KT_TRACE_ONLY

}  // namespace KT_TRACE_NS
