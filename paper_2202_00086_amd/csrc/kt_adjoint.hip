// kt_adjoint.hip -- discrete adjoint of the disk image (observed intensity
// per pixel) with respect to the spin a, the inclination and the disk's
// inner radius.
//
// Per ray (one per lane; lanes take rays from an atomic ticket over a list of
// the differentiated rays sorted by forward step count):
//   1. re-integrate from the camera with the trace kernel's own stepper and
//      controller (bit-identical steps), keeping a checkpoint (state, trial
//      step) every 2^ck_shift accepted steps (64 by default), up to the
//      located disk crossing;
//   2. seed the cotangent of the crossing state from the intensity's
//      derivatives, with the crossing-time correction that keeps theta on
//      the equatorial plane;
//   3. run the vector-Jacobian products of the Dormand-Prince steps backward
//      with the accepted step sizes frozen: the located partial step first,
//      then each segment between checkpoints, recomputed forward from its
//      checkpoint;
//   4. chain the cotangents of the initial state and of (E, L) through the
//      camera's dependence on (a, inclination).
// With the forward step counts, the longest rays (the head of the list) can
// have their step 3 split over several lanes instead: step 1 stores every
// accepted step, then each 64-step segment is swept backward from four
// basis cotangents at once, one lane each (the segment's transposed
// Jacobian, a linear map since the steps are frozen), and a last pass
// applies the segments' maps to the ray's seeded cotangent in order.  The
// backward sweep of a ray is otherwise one lane's sequential work, and the
// longest ray's sets the run time of the whole adjoint.
// The results are the per-pixel products cot_I * dI/d(a, incl, r_in) and,
// on request, their three sums over the image (a fixed-order block-then-grid
// reduction, so the sums do not depend on which lane ran which ray).
#include <hip/hip_runtime.h>

#include "kt_adjoint_math.h"
#include "kt_device.h"
#include "kt_internal.h"
#include "kt_ray.h"
#include "kt_sort.h"

namespace kt {

enum : int { ADJ_OK = 0, ADJ_FAIL = 1, ADJ_OVERFLOW = 2, ADJ_MISMATCH = 3 };

// Where the forward pass keeps states: entry idx at p + idx * istride, its
// field f (0..4 the state, 5 a step size) at + f * fstride, at most cap
// entries.  With shift > 0 entry c is the state after c * 2^shift accepted
// steps and the trial size of the next step (entry 0 the start); with shift
// 0 entry j is the start state of accepted step j and its accepted size.
// A lane's checkpoints and segment slots sit in [index][field][lane]
// arrays; a split ray's steps in its own range of the split-ray store.
struct StepStore {
    double* p;
    size_t istride, fstride;
    int32_t cap, shift;
    __device__ double* at(int idx) const { return p + static_cast<size_t>(idx) * istride; }
};
__device__ __forceinline__ void put6(double* p, size_t fstride, const double y[5], double h) {
#pragma unroll
    for (int f = 0; f < 5; ++f) p[f * fstride] = y[f];
    p[5 * fstride] = h;
}
__device__ __forceinline__ void get6(const double* p, size_t fstride, double y[5], double* h) {
#pragma unroll
    for (int f = 0; f < 5; ++f) y[f] = p[f * fstride];
    *h = p[5 * fstride];
}

// One attempt of the adaptive step as the trace kernel takes it.  Returns 1
// for an accepted step (yn, kn, dg, h_next set), 0 for a rejection (h
// shrunk), -1 for a failure.
__device__ __forceinline__ int try_step(const Spacetime& st, const RayConst& rc, const AdjParams& P,
                                        const double y[5], const double k1[5], double s0, double c0, double* h,
                                        bool* rejected, double yn[5], double kn[5], Diag* dg, double* h_next) {
    double er[5];
    dp45_step(st, rc, y, k1, s0, c0, *h, yn, kn, er, dg);
    bool finite = true;
#pragma unroll
    for (int i = 0; i < 5; ++i) finite = finite && isfinite(yn[i]);
    if (!finite) return -1;
    double sc[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) sc[i] = fma(P.rtol, fmax(fabs(y[i]), fabs(yn[i])), P.atol);
    const double msq = error_msq(er, sc);
    if (isnan(msq)) return -1;
    if (msq > 1.0) {
        *h *= reject_factor<KT_DP45>(msq);
        *rejected = true;
        return 0;
    }
    double fac = accept_factor<KT_DP45>(msq);
    if (*rejected) fac = fmin(fac, 1.0);
    *h_next = *h * fac;
    return 1;
}

constexpr int ADJ_BLOCK = 256;

// What the forward pass leaves for the backward one.
struct Fwd {
    double y[5];  // start of the located partial step
    double E, L;
    double zs[5], ks[5], hstar;  // crossing state, the field there, the partial step's size
    int n;                       // accepted steps before the crossing
};

// 1. Forward from the camera to the disk crossing, storing states in `sto`.
__device__ __forceinline__ int forward_to_hit(const AdjParams& P, const Spacetime& st, int32_t ray,
                                              const StepStore& sto, Fwd* f) {
    const Image& im = P.im;
    double* y = f->y;
    camera_state(im, ray, y, &f->E, &f->L);
    const RayConst rc = make_ray_const(st, f->E, f->L);
    const int ck_mask = (1 << sto.shift) - 1;
    double k1[5];
    Diag dg;
    rhs<true, false>(st, rc, y, k1, &dg);
    double s0 = dg.s, c0 = dg.c, h = P.h_init;
    bool rej = false;
    int n = 0;  // accepted steps
    if (sto.shift > 0) put6(sto.at(0), sto.fstride, y, h);
    bool hit = false;
    for (int64_t guard = 0; guard < P.max_attempts && !hit; ++guard) {
        double yn[5], kn[5], hn = 0.0;
        Diag dn;
        const int ok = try_step(st, rc, P, y, k1, s0, c0, &h, &rej, yn, kn, &dn, &hn);
        if (ok < 0) return ADJ_FAIL;
        if (ok == 0) continue;
        const double fa0 = y[1] - HALF_PI, fb0 = yn[1] - HALF_PI;
        if (fa0 * fb0 < 0.0) {
            // Illinois regula falsi on theta - pi/2, trial steps from y
            double A = 0.0, FA = fa0, B = h, FB = fb0, C = h - fb0 * h / (fb0 - fa0);
            double zc[5], kc[5];
            for (int it = 1;; ++it) {
                double ec[5];
                Diag dc;
                dp45_step(st, rc, y, k1, s0, c0, C, zc, kc, ec, &dc);
                const double fc = zc[1] - HALF_PI;
                if (fabs(fc) <= 1e-14 || it >= 64) break;
                if (fc * FB < 0.0) {
                    A = B;
                    FA = FB;
                } else {
                    FA *= 0.5;
                }
                B = C;
                FB = fc;
                C = B - FB * (B - A) / (FB - FA);
            }
            if (zc[0] >= im.r_in && zc[0] <= im.r_out) {
                hit = true;
                f->hstar = C;
#pragma unroll
                for (int i = 0; i < 5; ++i) {
                    f->zs[i] = zc[i];
                    f->ks[i] = kc[i];
                }
                break;
            }
        } else if (fb0 == 0.0 && yn[0] >= im.r_in && yn[0] <= im.r_out) {
            hit = true;
            f->hstar = h;
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                f->zs[i] = yn[i];
                f->ks[i] = kn[i];
            }
            break;
        }
        if (yn[0] < im.r_cap || yn[0] > im.r_esc) return ADJ_MISMATCH;
        if (sto.shift == 0) {
            // every accepted step: its start state and its accepted size
            if (n >= sto.cap) return ADJ_OVERFLOW;
            put6(sto.at(n), sto.fstride, y, h);
        }
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            y[i] = yn[i];
            k1[i] = kn[i];
        }
        s0 = dn.s;
        c0 = dn.c;
        h = hn;
        rej = false;
        ++n;
        if (sto.shift > 0 && (n & ck_mask) == 0) {
            if ((n >> sto.shift) >= sto.cap) return ADJ_OVERFLOW;
            put6(sto.at(n >> sto.shift), sto.fstride, y, h);
        }
    }
    if (!hit) return ADJ_FAIL;
    if (P.r_hit && !(f->zs[0] == P.r_hit[ray])) return ADJ_MISMATCH;
    f->n = n;
    return ADJ_OK;
}

// 2. Seeds from the intensity with the crossing-time correction, then the
// vector-Jacobian product of the located partial step.
__device__ __forceinline__ void seed_partial(const AdjParams& P, const Fwd& f, double w, double zb[5],
                                             adj::ParBar* pb, double* gr) {
    const Image& im = P.im;
    const Dual<5> I = adj::disk_intensity(P.dm, f.zs[0], f.E, f.L, im.a, im.r_in);
    *pb = adj::ParBar{w * I.d[1], w * I.d[2], w * I.d[3]};
    *gr = w * I.d[4];
    const double rbar = w * I.d[0];
    // r_c = r(lambda*) with theta(lambda*) = pi/2: dr_c = dr - (r' / theta') dtheta
    zb[0] = rbar;
    zb[1] = -rbar * f.ks[0] / f.ks[1];
    zb[2] = zb[3] = zb[4] = 0.0;
    adj::dp_step_vjp(im.M, im.a, f.E, f.L, f.y, f.hstar, zb, pb);
}

// 3. The rest of the reverse sweep with frozen steps, from the lane's own
// checkpoints: stored steps are read back; otherwise each segment between
// checkpoints is recomputed forward from its checkpoint into the lane's
// segment slots first.
__device__ __forceinline__ int sweep_lane(const AdjParams& P, const Spacetime& st, int lane, const Fwd& f,
                                          double zb[5], adj::ParBar* pb) {
    const Image& im = P.im;
    const size_t fs = static_cast<size_t>(P.n_lanes), is = 6u * fs;
    int n = f.n;
    if (P.ck_shift == 0) {
        // every step was stored: no recomputation
        for (int j = n - 1; j >= 0; --j) {
            double yj[5], hj;
            get6(P.ckpt + j * is + lane, fs, yj, &hj);
            adj::dp_step_vjp(im.M, im.a, f.E, f.L, yj, hj, zb, pb);
        }
        return ADJ_OK;
    }
    const RayConst rc = make_ray_const(st, f.E, f.L);
    const int ck_mask = (1 << P.ck_shift) - 1;
    for (int s = (n - 1) >> P.ck_shift; n > 0 && s >= 0; --s) {
        const int first = s << P.ck_shift, last = min(n, first + ck_mask + 1);
        double ys[5], hs;
        get6(P.ckpt + s * is + lane, fs, ys, &hs);
        double kk[5];
        Diag dr;
        rhs<true, false>(st, rc, ys, kk, &dr);
        double ss = dr.s, cc = dr.c;
        bool rj = false;
        int attempts = 0;
        for (int j = first; j < last;) {
            // the recomputation repeats the forward's attempts exactly; the
            // bound only guarantees that the loop ends
            if (++attempts > 64 * (ck_mask + 1)) return ADJ_FAIL;
            double yn[5], kn[5], hn = 0.0;
            Diag dn;
            const int ok = try_step(st, rc, P, ys, kk, ss, cc, &hs, &rj, yn, kn, &dn, &hn);
            if (ok < 0) return ADJ_FAIL;
            if (ok == 0) continue;
            put6(P.seg + (j - first) * is + lane, fs, ys, hs);
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                ys[i] = yn[i];
                kk[i] = kn[i];
            }
            ss = dn.s;
            cc = dn.c;
            hs = hn;
            rj = false;
            ++j;
        }
        for (int j = last - 1; j >= first; --j) {
            double yj[5], hj;
            get6(P.seg + (j - first) * is + lane, fs, yj, &hj);
            adj::dp_step_vjp(im.M, im.a, f.E, f.L, yj, hj, zb, pb);
        }
    }
    return ADJ_OK;
}

// 4. The camera: z0 = (r0, incl, 0, p_r, p_th), E, L of (a, incl).
__device__ __forceinline__ void camera_chain(const AdjParams& P, int32_t ray, const double zb[5],
                                             const adj::ParBar& pb, double* ga, double* gi) {
    const Image& im = P.im;
    const int32_t jj = ray / im.nx, ii = ray - jj * im.nx;
    const double x = -im.fov_x + (static_cast<double>(ii) + 0.5) * im.dx;
    const double yy = -im.fov_y + (static_cast<double>(jj) + 0.5) * im.dy;
    const double rad = 1.0 - (yy / im.r0) * (yy / im.r0) - (x / im.r0) * (x / im.r0);
    const double pr0 = -sqrt(im.g_rr * rad);
    double g2[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double dE = P.dcam[0][k] + x * P.dcam[1][k];
        const double dL = x * P.dcam[2][k];
        const double dpth = yy * P.dcam[3][k];
        const double dpr = 0.5 * pr0 * P.dcam[4][k] / im.g_rr;
        g2[k] = pb.E * dE + pb.L * dL + zb[3] * dpr + zb[4] * dpth;
    }
    *ga = pb.a + g2[0];
    *gi = zb[1] + g2[1];
}

__device__ __forceinline__ void put_grads(const AdjParams& P, int32_t ray, int status, double ga, double gi,
                                          double gr) {
    if (status != ADJ_OK) ga = gi = gr = 0.0;
    atomicAdd(P.stats + status, 1ull);
    if (P.grad_a) P.grad_a[ray] = ga;
    if (P.grad_incl) P.grad_incl[ray] = gi;
    if (P.grad_rin) P.grad_rin[ray] = gr;
}

// One entry t of the work list on this lane.  An entry among the first
// n_long (the split rays) that fits the split-ray store runs the forward
// pass into the store, seeds its cotangent, reserves its segment items and
// leaves the rest to the segment and combine kernels; every other entry
// runs the whole adjoint of its ray on this lane.
__device__ __forceinline__ void adjoint_entry(const AdjParams& P, const Spacetime& st, int lane, uint32_t t,
                                              uint32_t n_long) {
    const int32_t ray = static_cast<int32_t>(P.list[t]);
    const size_t fs = static_cast<size_t>(P.n_lanes);
    StepStore sto{P.ckpt + lane, 6u * fs, fs, P.max_ckpt, P.ck_shift};
    bool split = false;
    if (t < n_long) {
        // a split ray: every step into its own range of the store
        AdjLong& rec = P.longs[t];
        rec.ray = ray;
        rec.status = ADJ_LONG_DONE;
        const int32_t steps = P.n_steps[ray];
        const uint32_t cap = steps >= 0 ? static_cast<uint32_t>(steps) + 2u : 0u;
        if (cap > 2u && cap <= static_cast<uint32_t>(ADJ_SEG * ADJ_SEG_MAX)) {
            const uint32_t base = atomicAdd(P.counters + 1, cap);
            if (static_cast<uint64_t>(base) + cap <= P.long_cap) {
                sto = StepStore{P.long_store + static_cast<size_t>(base) * 6u, 6u, 1u, static_cast<int32_t>(cap), 0};
                rec.base = base;
                split = true;
            }
        }
    }
    Fwd f;
    double zb[5], ga = 0.0, gi = 0.0, gr = 0.0;
    adj::ParBar pb;
    int status = forward_to_hit(P, st, ray, sto, &f);
    if (status == ADJ_OK) seed_partial(P, f, P.cot[ray], zb, &pb, &gr);
    if (split && status == ADJ_OK) {
        AdjLong& rec = P.longs[t];
        const int n_seg = (f.n + ADJ_SEG - 1) / ADJ_SEG;
        const uint32_t n_items = 4u * static_cast<uint32_t>(n_seg);
        const uint32_t ib = atomicAdd(P.counters + 2, n_items);
        if (static_cast<uint64_t>(ib) + n_items <= P.item_cap) {
            for (uint32_t i = 0; i < n_items; ++i) P.owner[ib + i] = t;
            rec.n = f.n;
            rec.n_seg = n_seg;
            rec.item_base = ib;
            rec.zb[0] = zb[0];
            rec.zb[1] = zb[1];
            rec.zb[2] = zb[3];
            rec.zb[3] = zb[4];
            rec.pb[0] = pb.E;
            rec.pb[1] = pb.L;
            rec.pb[2] = pb.a;
            rec.gr = gr;
            rec.E = f.E;
            rec.L = f.L;
            rec.status = ADJ_LONG_SPLIT;
            return;  // the combine kernel finishes this ray
        }
        status = ADJ_OVERFLOW;  // cannot happen: the item space covers the store
    }
    if (!split && status == ADJ_OK) status = sweep_lane(P, st, lane, f, zb, &pb);
    if (status == ADJ_OK) camera_chain(P, ray, zb, pb, &ga, &gi);
    put_grads(P, ray, status, ga, gi, gr);
}

// One wave per SIMD: the unrolled step VJP wants about 500 VGPRs, and a
// two-wave budget (256) spills enough to run 1.6x slower.
#ifndef KT_ADJ_WAVES_PER_EU
#define KT_ADJ_WAVES_PER_EU 1
#endif
// Lanes take entries of the work list from an atomic ticket.
__global__ void __launch_bounds__(ADJ_BLOCK) __attribute__((amdgpu_waves_per_eu(KT_ADJ_WAVES_PER_EU)))
adjoint_kernel(const AdjParams P) {
    const int lane = blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= P.n_lanes) return;
    const Spacetime st{P.im.M, P.im.a, P.im.a2, P.im.two_a2};
    const uint32_t n_list = P.hist[SORT_BINS];
    const uint32_t n_long = P.max_long > 0 ? P.counters[0] : 0u;
    for (;;) {
        const uint32_t t = atomicAdd(P.ticket, 1u);
        if (t >= n_list) break;
        adjoint_entry(P, st, lane, t, n_long);
    }
}

// The split threshold and n_long, from the sorted work list's bins (one
// block, after the sort: hist[k] is then the end of bin k, and bin k holds
// the rays of 4 v to 4 v + 3 forward steps, v = SORT_BINS - 1 - k, bin 0
// also every longer ray).  The automatic threshold is 0.85 times the mean
// step count per lane of the grid: rays near that length or longer would
// outlast the rest of the list.  The split rays are whole bins, longest
// first, as many as the records and the split-ray store hold for certain (a
// ray of bin v takes at most 4 v + 5 entries of the store; rays beyond
// ADJ_SEG * ADJ_SEG_MAX - 2 steps are never split): which rays are split
// then does not depend on the order in which lanes take them, and neither
// do the gradients.  The store's size (ADJ_LONG_STEPS_PER_LANE steps per
// lane) thereby bounds the extra work of the basis sweeps, four step VJPs
// per stored step.
__global__ void __launch_bounds__(SORT_BLOCK) adjoint_split_kernel(const AdjParams P) {
    constexpr int PER = SORT_BINS / SORT_BLOCK;  // consecutive bins per thread
    static_assert(SORT_BINS % SORT_BLOCK == 0, "bins must split evenly over the block");
    __shared__ unsigned long long part[SORT_BLOCK];
    __shared__ long long thr;
    __shared__ int stop;
    const int t = threadIdx.x;
    uint32_t cnt[PER];
    unsigned long long steps = 0;
    for (int i = 0; i < PER; ++i) {
        const int k = t * PER + i;
        cnt[i] = P.hist[k] - (k > 0 ? P.hist[k - 1] : 0u);
        steps += static_cast<unsigned long long>(cnt[i]) * static_cast<unsigned long long>(4 * (SORT_BINS - 1 - k) + 2);
    }
    part[t] = steps;
    if (t == 0) stop = SORT_BINS;
    __syncthreads();
    for (int w = SORT_BLOCK / 2; w > 0; w >>= 1) {
        if (t < w) part[t] += part[t + w];
        __syncthreads();
    }
    if (t == 0) {
        long long T = P.split_above;
        if (T <= 0) {
            T = static_cast<long long>((17ull * part[0]) / (20ull * static_cast<unsigned long long>(P.n_lanes)));
            if (T < ADJ_SPLIT_MIN) T = ADJ_SPLIT_MIN;
        }
        thr = T;
    }
    __syncthreads();
    // bins above the threshold's: keys below kT; their store demand, at
    // most 4 v + 5 entries per ray of bin v, for bins that can hold a ray
    // short enough to split
    const long long kT = SORT_BINS - 1 - (thr >> 2);
    unsigned long long demand = 0;
    for (int i = 0; i < PER; ++i) {
        const int k = t * PER + i;
        const long long v = SORT_BINS - 1 - k;
        if (k < kT && 4 * v + 2 <= ADJ_SEG * ADJ_SEG_MAX)
            demand += static_cast<unsigned long long>(cnt[i]) *
                      static_cast<unsigned long long>(4 * v + 5 < ADJ_SEG * ADJ_SEG_MAX ? 4 * v + 5 : ADJ_SEG * ADJ_SEG_MAX);
    }
    // exclusive scan of the threads' demands (Hillis-Steele)
    __syncthreads();
    part[t] = demand;
    __syncthreads();
    for (int off = 1; off < SORT_BLOCK; off <<= 1) {
        const unsigned long long add = t >= off ? part[t - off] : 0ull;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    unsigned long long run = part[t] - demand;
    // the first bin that is past the threshold, or whose end passes the
    // records or whose demand passes the store
    for (int i = 0; i < PER; ++i) {
        const int k = t * PER + i;
        const long long v = SORT_BINS - 1 - k;
        if (k < kT && 4 * v + 2 <= ADJ_SEG * ADJ_SEG_MAX)
            run += static_cast<unsigned long long>(cnt[i]) *
                   static_cast<unsigned long long>(4 * v + 5 < ADJ_SEG * ADJ_SEG_MAX ? 4 * v + 5 : ADJ_SEG * ADJ_SEG_MAX);
        if (k >= kT || P.hist[k] > static_cast<uint32_t>(P.max_long) || run > P.long_cap) {
            atomicMin(&stop, k);
            break;
        }
    }
    __syncthreads();
    if (t == 0) P.counters[0] = stop > 0 ? P.hist[stop - 1] : 0u;
}

// The segments of the split rays: item w sweeps segment s of its ray
// backward from the basis cotangent e_b (b over r, theta, p_r, p_theta)
// with zero parameter cotangents, and stores the resulting cotangents of
// (r, theta, p_r, p_theta, E, L, a, phi): column b of the segment's
// transposed Jacobian.  Every item of a wave sweeps the same number of
// steps, and the four of a segment the same states.
__global__ void __launch_bounds__(ADJ_BLOCK) __attribute__((amdgpu_waves_per_eu(KT_ADJ_WAVES_PER_EU)))
adjoint_segment_kernel(const AdjParams P) {
    const Image& im = P.im;
    const uint32_t used = P.counters[2];
    const uint32_t total = used < P.item_cap ? used : P.item_cap;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < total; w += stride) {
        const uint32_t k = P.owner[w];
        if (k >= static_cast<uint32_t>(P.max_long)) continue;
        const AdjLong& rec = P.longs[k];
        if (rec.status != ADJ_LONG_SPLIT) continue;
        const uint32_t local = w - rec.item_base;
        if (local >= 4u * static_cast<uint32_t>(rec.n_seg)) continue;
        const int s = static_cast<int>(local >> 2), b = static_cast<int>(local & 3u);
        const int first = s * ADJ_SEG, last = min(rec.n, first + ADJ_SEG);
        double yb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        yb[b < 2 ? b : b + 1] = 1.0;
        adj::ParBar pb{0.0, 0.0, 0.0};
        const double* base = P.long_store + static_cast<size_t>(rec.base) * 6u;
        for (int j = last - 1; j >= first; --j) {
            double yj[5], hj;
            get6(base + static_cast<size_t>(j) * 6u, 1u, yj, &hj);
            adj::dp_step_vjp(im.M, im.a, rec.E, rec.L, yj, hj, yb, &pb);
        }
        double* o = P.items + static_cast<size_t>(w) * 8u;
        o[0] = yb[0];
        o[1] = yb[1];
        o[2] = yb[3];
        o[3] = yb[4];
        o[4] = pb.E;
        o[5] = pb.L;
        o[6] = pb.a;
        o[7] = yb[2];
    }
}

// Each split ray: its seeded cotangent through the segments' maps, last
// segment first (cotangent' = sum_b cotangent_b * column_b, parameter
// cotangents += sum_b cotangent_b * their column_b), then the camera.
__global__ void __launch_bounds__(ADJ_BLOCK) adjoint_combine_kernel(const AdjParams P) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.counters[0]) return;
    const AdjLong& rec = P.longs[k];
    if (rec.status != ADJ_LONG_SPLIT) return;
    double v[4] = {rec.zb[0], rec.zb[1], rec.zb[2], rec.zb[3]};
    adj::ParBar pb{rec.pb[0], rec.pb[1], rec.pb[2]};
    for (int s = rec.n_seg - 1; s >= 0; --s) {
        const double* o = P.items + (static_cast<size_t>(rec.item_base) + 4u * static_cast<size_t>(s)) * 8u;
        double nv[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const double* c = o + 8 * b;
#pragma unroll
            for (int i = 0; i < 4; ++i) nv[i] = fma(v[b], c[i], nv[i]);
            pb.E = fma(v[b], c[4], pb.E);
            pb.L = fma(v[b], c[5], pb.L);
            pb.a = fma(v[b], c[6], pb.a);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = nv[i];
    }
    const double zb[5] = {v[0], v[1], 0.0, v[2], v[3]};
    double ga, gi;
    camera_chain(P, rec.ray, zb, pb, &ga, &gi);
    put_grads(P, rec.ray, ADJ_OK, ga, gi, rec.gr);
}

// Clears the ticket, the statistics, the split counters and the sort's
// histogram (block 0), and marks every segment item unused.
__global__ void adjoint_init_kernel(const AdjParams P) {
    const int t = threadIdx.x;
    if (blockIdx.x == 0) {
        if (t == 0) *P.ticket = 0u;
        if (t < 4) P.stats[t] = 0ull;
        if (t < 3 && P.max_long > 0) P.counters[t] = 0u;
        for (int b = t; b <= SORT_BINS; b += blockDim.x) P.hist[b] = 0u;
    }
    if (P.max_long > 0)
        for (uint32_t w = blockIdx.x * blockDim.x + t; w < P.item_cap; w += gridDim.x * blockDim.x)
            P.owner[w] = 0xffffffffu;
}

// ---- work list ------------------------------------------------------------
// The lanes of a wave run their rays' loops in step, so a wave costs as much
// as its longest ray.  The differentiated rays (disk hits with a nonzero
// cotangent) are compacted into a list sorted by the forward render's step
// count, longest first (a counting sort over SORT_BINS bins of 4 steps):
// neighbouring lanes then take rays of nearly equal length.  Pixels outside
// the list get zero gradients from the key function.
struct StepKey {
    const uint8_t* fate;
    const double* cot;
    const int32_t* n_steps;  // may be NULL: every listed ray gets the same key
    double *ga, *gi, *gr;
    __device__ int operator()(int64_t ray) const {
        if (fate[ray] == KT_FATE_DISK && cot[ray] != 0.0) {
            int steps = n_steps ? n_steps[ray] >> 2 : 0;
            steps = steps < 0 ? 0 : steps > SORT_BINS - 1 ? SORT_BINS - 1 : steps;
            return SORT_BINS - 1 - steps;
        }
        if (ga) ga[ray] = 0.0;
        if (gi) gi[ray] = 0.0;
        if (gr) gr[ray] = 0.0;
        return SORT_SKIP;
    }
};

// ---- the image sums of the three gradient maps ---------------------------
// A fixed grid of ADJ_RED_BLOCKS blocks: thread t of block b adds pixels
// t + 256 b, t + 256 (b + ADJ_RED_BLOCKS), ... in that order, the block adds
// its 256 partial sums by a fixed tree in LDS, and one block then adds the
// ADJ_RED_BLOCKS block sums by the same tree.  Every sum is taken in one
// order whatever the device or the lanes that ran the rays.
constexpr int RED_THREADS = 256;

__device__ __forceinline__ void tree_sum3(double (*v)[RED_THREADS], int t) {
#pragma unroll
    for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
        __syncthreads();
        if (t < w) {
#pragma unroll
            for (int c = 0; c < 3; ++c) v[c][t] += v[c][t + w];
        }
    }
    __syncthreads();
}

__global__ void __launch_bounds__(RED_THREADS) grad_block_sum_kernel(const double* __restrict__ ga,
                                                                     const double* __restrict__ gi,
                                                                     const double* __restrict__ gr, int64_t n,
                                                                     double* __restrict__ partials) {
    __shared__ double v[3][RED_THREADS];
    const int t = threadIdx.x;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * RED_THREADS + t; k < n;
         k += static_cast<int64_t>(ADJ_RED_BLOCKS) * RED_THREADS) {
        s0 += ga[k];
        s1 += gi[k];
        s2 += gr[k];
    }
    v[0][t] = s0;
    v[1][t] = s1;
    v[2][t] = s2;
    tree_sum3(v, t);
    if (t < 3) partials[t * ADJ_RED_BLOCKS + blockIdx.x] = v[t][0];
}

__global__ void __launch_bounds__(RED_THREADS) grad_final_sum_kernel(const double* __restrict__ partials,
                                                                     double* __restrict__ out) {
    static_assert(ADJ_RED_BLOCKS == RED_THREADS, "one partial per thread");
    __shared__ double v[3][RED_THREADS];
    const int t = threadIdx.x;
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c][t] = partials[c * ADJ_RED_BLOCKS + t];
    tree_sum3(v, t);
    if (t < 3) out[t] = v[t][0];
}

int launch_adjoint(const AdjParams& p, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool split = p.max_long > 0;
    const uint32_t fill_blocks = split ? (p.item_cap + 255u) / 256u : 1u;
    hipLaunchKernelGGL(adjoint_init_kernel, dim3(fill_blocks < 1u ? 1u : fill_blocks), dim3(256), 0, s, p);
    if (hipGetLastError() != hipSuccess) return -1;
    const SortBufs b{p.n_rays, p.hist, p.keys, p.list};
    if (launch_sort(b, StepKey{p.fate, p.cot, p.n_steps, p.grad_a, p.grad_incl, p.grad_rin}, s)) return -1;
    if (split) {
        hipLaunchKernelGGL(adjoint_split_kernel, dim3(1), dim3(SORT_BLOCK), 0, s, p);
        if (hipGetLastError() != hipSuccess) return -1;
    }
    const int grid = (p.n_lanes + ADJ_BLOCK - 1) / ADJ_BLOCK;
    hipLaunchKernelGGL(adjoint_kernel, dim3(grid), dim3(ADJ_BLOCK), 0, s, p);
    if (hipGetLastError() != hipSuccess) return -1;
    if (split) {
        hipLaunchKernelGGL(adjoint_segment_kernel, dim3(grid), dim3(ADJ_BLOCK), 0, s, p);
        if (hipGetLastError() != hipSuccess) return -1;
        hipLaunchKernelGGL(adjoint_combine_kernel, dim3((p.max_long + ADJ_BLOCK - 1) / ADJ_BLOCK), dim3(ADJ_BLOCK),
                           0, s, p);
        if (hipGetLastError() != hipSuccess) return -1;
    }
    if (p.grad_sum) {
        hipLaunchKernelGGL(grad_block_sum_kernel, dim3(ADJ_RED_BLOCKS), dim3(RED_THREADS), 0, s, p.grad_a,
                           p.grad_incl, p.grad_rin, static_cast<int64_t>(p.n_rays), p.partials);
        if (hipGetLastError() != hipSuccess) return -1;
        hipLaunchKernelGGL(grad_final_sum_kernel, dim3(1), dim3(RED_THREADS), 0, s, p.partials, p.grad_sum);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace kt
