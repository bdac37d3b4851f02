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

// Checkpoint c (after c * 2^ck_shift accepted steps) and segment slot j of a
// lane: [index][field][lane], fields 0..4 the state, 5 the step size.
__device__ __forceinline__ double* slot(double* base, int idx, int lane, int n_lanes) {
    return base + static_cast<size_t>(idx) * 6u * static_cast<size_t>(n_lanes) + lane;
}
__device__ __forceinline__ void put6(double* p, int n_lanes, const double y[5], double h) {
#pragma unroll
    for (int f = 0; f < 5; ++f) p[static_cast<size_t>(f) * n_lanes] = y[f];
    p[static_cast<size_t>(5) * n_lanes] = h;
}
__device__ __forceinline__ void get6(const double* p, int n_lanes, double y[5], double* h) {
#pragma unroll
    for (int f = 0; f < 5; ++f) y[f] = p[static_cast<size_t>(f) * n_lanes];
    *h = p[static_cast<size_t>(5) * n_lanes];
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

__device__ int adjoint_ray(const AdjParams& P, const Spacetime& st, int lane, int32_t ray, double w, double* ga,
                           double* gi, double* gr) {
    const Image& im = P.im;
    double y[5], E, L;
    camera_state(im, ray, y, &E, &L);
    const RayConst rc = make_ray_const(st, E, L);
    const int ck_mask = (1 << P.ck_shift) - 1;
    double k1[5];
    Diag dg;
    rhs<true, false>(st, rc, y, k1, &dg);
    double s0 = dg.s, c0 = dg.c, h = P.h_init;
    bool rej = false;
    int n = 0;  // accepted steps
    put6(slot(P.ckpt, 0, lane, P.n_lanes), P.n_lanes, y, h);

    // ---- 1. forward to the disk crossing --------------------------------
    double zs[5], ks[5], hstar = 0.0;
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
                hstar = C;
#pragma unroll
                for (int i = 0; i < 5; ++i) {
                    zs[i] = zc[i];
                    ks[i] = kc[i];
                }
                break;
            }
        } else if (fb0 == 0.0 && yn[0] >= im.r_in && yn[0] <= im.r_out) {
            hit = true;
            hstar = h;
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                zs[i] = yn[i];
                ks[i] = kn[i];
            }
            break;
        }
        if (yn[0] < im.r_cap || yn[0] > im.r_esc) return ADJ_MISMATCH;
        if (P.ck_shift == 0) {
            // every accepted step: its start state and its accepted size
            if (n >= P.max_ckpt) return ADJ_OVERFLOW;
            put6(slot(P.ckpt, n, lane, P.n_lanes), P.n_lanes, y, h);
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
        if (P.ck_shift > 0 && (n & ck_mask) == 0) {
            if ((n >> P.ck_shift) >= P.max_ckpt) return ADJ_OVERFLOW;
            put6(slot(P.ckpt, n >> P.ck_shift, lane, P.n_lanes), P.n_lanes, y, h);
        }
    }
    if (!hit) return ADJ_FAIL;
    if (P.r_hit && !(zs[0] == P.r_hit[ray])) return ADJ_MISMATCH;

    // ---- 2. seeds from the intensity and the crossing-time correction ---
    const Dual<5> I = adj::disk_intensity(P.dm, zs[0], E, L, im.a, im.r_in);
    adj::ParBar pb{w * I.d[1], w * I.d[2], w * I.d[3]};
    *gr = w * I.d[4];
    const double rbar = w * I.d[0];
    // r_c = r(lambda*) with theta(lambda*) = pi/2: dr_c = dr - (r' / theta') dtheta
    double zb[5] = {rbar, -rbar * ks[0] / ks[1], 0.0, 0.0, 0.0};

    // ---- 3. reverse sweep with frozen steps ------------------------------
    adj::dp_step_vjp(im.M, im.a, E, L, y, hstar, zb, &pb);
    if (P.ck_shift == 0) {
        // every step was stored: no recomputation
        for (int j = n - 1; j >= 0; --j) {
            double yj[5], hj;
            get6(slot(P.ckpt, j, lane, P.n_lanes), P.n_lanes, yj, &hj);
            adj::dp_step_vjp(im.M, im.a, E, L, yj, hj, zb, &pb);
        }
        n = 0;  // the segment sweep below has nothing left to do
    }
    for (int s = (n - 1) >> P.ck_shift; n > 0 && s >= 0; --s) {
        const int first = s << P.ck_shift, last = min(n, first + ck_mask + 1);
        double ys[5], hs;
        get6(slot(P.ckpt, s, lane, P.n_lanes), P.n_lanes, ys, &hs);
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
            put6(slot(P.seg, j - first, lane, P.n_lanes), P.n_lanes, ys, hs);
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
            get6(slot(P.seg, j - first, lane, P.n_lanes), P.n_lanes, yj, &hj);
            adj::dp_step_vjp(im.M, im.a, E, L, yj, hj, zb, &pb);
        }
    }

    // ---- 4. the camera: z0 = (r0, incl, 0, p_r, p_th), E, L of (a, incl) --
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
    return ADJ_OK;
}

// One wave per SIMD: the unrolled step VJP wants about 500 VGPRs, and a
// two-wave budget (256) spills enough to run 1.6x slower.
#ifndef KT_ADJ_WAVES_PER_EU
#define KT_ADJ_WAVES_PER_EU 1
#endif
__global__ void __launch_bounds__(ADJ_BLOCK) __attribute__((amdgpu_waves_per_eu(KT_ADJ_WAVES_PER_EU)))
adjoint_kernel(const AdjParams P) {
    const int lane = blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= P.n_lanes) return;
    const Image& im = P.im;
    const Spacetime st{im.M, im.a, im.a2, im.two_a2};
    const uint32_t n_list = P.hist[SORT_BINS];
    for (;;) {
        const uint32_t t = atomicAdd(P.ticket, 1u);
        if (t >= n_list) break;
        const int32_t ray = static_cast<int32_t>(P.list[t]);
        double ga = 0.0, gi = 0.0, gr = 0.0;
        const int status = adjoint_ray(P, st, lane, ray, P.cot[ray], &ga, &gi, &gr);
        if (status != ADJ_OK) ga = gi = gr = 0.0;
        atomicAdd(P.stats + status, 1ull);
        if (P.grad_a) P.grad_a[ray] = ga;
        if (P.grad_incl) P.grad_incl[ray] = gi;
        if (P.grad_rin) P.grad_rin[ray] = gr;
    }
}

__global__ void adjoint_init_kernel(uint32_t* ticket, unsigned long long* stats, uint32_t* hist) {
    const int t = threadIdx.x;
    if (t == 0) *ticket = 0u;
    if (t < 4) stats[t] = 0ull;
    for (int b = t; b <= SORT_BINS; b += blockDim.x) hist[b] = 0u;
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
    hipLaunchKernelGGL(adjoint_init_kernel, dim3(1), dim3(256), 0, s, p.ticket, p.stats, p.hist);
    if (hipGetLastError() != hipSuccess) return -1;
    const SortBufs b{p.n_rays, p.hist, p.keys, p.list};
    if (launch_sort(b, StepKey{p.fate, p.cot, p.n_steps, p.grad_a, p.grad_incl, p.grad_rin}, s)) return -1;
    const int grid = (p.n_lanes + ADJ_BLOCK - 1) / ADJ_BLOCK;
    hipLaunchKernelGGL(adjoint_kernel, dim3(grid), dim3(ADJ_BLOCK), 0, s, p);
    if (hipGetLastError() != hipSuccess) return -1;
    if (p.grad_sum) {
        hipLaunchKernelGGL(grad_block_sum_kernel, dim3(ADJ_RED_BLOCKS), dim3(RED_THREADS), 0, s, p.grad_a,
                           p.grad_incl, p.grad_rin, static_cast<int64_t>(p.n_rays), p.partials);
        if (hipGetLastError() != hipSuccess) return -1;
        hipLaunchKernelGGL(grad_final_sum_kernel, dim3(1), dim3(RED_THREADS), 0, s, p.partials, p.grad_sum);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace kt
