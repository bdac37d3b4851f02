// kt_ray.h -- per-ray pieces shared by the trace and adjoint kernels: the
// camera's initial state, the step-size controller's arithmetic.  Both
// kernels must take bit-identical steps for the same ray, so they share
// these definitions.
#pragma once

#include <hip/hip_runtime.h>

#include "kt_device.h"
#include "kt_internal.h"

namespace kt {

constexpr double HALF_PI = 1.57079632679489661923;

// Initial state of pixel `pix` of image `im` (second eq:momentums with p_r
// ingoing).  Returns false when x^2 + y^2 >= r0^2 (no real p_r).
__device__ __forceinline__ bool camera_state(const Image& im, int32_t pix, double z[5], double* E,
                                             double* L) {
    // separate roundings, no FMA: the pixel centre is the same double the
    // plain expression -fov + (i + 1/2) dx gives on any IEEE machine
#pragma clang fp contract(off)
    const int32_t j = pix / im.nx;
    const int32_t i = pix - j * im.nx;
    const double x = -im.fov_x + (static_cast<double>(i) + 0.5) * im.dx;
    const double y = -im.fov_y + (static_cast<double>(j) + 0.5) * im.dy;
    const double Pth = y / im.r0;   // observer-frame P^theta with P^t = 1
    const double Pph = -x / im.r0;  // observer-frame P^phi
    const double rad = 1.0 - Pth * Pth - Pph * Pph;
    *E = im.E0 + x * im.cE;
    *L = x * im.cL;
    z[0] = im.r0;
    z[1] = im.incl;
    z[2] = 0.0;
    z[3] = rad > 0.0 ? -sqrt(im.g_rr * rad) : 0.0;
    z[4] = y * im.cth;
    return rad > 0.0;
}

// Evaluations per step and the step-size controller exponent 1/(q + 1), q
// the order of the method's error estimate (4 for the Runge-Kutta pairs,
// 2K - 2 for Bulirsch-Stoer with K columns).
template <int METHOD>
constexpr int evals_per_step() {
    return METHOD == KT_RK4_S ? 4 : (METHOD == KT_BS || METHOD == KT_BS_RAT) ? BS_COLUMNS * BS_COLUMNS + 1 : 6;
}
template <int METHOD>
constexpr float controller_exponent() {
    return (METHOD == KT_BS || METHOD == KT_BS_RAT) ? 1.0f / (2 * BS_COLUMNS - 1) : 0.2f;
}

// Whether the step-size control runs entirely in FP64.  For the Runge-Kutta
// pairs the factor only steers the step size and is taken in FP32 (with one
// hardware reciprocal estimate in the error norm).  Bulirsch-Stoer takes
// about 60 long steps per ray, and where its steps land moves the swept
// angle by up to 1e-5 under a 1e-7 change of the step size, so its control
// follows the plain FP64 arithmetic: refined reciprocals, an FP64 power and
// FP64 clamps.
template <int METHOD>
constexpr bool fp64_control() {
    return METHOD == KT_BS || METHOD == KT_BS_RAT;
}

// Step-size factor 0.9 err^(-1/(q+1)) from the mean-square error msq = err^2,
// evaluated in FP32: it only steers the step size.
template <int METHOD>
__device__ __forceinline__ float step_factor(double msq) {
    constexpr float x = -0.5f * controller_exponent<METHOD>();
    return 0.9f * __builtin_amdgcn_exp2f(x * __builtin_amdgcn_logf(static_cast<float>(msq)));
}

// The same factor in FP64: 0.9 exp(-ln(msq) / (2 (q + 1))) with the kernel's
// own logarithm and exponential (about an ulp each).
template <int METHOD>
__device__ __forceinline__ double step_factor64(double msq) {
    constexpr double x = -0.5 / ((METHOD == KT_BS || METHOD == KT_BS_RAT) ? 2 * BS_COLUMNS - 1 : 5);
    return 0.9 * exp_fast(x * log_fast(msq));
}

// h multiplier after a rejected step: max(0.2, factor).
template <int METHOD>
__device__ __forceinline__ double reject_factor(double msq) {
    if constexpr (fp64_control<METHOD>())
        return fmax(0.2, step_factor64<METHOD>(msq));
    else
        return static_cast<double>(fmaxf(0.2f, step_factor<METHOD>(msq)));
}

// h multiplier after an accepted step: 5 for a negligible error (err below
// 1e-10), else the factor clamped to [0.2, 5].
template <int METHOD>
__device__ __forceinline__ double accept_factor(double msq) {
    if (!(msq >= 1e-20)) return 5.0;
    if constexpr (fp64_control<METHOD>())
        return fmin(5.0, fmax(0.2, step_factor64<METHOD>(msq)));
    else
        return static_cast<double>(fminf(5.0f, fmaxf(0.2f, step_factor<METHOD>(msq))));
}

// Mean square of err_i / sc_i over the five components.  The five
// reciprocals come from one reciprocal of the product of the scales: the
// hardware estimate (relative error ~5e-8: this number only steers the step
// size), or with REFINED that estimate refined to about an ulp.
template <bool REFINED = false>
__device__ __forceinline__ double error_msq(const double er[5], const double sc[5]) {
    const double p01 = sc[0] * sc[1], p34 = sc[3] * sc[4];
    const double p012 = p01 * sc[2];
    const double q = REFINED ? rcp(p012 * p34) : __builtin_amdgcn_rcp(p012 * p34);
    const double q012 = q * p34;           // 1 / (sc0 sc1 sc2)
    const double q34 = q * p012;           // 1 / (sc3 sc4)
    const double q01 = q012 * sc[2];       // 1 / (sc0 sc1)
    const double e0 = er[0] * (q01 * sc[1]);
    const double e1 = er[1] * (q01 * sc[0]);
    const double e2 = er[2] * (q012 * p01);
    const double e3 = er[3] * (q34 * sc[4]);
    const double e4 = er[4] * (q34 * sc[3]);
    return 0.2 * fma(e0, e0, fma(e1, e1, fma(e2, e2, fma(e3, e3, e4 * e4))));
}

}  // namespace kt
