// kt_elem.h -- the elementary functions the trace kernel shares with the
// adjoint: the reciprocal and sin/cos of the polar angle.  sincos_theta is
// plain arithmetic and compiles on the host as well; rcp has a device form
// (the hardware estimate, refined) and a host form (a division), chosen by
// the side that calls it.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace kt {

// 1/x from the hardware reciprocal estimate y (relative error e) refined by
// one third-order step y (1 + e + e^2), which cubes the error (below 1e-21
// from the estimate's ~5e-8): the result is within about an ulp.
__device__ __forceinline__ double rcp(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, y, 1.0);
    return fma(y, fma(e, e, e), y);
}
__host__ inline double rcp(double x) { return 1.0 / x; }

// sin and cos of the polar angle theta.  theta is folded to t in [-pi, pi]
// by t = theta - 2 pi rint(theta / 2 pi) (t = theta exactly on [0, pi), the
// range of every ray that does not pass over the polar axis); then with
// u = |t| - pi/2 in [-pi/2, pi/2]: sin theta = copysign(cos u, t) and
// cos theta = -sin u.  cos u = 1 - x C(x) and sin u = u - u x S(x), x = u^2,
// with minimax polynomials C and S of degree 7 for |u| <= pi/2 (coefficients
// from minimax_coefs.py, the constant term of C held at 1/2).  With the
// coefficients rounded to double the absolute error stays below 1.4e-17 for
// cos u and 4.1e-17 for sin u, under a third of an ulp of 1; Taylor's series
// needs two more terms each for the same.  No quadrant selects.
__host__ __device__ inline __attribute__((always_inline)) void sincos_theta(double th, double* s_out,
                                                                           double* c_out) {
    constexpr double INV_TWO_PI = 0.15915494309189533577;
    constexpr double TWO_PI_HI = 6.2831853071795862320e+00;  // 2 pi rounded to double
    constexpr double TWO_PI_LO = 2.4492935982947064e-16;     // 2 pi - TWO_PI_HI
    constexpr double PIO2_HI = 1.5707963267948965580e+00;
    constexpr double PIO2_LO = 6.1232339957367658e-17;
    const double n = __builtin_rint(th * INV_TWO_PI);
    double t = fma(-n, TWO_PI_HI, th);
    t = fma(-n, TWO_PI_LO, t);
    const double u = (fabs(t) - PIO2_HI) - PIO2_LO;
    const double u2 = u * u;
    double pc = 4.616135051438568e-14;
    pc = fma(pc, u2, -1.1463635437491283e-11);
    pc = fma(pc, u2, 2.0876592592498227e-09);
    pc = fma(pc, u2, -2.755731706851054e-07);
    pc = fma(pc, u2, 2.48015872857839e-05);
    pc = fma(pc, u2, -0.001388888888883005);
    pc = fma(pc, u2, 0.04166666666666583);
    pc = fma(pc, u2, -0.5);
    *s_out = __builtin_copysign(fma(pc, u2, 1.0), t);  // sin theta = +-cos u
    double ps = -2.7184963661503298e-15;
    ps = fma(ps, u2, 7.642712927256417e-13);
    ps = fma(ps, u2, -1.605892783643712e-10);
    ps = fma(ps, u2, 2.5052106606636936e-08);
    ps = fma(ps, u2, -2.755731920778693e-06);
    ps = fma(ps, u2, 0.00019841269841185962);
    ps = fma(ps, u2, -0.008333333333333115);
    ps = fma(ps, u2, 0.16666666666666666);
    *c_out = fma(ps * u2, u, -u);  // cos theta = -sin u
}

}  // namespace kt
