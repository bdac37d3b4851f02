// kt_device.h -- device math for the gfx950 Kerr ray tracer: fast FP64
// elementary functions (with the reciprocal and sin/cos of theta from
// kt_elem.h), the Hamiltonian right-hand side in Carter's separated form and
// that of the q-metric, and the Runge-Kutta and Bulirsch-Stoer steppers.
//
// Everything here runs one ray per lane in VGPRs; nothing touches memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kt_elem.h"

namespace kt {

// ---------------------------------------------------------------------------
// Elementary functions
// ---------------------------------------------------------------------------

// sin and cos of x for |x| < ~1e5.  Cody-Waite reduction by pi/2 with a
// two-part constant, then the Taylor series of sin through r^15 and of cos
// through r^16 on |r| <= pi/4 (truncation below 1e-16), and a quadrant swap.
__device__ __forceinline__ void sincos_fast(double x, double* s_out, double* c_out) {
    constexpr double TWO_OVER_PI = 0.63661977236758134308;
    constexpr double PIO2_HI = 1.5707963267948965580e+00;  // pi/2 rounded to double
    constexpr double PIO2_LO = 6.1232339957367658e-17;     // pi/2 - PIO2_HI
    const double n = __builtin_rint(x * TWO_OVER_PI);
    double r = fma(-n, PIO2_HI, x);
    r = fma(-n, PIO2_LO, r);
    const double r2 = r * r;
    // sin r = r (1 - r^2/3! + r^4/5! - ...), cos r = 1 - r^2/2! + r^4/4! - ...
    double ps = -1.0 / 1307674368000.0;        // -1/15!
    ps = fma(ps, r2, 1.0 / 6227020800.0);      //  1/13!
    ps = fma(ps, r2, -1.0 / 39916800.0);       // -1/11!
    ps = fma(ps, r2, 1.0 / 362880.0);          //  1/9!
    ps = fma(ps, r2, -1.0 / 5040.0);           // -1/7!
    ps = fma(ps, r2, 1.0 / 120.0);             //  1/5!
    ps = fma(ps, r2, -1.0 / 6.0);              // -1/3!
    const double sr = fma(ps * r2, r, r);
    double pc = 1.0 / 20922789888000.0;        //  1/16!
    pc = fma(pc, r2, -1.0 / 87178291200.0);    // -1/14!
    pc = fma(pc, r2, 1.0 / 479001600.0);       //  1/12!
    pc = fma(pc, r2, -1.0 / 3628800.0);        // -1/10!
    pc = fma(pc, r2, 1.0 / 40320.0);           //  1/8!
    pc = fma(pc, r2, -1.0 / 720.0);            // -1/6!
    pc = fma(pc, r2, 1.0 / 24.0);              //  1/4!
    pc = fma(pc, r2, -0.5);                    // -1/2!
    const double cr = fma(pc, r2, 1.0);
    const int q = static_cast<int>(n) & 3;
    const double s0 = (q & 1) ? cr : sr;
    const double c0 = (q & 1) ? sr : cr;
    *s_out = (q & 2) ? -s0 : s0;
    *c_out = ((q + 1) & 2) ? -c0 : c0;
}

// sqrt(q) for q >= 0 from the hardware reciprocal-square-root estimate and
// two Newton steps on 1/sqrt (within an ulp or two); 0 for q = 0.
__device__ __forceinline__ double sqrt_fast(double q) {
    double y = __builtin_amdgcn_rsq(q);
    y = y * fma(-0.5 * q * y, y, 1.5);
    y = y * fma(-0.5 * q * y, y, 1.5);
    return q > 0.0 ? q * y : 0.0;
}

// atan t for |t| <= 1: two half-angle reductions, atan t = 2 atan(t / (1 +
// sqrt(1 + t^2))), bring |t| below tan(pi/16) = 0.199, where the Taylor
// series through t^23 is exact to < 1e-18.
__device__ __forceinline__ double atan_unit(double t) {
    t = t / (1.0 + sqrt(fma(t, t, 1.0)));
    t = t / (1.0 + sqrt(fma(t, t, 1.0)));
    const double t2 = t * t;
    double p = -1.0 / 23;
    p = fma(p, t2, 1.0 / 21);
    p = fma(p, t2, -1.0 / 19);
    p = fma(p, t2, 1.0 / 17);
    p = fma(p, t2, -1.0 / 15);
    p = fma(p, t2, 1.0 / 13);
    p = fma(p, t2, -1.0 / 11);
    p = fma(p, t2, 1.0 / 9);
    p = fma(p, t2, -1.0 / 7);
    p = fma(p, t2, 1.0 / 5);
    p = fma(p, t2, -1.0 / 3);
    return 4.0 * fma(p * t2, t, t);
}

// atan2(y, x) for y >= 0 (an angle in [0, pi]).
__device__ __forceinline__ double atan2_upper(double y, double x) {
    constexpr double PI = 3.14159265358979323846, HALF_PI = 1.57079632679489661923;
    if (x >= y) return atan_unit(y / x);
    if (x >= -y) return HALF_PI - atan_unit(x / y);
    return PI + atan_unit(y / x);
}

// Coefficient k of the series asin x = sum_k c_k x^(2k+1),
// c_k = (2k)! / (4^k (k!)^2 (2k+1)), from c_0 = 1 and
// c_k = c_(k-1) (2k-1)^2 / ((2k)(2k+1)).
constexpr double asin_coef(int k) {
    double c = 1.0;
    for (int j = 1; j <= k; ++j) c *= static_cast<double>((2 * j - 1) * (2 * j - 1)) / ((2.0 * j) * (2.0 * j + 1));
    return c;
}

// asin x for 0 <= x <= 1/16 from the series through x^13 (truncation below
// 2e-19 relative).
__device__ __forceinline__ double asin_small(double x) {
    constexpr double C1 = asin_coef(1), C2 = asin_coef(2), C3 = asin_coef(3), C4 = asin_coef(4),
                     C5 = asin_coef(5), C6 = asin_coef(6);
    const double x2 = x * x;
    double p = C6;
    p = fma(p, x2, C5);
    p = fma(p, x2, C4);
    p = fma(p, x2, C3);
    p = fma(p, x2, C2);
    p = fma(p, x2, C1);
    return fma(p * x2, x, x);
}

// ---------------------------------------------------------------------------
// Per-launch and per-ray constants
// ---------------------------------------------------------------------------

struct Spacetime {
    double M, a, a2, two_a2;
};

struct RayConst {
    double E, L;    // -p_t, p_phi
    double aE, aL;  // a E, a L
    double twoE;    // 2 E
    double Wc;      // a^2 E - a L, so that W = (r^2 + a^2) E - a L = r^2 E + Wc
};

__device__ __forceinline__ RayConst make_ray_const(const Spacetime& st, double E, double L) {
    RayConst rc;
    rc.E = E;
    rc.L = L;
    rc.aE = st.a * E;
    rc.aL = st.a * L;
    rc.twoE = 2.0 * E;
    rc.Wc = fma(st.a2, E, -rc.aL);
    return rc;
}

// By-products of an RHS evaluation used at accepted states.
struct Diag {
    double H;       // Hamiltonian
    double Kabs;    // |2 Sigma H| (|2H| for the q-metric)
    double D;       // the sum of the magnitudes of its terms: |H|_rel = Kabs / D
    double s, c;    // sin, cos of theta
    __device__ double rel() const { return Kabs * rcp(D); }
};

// ---------------------------------------------------------------------------
// Hamilton's equations in Carter's separated form.
//   2 Sigma H = K = Delta p_r^2 + p_th^2 + T^2 - W^2/Delta,
//   T = L/sin - a E sin,  W = (r^2 + a^2) E - a L.
// State z = (r, theta, phi, p_r, p_theta); dz = (dH/dp_r, dH/dp_th, dH/dL,
// -dH/dr, -dH/dtheta), with the exact -H dSigma/Sigma terms kept so the flow
// is the Hamiltonian flow of H itself (H is then conserved to truncation).
// S_TIME scales the field by d(lambda)/ds = Delta/r.
// ---------------------------------------------------------------------------
template <bool WANT_DIAG, bool S_TIME>
__device__ __forceinline__ void rhs_sc(const Spacetime& st, const RayConst& rc, const double z[5], double s,
                                       double c, double dz[5], Diag* dg) {
    const double r = z[0], pr = z[3], pth = z[4];
    const double r2 = r * r;
    const double Sig = fma(st.a2 * c, c, r2);
    const double Del = fma(r, r - 2.0 * st.M, st.a2);
    // 1/sin, 1/Sigma, 1/Delta (and 1/r for the s-time scaling) from one
    // reciprocal of their product
    const double SD = Sig * Del;
    const double P = S_TIME ? SD * s * r : SD * s;
    const double q = rcp(P);
    const double inv_s = S_TIME ? SD * r * q : SD * q;
    const double inv_SD = S_TIME ? s * r * q : s * q;
    const double inv_Sig = Del * inv_SD;
    const double inv_Del = Sig * inv_SD;
    const double W = fma(r2, rc.E, rc.Wc);
    const double T = fma(rc.L, inv_s, -rc.aE * s);
    const double Wd = W * inv_Del;
    const double pr2 = pr * pr;
    const double WWd = W * Wd;
    const double K = fma(Del, pr2, fma(pth, pth, fma(T, T, -WWd)));
    const double H2 = K * inv_Sig;  // 2H
    // (1/2) d K / d r = (r - M) (p_r^2 + Wd^2) - 2 r E Wd
    const double hdK = fma(r - st.M, fma(Wd, Wd, pr2), -(rc.twoE * r) * Wd);
    // d T / d theta = -cos Q, Q = L / sin^2 + a E
    const double Q = fma(rc.L, inv_s * inv_s, rc.aE);
    double d0 = Del * pr * inv_Sig;
    double d1 = pth * inv_Sig;
    double d2 = fma(T, inv_s, st.a * Wd) * inv_Sig;
    // -dH/dr = (2 r H - (1/2) dK/dr) / Sigma;  -dH/dtheta = cos (T Q - a^2 sin 2H) / Sigma
    double d3 = fma(r, H2, -hdK) * inv_Sig;
    double d4 = (c * inv_Sig) * fma(T, Q, -(st.a2 * H2) * s);
    if (S_TIME) {
        const double w = Del * (s * SD * q);  // Delta / r
        d0 *= w;
        d1 *= w;
        d2 *= w;
        d3 *= w;
        d4 *= w;
    }
    dz[0] = d0;
    dz[1] = d1;
    dz[2] = d2;
    dz[3] = d3;
    dz[4] = d4;
    if (WANT_DIAG) {
        const double D = fma(Del, pr2, fma(pth, pth, fma(T, T, WWd)));
        dg->H = 0.5 * H2;
        dg->Kabs = fabs(K);
        dg->D = D;
        dg->s = s;
        dg->c = c;
    }
}

// The RHS at z with sin/cos of theta computed from theta itself.
// ---------------------------------------------------------------------------
// The q-metric of the appendix (eq:q-metric, signature (-,+,+,+)): static and
// diagonal, with f = 1 - 2M/r, D = 1 + M^2 sin^2 / (r^2 f), P = q (2 + q),
//   g^tt = -f^-(1+q), g^rr = f^(1+q) D^P, g^thth = f^q D^P / r^2,
//   g^phph = f^q / (r^2 sin^2).
// H = (-E^2 G + p_r^2 A + p_th^2 B + L^2 C) / 2 with those magnitudes, and
// each term's r- and theta-derivative is the term times the log-derivative
// of its factor.
// ---------------------------------------------------------------------------
struct QSpacetime {
    double M, q, P;
};

__device__ __forceinline__ RayConst make_ray_const(const QSpacetime&, double E, double L) {
    RayConst rc;
    rc.E = E;
    rc.L = L;
    rc.aE = 0.0;
    rc.aL = 0.0;
    rc.twoE = 2.0 * E;
    rc.Wc = 0.0;
    return rc;
}

// e^x for |x| < ~700: x = n ln 2 + t with |t| <= (ln 2)/2 (Cody-Waite with a
// two-part ln 2), e^t = 1 + t + t^2 G(t) with G a degree-9 minimax polynomial
// (coefficients from minimax_coefs.py; relative error below 1e-17 with the
// coefficients rounded to double, where Taylor's series needs through t^13),
// scaled by 2^n.  About 1 ulp.
__device__ __forceinline__ double exp_fast(double x) {
    constexpr double LOG2E = 1.4426950408889634074;
    constexpr double LN2_HI = 6.93147180369123816490e-01;  // 32 significant bits
    constexpr double LN2_LO = 1.90821492927058770002e-10;
    const double n = __builtin_rint(x * LOG2E);
    const double t = fma(-n, LN2_LO, fma(-n, LN2_HI, x));
    double p = 2.511003970895208e-08;
    p = fma(p, t, 2.763264062648625e-07);
    p = fma(p, t, 2.755724236405712e-06);
    p = fma(p, t, 2.4801487366143253e-05);
    p = fma(p, t, 0.00019841269886566477);
    p = fma(p, t, 0.001388888894778543);
    p = fma(p, t, 0.008333333333322215);
    p = fma(p, t, 0.041666666666522106);
    p = fma(p, t, 0.16666666666666674);
    p = fma(p, t, 0.500000000000001);
    p = fma(p, t, 1.0);  // 1 + t G
    p = fma(p, t, 1.0);  // 1 + t + t^2 G
    return __builtin_amdgcn_ldexp(p, static_cast<int>(n));
}

// ln x = e ln 2 + ln m for x = 2^e m, m in [1/sqrt 2, sqrt 2), and
// ln m = 2 atanh s = 2 s + 2 s s^2 L(s^2) with s = (m - 1)/(m + 1),
// |s| <= 0.172, L a degree-6 minimax polynomial (coefficients from
// minimax_coefs.py; relative error below 2e-18 with the coefficients rounded
// to double, where the atanh series needs through s^21).  log_split takes x
// apart; log_join adds the pieces once the caller has s (so that several
// logarithms can share one reciprocal).  NaN for x <= 0.
struct LogSplit {
    double x, m, e;
};

__device__ __forceinline__ LogSplit log_split(double x) {
    double m = __builtin_amdgcn_frexp_mant(x);  // [1/2, 1)
    int e = __builtin_amdgcn_frexp_exp(x);
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    return LogSplit{x, m, static_cast<double>(e)};
}

__device__ __forceinline__ double log_join(const LogSplit& ls, double s) {
    constexpr double LN2_HI = 6.93147180369123816490e-01;
    constexpr double LN2_LO = 1.90821492927058770002e-10;
    const double s2 = s * s;
    double p = 0.07397974873252054;
    p = fma(p, s2, 0.07657025269735923);
    p = fma(p, s2, 0.09091782163503512);
    p = fma(p, s2, 0.11111099286578859);
    p = fma(p, s2, 0.14285714371194005);
    p = fma(p, s2, 0.19999999999707338);
    p = fma(p, s2, 0.3333333333333367);
    const double lm = fma((2.0 * s) * s2, p, 2.0 * s);
    const double r = fma(ls.e, LN2_HI, fma(ls.e, LN2_LO, lm));
    return ls.x > 0.0 ? r : __builtin_nan("");
}

__device__ __forceinline__ double log_fast(double x) {
    const LogSplit ls = log_split(x);
    return log_join(ls, (ls.m - 1.0) * rcp(ls.m + 1.0));
}

template <bool WANT_DIAG>
__device__ __forceinline__ void rhs_q(const QSpacetime& st, const RayConst& rc, const double z[5], double s,
                                      double c, double dz[5], Diag* dg) {
    const double r = z[0], pr = z[3], pth = z[4], M = st.M;
    const double rf = r * (r - 2.0 * M);  // r^2 f
    // 1/r, 1/(r^2 f) and 1/sin from one reciprocal of their product
    const double X = r * rf;
    const double qX = rcp(X * s);
    const double ir = rf * s * qX;
    const double irf = r * s * qX;
    const double is = X * qX;
    const double f = rf * ir * ir;
    const double Dm1 = (M * M) * (s * s) * irf;  // D - 1
    const double D = 1.0 + Dm1;
    // ln f, ln D and 1/D with one reciprocal: that of (m_f + 1)(m_D + 1) D,
    // m_f and m_D the logarithms' mantissas
    const LogSplit sf = log_split(f), sd = log_split(D);
    const double af = sf.m + 1.0, ad = sd.m + 1.0;
    const double afad = af * ad;
    const double q3 = rcp(afad * D);
    const double iD = afad * q3;
    const double qD = D * q3;  // 1 / ((m_f + 1)(m_D + 1))
    const double lf = log_join(sf, (sf.m - 1.0) * (ad * qD));
    const double fq = exp_fast(st.q * lf);                                // f^q
    const double DP = exp_fast(st.P * log_join(sd, (sd.m - 1.0) * (af * qD)));  // D^P
    const double ir2 = ir * ir;
    const double A = f * fq * DP;
    const double B = fq * DP * ir2;
    const double C = fq * ir2 * is * is;
    const double G = rcp(f * fq);
    const double tG = rc.E * rc.E * G, tA = pr * pr * A, tB = pth * pth * B, tC = rc.L * rc.L * C;
    const double lf_r = 2.0 * M * irf;                          // d ln f / dr
    const double PlD_r = -st.P * Dm1 * (2.0 * (r - M)) * irf * iD;  // P d ln D / dr
    const double PlD_th = 2.0 * st.P * Dm1 * c * is * iD;          // P d ln D / dtheta
    const double tAB = tA + tB, tBC = tB + tC;
    // 2 dH/dr and 2 dH/dtheta
    const double Hr2 = fma((1.0 + st.q) * lf_r, tG + tA, fma(st.q * lf_r, tBC, fma(PlD_r, tAB, -2.0 * ir * tBC)));
    const double Hth2 = fma(PlD_th, tAB, -2.0 * c * is * tC);
    dz[0] = A * pr;
    dz[1] = B * pth;
    dz[2] = C * rc.L;
    dz[3] = -0.5 * Hr2;
    dz[4] = -0.5 * Hth2;
    if (WANT_DIAG) {
        const double K = (tA - tG) + (tB + tC);
        dg->H = 0.5 * K;
        dg->Kabs = fabs(K);
        dg->D = tG + tA + tB + tC;
        dg->s = s;
        dg->c = c;
    }
}

// The RHS of either spacetime at z, given sin/cos of theta.
template <bool WANT_DIAG>
__device__ __forceinline__ void field_at(const Spacetime& st, const RayConst& rc, const double z[5], double s,
                                         double c, double dz[5], Diag* dg) {
    rhs_sc<WANT_DIAG, false>(st, rc, z, s, c, dz, dg);
}
template <bool WANT_DIAG>
__device__ __forceinline__ void field_at(const QSpacetime& st, const RayConst& rc, const double z[5], double s,
                                         double c, double dz[5], Diag* dg) {
    rhs_q<WANT_DIAG>(st, rc, z, s, c, dz, dg);
}

template <bool WANT_DIAG, bool S_TIME, class ST>
__device__ __forceinline__ void rhs(const ST& st, const RayConst& rc, const double z[5], double dz[5], Diag* dg) {
    double s, c;
    sincos_theta(z[1], &s, &c);
    if constexpr (S_TIME)
        rhs_sc<WANT_DIAG, true>(st, rc, z, s, c, dz, dg);
    else
        field_at<WANT_DIAG>(st, rc, z, s, c, dz, dg);
}

// sin and cos of theta0 + d from those of theta0 by angle addition, with
// sin d = d - d x S(x) and cos d - 1 = -x C(x), x = d^2, where S and C are
// minimax polynomials for |d| <= 1/2 (degrees 4 and 5, coefficients from
// minimax_coefs.py).  With the coefficients rounded to double the relative
// error of sin d stays below 2.6e-17 and the absolute error of cos d below
// 6e-18 there, within a quarter ulp, as Taylor's series does with one more
// term each.  That range covers the angle change between a step's start and
// any of its stages: accepted steps of the embedded pairs change theta by at
// most 0.045 rad on the 1024^2 image and 0.10 rad over random images at rtol
// down to 1e-10.  Beyond it the error grows like d^13 (2e-14 relative at
// |d| = 0.6, 8e-11 at 1) for the wild stages of steps that get rejected.
__device__ __forceinline__ void sincos_shift(double s0, double c0, double d, double* s_out, double* c_out) {
    const double d2 = d * d;
    double ps = 2.49340193295306e-08;
    ps = fma(ps, d2, -2.7556995708658808e-06);
    ps = fma(ps, d2, 0.00019841269438799643);
    ps = fma(ps, d2, -0.008333333333114794);
    ps = fma(ps, d2, 0.1666666666666628);
    const double sd = fma(-ps * d2, d, d);  // sin d
    double pc = -2.0777882749707575e-09;
    pc = fma(pc, d2, 2.755698550128358e-07);
    pc = fma(pc, d2, -2.480158674730891e-05);
    pc = fma(pc, d2, 0.0013888888888423405);
    pc = fma(pc, d2, -0.04166666666666487);
    pc = fma(pc, d2, 0.5);
    const double cdm1 = -pc * d2;  // cos d - 1
    *s_out = fma(s0, cdm1, fma(c0, sd, s0));
    *c_out = fma(c0, cdm1, fma(-s0, sd, c0));
}

// ---------------------------------------------------------------------------
// Split form for the mixed-precision policy: H = H0 + HM with
//   H0 = 1/2 [-E^2 + (rho2 p_r^2 + p_th^2)/Sigma + L^2/(rho2 sin^2)]   (M = 0 part)
//   HM = -(M r / Sigma) [W^2 / (rho2 Delta) + p_r^2]                    (mass part)
// (rho2 = r^2 + a^2; H0 + HM equals the Carter form identically).  The flow
// of H0 is evaluated in FP64 and that of HM in FP32; HM carries a factor
// M/r, so its FP32 rounding is small where r is large.  With WANT_DIAG the
// constraint diagnostics are computed from the full Carter form in FP64.
// ---------------------------------------------------------------------------
struct Spacetime32 {
    float M, a, a2;
};

template <bool WANT_DIAG>
__device__ __forceinline__ void rhs_split(const Spacetime& st, const Spacetime32& sf, const RayConst& rc,
                                          const double z[5], double s, double c, double dz[5], Diag* dg) {
    const double r = z[0], pr = z[3], pth = z[4];
    const double r2 = r * r;
    const double rho2 = r2 + st.a2;
    const double Sig = fma(st.a2 * c, c, r2);
    // 1/sin, 1/Sigma, 1/rho2 from one reciprocal of the product
    const double SR = Sig * rho2;
    const double q = rcp(SR * s);
    const double inv_s = SR * q;
    const double inv_SR = s * q;
    const double inv_Sig = rho2 * inv_SR;
    const double inv_rho2 = Sig * inv_SR;
    const double pr2 = pr * pr;
    const double A = fma(rho2, pr2, pth * pth);
    const double inv_s2 = inv_s * inv_s;
    const double L2r = rc.L * rc.L * inv_rho2 * inv_s2;  // L^2 / (rho2 sin^2)
    const double AS2 = A * inv_Sig * inv_Sig;            // A / Sigma^2
    double d0 = rho2 * pr * inv_Sig;
    double d1 = pth * inv_Sig;
    double d2 = rc.L * inv_rho2 * inv_s2;
    double d3 = r * (AS2 - pr2 * inv_Sig + L2r * inv_rho2);
    double d4 = c * (L2r * inv_s - st.a2 * s * AS2);

    // mass part in FP32
    const float rf = static_cast<float>(r), sfl = static_cast<float>(s), cf = static_cast<float>(c);
    const float prf = static_cast<float>(pr), Ef = static_cast<float>(rc.E), Lf = static_cast<float>(rc.L);
    const float rho2f = rf * rf + sf.a2;
    const float Sigf = fmaf(sf.a2 * cf, cf, rf * rf);
    const float Delf = fmaf(rf, rf - 2.0f * sf.M, sf.a2);
    const float inv_Sigf = __builtin_amdgcn_rcpf(Sigf);
    const float inv_RDf = __builtin_amdgcn_rcpf(rho2f * Delf);
    const float Wf = fmaf(rho2f, Ef, -sf.a * Lf);
    const float WR = Wf * inv_RDf;                        // W / (rho2 Delta)
    const float G = fmaf(Wf, WR, prf * prf);              // W^2/(rho2 Delta) + p_r^2
    const float qm = sf.M * rf * inv_Sigf;                // M r / Sigma
    // d G / d r = 4 r E W/(rho2 Delta) - W^2 (2 r Delta + 2 rho2 (r - M)) / (rho2 Delta)^2
    const float dG = fmaf(4.0f * rf * Ef, WR, -WR * WR * 2.0f * fmaf(rf, Delf, rho2f * (rf - sf.M)));
    const float m0 = -2.0f * qm * prf;
    const float m2 = 2.0f * sf.a * qm * WR;
    const float m3 = fmaf(sf.M * inv_Sigf * G, fmaf(-2.0f * rf * rf, inv_Sigf, 1.0f), qm * dG);
    const float m4 = 2.0f * sf.a2 * sfl * cf * qm * G * inv_Sigf;
    dz[0] = d0 + static_cast<double>(m0);
    dz[1] = d1;
    dz[2] = d2 + static_cast<double>(m2);
    dz[3] = d3 + static_cast<double>(m3);
    dz[4] = d4 + static_cast<double>(m4);
    if (WANT_DIAG) {
        const double Del = fma(r, r - 2.0 * st.M, st.a2);
        const double W = fma(rho2, rc.E, -rc.aL);
        const double T = fma(rc.L, inv_s, -rc.aE * s);
        const double WWd = W * W * rcp(Del);
        const double K = fma(Del, pr2, fma(pth, pth, fma(T, T, -WWd)));
        const double D = fma(Del, pr2, fma(pth, pth, fma(T, T, WWd)));
        dg->H = 0.5 * K * inv_Sig;
        dg->Kabs = fabs(K);
        dg->D = D;
        dg->s = s;
        dg->c = c;
    }
}

// The right-hand side of the stepper: Carter form in FP64, or the split form.
// at stage state z.  Inner stages take sin/cos of theta from those (s0, c0)
// at the step's start angle th0; the last stage (D: the step's end, whose
// sin/cos seed the next step) computes them from theta itself, so the
// shifts never accumulate.
template <bool SPLIT, bool D, class ST>
__device__ __forceinline__ void eval_rhs(const ST& st, const Spacetime32* sf, const RayConst& rc,
                                         const double* z, double th0, double s0, double c0, double* out,
                                         Diag* dg) {
    double s, c;
    if constexpr (D)
        sincos_theta(z[1], &s, &c);
    else
        sincos_shift(s0, c0, z[1] - th0, &s, &c);
    if constexpr (SPLIT)
        rhs_split<D>(st, *sf, rc, z, s, c, out, dg);
    else
        field_at<D>(st, rc, z, s, c, out, dg);
}

// ---------------------------------------------------------------------------
// Dormand & Prince (1980) RK5(4)7M, first-same-as-last.
// ---------------------------------------------------------------------------
namespace dp {
constexpr double A21 = 1.0 / 5;
constexpr double A31 = 3.0 / 40, A32 = 9.0 / 40;
constexpr double A41 = 44.0 / 45, A42 = -56.0 / 15, A43 = 32.0 / 9;
constexpr double A51 = 19372.0 / 6561, A52 = -25360.0 / 2187, A53 = 64448.0 / 6561,
                 A54 = -212.0 / 729;
constexpr double A61 = 9017.0 / 3168, A62 = -355.0 / 33, A63 = 46732.0 / 5247, A64 = 49.0 / 176,
                 A65 = -5103.0 / 18656;
// 5th-order weights; the 7th stage is evaluated at the 5th-order solution.
constexpr double B1 = 35.0 / 384, B3 = 500.0 / 1113, B4 = 125.0 / 192, B5 = -2187.0 / 6784,
                 B6 = 11.0 / 84;
// error weights: 5th-order minus embedded 4th-order weights
constexpr double E1 = 71.0 / 57600, E3 = -71.0 / 16695, E4 = 71.0 / 1920,
                 E5 = -17253.0 / 339200, E6 = 22.0 / 525, E7 = -1.0 / 40;
}  // namespace dp

// One DP5(4) step of size h from y with k1 = f(y).  Writes the 5th-order
// solution yn, kn = f(yn) with its diagnostics, and the error vector err.
// Six RHS evaluations.
// (s0, c0) are sin and cos of y[1].
template <bool SPLIT = false, class ST = Spacetime>
__device__ __forceinline__ void dp45_step(const ST& st, const RayConst& rc, const double y[5],
                                          const double k1[5], double s0, double c0, double h, double yn[5],
                                          double kn[5], double err[5], Diag* dg,
                                          const Spacetime32* sf = nullptr) {
    using namespace dp;
    double k2[5], k3[5], k4[5], k5[5], k6[5], ys[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) ys[i] = fma(h, A21 * k1[i], y[i]);
    eval_rhs<SPLIT, false>(st, sf, rc, ys, y[1], s0, c0, k2, dg);
#pragma unroll
    for (int i = 0; i < 5; ++i) ys[i] = fma(h, fma(A31, k1[i], A32 * k2[i]), y[i]);
    eval_rhs<SPLIT, false>(st, sf, rc, ys, y[1], s0, c0, k3, dg);
#pragma unroll
    for (int i = 0; i < 5; ++i) ys[i] = fma(h, fma(A41, k1[i], fma(A42, k2[i], A43 * k3[i])), y[i]);
    eval_rhs<SPLIT, false>(st, sf, rc, ys, y[1], s0, c0, k4, dg);
#pragma unroll
    for (int i = 0; i < 5; ++i)
        ys[i] = fma(h, fma(A51, k1[i], fma(A52, k2[i], fma(A53, k3[i], A54 * k4[i]))), y[i]);
    eval_rhs<SPLIT, false>(st, sf, rc, ys, y[1], s0, c0, k5, dg);
#pragma unroll
    for (int i = 0; i < 5; ++i)
        ys[i] = fma(h, fma(A61, k1[i], fma(A62, k2[i], fma(A63, k3[i], fma(A64, k4[i], A65 * k5[i])))),
                    y[i]);
    eval_rhs<SPLIT, false>(st, sf, rc, ys, y[1], s0, c0, k6, dg);
    // error partial sums before stage 7 so that k3..k6 are dead across it
    double ep[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        yn[i] = fma(h, fma(B1, k1[i], fma(B3, k3[i], fma(B4, k4[i], fma(B5, k5[i], B6 * k6[i])))), y[i]);
        ep[i] = fma(E1, k1[i], fma(E3, k3[i], fma(E4, k4[i], fma(E5, k5[i], E6 * k6[i]))));
    }
    eval_rhs<SPLIT, true>(st, sf, rc, yn, y[1], s0, c0, kn, dg);
#pragma unroll
    for (int i = 0; i < 5; ++i) err[i] = h * fma(E7, kn[i], ep[i]);
}

// ---------------------------------------------------------------------------
// Six-stage embedded pairs without FSAL, compared with DP5(4) in Sect. 3.1.
// a(i, j): stage rows; b(j): weights of the propagated solution; e(j):
// propagated minus embedded weights (the error estimate's weights).
// ---------------------------------------------------------------------------
// Fehlberg (1969) RK4(5): the 4th-order solution is propagated.
struct Fehlberg45 {
    static constexpr double a(int i, int j) {
        constexpr double t[6][5] = {{0, 0, 0, 0, 0},
                                    {1.0 / 4, 0, 0, 0, 0},
                                    {3.0 / 32, 9.0 / 32, 0, 0, 0},
                                    {1932.0 / 2197, -7200.0 / 2197, 7296.0 / 2197, 0, 0},
                                    {439.0 / 216, -8.0, 3680.0 / 513, -845.0 / 4104, 0},
                                    {-8.0 / 27, 2.0, -3544.0 / 2565, 1859.0 / 4104, -11.0 / 40}};
        return t[i][j];
    }
    static constexpr double b(int j) {
        constexpr double t[6] = {25.0 / 216, 0, 1408.0 / 2565, 2197.0 / 4104, -1.0 / 5, 0};
        return t[j];
    }
    static constexpr double e(int j) {
        constexpr double t[6] = {25.0 / 216 - 16.0 / 135, 0, 1408.0 / 2565 - 6656.0 / 12825,
                                 2197.0 / 4104 - 28561.0 / 56430, -1.0 / 5 + 9.0 / 50, -2.0 / 55};
        return t[j];
    }
};

// Cash & Karp (1990) RK5(4): the 5th-order solution is propagated.
struct CashKarp45 {
    static constexpr double a(int i, int j) {
        constexpr double t[6][5] = {{0, 0, 0, 0, 0},
                                    {1.0 / 5, 0, 0, 0, 0},
                                    {3.0 / 40, 9.0 / 40, 0, 0, 0},
                                    {3.0 / 10, -9.0 / 10, 6.0 / 5, 0, 0},
                                    {-11.0 / 54, 5.0 / 2, -70.0 / 27, 35.0 / 27, 0},
                                    {1631.0 / 55296, 175.0 / 512, 575.0 / 13824, 44275.0 / 110592,
                                     253.0 / 4096}};
        return t[i][j];
    }
    static constexpr double b(int j) {
        constexpr double t[6] = {37.0 / 378, 0, 250.0 / 621, 125.0 / 594, 0, 512.0 / 1771};
        return t[j];
    }
    static constexpr double e(int j) {
        constexpr double t[6] = {37.0 / 378 - 2825.0 / 27648, 0, 250.0 / 621 - 18575.0 / 48384,
                                 125.0 / 594 - 13525.0 / 55296, -277.0 / 14336, 512.0 / 1771 - 1.0 / 4};
        return t[j];
    }
};

// One step of a six-stage pair of size h from y with k1 = f(y): the
// propagated solution yn, kn = f(yn) with its diagnostics, and err = h sum
// e_j k_j.  Inner stages take sin/cos of theta by angle addition from
// (s0, c0); f(yn) computes them from theta.  Six RHS evaluations.
template <class TAB, class ST>
__device__ __forceinline__ void erk6_step(const ST& st, const RayConst& rc, const double y[5],
                                          const double k1[5], double s0, double c0, double h, double yn[5],
                                          double kn[5], double err[5], Diag* dg) {
    double k[6][5];
#pragma unroll
    for (int i = 0; i < 5; ++i) k[0][i] = k1[i];
#pragma unroll
    for (int stg = 1; stg < 6; ++stg) {
        double ys[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            double acc = TAB::a(stg, 0) * k[0][i];
#pragma unroll
            for (int j = 1; j < stg; ++j)
                if (TAB::a(stg, j) != 0.0) acc = fma(TAB::a(stg, j), k[j][i], acc);
            ys[i] = fma(h, acc, y[i]);
        }
        eval_rhs<false, false>(st, nullptr, rc, ys, y[1], s0, c0, k[stg], dg);
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        double acc = 0.0, ea = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            if (TAB::b(j) != 0.0) acc = fma(TAB::b(j), k[j][i], acc);
            if (TAB::e(j) != 0.0) ea = fma(TAB::e(j), k[j][i], ea);
        }
        yn[i] = fma(h, acc, y[i]);
        err[i] = h * ea;
    }
    eval_rhs<false, true>(st, nullptr, rc, yn, y[1], s0, c0, kn, dg);
}

// ---------------------------------------------------------------------------
// Bulirsch-Stoer extrapolation (the third scheme of Sect. 3.1).  For
// k = 1..BS_COLUMNS the modified midpoint chain with n_k = 2k substeps
// across [0, h] starts from y; its end is extrapolated to zero substep size
// with the earlier chains' ends, in x = (1/n_k)^2, one tableau row at a time
// kept in place: by Aitken-Neville polynomials, or (RATIONAL) by Stoer and
// Bulirsch's recursion for rational functions,
//   T[k][j] = T[k][j-1] + d / (rho (1 - d / (T[k][j-1] - T[k-1][j-2])) - 1),
//   d = T[k][j-1] - T[k-1][j-1],  rho = (n_k / n_(k-j))^2,  T[k-1][-1] = 0,
// with no correction where a denominator vanishes.  The last diagonal entry
// (order 2K) is the step's result; the error vector is its difference to the
// entry before it.  Chains span the whole step, so every evaluation takes
// sin/cos of theta from theta itself.  K^2 + 1 RHS evaluations.
// ---------------------------------------------------------------------------
constexpr int BS_COLUMNS = 5;

// (n_k / n_(k-j))^2 with n = 2k, k = 1..BS_COLUMNS (as indices k, j from 0),
// and the Aitken-Neville weight 1 / (that - 1).
constexpr double bs_ratio2(int k, int j) {
    return static_cast<double>((k + 1) * (k + 1)) / static_cast<double>((k - j + 1) * (k - j + 1));
}
constexpr double bs_weight(int k, int j) { return 1.0 / (bs_ratio2(k, j) - 1.0); }

template <bool RATIONAL = false, class ST>
__device__ __forceinline__ void bs_step(const ST& st, const RayConst& rc, const double y[5],
                                        const double k1[5], double h, double yn[5], double kn[5],
                                        double err[5], Diag* dg) {
    double T[BS_COLUMNS][5];  // row k of the tableau after chain k
#pragma unroll
    for (int k = 0; k < BS_COLUMNS; ++k) {
        const int ns = 2 * (k + 1);
        const double hs = h * (1.0 / ns);
        const double h2 = 2.0 * hs;
        double zp[5], zc[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            zp[i] = y[i];
            zc[i] = fma(hs, k1[i], y[i]);
        }
#pragma unroll 1
        for (int m = 1; m < ns; ++m) {
            double fz[5];
            rhs<false, false>(st, rc, zc, fz, nullptr);
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                const double zn = fma(h2, fz[i], zp[i]);
                zp[i] = zc[i];
                zc[i] = zn;
            }
        }
        // row k from row k - 1, in place: `carry` is T[k][j-1], `below` the
        // overwritten T[k-1][j-2]
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            double carry = zc[i];
            double below = 0.0;
#pragma unroll
            for (int j = 1; j <= k; ++j) {
                const double old = T[j - 1][i];
                T[j - 1][i] = carry;
                const double d = carry - old;
                if constexpr (RATIONAL) {
                    const double din = carry - below;
                    const double den = fma(bs_ratio2(k, j), fma(-d, rcp(din), 1.0), -1.0);
                    const double upd = d * rcp(den);
                    carry = (din != 0.0 && den != 0.0) ? carry + upd : carry;
                    below = old;
                } else {
                    carry = fma(d, bs_weight(k, j), carry);
                }
            }
            T[k][i] = carry;
        }
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        yn[i] = T[BS_COLUMNS - 1][i];
        err[i] = T[BS_COLUMNS - 1][i] - T[BS_COLUMNS - 2][i];
    }
    rhs<true, false>(st, rc, yn, kn, dg);
}

// One classic RK4 step of size h (in s) from y with k1 = F(y), F the field
// scaled by Delta/r.  Writes yn and kn = F(yn) with diagnostics.  Four RHS
// evaluations.
__device__ __forceinline__ void rk4s_step(const Spacetime& st, const RayConst& rc, const double y[5],
                                          const double k1[5], double h, double yn[5], double kn[5],
                                          Diag* dg) {
    double k2[5], k3[5], k4[5], ys[5];
    const double hh = 0.5 * h;
#pragma unroll
    for (int i = 0; i < 5; ++i) ys[i] = fma(hh, k1[i], y[i]);
    rhs<false, true>(st, rc, ys, k2, nullptr);
#pragma unroll
    for (int i = 0; i < 5; ++i) ys[i] = fma(hh, k2[i], y[i]);
    rhs<false, true>(st, rc, ys, k3, nullptr);
#pragma unroll
    for (int i = 0; i < 5; ++i) ys[i] = fma(h, k3[i], y[i]);
    rhs<false, true>(st, rc, ys, k4, nullptr);
    const double h6 = h * (1.0 / 6.0);
#pragma unroll
    for (int i = 0; i < 5; ++i) yn[i] = fma(h6, k1[i] + 2.0 * (k2[i] + k3[i]) + k4[i], y[i]);
    rhs<true, true>(st, rc, yn, kn, dg);
}

}  // namespace kt
