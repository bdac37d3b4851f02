// kt_adjoint_math.h -- the pieces of the discrete adjoint that are pure
// arithmetic: the gradient of the Hamiltonian in all its arguments, the
// vector-Jacobian product of the RHS as a Hessian-vector product, one
// Dormand-Prince step as a map y -> y' with frozen step size and its
// vector-Jacobian product, and the disk observables with their derivatives.
// Host and device: the same templates serve a host-side self-check.
#pragma once

#include "kt_dual.h"
#include "kt_elem.h"

namespace kt {
namespace adj {

// sin and cos of theta from their values (sv, cv): for a dual theta the
// tangents follow from d sin = cos d theta, d cos = -sin d theta.
__host__ __device__ inline void sincos_from(const double&, double sv, double cv, double* s, double* c) {
    *s = sv;
    *c = cv;
}
template <int N>
__host__ __device__ inline void sincos_from(const Dual<N>& th, double sv, double cv, Dual<N>* s, Dual<N>* c) {
    *s = Dual<N>(sv);
    *c = Dual<N>(cv);
    for (int i = 0; i < N; ++i) {
        s->d[i] = cv * th.d[i];
        c->d[i] = -sv * th.d[i];
    }
}

// Gradient of H = K / (2 Sigma), K = Delta p_r^2 + p_th^2 + T^2 - W^2/Delta
// (Carter's separated form, T = L/sin - aE sin, W = (r^2 + a^2)E - aL), with
// respect to X = (r, theta, p_r, p_theta, L, E, a); M is a constant.  (sv, cv)
// are sin and cos of theta's value.  1/sin, 1/Sigma and 1/Delta come from one
// reciprocal of their product.  E and a are plain numbers: the dual form is
// only ever taken along directions in (r, theta, p_r, p_theta, L).
template <class T>
__host__ __device__ inline void grad_H(double M, const T& r, const T& th, const T& pr, const T& pth,
                                       const T& L, double E, double a, double sv, double cv, T g[7]) {
    T s, c;
    sincos_from(th, sv, cv, &s, &c);
    const T r2 = r * r;
    const double a2 = a * a;
    const T Sig = r2 + a2 * c * c;
    const T Del = r2 - 2.0 * M * r + a2;
    const T rho2 = r2 + a2;
    const T SD = Sig * Del;
    const T R = recip(SD * s);
    const T iS = Del * s * R, iD = Sig * s * R, is = SD * R;
    const T Lis = L * is;
    const T Tt = Lis - a * E * s;
    const T W = rho2 * E - a * L;
    const T pr2 = pr * pr;
    const T WiD = W * iD;
    const T K = Del * pr2 + pth * pth + Tt * Tt - W * WiD;
    const T H2 = K * iS;  // 2H
    const T rM2 = 2.0 * (r - M);
    const T Kr = rM2 * pr2 - 4.0 * r * E * WiD + WiD * WiD * rM2;
    const T Kth = -2.0 * Tt * c * (Lis * is + a * E);
    const T Ka = 2.0 * a * pr2 - 2.0 * Tt * E * s - 2.0 * WiD * (2.0 * a * E - L) + WiD * WiD * (2.0 * a);
    g[0] = 0.5 * (Kr - 2.0 * r * H2) * iS;
    g[1] = 0.5 * (Kth + 2.0 * a2 * s * c * H2) * iS;
    g[2] = Del * pr * iS;
    g[3] = pth * iS;
    g[4] = (Tt * is + a * WiD) * iS;
    g[5] = (-(a * s * Tt) - rho2 * WiD) * iS;
    g[6] = 0.5 * (Ka - 2.0 * a * c * c * H2) * iS;
}

// Hamilton's equations from the gradient: d/dlambda (r, th, phi, p_r, p_th).
// Returns sin and cos of theta (the trace kernel's own sincos_theta), which
// the step VJP reuses.
__host__ __device__ inline void field(double M, double a, double E, double L, const double z[5], double f[5],
                                      double* sv, double* cv) {
    sincos_theta(z[1], sv, cv);
    double g[7];
    grad_H<double>(M, z[0], z[1], z[3], z[4], L, E, a, *sv, *cv, g);
    f[0] = g[2];
    f[1] = g[3];
    f[2] = g[4];
    f[3] = -g[0];
    f[4] = -g[1];
}

// Parameter cotangents accumulated along a ray.
struct ParBar {
    double E, L, a;
};

// Vector-Jacobian product of the field at z: zbar += (df/dz)^T v and the
// parameter cotangents += (df/d(E, L, a))^T v.  The field is S grad H, so
// this is the Hessian-vector product of H along u = (-v_pr, -v_th, v_r, v_th,
// v_phi, 0, 0) in (r, th, p_r, p_th, L, E, a), taken by forward-mode duals
// on grad_H.
__host__ __device__ inline void field_vjp(double M, double a, double E, double L, const double z[5], double sv,
                                          double cv, const double v[5], double zbar[5], ParBar* pb) {
    using D = Dual<1>;
    D rr(z[0]), tt(z[1]), pp(z[3]), qq(z[4]), LL(L);
    rr.d[0] = -v[3];
    tt.d[0] = -v[4];
    pp.d[0] = v[0];
    qq.d[0] = v[1];
    LL.d[0] = v[2];
    D g[7];
    grad_H<D>(M, rr, tt, pp, qq, LL, E, a, sv, cv, g);
    zbar[0] += g[0].d[0];
    zbar[1] += g[1].d[0];
    zbar[3] += g[2].d[0];
    zbar[4] += g[3].d[0];
    pb->L += g[4].d[0];
    pb->E += g[5].d[0];
    pb->a += g[6].d[0];
}

// Dormand & Prince (1980) RK5(4)7M: the rows and 5th-order weights of the
// step map (the seventh stage only serves the error estimate and FSAL).
__host__ __device__ constexpr double dp_a(int i, int j) {
    constexpr double t[6][5] = {{0, 0, 0, 0, 0},
                                {1.0 / 5, 0, 0, 0, 0},
                                {3.0 / 40, 9.0 / 40, 0, 0, 0},
                                {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0},
                                {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0},
                                {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656}};
    return t[i][j];
}
__host__ __device__ constexpr double dp_b(int j) {
    constexpr double t[6] = {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84};
    return t[j];
}

// Vector-Jacobian product of one step with frozen h: given ybar at the
// step's end, returns ybar at its start (in place) and accumulates the
// parameter cotangents.  The stage states are rebuilt from y (the step's
// end value itself is not needed, so the last stage's field is skipped).
// Every loop is unrolled so that the stage arrays stay in registers: with
// run-time indices they would live in scratch memory, at half the speed.
__host__ __device__ inline void dp_step_vjp(double M, double a, double E, double L, const double y[5], double h,
                                            double ybar[5], ParBar* pb) {
    double Y[6][5], K[5][5], S[6], C[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l < j; ++l) acc += dp_a(j, l) * K[l][i];
            Y[j][i] = y[i] + h * acc;
        }
        if (j < 5)
            field(M, a, E, L, Y[j], K[j], &S[j], &C[j]);
        else
            sincos_theta(Y[j][1], &S[j], &C[j]);
    }
    double kb[6][5];
#pragma unroll
    for (int j = 0; j < 6; ++j)
#pragma unroll
        for (int i = 0; i < 5; ++i) kb[j][i] = h * dp_b(j) * ybar[i];
#pragma unroll
    for (int j = 5; j >= 0; --j) {
        double Yb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        field_vjp(M, a, E, L, Y[j], S[j], C[j], kb[j], Yb, pb);
#pragma unroll
        for (int i = 0; i < 5; ++i) ybar[i] += Yb[i];
#pragma unroll
        for (int l = 0; l < j; ++l)
#pragma unroll
            for (int i = 0; i < 5; ++i) kb[l][i] += h * dp_a(j, l) * Yb[i];
    }
}

// Observed intensity of a disk hit at radius r for a ray with constants
// (E, L), spin a and inner edge r_in (Keplerian rotation, or constant l0),
// as a dual number in (r, E, L, a, r_in).
struct DiskModel {
    double M, r_out, emis_q, l0;
    int rotation, emis_model;
};

__host__ __device__ inline Dual<5> disk_intensity(const DiskModel& dm, double r_, double E_, double L_, double a_,
                                                  double rin_) {
    using D = Dual<5>;
    const D r = D::var(r_, 0), E = D::var(E_, 1), L = D::var(L_, 2), a = D::var(a_, 3), rin = D::var(rin_, 4);
    const double M = dm.M;
    const D ir = 1.0 / r;
    const D gtt = -(1.0 - 2.0 * M * ir);
    const D gtp = -2.0 * M * a * ir;
    const D gpp = r * r + a * a + 2.0 * M * a * a * ir;
    D Om;
    if (dm.rotation == 1) {
        Om = -(gtp + dm.l0 * gtt) / (gpp + dm.l0 * gtp);
    } else {
        const double sM = sqrt(M);
        Om = sM / (r * dsqrt(r) + a * sM);
    }
    const D norm = -gtt - 2.0 * Om * gtp - Om * Om * gpp;
    const D g = dsqrt(norm) / (E - Om * L);
    D em;
    if (dm.emis_model == 1) {
        const D mr = M * ir;
        em = mr * mr * (1.0 - dsqrt(rin * ir));
        const D sv = (dm.r_out - r) / (2.0 * M);
        if (sv.v < 1.0) em = em * sv * sv * (3.0 - 2.0 * sv);
    } else {
        const double e0 = pow(M / r_, dm.emis_q);
        em = D(e0);
        em.d[0] = -dm.emis_q * e0 / r_;
    }
    return g * g * g * em;
}

}  // namespace adj
}  // namespace kt
