// kt_dual.h -- forward-mode dual numbers for the adjoint: a value and N
// directional derivatives, carried through + - * / sqrt sin cos.  Used on the
// device for Hessian-vector products of the Hamiltonian and for the
// derivatives of the disk observables, and on the host for the derivatives
// of the camera constants.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "kt_elem.h"

namespace kt {

template <int N>
struct Dual {
    double v;
    double d[N];

    __host__ __device__ Dual() : v(0.0) {
        for (int i = 0; i < N; ++i) d[i] = 0.0;
    }
    __host__ __device__ Dual(double x) : v(x) {  // a constant
        for (int i = 0; i < N; ++i) d[i] = 0.0;
    }
    // a variable with derivative 1 along direction k
    __host__ __device__ static Dual var(double x, int k) {
        Dual r(x);
        r.d[k] = 1.0;
        return r;
    }
    // a value with the given tangent along every direction
    __host__ __device__ static Dual with(double x, const double* t) {
        Dual r(x);
        for (int i = 0; i < N; ++i) r.d[i] = t[i];
        return r;
    }
};

template <int N>
__host__ __device__ inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r(a.v + b.v);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <int N>
__host__ __device__ inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r(a.v - b.v);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <int N>
__host__ __device__ inline Dual<N> operator-(const Dual<N>& a) {
    Dual<N> r(-a.v);
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <int N>
__host__ __device__ inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r(a.v * b.v);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <int N>
__host__ __device__ inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
    const double ib = rcp(b.v);  // one reciprocal for the value and all tangents
    const double q = a.v * ib;
    Dual<N> r(q);
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - q * b.d[i]) * ib;
    return r;
}
template <int N>
__host__ __device__ inline Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N>
__host__ __device__ inline Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N>
__host__ __device__ inline Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N>
__host__ __device__ inline Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N>
__host__ __device__ inline Dual<N> operator*(const Dual<N>& a, double b) {
    Dual<N> r(a.v * b);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
    return r;
}
template <int N>
__host__ __device__ inline Dual<N> operator*(double a, const Dual<N>& b) { return b * a; }
template <int N>
__host__ __device__ inline Dual<N> operator/(const Dual<N>& a, double b) { return a * rcp(b); }
template <int N>
__host__ __device__ inline Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }

// 1/x for plain and dual numbers
__host__ __device__ inline double recip(double x) { return rcp(x); }
template <int N>
__host__ __device__ inline Dual<N> recip(const Dual<N>& x) {
    return 1.0 / x;
}

template <int N>
__host__ __device__ inline Dual<N> dsqrt(const Dual<N>& a) {
    const double s = sqrt(a.v);
    Dual<N> r(s);
    const double h = 0.5 / s;
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * h;
    return r;
}
template <int N>
__host__ __device__ inline void dsincos(const Dual<N>& a, Dual<N>* s, Dual<N>* c) {
    const double sv = sin(a.v), cv = cos(a.v);
    *s = Dual<N>(sv);
    *c = Dual<N>(cv);
    for (int i = 0; i < N; ++i) {
        s->d[i] = cv * a.d[i];
        c->d[i] = -sv * a.d[i];
    }
}

// plain doubles through the same interface
__host__ __device__ inline double dsqrt(double a) { return sqrt(a); }
__host__ __device__ inline void dsincos(double a, double* s, double* c) {
    *s = sin(a);
    *c = cos(a);
}

}  // namespace kt
