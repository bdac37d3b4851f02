// flop.h -- a counting scalar for test-only FLOP counts.  A Flop holds a
// double and counts every arithmetic operation done on it: + - * / and sqrt
// count 1 each, sin and cos 1 each (a sincos pair 2), pow, atan2 and acos 2
// each (the convention of the measurement's algorithmic count).  Sign
// changes, comparisons, fabs, fmax, fmin, floor and round count nothing.
#pragma once

#include <cmath>
#include <cstdint>

struct FlopCounter {
    long long add = 0, mul = 0, div = 0, sqrt = 0, fn = 0;
    long long total() const { return add + mul + div + sqrt + fn; }
};
inline FlopCounter g_flops;

struct Flop {
    double v;
    Flop() = default;
    Flop(double x) : v(x) {}
    explicit operator double() const { return v; }
    explicit operator int() const { return static_cast<int>(v); }
    explicit operator long() const { return static_cast<long>(v); }
    explicit operator long long() const { return static_cast<long long>(v); }
    Flop& operator+=(Flop b) { ++g_flops.add; v += b.v; return *this; }
    Flop& operator-=(Flop b) { ++g_flops.add; v -= b.v; return *this; }
    Flop& operator*=(Flop b) { ++g_flops.mul; v *= b.v; return *this; }
    Flop& operator/=(Flop b) { ++g_flops.div; v /= b.v; return *this; }
};

#define KT_FLOP_BIN(OP, CTR)                                                            \
    inline Flop operator OP(Flop a, Flop b) { ++g_flops.CTR; return Flop(a.v OP b.v); } \
    inline Flop operator OP(Flop a, double b) { ++g_flops.CTR; return Flop(a.v OP b); } \
    inline Flop operator OP(double a, Flop b) { ++g_flops.CTR; return Flop(a OP b.v); }
KT_FLOP_BIN(+, add)
KT_FLOP_BIN(-, add)
KT_FLOP_BIN(*, mul)
KT_FLOP_BIN(/, div)
#undef KT_FLOP_BIN
inline Flop operator-(Flop a) { return Flop(-a.v); }

#define KT_FLOP_CMP(OP)                                                  \
    inline bool operator OP(Flop a, Flop b) { return a.v OP b.v; }       \
    inline bool operator OP(Flop a, double b) { return a.v OP b; }       \
    inline bool operator OP(double a, Flop b) { return a OP b.v; }
KT_FLOP_CMP(<)
KT_FLOP_CMP(<=)
KT_FLOP_CMP(>)
KT_FLOP_CMP(>=)
KT_FLOP_CMP(==)
KT_FLOP_CMP(!=)
#undef KT_FLOP_CMP

inline Flop sqrt(Flop a) { ++g_flops.sqrt; return Flop(std::sqrt(a.v)); }
inline Flop sin(Flop a) { ++g_flops.fn; return Flop(std::sin(a.v)); }
inline Flop cos(Flop a) { ++g_flops.fn; return Flop(std::cos(a.v)); }
inline Flop acos(Flop a) { g_flops.fn += 2; return Flop(std::acos(a.v)); }
inline Flop atan2(Flop a, Flop b) { g_flops.fn += 2; return Flop(std::atan2(a.v, b.v)); }
inline Flop pow(Flop a, Flop b) { g_flops.fn += 2; return Flop(std::pow(a.v, b.v)); }
inline Flop pow(Flop a, double b) { g_flops.fn += 2; return Flop(std::pow(a.v, b)); }
inline Flop pow(double a, Flop b) { g_flops.fn += 2; return Flop(std::pow(a, b.v)); }
inline Flop fabs(Flop a) { return Flop(std::fabs(a.v)); }
inline Flop fmax(Flop a, Flop b) { return Flop(std::fmax(a.v, b.v)); }
inline Flop fmin(Flop a, Flop b) { return Flop(std::fmin(a.v, b.v)); }
inline Flop floor(Flop a) { return Flop(std::floor(a.v)); }
inline Flop round(Flop a) { return Flop(std::round(a.v)); }
inline bool isfinite(Flop a) { return std::isfinite(a.v); }
inline bool isnan(Flop a) { return std::isnan(a.v); }
inline Flop fmax(Flop a, double b) { return Flop(std::fmax(a.v, b)); }
inline Flop fmax(double a, Flop b) { return Flop(std::fmax(a, b.v)); }
inline Flop fmin(Flop a, double b) { return Flop(std::fmin(a.v, b)); }
inline Flop fmin(double a, Flop b) { return Flop(std::fmin(a, b.v)); }
