/*
 * opcount.cpp -- the oracle's own source compiled with an operation-counting number
 * type in place of double, to measure the algorithmic floating-point work of one
 * time step (the definitional algorithm, before any fusion or reuse).
 *
 * TEST INFRASTRUCTURE, like the oracle itself: a measurement of the method, not part
 * of the product. Built on request by oracle/opcount.py; exports the oracle's API
 * (same struct layouts: the counting type is one double) plus opc_reset / opc_read.
 *
 * Counted: + and - (add), * (mul), / (div), sqrt and transcendental calls (special),
 * comparisons, min/max/abs/clamp-type selects (cmp). Unary minus and copies are free.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

namespace opc {
static long long n_add, n_mul, n_div, n_special, n_cmp;
}

struct Cnt {
    double v;
    Cnt() = default;
    Cnt(double x) : v(x) {}
    explicit operator int() const { return (int)v; }
    explicit operator long() const { return (long)v; }
    explicit operator long long() const { return (long long)v; }
    explicit operator float() const { return (float)v; }
    explicit operator double() const { return v; }
    Cnt& operator+=(Cnt b) { ++opc::n_add; v += b.v; return *this; }
    Cnt& operator-=(Cnt b) { ++opc::n_add; v -= b.v; return *this; }
    Cnt& operator*=(Cnt b) { ++opc::n_mul; v *= b.v; return *this; }
    Cnt& operator/=(Cnt b) { ++opc::n_div; v /= b.v; return *this; }
};
static_assert(sizeof(Cnt) == sizeof(double), "layout must match the FP64 oracle");

inline Cnt operator+(Cnt a, Cnt b) { ++opc::n_add; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++opc::n_add; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++opc::n_mul; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++opc::n_div; return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt operator+(Cnt a) { return a; }
inline bool operator<(Cnt a, Cnt b) { ++opc::n_cmp; return a.v < b.v; }
inline bool operator>(Cnt a, Cnt b) { ++opc::n_cmp; return a.v > b.v; }
inline bool operator<=(Cnt a, Cnt b) { ++opc::n_cmp; return a.v <= b.v; }
inline bool operator>=(Cnt a, Cnt b) { ++opc::n_cmp; return a.v >= b.v; }
inline bool operator==(Cnt a, Cnt b) { ++opc::n_cmp; return a.v == b.v; }
inline bool operator!=(Cnt a, Cnt b) { ++opc::n_cmp; return a.v != b.v; }

inline Cnt sqrt(Cnt a) { ++opc::n_special; return Cnt(::sqrt(a.v)); }
inline Cnt tanh(Cnt a) { ++opc::n_special; return Cnt(::tanh(a.v)); }
inline Cnt cos(Cnt a) { ++opc::n_special; return Cnt(::cos(a.v)); }
inline Cnt sin(Cnt a) { ++opc::n_special; return Cnt(::sin(a.v)); }
inline Cnt exp(Cnt a) { ++opc::n_special; return Cnt(::exp(a.v)); }
inline Cnt atan2(Cnt a, Cnt b) { ++opc::n_special; return Cnt(::atan2(a.v, b.v)); }
inline Cnt floor(Cnt a) { ++opc::n_cmp; return Cnt(::floor(a.v)); }
inline Cnt fabs(Cnt a) { ++opc::n_cmp; return Cnt(::fabs(a.v)); }
inline Cnt fmin(Cnt a, Cnt b) { ++opc::n_cmp; return Cnt(::fmin(a.v, b.v)); }
inline Cnt fmax(Cnt a, Cnt b) { ++opc::n_cmp; return Cnt(::fmax(a.v, b.v)); }
inline bool isfinite(Cnt a) { return ::isfinite(a.v); }
inline bool isnan(Cnt a) { return ::isnan(a.v); }

#define double Cnt
#include "lbfs_oracle.c"
#undef double

extern "C" void opc_reset(void)
{
    opc::n_add = opc::n_mul = opc::n_div = opc::n_special = opc::n_cmp = 0;
}

/* out[5] = {add, mul, div, special, cmp} since the last reset */
extern "C" void opc_read(long long* out)
{
    out[0] = opc::n_add;
    out[1] = opc::n_mul;
    out[2] = opc::n_div;
    out[3] = opc::n_special;
    out[4] = opc::n_cmp;
}
