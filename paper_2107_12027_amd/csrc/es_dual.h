// Forward-mode dual numbers for the local Jacobians of the adjoint: a value and
// K tangent components, propagated by the chain rule through the same device
// arithmetic as the residual (the pair flux and the face eigen-structure are
// templated on their real type).  Comparisons and branch decisions use the
// value only, so a tangent is the derivative of the branch the value takes.
#pragma once

#include "es_common.h"

namespace es {

// the overloads below for Dual would otherwise hide the double/float ones
using ::fabs;
using ::fma;
using ::fmax;
using ::fmin;

template <int K>
struct Dual {
    double v;
    double d[K];
    __device__ __forceinline__ Dual() : v(0.0) {
#pragma unroll
        for (int k = 0; k < K; ++k) d[k] = 0.0;
    }
    __device__ __forceinline__ Dual(double x) : v(x) {
#pragma unroll
        for (int k = 0; k < K; ++k) d[k] = 0.0;
    }
    // value x with tangent component `which` equal to one
    __device__ __forceinline__ static Dual seed(double x, int which) {
        Dual r(x);
#pragma unroll
        for (int k = 0; k < K; ++k) r.d[k] = k == which ? 1.0 : 0.0;
        return r;
    }
};

template <int K>
__device__ __forceinline__ Dual<K> operator+(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r(a.v + b.v);
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator-(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r(a.v - b.v);
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator-(const Dual<K>& a) {
    Dual<K> r(-a.v);
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator*(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r(a.v * b.v);
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) {
    const double ib = 1.0 / b.v;
    const double q = a.v * ib;
    Dual<K> r(q);
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - q * b.d[k]) * ib;
    return r;
}
template <int K> __device__ __forceinline__ Dual<K> operator+(const Dual<K>& a, double b) { return a + Dual<K>(b); }
template <int K> __device__ __forceinline__ Dual<K> operator+(double a, const Dual<K>& b) { return Dual<K>(a) + b; }
template <int K> __device__ __forceinline__ Dual<K> operator-(const Dual<K>& a, double b) { return a - Dual<K>(b); }
template <int K> __device__ __forceinline__ Dual<K> operator-(double a, const Dual<K>& b) { return Dual<K>(a) - b; }
template <int K>
__device__ __forceinline__ Dual<K> operator*(const Dual<K>& a, double b) {
    Dual<K> r(a.v * b);
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b;
    return r;
}
template <int K> __device__ __forceinline__ Dual<K> operator*(double a, const Dual<K>& b) { return b * a; }
template <int K> __device__ __forceinline__ Dual<K> operator/(const Dual<K>& a, double b) { return a * (1.0 / b); }
template <int K> __device__ __forceinline__ Dual<K> operator/(double a, const Dual<K>& b) { return Dual<K>(a) / b; }
template <int K> __device__ __forceinline__ Dual<K>& operator+=(Dual<K>& a, const Dual<K>& b) { a = a + b; return a; }
template <int K> __device__ __forceinline__ Dual<K>& operator-=(Dual<K>& a, const Dual<K>& b) { a = a - b; return a; }
template <int K> __device__ __forceinline__ Dual<K>& operator*=(Dual<K>& a, const Dual<K>& b) { a = a * b; return a; }

template <int K> __device__ __forceinline__ bool operator<(const Dual<K>& a, const Dual<K>& b) { return a.v < b.v; }
template <int K> __device__ __forceinline__ bool operator>(const Dual<K>& a, const Dual<K>& b) { return a.v > b.v; }
template <int K> __device__ __forceinline__ bool operator<=(const Dual<K>& a, const Dual<K>& b) { return a.v <= b.v; }
template <int K> __device__ __forceinline__ bool operator>=(const Dual<K>& a, const Dual<K>& b) { return a.v >= b.v; }
template <int K> __device__ __forceinline__ bool operator==(const Dual<K>& a, const Dual<K>& b) { return a.v == b.v; }
template <int K> __device__ __forceinline__ bool operator<(const Dual<K>& a, double b) { return a.v < b; }
template <int K> __device__ __forceinline__ bool operator>(const Dual<K>& a, double b) { return a.v > b; }
template <int K> __device__ __forceinline__ bool operator<(double a, const Dual<K>& b) { return a < b.v; }
template <int K> __device__ __forceinline__ bool operator>(double a, const Dual<K>& b) { return a > b.v; }

// f(a) with f' given: value fv, derivative fp
template <int K>
__device__ __forceinline__ Dual<K> chain(const Dual<K>& a, double fv, double fp) {
    Dual<K> r(fv);
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = fp * a.d[k];
    return r;
}

template <int K>
__device__ __forceinline__ Dual<K> xsqrt(const Dual<K>& a) {
    const double s = sqrt(a.v);
    return chain(a, s, 0.5 / s);
}
template <int K>
__device__ __forceinline__ Dual<K> xexp(const Dual<K>& a) {
    const double e = exp(a.v);
    return chain(a, e, e);
}
template <int K>
__device__ __forceinline__ Dual<K> xlog(const Dual<K>& a) {
    return chain(a, log(a.v), 1.0 / a.v);
}
template <int K>
__device__ __forceinline__ Dual<K> frcp(const Dual<K>& a) {
    const double r = 1.0 / a.v;
    return chain(a, r, -r * r);
}
// positive-argument forms of the forward path: the same values through the
// general square root here (the adjoint's tangents need only the derivative)
template <int K>
__device__ __forceinline__ Dual<K> psqrt(const Dual<K>& a) {
    return xsqrt(a);
}
template <int K>
__device__ __forceinline__ Dual<K> frsqrt(const Dual<K>& a) {
    return frcp(xsqrt(a));
}
template <int K>
__device__ __forceinline__ Dual<K> fabs(const Dual<K>& a) {
    return a.v < 0.0 ? -a : a;
}
template <int K>
__device__ __forceinline__ Dual<K> fmax(const Dual<K>& a, const Dual<K>& b) {
    return a.v >= b.v ? a : b;
}
template <int K>
__device__ __forceinline__ Dual<K> fmin(const Dual<K>& a, const Dual<K>& b) {
    return a.v <= b.v ? a : b;
}
template <int K>
__device__ __forceinline__ Dual<K> fma(const Dual<K>& a, const Dual<K>& b, const Dual<K>& c) {
    return a * b + c;
}
template <int K> __device__ __forceinline__ Dual<K> fma(const Dual<K>& a, double b, double c) { return a * b + c; }
template <int K> __device__ __forceinline__ Dual<K> fma(const Dual<K>& a, const Dual<K>& b, double c) { return a * b + c; }

template <int K>
__device__ __forceinline__ double value_of(const Dual<K>& x) { return x.v; }

template <typename R>
struct RealTraits;
template <int K>
struct RealTraits<Dual<K>> {
    static constexpr double ytol = 1e-10;
    static constexpr bool wide_range = true;
};

}  // namespace es
