// Forward-mode dual numbers for the per-point setup on the GPU.
//
// Dual<N> carries a value and N directional derivatives.  The setup code is written
// once as a template over the scalar type: instantiated with `double` it produces the
// per-point coefficient record, with Dual<N> it also produces that record's tangents
// along N input directions (parameters theta, or the 19 fit parameters).
#pragma once
#include <hip/hip_runtime.h>

namespace pd {

template <int N>
struct Dual {
    double v;
    double d[N];
};

template <int N>
__device__ __forceinline__ Dual<N> dconst(double x) {
    Dual<N> r;
    r.v = x;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = 0.0;
    return r;
}

// ---- arithmetic ---------------------------------------------------------------
template <int N>
__device__ __forceinline__ Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N>& a) {
    Dual<N> r;
    r.v = -a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r;
    const double inv = 1.0 / b.v;
    r.v = a.v * inv;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * inv;
    return r;
}
// mixed with double
template <int N>
__device__ __forceinline__ Dual<N> operator+(const Dual<N>& a, double b) {
    Dual<N> r = a;
    r.v += b;
    return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator+(double b, const Dual<N>& a) { return a + b; }
template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N>& a, double b) {
    Dual<N> r = a;
    r.v -= b;
    return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(double b, const Dual<N>& a) {
    Dual<N> r;
    r.v = b - a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(const Dual<N>& a, double b) {
    Dual<N> r;
    r.v = a.v * b;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
    return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(double b, const Dual<N>& a) { return a * b; }
template <int N>
__device__ __forceinline__ Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N>
__device__ __forceinline__ Dual<N> operator/(double a, const Dual<N>& b) {
    Dual<N> r;
    const double inv = 1.0 / b.v;
    r.v = a * inv;
    const double s = -r.v * inv;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = s * b.d[i];
    return r;
}

// ---- elementary functions (chain rule on the value's derivative) --------------
template <int N>
__device__ __forceinline__ Dual<N> chain(const Dual<N>& a, double fv, double dfv) {
    Dual<N> r;
    r.v = fv;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = dfv * a.d[i];
    return r;
}

// typed constant: K<T>(c) is c as a double or as a dual with zero tangent
template <class T>
struct KT {
    static __device__ __forceinline__ T make(double c) { return c; }
};
template <int N>
struct KT<Dual<N>> {
    static __device__ __forceinline__ Dual<N> make(double c) { return dconst<N>(c); }
};
template <class T>
__device__ __forceinline__ T K(double c) { return KT<T>::make(c); }

__device__ __forceinline__ double val(double x) { return x; }
template <int N>
__device__ __forceinline__ double val(const Dual<N>& x) { return x.v; }

__device__ __forceinline__ double dsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ double dlog(double x) { return log(x); }
__device__ __forceinline__ double dexp(double x) { return exp(x); }
__device__ __forceinline__ double datan(double x) { return atan(x); }
__device__ __forceinline__ double dcbrt(double x) { return cbrt(x); }
__device__ __forceinline__ double dpow(double x, double a) { return pow(x, a); }

template <int N>
__device__ __forceinline__ Dual<N> dsqrt(const Dual<N>& a) {
    const double s = sqrt(a.v);
    return chain(a, s, 0.5 / s);
}
template <int N>
__device__ __forceinline__ Dual<N> dlog(const Dual<N>& a) {
    return chain(a, log(a.v), 1.0 / a.v);
}
template <int N>
__device__ __forceinline__ Dual<N> dexp(const Dual<N>& a) {
    const double e = exp(a.v);
    return chain(a, e, e);
}
template <int N>
__device__ __forceinline__ Dual<N> datan(const Dual<N>& a) {
    return chain(a, atan(a.v), 1.0 / (1.0 + a.v * a.v));
}
template <int N>
__device__ __forceinline__ Dual<N> dcbrt(const Dual<N>& a) {
    const double c = cbrt(a.v);
    return chain(a, c, c / (3.0 * a.v));
}
template <int N>
__device__ __forceinline__ Dual<N> dpow(const Dual<N>& a, double e) {
    const double p = pow(a.v, e);
    return chain(a, p, e * p / a.v);
}

}  // namespace pd
