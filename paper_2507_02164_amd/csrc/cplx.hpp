// cplx.hpp -- register-resident complex arithmetic for the gfx950 kernels.
//
// Plain structs of two scalars so that every entry of a per-lane matrix is
// two VGPRs (FP32) or four (FP64) and the compiler sees each real
// multiply-add explicitly.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace proots {

template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }

template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }

template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }

template <typename T>
__device__ __forceinline__ T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }

// |Re z| + |Im z|, evaluated in FP64 whatever the storage precision.
template <typename T>
__device__ __forceinline__ double cabs1_d(cx<T> a)
{
    return fabs((double)a.re) + fabs((double)a.im);
}

// |x| in x's own precision (__builtin_fabs would take a float through FP64).
__device__ __forceinline__ float abs_t(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double abs_t(double x) { return __builtin_fabs(x); }

template <typename T>
__device__ __forceinline__ bool finite(cx<T> a) { return isfinite(a.re) && isfinite(a.im); }

// a / b by Smith's method (no overflow of |b|^2 for large b).
__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b)
{
    if (fabs(b.re) >= fabs(b.im)) {
        double r = b.im / b.re;
        double den = b.re + b.im * r;
        return {(a.re + a.im * r) / den, (a.im - a.re * r) / den};
    }
    double r = b.re / b.im;
    double den = b.re * r + b.im;
    return {(a.re * r + a.im) / den, (a.im * r - a.re) / den};
}

// Read-once and write-once streams (a kernel's inputs and outputs that no
// later access of the same launch reuses): nontemporal accesses, which keep
// them from displacing reusable lines in the caches.
typedef double nt_double2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double2 load_stream(const double2* p)
{
    const nt_double2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_double2*>(p));
    return make_double2(v.x, v.y);
}

__device__ __forceinline__ void store_stream(double2* p, double2 v)
{
    __builtin_nontemporal_store(nt_double2{v.x, v.y}, reinterpret_cast<nt_double2*>(p));
}

}  // namespace proots
