// backward.hip -- coefficient cotangents from root cotangents (gfx950).
//
// At a simple root r of p(z) = sum_k a_k z^k, differentiating p(r(a); a) = 0
// gives dr/da_k = -r^k / p'(r).  For a real loss with root cotangent
// g = dL/dRe r + i dL/dIm r, the coefficient cotangent in the same
// convention is conj(dr/da_k) g = conj(r)^k q with q = -g / conj(p'(r)),
// summed over the roots of the polynomial.
//
// One lane per polynomial: coefficients, roots and cotangents are read as
// coalesced SoA rows, p'(r) comes from Horner in FP64, and each root adds
// q, q conj(r), q conj(r)^2, ... to the running sums.  No cross-lane
// reduction and no atomics: the kernel streams HBM.
#include <hip/hip_runtime.h>

#include "cplx.hpp"
#include "internal.hpp"

namespace proots {
namespace {

constexpr int kBlock = kBackwardBlock;

template <int DM>
__global__ __launch_bounds__(kBlock) void backward_kernel(
    const double2* __restrict__ coeffs, const int32_t* __restrict__ degrees,
    const double2* __restrict__ roots, const double2* __restrict__ grad_roots, int64_t n,
    double2* __restrict__ grad_coeffs, uint32_t* __restrict__ status)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const int d = degrees ? degrees[i] : DM;
    // the rows are loaded before the status word is looked at, so that no
    // load waits on another; rows k <= min(d, DM) are in bounds for any d
    cx<double> a[DM + 1], r[DM], gr[DM];
#pragma unroll
    for (int k = 0; k <= DM; ++k) {
        a[k] = {0.0, 0.0};
        if (d >= 1 && k <= d) {
            const double2 v = load_stream(coeffs + (int64_t)k * n + i);
            a[k] = {v.x, v.y};
        }
    }
#pragma unroll
    for (int j = 0; j < DM; ++j) {
        r[j] = gr[j] = {0.0, 0.0};
        if (j < d) {
            const double2 rv = load_stream(roots + (int64_t)j * n + i);
            const double2 gv = load_stream(grad_roots + (int64_t)j * n + i);
            r[j] = {rv.x, rv.y};
            gr[j] = {gv.x, gv.y};
        }
    }
    uint32_t st = status[i];
    cx<double> g[DM + 1];
#pragma unroll
    for (int k = 0; k <= DM; ++k)
        g[k] = {0.0, 0.0};
    const bool valid = d >= 1 && d <= DM &&
                       !(st & (PR_ST_BAD_DEGREE | PR_ST_NONFINITE | PR_ST_ZERO_LEADING));
    if (valid) {
#pragma unroll
        for (int j = 0; j < DM; ++j) {
            if (j < d) {
                // p'(r) by Horner over k = DM..1 (a_k = 0 above the degree)
                cx<double> dp = {DM * a[DM].re, DM * a[DM].im};
#pragma unroll
                for (int k = DM - 1; k >= 1; --k)
                    dp = dp * r[j] + cx<double>{k * a[k].re, k * a[k].im};
                const bool singular = !finite(dp) || (dp.re == 0.0 && dp.im == 0.0);
                if (singular)
                    st |= PR_ST_SINGULAR_DERIV;
                // q = -g / conj(dp); a singular root contributes nothing
                cx<double> q = cdiv(cx<double>{-gr[j].re, -gr[j].im}, conj(dp));
                q = singular ? cx<double>{0.0, 0.0} : q;
                const cx<double> rc = conj(r[j]);
#pragma unroll
                for (int k = 0; k <= DM; ++k) {
                    if (k <= d)
                        g[k] = g[k] + q;
                    q = q * rc;
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k <= DM; ++k)
        store_stream(grad_coeffs + (int64_t)k * n + i, make_double2(g[k].re, g[k].im));
    status[i] = st;
}

template <int DM>
hipError_t launch_dm(const BackwardArgs& a, hipStream_t stream)
{
    const int64_t blocks = (a.n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(backward_kernel<DM>, dim3((unsigned)blocks), dim3(kBlock), 0, stream,
                       reinterpret_cast<const double2*>(a.coeffs), a.degrees,
                       reinterpret_cast<const double2*>(a.roots),
                       reinterpret_cast<const double2*>(a.grad_roots), a.n,
                       reinterpret_cast<double2*>(a.grad_coeffs), a.status);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_backward(const BackwardArgs& a, hipStream_t stream)
{
    switch (a.dmax) {
    case 1: return launch_dm<1>(a, stream);
    case 2: return launch_dm<2>(a, stream);
    case 3: return launch_dm<3>(a, stream);
    case 4: return launch_dm<4>(a, stream);
    case 5: return launch_dm<5>(a, stream);
    case 6: return launch_dm<6>(a, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace proots
