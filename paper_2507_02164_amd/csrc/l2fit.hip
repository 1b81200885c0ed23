// l2fit.hip -- polynomial approximation front-end (arXiv 2507.02164,
// Sec. II-A): least-squares (L2) polynomial approximation of a sampled
// complex function on each of many small disks.
//
// On the unit disk with <g, h> = integral of g conj(h) dA the monomials are
// orthogonal: G_jk = <w^j, w^k> = pi/(j+1) delta_jk, so the normal
// equations G a = b give a_j = (j+1)/pi * b_j with b_j = <f, w^j>.  b_j comes
// from a product quadrature in polar coordinates (Gauss-Legendre in the
// radius, equally spaced angles): b_j = sum_q omega_q f(w_q) conj(w_q)^j.
//
// One lane per disk.  Sample row q of all disks is one coalesced read; the
// lane forms conj(w_q)^j by repeated multiplication and accumulates the
// degree+1 sums in registers.  The quadrature table (radii, weights and the
// nt angles) is uniform across the grid: radii and weights arrive as kernel
// arguments, the angles are built once per block in LDS.  The kernel streams
// HBM (16 bytes read per sample, about 2 FLOP per byte).
#include <hip/hip_runtime.h>

#include <cmath>

#include "cplx.hpp"
#include "internal.hpp"

namespace proots {
namespace {

constexpr int kBlock = kL2fitBlock;
constexpr int kBatch = 8;

template <int DEG>
__global__ __launch_bounds__(kBlock) void l2fit_kernel(const double2* __restrict__ samples,
                                                        int64_t n, L2Quad qd,
                                                        double2* __restrict__ coeffs)
{
    __shared__ double cs[kMaxNt], sn[kMaxNt];
    for (int t = threadIdx.x; t < qd.nt; t += kBlock)
        sincospi(2.0 * t / qd.nt, &sn[t], &cs[t]);
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    cx<double> acc[DEG + 1];
#pragma unroll
    for (int j = 0; j <= DEG; ++j)
        acc[j] = {0.0, 0.0};
    for (int ir = 0; ir < qd.nr; ++ir) {
        const double r = qd.r[ir], om = qd.w[ir];
        int it = 0;
        // the samples of kBatch angles are loaded before any is used, so a
        // wave keeps kBatch loads in flight instead of one
        for (; it + kBatch <= qd.nt; it += kBatch) {
            double2 f[kBatch];
#pragma unroll
            for (int b = 0; b < kBatch; ++b)
                f[b] = load_stream(samples + (int64_t)(ir * qd.nt + it + b) * n + i);
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const cx<double> cw = {r * cs[it + b], -r * sn[it + b]};  // conj(w_q)
                cx<double> t = {f[b].x * om, f[b].y * om};
#pragma unroll
                for (int j = 0; j <= DEG; ++j) {
                    acc[j] = acc[j] + t;
                    t = t * cw;
                }
            }
        }
        for (; it < qd.nt; ++it) {
            const double2 f = load_stream(samples + (int64_t)(ir * qd.nt + it) * n + i);
            const cx<double> cw = {r * cs[it], -r * sn[it]};  // conj(w_q)
            cx<double> t = {f.x * om, f.y * om};
#pragma unroll
            for (int j = 0; j <= DEG; ++j) {
                acc[j] = acc[j] + t;
                t = t * cw;
            }
        }
    }
#pragma unroll
    for (int j = 0; j <= DEG; ++j) {
        const double s = (j + 1) / M_PI;
        store_stream(coeffs + (int64_t)j * n + i, make_double2(acc[j].re * s, acc[j].im * s));
    }
}

template <int DEG>
hipError_t launch_deg(const L2FitArgs& a, hipStream_t stream)
{
    const int64_t blocks = (a.n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(l2fit_kernel<DEG>, dim3((unsigned)blocks), dim3(kBlock), 0, stream,
                       reinterpret_cast<const double2*>(a.samples), a.n, a.quad,
                       reinterpret_cast<double2*>(a.coeffs));
    return hipGetLastError();
}

}  // namespace

// Gauss-Legendre rule on [-1, 1]: the nodes are the zeros of P_n, found by
// Newton's method from the estimate cos(pi (k + 3/4) / (n + 1/2)) with P_n
// and P_n' from the three-term recurrence; weights 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, double* x, double* w)
{
    for (int k = 0; k < n; ++k) {
        double z = std::cos(M_PI * (k + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;  // P_0, P_1
            for (int j = 2; j <= n; ++j) {
                const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) {
                p0 = 1.0;
                p1 = z;
            }
            dp = n * (z * p1 - p0) / ((z - 1.0) * (z + 1.0));
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) <= 1e-16)
                break;
        }
        // P_n' at the final node
        double p0 = 1.0, p1 = z;
        for (int j = 2; j <= n; ++j) {
            const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / ((z - 1.0) * (z + 1.0));
        x[k] = z;
        w[k] = 2.0 / ((1.0 - z) * (1.0 + z) * dp * dp);
    }
}

void l2_quadrature(int nr, int nt, L2Quad& q)
{
    double x[kMaxNr], w[kMaxNr];
    gauss_legendre(nr, x, w);
    q.nr = nr;
    q.nt = nt;
    for (int k = 0; k < nr; ++k) {
        // radius in (0, 1), weight for the r dr dtheta area element
        const int kk = nr - 1 - k;  // increasing radius
        q.r[k] = 0.5 * (1.0 + x[kk]);
        q.w[k] = 0.5 * w[kk] * q.r[k] * (2.0 * M_PI / nt);
    }
}

hipError_t launch_l2fit(const L2FitArgs& a, hipStream_t stream)
{
    switch (a.degree) {
    case 1: return launch_deg<1>(a, stream);
    case 2: return launch_deg<2>(a, stream);
    case 3: return launch_deg<3>(a, stream);
    case 4: return launch_deg<4>(a, stream);
    case 5: return launch_deg<5>(a, stream);
    case 6: return launch_deg<6>(a, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace proots
