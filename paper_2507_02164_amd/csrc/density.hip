// density.hip -- roots to root-density image (arXiv 2507.02164, Sec. III:
// each eigenvalue is converted to a pixel coordinate and accumulated in
// video memory).
//
// A root counts iff u = (re - x0) * sx and v = (im - y0) * sy satisfy
// 0 <= u < width and 0 <= v < height (NaN fails every comparison); it adds
// 1 to pixel (floor(v), floor(u)).  sx and sy come from the host; the
// subtract and the multiply are each rounded (contraction is off), so every
// pixel decision is reproducible from the root array alone, and integer
// addition makes the image independent of the order of the additions.
//
// One lane per polynomial.  All of a lane's root rows are loaded first
// (coalesced 16-byte-per-lane reads, all in flight together), then binned.
// Neighbouring polynomials of a smooth family put their roots into the same
// few pixels, and 64 lanes hammering one address serialise in the memory
// system, so for each root row the wave merges equal pixels: the lowest
// pending lane's pixel is broadcast, every lane holding it is counted with
// one ballot, and one lane adds the count.  After kRounds merges the
// remaining lanes add 1 each directly, so a row of 64 distinct pixels
// (random roots) costs little more than plain atomics.
//
// Local form (the front-end's roots, in each disk's variable w): a root
// counts only when |w|^2 < rmax2, at z = c + rho w (each part a rounded
// multiply then a rounded add), then binned as above.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace proots {
namespace {

constexpr int kBlock = 256;
constexpr int kRounds = 8;
#ifndef PR_DENSITY_XCD_REMAP
#define PR_DENSITY_XCD_REMAP 1
#endif

template <int DM, bool LOCAL>
__global__ __launch_bounds__(kBlock) void density_kernel(
    const double2* __restrict__ roots, const int32_t* __restrict__ degrees,
    const uint32_t* __restrict__ status, uint32_t skip_mask, int64_t n, double x0, double y0,
    double sx, double sy, int width, int height, int32_t* __restrict__ hist,
    const double2* __restrict__ centers, const double* __restrict__ radii, double rmax2)
{
#pragma clang fp contract(off)
#if PR_DENSITY_XCD_REMAP
    // consecutive blocks are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous range of polynomials instead, so that neighbouring
    // polynomials (which hit the same pixels) run on the same XCD
    const int64_t nb = gridDim.x, per = (nb + 7) / 8;
    const int64_t b = blockIdx.x;
    const int64_t bb = (b % 8) * per + b / 8;
    const int64_t i = bb * kBlock + threadIdx.x;
#else
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
#endif
    int d = 0;
    if (i < n && !(status && (status[i] & skip_mask))) {
        d = degrees ? degrees[i] : DM;
        d = d > DM ? DM : d;
    }
    const double w = (double)width, hgt = (double)height;
    double2 c = make_double2(0.0, 0.0);
    double rho = 0.0;
    if (LOCAL && d > 0) {
        c = centers[i];
        rho = radii[i];
    }
    int bin[DM];
#pragma unroll
    for (int k = 0; k < DM; ++k) {
        bin[k] = -1;
        if (k < d) {
            double2 z = roots[(int64_t)k * n + i];
            if (LOCAL) {
                // local root w: keep it only inside the disk, then z = c + rho w
                const bool inside = z.x * z.x + z.y * z.y < rmax2;
                z = make_double2(c.x + rho * z.x, c.y + rho * z.y);
                if (!inside)
                    z = make_double2(__builtin_nan(""), 0.0);
            }
            const double u = (z.x - x0) * sx;
            const double v = (z.y - y0) * sy;
            if (u >= 0.0 && u < w && v >= 0.0 && v < hgt)
                bin[k] = (int)v * width + (int)u;
        }
    }
    const int lane = __lane_id();
#pragma unroll
    for (int k = 0; k < DM; ++k) {
        int b = bin[k];
        uint64_t pending = __ballot(b >= 0);
        for (int round = 0; round < kRounds && pending; ++round) {
            const int leader = __builtin_ctzll(pending);
            const int lb = __builtin_amdgcn_readlane(b, leader);
            const uint64_t same = __ballot(b == lb);
            if (lane == leader)
                atomicAdd(hist + lb, __builtin_popcountll(same));
            if (b == lb)
                b = -1;
            pending &= ~same;
        }
        if (b >= 0)
            atomicAdd(hist + b, 1);
    }
}

template <int DM>
hipError_t launch_dm(const DensityArgs& a, hipStream_t stream)
{
    int64_t blocks = (a.n + kBlock - 1) / kBlock;
#if PR_DENSITY_XCD_REMAP
    blocks = (blocks + 7) / 8 * 8;
#endif
    if (a.centers)
        hipLaunchKernelGGL((density_kernel<DM, true>), dim3((unsigned)blocks), dim3(kBlock), 0,
                           stream, reinterpret_cast<const double2*>(a.roots), a.degrees,
                           a.status, a.skip_mask, a.n, a.x0, a.y0, a.sx, a.sy, a.width,
                           a.height, a.hist, reinterpret_cast<const double2*>(a.centers),
                           a.radii, a.rmax2);
    else
        hipLaunchKernelGGL((density_kernel<DM, false>), dim3((unsigned)blocks), dim3(kBlock), 0,
                           stream, reinterpret_cast<const double2*>(a.roots), a.degrees,
                           a.status, a.skip_mask, a.n, a.x0, a.y0, a.sx, a.sy, a.width,
                           a.height, a.hist, nullptr, nullptr, 0.0);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_density(const DensityArgs& a, hipStream_t stream)
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
