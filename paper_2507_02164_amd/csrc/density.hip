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
// One lane per polynomial; the wave walks the root rows together, so each
// row load is a coalesced 16-byte-per-lane read.  Neighbouring polynomials
// of a smooth family put their roots into the same few pixels, and 64 lanes
// hammering one address serialise in the memory system.  So each wave first
// merges equal pixels: the lowest pending lane's pixel is broadcast, every
// lane holding that pixel is counted with one ballot, and one lane adds the
// count.  After kRounds merges the remaining lanes add 1 each directly, so a
// wave of 64 distinct pixels (random roots) costs little more than plain
// atomics.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace proots {
namespace {

constexpr int kBlock = 256;
constexpr int kRounds = 8;

__global__ __launch_bounds__(kBlock) void density_kernel(
    const double2* __restrict__ roots, const int32_t* __restrict__ degrees,
    const uint32_t* __restrict__ status, uint32_t skip_mask, int64_t n, int dmax, double x0,
    double y0, double sx, double sy, int width, int height, int32_t* __restrict__ hist)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int d = 0;
    if (i < n && !(status && (status[i] & skip_mask))) {
        d = degrees ? degrees[i] : dmax;
        d = d > dmax ? dmax : d;
    }
    const double w = (double)width, hgt = (double)height;
    const int lane = __lane_id();
    for (int k = 0; k < dmax; ++k) {          // dmax is uniform: every lane takes every trip
        int bin = -1;
        if (k < d) {
            const double2 z = roots[(int64_t)k * n + i];
            const double u = (z.x - x0) * sx;
            const double v = (z.y - y0) * sy;
            if (u >= 0.0 && u < w && v >= 0.0 && v < hgt)
                bin = (int)v * width + (int)u;
        }
        uint64_t pending = __ballot(bin >= 0);
        for (int round = 0; round < kRounds && pending; ++round) {
            const int leader = __builtin_ctzll(pending);
            const int b = __builtin_amdgcn_readlane(bin, leader);
            const uint64_t same = __ballot(bin == b);
            if (lane == leader)
                atomicAdd(hist + b, __builtin_popcountll(same));
            if (bin == b)
                bin = -1;
            pending &= ~same;
        }
        if (bin >= 0)
            atomicAdd(hist + bin, 1);
    }
}

}  // namespace

hipError_t launch_density(const DensityArgs& a, hipStream_t stream)
{
    const int64_t blocks = (a.n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(density_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, stream,
                       reinterpret_cast<const double2*>(a.roots), a.degrees, a.status,
                       a.skip_mask, a.n, a.dmax, a.x0, a.y0, a.sx, a.sy, a.width, a.height,
                       a.hist);
    return hipGetLastError();
}

}  // namespace proots
