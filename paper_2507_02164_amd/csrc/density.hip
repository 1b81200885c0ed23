// density.hip -- roots to root-density image (arXiv 2507.02164, Sec. III:
// each eigenvalue is converted to a pixel coordinate and accumulated in
// video memory).
//
// One lane per polynomial; the lane walks the polynomial's root rows, so
// each row load is a coalesced 16-byte-per-lane read.  A root counts iff
// u = (re - x0) * sx and v = (im - y0) * sy satisfy 0 <= u < width and
// 0 <= v < height (NaN fails every comparison); it adds 1 to pixel
// (floor(v), floor(u)) with an integer atomic, so the image does not depend
// on the order of the additions.  sx and sy come from the host; the
// subtract and the multiply are each rounded (contraction is off), which
// makes every pixel decision reproducible from the root array alone.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace proots {
namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void density_kernel(
    const double2* __restrict__ roots, const int32_t* __restrict__ degrees,
    const uint32_t* __restrict__ status, uint32_t skip_mask, int64_t n, int dmax, double x0,
    double y0, double sx, double sy, int width, int height, int32_t* __restrict__ hist)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    if (status && (status[i] & skip_mask))
        return;
    int d = degrees ? degrees[i] : dmax;
    d = d > dmax ? dmax : d;
    const double w = (double)width, hgt = (double)height;
    for (int k = 0; k < d; ++k) {
        const double2 z = roots[(int64_t)k * n + i];
        const double u = (z.x - x0) * sx;
        const double v = (z.y - y0) * sy;
        if (u >= 0.0 && u < w && v >= 0.0 && v < hgt) {
            const int64_t pix = (int64_t)(int)v * width + (int)u;
            atomicAdd(hist + pix, 1);
        }
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
