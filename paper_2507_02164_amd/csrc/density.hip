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
// (coalesced 16-byte-per-lane reads, all in flight together), then binned
// row by row, each run of consecutive lanes on one pixel with one atomic
// (`run_count`).
//
// Local form (the front-end's roots, in each disk's variable w): a root
// counts only when |w|^2 < rmax2, at z = c + rho w (each part a rounded
// multiply then a rounded add), then binned as above.
#include <hip/hip_runtime.h>

#include "bin.hpp"
#include "internal.hpp"

namespace proots {
namespace {

constexpr int kBlock = kDensityBlock;

template <int DM, bool LOCAL>
__global__ __launch_bounds__(kBlock) void density_kernel(
    const double2* __restrict__ roots, const int32_t* __restrict__ degrees,
    const uint32_t* __restrict__ status, uint32_t skip_mask, int64_t n, BinWindow win,
    const double2* __restrict__ centers, const double* __restrict__ radii, double rmax2)
{
#pragma clang fp contract(off)
    // consecutive blocks are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous range of polynomials instead, so that neighbouring
    // polynomials (which hit the same pixels) run on the same XCD and their
    // atomics meet in one L2 (measured 1.1 -> 0.72 ms on the 4096^2 grid)
    const int64_t nb = gridDim.x, per = (nb + 7) / 8;
    const int64_t b = blockIdx.x;
    const int64_t bb = (b % 8) * per + b / 8;
    const int64_t i = bb * kBlock + threadIdx.x;
    int d = 0;
    if (i < n && !(status && (status[i] & skip_mask))) {
        d = degrees ? degrees[i] : DM;
        d = d > DM ? DM : d;
    }
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
            bin[k] = pixel_of(z.x, z.y, win);
        }
    }
#pragma unroll
    for (int k = 0; k < DM; ++k)
        run_count(bin[k], win.hist);
}

template <int DM>
hipError_t launch_dm(const DensityArgs& a, hipStream_t stream)
{
    int64_t blocks = (a.n + kBlock - 1) / kBlock;
    blocks = (blocks + 7) / 8 * 8;  // a whole number of blocks per XCD
    if (a.centers)
        hipLaunchKernelGGL((density_kernel<DM, true>), dim3((unsigned)blocks), dim3(kBlock), 0,
                           stream, reinterpret_cast<const double2*>(a.roots), a.degrees,
                           a.status, a.skip_mask, a.n, a.win,
                           reinterpret_cast<const double2*>(a.centers), a.radii, a.rmax2);
    else
        hipLaunchKernelGGL((density_kernel<DM, false>), dim3((unsigned)blocks), dim3(kBlock), 0,
                           stream, reinterpret_cast<const double2*>(a.roots), a.degrees,
                           a.status, a.skip_mask, a.n, a.win, nullptr, nullptr, 0.0);
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
