// bin.hpp -- root to pixel, and wave-merged pixel counting (arXiv
// 2507.02164, Sec. III: each eigenvalue becomes a pixel coordinate whose
// count is incremented in video memory).  Shared by the density kernel and
// the solve kernel's binning epilogue, so that both decide every pixel with
// the same arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace proots {

// The image and its window: pixel (v, u) covers [x0 + u/sx, x0 + (u+1)/sx)
// x [y0 + v/sy, ...); sx = width / (x1 - x0), sy = height / (y1 - y0) are
// computed once on the host in FP64.
struct BinWindow {
    double x0, y0, sx, sy;
    int32_t width, height;
    int32_t* hist;  // [height][width], counts are added
};

// Pixel index of z, or -1 when z is outside the window (or NaN, which fails
// every comparison).  u = (re - x0) * sx and v = (im - y0) * sy, each a
// rounded subtract then a rounded multiply (no contraction), so the decision
// depends on the root alone.
__device__ __forceinline__ int pixel_of(double re, double im, const BinWindow& w)
{
#pragma clang fp contract(off)
    const double u = (re - w.x0) * w.sx;
    const double v = (im - w.y0) * w.sy;
    if (u >= 0.0 && u < (double)w.width && v >= 0.0 && v < (double)w.height)
        return (int)v * w.width + (int)u;
    return -1;
}

// Add 1 at pixel b (b < 0: nothing) for every lane of the wave, merging
// runs of consecutive lanes that hold the same pixel; all lanes must call it
// together.  A lane starts a run where its pixel differs from the previous
// lane's (lane 0 always); the run ends before the next such lane, and its
// first lane adds the run's length with one atomic.  Every lane with b >= 0
// lies in exactly one run that starts at or before it with the same pixel,
// so each is counted once.  Where lanes hold consecutive polynomials of a
// smooth family, a root moves through its pixels in runs, which this merges
// at a fixed cost of a few instructions; distinct pixels cost one atomic
// each, as plain atomics would.
__device__ __forceinline__ void run_count(int b, int32_t* __restrict__ hist)
{
    const int lane = __lane_id();
    const int prev = __shfl_up(b, 1);
    const uint64_t starts = __ballot(lane == 0 || b != prev);
    const uint64_t after = lane == 63 ? 0ull : starts >> (lane + 1);
    const int len = after ? __builtin_ctzll(after) + 1 : 64 - lane;
    if (b >= 0 && (lane == 0 || b != prev))
        atomicAdd(hist + b, len);
}

}  // namespace proots
