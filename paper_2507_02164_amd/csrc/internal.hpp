// internal.hpp -- launchers shared between the C-ABI layer and the kernel
// translation units.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "proots.h"

namespace proots {

struct SolveArgs {
    const pr_complex* coeffs;
    const int32_t* degrees;
    int64_t n;
    int32_t dmax;
    pr_complex* roots;
    uint32_t* status;
    int32_t* iters;
    int32_t cap;
    uint32_t flags;
    int32_t polish_steps;
    double polish_tol;
    int32_t tile;         // > 0 with degrees: persistent degree-bucketed launch
    int32_t grid_blocks;  // persistent launch: number of one-wave blocks (0 = one per tile)
};

int max_tile();
hipError_t launch_solve_fp64(const SolveArgs& a, hipStream_t stream);
hipError_t launch_solve_fp32_polish(const SolveArgs& a, hipStream_t stream);

struct DensityArgs {
    const pr_complex* roots;
    const int32_t* degrees;
    const uint32_t* status;
    uint32_t skip_mask;
    int64_t n;
    int32_t dmax;
    double x0, y0, sx, sy;
    int32_t width, height;
    int32_t* hist;
};

hipError_t launch_density(const DensityArgs& a, hipStream_t stream);

struct BackwardArgs {
    const pr_complex* coeffs;
    const int32_t* degrees;
    const pr_complex* roots;
    const pr_complex* grad_roots;
    int64_t n;
    int32_t dmax;
    pr_complex* grad_coeffs;
    uint32_t* status;
};

hipError_t launch_backward(const BackwardArgs& a, hipStream_t stream);

}  // namespace proots
