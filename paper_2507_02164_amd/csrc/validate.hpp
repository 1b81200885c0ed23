// validate.hpp -- host-side argument checks of the C ABI (include/proots.h).
//
// Plain C++ with no HIP dependency, so that the checks can be compiled and
// exercised on their own (the CPU test-suite builds them with address and
// undefined-behaviour sanitizers).  Each returns a pr_error code.
#pragma once

#include <cmath>
#include <cstdint>

#include "proots.h"

namespace proots {

// Batch shape shared by every batched call.
inline int check_batch(int64_t n, int32_t dmax)
{
    return (n < 0 || dmax < 1 || dmax > 6) ? PR_ERR_INVALID_ARG : PR_OK;
}

// Window [x0, x1) x [y0, y1) split into width x height pixels, and the image
// pointer: finite bounds in increasing order, a non-empty image of at most
// 2^31 - 1 pixels, and finite pixel scales sx = width / (x1 - x0),
// sy = height / (y1 - y0) (returned).
inline int check_window(double x0, double x1, double y0, double y1, int32_t width,
                        int32_t height, const void* hist, double& sx, double& sy)
{
    if (!hist)
        return PR_ERR_INVALID_ARG;
    if (!std::isfinite(x0) || !std::isfinite(x1) || !std::isfinite(y0) || !std::isfinite(y1))
        return PR_ERR_INVALID_ARG;
    if (!(x1 > x0) || !(y1 > y0) || width <= 0 || height <= 0)
        return PR_ERR_INVALID_ARG;
    if ((int64_t)width * (int64_t)height > 0x7fffffffLL)
        return PR_ERR_INVALID_ARG;
    sx = (double)width / (x1 - x0);
    sy = (double)height / (y1 - y0);
    if (!std::isfinite(sx) || !std::isfinite(sy))
        return PR_ERR_INVALID_ARG;
    return PR_OK;
}

// Options of pr_solve / pr_solve_bin (NULL = defaults), copied into `o`.
inline int check_solve_opts(const pr_solve_opts* opts, int max_tile, pr_solve_opts& o)
{
    o = pr_solve_opts{};
    if (opts)
        o = *opts;
    if (o.precision != PR_FP64 && o.precision != PR_FP32_POLISH)
        return PR_ERR_UNSUPPORTED;
    if (o.max_iter_per_level < 0 || o.max_iter_per_level > 1000)
        return PR_ERR_INVALID_ARG;
    if (o.polish_steps < 0 || o.polish_steps > 8)
        return PR_ERR_INVALID_ARG;
    if (!(o.polish_tol >= 0.0 && o.polish_tol < 1.0))
        return PR_ERR_INVALID_ARG;
    if (o.flags &
        ~(uint32_t)(PR_FLAG_NO_EXCEPTIONAL_SHIFT | PR_FLAG_FIXED_STEPS | PR_FLAG_FP64_FALLBACK |
                    PR_FLAG_RAYLEIGH_SHIFT | PR_FLAG_PAIRED_LANES |
                    PR_FLAG_RUN_AHEAD))
        return PR_ERR_UNSUPPORTED;
    if (o.tile < -1 || o.tile > max_tile || o.grid_blocks < 0)
        return PR_ERR_INVALID_ARG;
    return PR_OK;
}

}  // namespace proots
