// api.hip -- the C ABI declared in include/proots.h: argument validation on
// the host, then one kernel launch on the caller's stream.  Nothing here
// allocates, synchronises or throws.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>

#include "internal.hpp"
#include "proots.h"
#include "validate.hpp"

using namespace proots;

namespace {

constexpr int kDefaultCap = 30;
constexpr int kDefaultPolishSteps = 2;
constexpr double kDefaultPolishTol = 1e-6;
constexpr int kDefaultTile = 2048;
constexpr int kDefaultBlocksPerCU = 8;
constexpr int kMaxDevices = 64;

inline int hip_status(hipError_t e) { return e == hipSuccess ? PR_OK : PR_ERR_HIP; }

// Compute-unit count of the current device, looked up once per device (calls
// from several host threads may look it up together; they store the same
// value).
int cu_count()
{
    static std::atomic<int> cached[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return 256;
    int cus = cached[dev].load(std::memory_order_relaxed);
    if (cus == 0) {
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        cached[dev].store(cus, std::memory_order_relaxed);
    }
    return cus;
}

}  // namespace

// Window validation shared by the density and binning entry points.
static int make_window(double x0, double x1, double y0, double y1, int32_t width,
                       int32_t height, int32_t* hist, BinWindow& w)
{
    double sx = 0.0, sy = 0.0;
    const int rc = check_window(x0, x1, y0, y1, width, height, hist, sx, sy);
    if (rc != PR_OK)
        return rc;
    w.x0 = x0;
    w.y0 = y0;
    w.sx = sx;
    w.sy = sy;
    w.width = width;
    w.height = height;
    w.hist = hist;
    return PR_OK;
}

// win == nullptr: plain solve; else the binning epilogue (roots optional).
static int solve_common(const pr_complex* coeffs, const int32_t* degrees, int64_t n,
                        int32_t dmax, pr_complex* roots, uint32_t* status,
                        const pr_solve_opts* opts, const BinWindow* win, uint32_t skip_mask,
                        void* stream)
{
    if (check_batch(n, dmax) != PR_OK)
        return PR_ERR_INVALID_ARG;
    if (n > 0 && (!coeffs || (!roots && !win) || !status))
        return PR_ERR_INVALID_ARG;
    pr_solve_opts o;
    const int orc = check_solve_opts(opts, max_tile(), o);
    if (orc != PR_OK)
        return orc;
    if (n == 0)
        return PR_OK;
    if (n > kMaxSolveBatch)
        return PR_ERR_INVALID_ARG;
    SolveArgs a;
    a.coeffs = coeffs;
    a.degrees = degrees;
    a.n = n;
    a.dmax = dmax;
    a.roots = roots;
    a.status = status;
    a.iters = o.iter_counts;
    a.cap = o.max_iter_per_level ? o.max_iter_per_level : kDefaultCap;
    a.flags = o.flags;
    a.polish_steps = o.polish_steps ? o.polish_steps : kDefaultPolishSteps;
    a.polish_tol = o.polish_tol > 0.0 ? o.polish_tol : kDefaultPolishTol;
    a.tile = o.tile == 0 ? kDefaultTile : (o.tile < 0 ? 0 : o.tile);
    a.grid_blocks = o.grid_blocks;  // 0: one block per (tile, slice)
    a.win = win ? *win : BinWindow{0.0, 0.0, 0.0, 0.0, 0, 0, nullptr};
    a.skip_mask = skip_mask;
    a.fallback_tile = a.tile > 0 ? a.tile : kDefaultTile;
    a.fallback_grid = o.grid_blocks > 0 ? o.grid_blocks : kDefaultBlocksPerCU * cu_count();
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (o.precision == PR_FP64)
        return hip_status(launch_solve_fp64(a, s));
    return hip_status(launch_solve_fp32_polish(a, s));
}

extern "C" int pr_solve(const pr_complex* coeffs, const int32_t* degrees, int64_t n,
                        int32_t dmax, pr_complex* roots, uint32_t* status,
                        const pr_solve_opts* opts, void* stream)
{
    return solve_common(coeffs, degrees, n, dmax, roots, status, opts, nullptr, 0, stream);
}

extern "C" int pr_solve_bin(const pr_complex* coeffs, const int32_t* degrees, int64_t n,
                            int32_t dmax, pr_complex* roots, uint32_t* status,
                            const pr_solve_opts* opts, uint32_t skip_mask, double x0, double x1,
                            double y0, double y1, int32_t width, int32_t height, int32_t* hist,
                            void* stream)
{
    BinWindow w;
    const int rc = make_window(x0, x1, y0, y1, width, height, hist, w);
    if (rc != PR_OK)
        return rc;
    return solve_common(coeffs, degrees, n, dmax, roots, status, opts, &w, skip_mask, stream);
}

// Argument checks shared by the density entry points; fills `a` (a.n == 0:
// nothing to enqueue).
static int density_args(const pr_complex* roots, const int32_t* degrees, const uint32_t* status,
                        uint32_t skip_mask, int64_t n, int32_t dmax, double x0, double x1,
                        double y0, double y1, int32_t width, int32_t height, int32_t* hist,
                        DensityArgs& a)
{
    if (check_batch(n, dmax) != PR_OK)
        return PR_ERR_INVALID_ARG;
    if (n > 0 && !roots)
        return PR_ERR_INVALID_ARG;
    BinWindow w;
    const int rc = make_window(x0, x1, y0, y1, width, height, hist, w);
    if (rc != PR_OK)
        return rc;
    if (n > kMaxDensityBatch)
        return PR_ERR_INVALID_ARG;
    a.roots = roots;
    a.degrees = degrees;
    a.status = status;
    a.skip_mask = skip_mask;
    a.n = n;
    a.dmax = dmax;
    a.win = w;
    a.centers = nullptr;
    a.radii = nullptr;
    a.rmax2 = 0.0;
    return PR_OK;
}

extern "C" int pr_density(const pr_complex* roots, const int32_t* degrees,
                          const uint32_t* status, uint32_t skip_mask, int64_t n, int32_t dmax,
                          double x0, double x1, double y0, double y1, int32_t width,
                          int32_t height, int32_t* hist, void* stream)
{
    DensityArgs a;
    const int rc = density_args(roots, degrees, status, skip_mask, n, dmax, x0, x1, y0, y1, width,
                                height, hist, a);
    if (rc != PR_OK || n == 0)
        return rc;
    return hip_status(launch_density(a, static_cast<hipStream_t>(stream)));
}

extern "C" int64_t pr_density_sorted_workspace(int64_t n, int32_t dmax, int32_t width,
                                               int32_t height)
{
    if (n < 0 || dmax < 1 || dmax > 6 || width <= 0 || height <= 0 ||
        (int64_t)width * (int64_t)height > 0x7fffffffLL || n > kMaxDensityBatch)
        return PR_ERR_INVALID_ARG;
    return sortbin_workspace(n, dmax, width, height);
}

extern "C" int pr_density_sorted(const pr_complex* roots, const int32_t* degrees,
                                 const uint32_t* status, uint32_t skip_mask, int64_t n,
                                 int32_t dmax, double x0, double x1, double y0, double y1,
                                 int32_t width, int32_t height, int32_t* hist, void* workspace,
                                 int64_t workspace_bytes, void* stream)
{
    DensityArgs a;
    const int rc = density_args(roots, degrees, status, skip_mask, n, dmax, x0, x1, y0, y1, width,
                                height, hist, a);
    if (rc != PR_OK || n == 0)
        return rc;
    const int64_t need = sortbin_workspace(n, dmax, width, height);
    if (need > 0) {
        if (!workspace || workspace_bytes < need)
            return PR_ERR_NO_MEMORY;
        if (reinterpret_cast<uintptr_t>(workspace) & 255)
            return PR_ERR_INVALID_ARG;
    }
    return hip_status(
        launch_density_sorted(a, workspace, cu_count(), static_cast<hipStream_t>(stream)));
}

extern "C" int pr_density_sorted_noalloc(const pr_complex* roots, const int32_t* degrees,
                                         const uint32_t* status, uint32_t skip_mask, int64_t n,
                                         int32_t dmax, double x0, double x1, double y0,
                                         double y1, int32_t width, int32_t height, int32_t* hist,
                                         void* stream)
{
    DensityArgs a;
    const int rc = density_args(roots, degrees, status, skip_mask, n, dmax, x0, x1, y0, y1, width,
                                height, hist, a);
    if (rc != PR_OK || n == 0)
        return rc;
    const int64_t need = sortbin_workspace(n, dmax, width, height);
    if (need > kSortScratchBytes)
        return PR_ERR_NO_MEMORY;
    void* ws = nullptr;
    if (need > 0 && (ws = sortbin_scratch()) == nullptr)
        return PR_ERR_HIP;
    return hip_status(launch_density_sorted(a, ws, cu_count(), static_cast<hipStream_t>(stream)));
}

extern "C" int pr_density_local(const pr_complex* roots, const int32_t* degrees,
                                const uint32_t* status, uint32_t skip_mask, int64_t n,
                                int32_t dmax, const pr_complex* centers, const double* radii,
                                double rmax2, double x0, double x1, double y0, double y1,
                                int32_t width, int32_t height, int32_t* hist, void* stream)
{
    if (!(rmax2 > 0.0) || !std::isfinite(rmax2))
        return PR_ERR_INVALID_ARG;
    if (n > 0 && (!centers || !radii))
        return PR_ERR_INVALID_ARG;
    DensityArgs a;
    const int rc = density_args(roots, degrees, status, skip_mask, n, dmax, x0, x1, y0, y1, width,
                                height, hist, a);
    if (rc != PR_OK || n == 0)
        return rc;
    a.centers = centers;
    a.radii = radii;
    a.rmax2 = rmax2;
    return hip_status(launch_density(a, static_cast<hipStream_t>(stream)));
}

extern "C" int pr_l2fit_nodes(int32_t nr, int32_t nt, double* nodes, double* weights)
{
    if (!nodes || !weights || nr < 1 || nr > kMaxNr || nt < 1 || nt > kMaxNt)
        return PR_ERR_INVALID_ARG;
    L2Quad q;
    l2_quadrature(nr, nt, q);
    for (int ir = 0; ir < nr; ++ir)
        for (int it = 0; it < nt; ++it) {
            const int k = ir * nt + it;
            const double th = 2.0 * M_PI * it / nt;
            nodes[2 * k] = q.r[ir] * std::cos(th);
            nodes[2 * k + 1] = q.r[ir] * std::sin(th);
            weights[k] = q.w[ir];
        }
    return PR_OK;
}

extern "C" int pr_l2fit(const pr_complex* samples, int64_t n, int32_t degree, int32_t nr,
                        int32_t nt, pr_complex* coeffs, void* stream)
{
    if (n < 0 || degree < 1 || degree > 6 || nr < 1 || nr > kMaxNr || nt < 1 || nt > kMaxNt)
        return PR_ERR_INVALID_ARG;
    if (n > 0 && (!samples || !coeffs))
        return PR_ERR_INVALID_ARG;
    if (n == 0)
        return PR_OK;
    if (n > kMaxL2fitBatch)
        return PR_ERR_INVALID_ARG;
    L2FitArgs a;
    a.samples = samples;
    a.n = n;
    a.degree = degree;
    l2_quadrature(nr, nt, a.quad);
    a.coeffs = coeffs;
    return hip_status(launch_l2fit(a, static_cast<hipStream_t>(stream)));
}

extern "C" int pr_backward(const pr_complex* coeffs, const int32_t* degrees,
                           const pr_complex* roots, const pr_complex* grad_roots, int64_t n,
                           int32_t dmax, pr_complex* grad_coeffs, uint32_t* status,
                           void* stream)
{
    if (n < 0 || dmax < 1 || dmax > 6)
        return PR_ERR_INVALID_ARG;
    if (n > 0 && (!coeffs || !roots || !grad_roots || !grad_coeffs || !status))
        return PR_ERR_INVALID_ARG;
    if (n == 0)
        return PR_OK;
    if (n > kMaxBackwardBatch)
        return PR_ERR_INVALID_ARG;
    BackwardArgs a;
    a.coeffs = coeffs;
    a.degrees = degrees;
    a.roots = roots;
    a.grad_roots = grad_roots;
    a.n = n;
    a.dmax = dmax;
    a.grad_coeffs = grad_coeffs;
    a.status = status;
    return hip_status(launch_backward(a, static_cast<hipStream_t>(stream)));
}

extern "C" const char* pr_strerror(int code)
{
    switch (code) {
    case PR_OK: return "success";
    case PR_ERR_INVALID_ARG: return "invalid argument";
    case PR_ERR_UNSUPPORTED: return "unsupported option";
    case PR_ERR_HIP: return "HIP runtime error";
    case PR_ERR_NO_MEMORY: return "workspace (or the static scratch of an allocation-free call) too small for this call";
    }
    return "unknown error code";
}

extern "C" int pr_version(void) { return 100; }
