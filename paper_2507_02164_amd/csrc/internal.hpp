// internal.hpp -- launchers shared between the C-ABI layer and the kernel
// translation units.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bin.hpp"
#include "proots.h"

namespace proots {

// Block sizes of the one-pass kernels, and the largest batch each launch
// covers: a one-dimensional grid holds at most 2^31 - 1 blocks (the density
// grid is rounded up to a multiple of 8 blocks, one share per XCD).
constexpr int kDensityBlock = 256;
constexpr int kBackwardBlock = 128;  // measured 2-4% faster than 64, 256, 512 or 1024
constexpr int kL2fitBlock = 256;
constexpr int64_t kMaxGridBlocks = 0x7fffffff;
constexpr int64_t kMaxSolveBatch = kMaxGridBlocks * 64;  // one-wave blocks
constexpr int64_t kMaxDensityBatch = (kMaxGridBlocks - 7) * kDensityBlock;
constexpr int64_t kMaxBackwardBatch = kMaxGridBlocks * kBackwardBlock;
constexpr int64_t kMaxL2fitBatch = kMaxGridBlocks * kL2fitBlock;

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
    int32_t grid_blocks;  // 0: one one-wave block per (tile, slice); > 0: persistent blocks
    // binning epilogue: win.hist == nullptr for none; else every root of a
    // polynomial whose final status has no bit of skip_mask is counted into
    // win.hist exactly as the density kernel would count it (roots may then
    // be nullptr: not stored)
    BinWindow win;
    uint32_t skip_mask;
    // PR_FLAG_FP64_FALLBACK (FP32 form): layout of the second, FP64 launch
    int32_t fallback_tile;
    int32_t fallback_grid;
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
    BinWindow win;
    // local-coordinate form: root w of polynomial i counts iff |w|^2 < rmax2
    // and is binned at centers[i] + radii[i] * w (centers == nullptr: plain)
    const pr_complex* centers;
    const double* radii;
    double rmax2;
};

hipError_t launch_density(const DensityArgs& a, hipStream_t stream);

// Tile-sorted counting (sortbin.hip): bytes of workspace a batch needs (0:
// counted by launch_density, no workspace), and the launches.
int64_t sortbin_workspace(int64_t n, int dmax, int width, int height);
hipError_t launch_density_sorted(const DensityArgs& a, void* workspace, int cus,
                                 hipStream_t stream);

// The allocation-free variant's static per-GPU workspace: its size, and its
// device address on the current GPU (nullptr if the lookup fails).
constexpr int64_t kSortScratchBytes = (int64_t)64 << 20;
void* sortbin_scratch();

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

constexpr int kMaxNr = 64;
constexpr int kMaxNt = 256;

// Product quadrature on the unit disk: radii r[k] with weights w[k] that
// already carry the r dr area factor and the 2 pi / nt angular step.
struct L2Quad {
    int32_t nr, nt;
    double r[kMaxNr];
    double w[kMaxNr];
};

struct L2FitArgs {
    const pr_complex* samples;
    int64_t n;
    int32_t degree;
    L2Quad quad;
    pr_complex* coeffs;
};

void gauss_legendre(int n, double* x, double* w);
void l2_quadrature(int nr, int nt, L2Quad& q);
hipError_t launch_l2fit(const L2FitArgs& a, hipStream_t stream);

}  // namespace proots
