"""Batched complex polynomial roots and root-density images on AMD MI355X.

Implements the hot path of Tang & Quan, "Hardware-Accelerated Algorithm for
Complex Function Roots Density Graph Plotting" (arXiv 2507.02164):
companion-matrix eigenvalues by single-shift Givens QR iteration
(Sec. II-B/II-C, Alg. 1-2), roots binned into a density image (Sec. III),
plus the implicit-function root adjoint.

The computation lives in hand-written HIP kernels for gfx950 behind a C ABI
(include/proots.h, libproots.so); this package only marshals torch tensors
into it.  Build with ``python -m paper_2507_02164_amd.build``.
"""
from ._capi import (FLAG_FIXED_STEPS, FLAG_FP64_FALLBACK, FLAG_NO_EXCEPTIONAL_SHIFT,
                    FLAG_PAIRED_LANES, FLAG_RAYLEIGH_SHIFT, FLAG_RUN_AHEAD, FP32_POLISH, FP64,
                    NOALLOC_SCRATCH_BYTES, PR_ERR_HIP, PR_ERR_INVALID_ARG, PR_ERR_NO_MEMORY,
                    PR_ERR_UNSUPPORTED, PR_OK, ST_BAD_DEGREE, ST_NONFINITE, ST_NOT_CONVERGED,
                    ST_POLISH_UNCONVERGED, ST_RESOLVED_FP64, ST_SINGULAR_DERIV, ST_ZERO_LEADING,
                    ProotsError, SolveOpts, backward, density, density_local, density_sorted,
                    density_sorted_noalloc, density_sorted_workspace, l2fit, l2fit_nodes, lib,
                    solve, solve_bin, strerror, version)
from .autograd import RootsFn, roots

__all__ = [
    "solve", "solve_bin", "density", "density_sorted", "density_sorted_noalloc",
    "density_sorted_workspace", "backward", "l2fit", "l2fit_nodes", "density_local", "RootsFn",
    "roots", "lib", "strerror", "version", "ProotsError", "SolveOpts", "FP64", "FP32_POLISH",
    "FLAG_NO_EXCEPTIONAL_SHIFT", "FLAG_FIXED_STEPS", "FLAG_FP64_FALLBACK", "FLAG_RAYLEIGH_SHIFT",
    "FLAG_PAIRED_LANES", "FLAG_RUN_AHEAD",
    "NOALLOC_SCRATCH_BYTES", "PR_OK", "PR_ERR_INVALID_ARG", "PR_ERR_UNSUPPORTED", "PR_ERR_HIP",
    "PR_ERR_NO_MEMORY", "ST_BAD_DEGREE", "ST_NONFINITE", "ST_ZERO_LEADING", "ST_NOT_CONVERGED",
    "ST_POLISH_UNCONVERGED", "ST_SINGULAR_DERIV", "ST_RESOLVED_FP64",
]
