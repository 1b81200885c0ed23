"""ctypes binding of the C ABI in include/proots.h.

Argument marshalling only: torch supplies device memory and the current HIP
stream; every step of the computation runs in the HIP library.  There is no
CPU fallback -- without the built library or a GPU every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libproots.so")

PR_OK = 0
PR_ERR_INVALID_ARG = -1
PR_ERR_UNSUPPORTED = -2
PR_ERR_HIP = -3
PR_ERR_NO_MEMORY = -4

ST_BAD_DEGREE = 1 << 0
ST_NONFINITE = 1 << 1
ST_ZERO_LEADING = 1 << 2
ST_NOT_CONVERGED = 1 << 3
ST_POLISH_UNCONVERGED = 1 << 4
ST_SINGULAR_DERIV = 1 << 5
ST_RESOLVED_FP64 = 1 << 6

FP64 = 0
FP32_POLISH = 1
PRECISIONS = {"fp64": FP64, "fp32_polish": FP32_POLISH}

FLAG_NO_EXCEPTIONAL_SHIFT = 1 << 0
FLAG_FIXED_STEPS = 1 << 1
FLAG_FP64_FALLBACK = 1 << 2
FLAG_RAYLEIGH_SHIFT = 1 << 3
FLAG_PAIRED_LANES = 1 << 4
FLAG_RUN_AHEAD = 1 << 5


class ProotsError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} (code {code})")


class SolveOpts(ctypes.Structure):
    """Mirror of pr_solve_opts."""
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("max_iter_per_level", ctypes.c_int32),
        ("polish_steps", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("polish_tol", ctypes.c_double),
        ("iter_counts", ctypes.c_void_p),
        ("tile", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libproots.so (built by ``python -m paper_2507_02164_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2507_02164_amd.build` "
                              "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32, U32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
        L.pr_solve.argtypes = [P, P, I64, I32, P, P, ctypes.POINTER(SolveOpts), P]
        L.pr_solve.restype = ctypes.c_int
        L.pr_density.argtypes = [P, P, P, U32, I64, I32, D, D, D, D, I32, I32, P, P]
        L.pr_density.restype = ctypes.c_int
        L.pr_solve_bin.argtypes = [P, P, I64, I32, P, P, ctypes.POINTER(SolveOpts), U32, D, D, D,
                                   D, I32, I32, P, P]
        L.pr_solve_bin.restype = ctypes.c_int
        L.pr_backward.argtypes = [P, P, P, P, I64, I32, P, P, P]
        L.pr_backward.restype = ctypes.c_int
        L.pr_density_sorted.argtypes = [P, P, P, U32, I64, I32, D, D, D, D, I32, I32, P, P, I64, P]
        L.pr_density_sorted.restype = ctypes.c_int
        L.pr_density_sorted_noalloc.argtypes = [P, P, P, U32, I64, I32, D, D, D, D, I32, I32, P, P]
        L.pr_density_sorted_noalloc.restype = ctypes.c_int
        L.pr_density_sorted_workspace.argtypes = [I64, I32, I32, I32]
        L.pr_density_sorted_workspace.restype = ctypes.c_int64
        L.pr_density_local.argtypes = [P, P, P, U32, I64, I32, P, P, D, D, D, D, D, I32, I32, P, P]
        L.pr_density_local.restype = ctypes.c_int
        L.pr_l2fit_nodes.argtypes = [I32, I32, P, P]
        L.pr_l2fit_nodes.restype = ctypes.c_int
        L.pr_l2fit.argtypes = [P, I64, I32, I32, I32, P, P]
        L.pr_l2fit.restype = ctypes.c_int
        L.pr_strerror.argtypes = [ctypes.c_int]
        L.pr_strerror.restype = ctypes.c_char_p
        L.pr_version.argtypes = []
        L.pr_version.restype = ctypes.c_int
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().pr_strerror(code).decode()


def version() -> int:
    return lib().pr_version()


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check(t, name, dtype, shape=None, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor (the library has no CPU path)")
    if device is not None and t.device != device:
        # a pointer into another GPU's memory would be read by this GPU's kernel
        raise ValueError(f"{name} must be on {device} like the other arrays, got {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _prepare_solve(coeffs, degrees, precision, max_iter_per_level, polish_steps, polish_tol,
                   flags, iter_counts, roots, status, tile, grid_blocks, want_roots=True):
    """Shared argument checks, output allocation and options of pr_solve and
    pr_solve_bin."""
    _check(coeffs, "coeffs", torch.complex128)
    if coeffs.dim() != 2:
        raise ValueError("coeffs must be 2-D [dmax+1, n]")
    dmax = coeffs.shape[0] - 1
    n = coeffs.shape[1]
    dev = coeffs.device
    if degrees is not None:
        _check(degrees, "degrees", torch.int32, (n,), device=coeffs.device)
    if roots is None and want_roots:
        roots = torch.empty((max(dmax, 0), n), dtype=torch.complex128, device=dev)
    if roots is not None:
        _check(roots, "roots", torch.complex128, (dmax, n), device=coeffs.device)
    if status is None:
        status = torch.empty((n,), dtype=torch.int32, device=dev)
    _check(status, "status", torch.int32, (n,), device=coeffs.device)
    its = None
    if iter_counts:
        its = torch.empty((max(dmax - 1, 0), n), dtype=torch.int32, device=dev)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    if max_iter_per_level is None or tile is None or grid_blocks is None:
        from . import autotune
        name = {v: k for k, v in PRECISIONS.items()}.get(prec, str(prec))
        tuned = autotune.tuned_options(name, dmax, degrees is not None, dev, n)
        if max_iter_per_level is None:
            max_iter_per_level = tuned.get("max_iter_per_level", 0)
        # the tuned layout (tile, and its flags) only when the caller left
        # the layout to the tuner
        layout_tuned = tile is None
        if tile is None:
            tile = tuned.get("tile", 0)
        if grid_blocks is None:
            grid_blocks = tuned.get("grid_blocks", 0)
        if layout_tuned and tuned.get("paired") and tile == -1:
            flags |= FLAG_PAIRED_LANES
        if layout_tuned and tuned.get("ahead") and (tile == -1 or (tile > 0 and grid_blocks == 0)):
            flags |= FLAG_RUN_AHEAD
    opts = SolveOpts(prec, max_iter_per_level, polish_steps, flags, polish_tol,
                     None if its is None or its.numel() == 0 else its.data_ptr(), tile, grid_blocks)
    return dmax, n, roots, status, its, opts


def solve(coeffs, degrees=None, precision="fp64", *, max_iter_per_level=None, polish_steps=0,
          polish_tol=0.0, flags=0, iter_counts=False, roots=None, status=None, stream=None,
          tile=None, grid_blocks=None):
    """Roots of each column of ``coeffs`` (complex128 [dmax+1, n], row k =
    a_k).  Returns ``(roots complex128 [dmax, n], status int32 [n])``, plus
    the per-level QR step counts int32 [dmax-1, n] when ``iter_counts``.
    Status bits are the ST_* constants (the int32 holds the uint32 bits).
    Launch layout and iteration cap left as None come from the autotuner's
    cache for this GPU (library defaults when nothing was tuned)."""
    dmax, n, roots, status, its, opts = _prepare_solve(
        coeffs, degrees, precision, max_iter_per_level, polish_steps, polish_tol, flags,
        iter_counts, roots, status, tile, grid_blocks)
    with torch.cuda.device(coeffs.device):
        rc = lib().pr_solve(_ptr(coeffs), _ptr(degrees), n, dmax, _ptr(roots), _ptr(status),
                            ctypes.byref(opts), _stream(stream))
    if rc != PR_OK:
        raise ProotsError(rc, "pr_solve")
    if iter_counts:
        return roots, status, its
    return roots, status


def solve_bin(coeffs, window, shape, degrees=None, precision="fp64", *, skip_mask=0, out=None,
              store_roots=True, max_iter_per_level=None, polish_steps=0, polish_tol=0.0, flags=0,
              iter_counts=False, roots=None, status=None, stream=None, tile=None,
              grid_blocks=None):
    """``solve`` and ``density`` in one launch: the roots are counted into
    the int32 [height, width] image ``out`` (a new zeroed one when None) as
    they are found.  Returns ``(roots or None, status, image)`` (plus the
    step counts with ``iter_counts``); with ``store_roots=False`` and no
    ``roots`` array the roots are not written at all."""
    dmax, n, roots, status, its, opts = _prepare_solve(
        coeffs, degrees, precision, max_iter_per_level, polish_steps, polish_tol, flags,
        iter_counts, roots, status, tile, grid_blocks, want_roots=store_roots)
    x0, x1, y0, y1 = (float(v) for v in window)
    width, height = (int(v) for v in shape)
    if out is None:
        out = torch.zeros((height, width), dtype=torch.int32, device=coeffs.device)
    _check(out, "out", torch.int32, (height, width), device=coeffs.device)
    with torch.cuda.device(coeffs.device):
        rc = lib().pr_solve_bin(_ptr(coeffs), _ptr(degrees), n, dmax, _ptr(roots), _ptr(status),
                                ctypes.byref(opts), skip_mask & 0xFFFFFFFF, x0, x1, y0, y1, width,
                                height, _ptr(out), _stream(stream))
    if rc != PR_OK:
        raise ProotsError(rc, "pr_solve_bin")
    if iter_counts:
        return roots, status, out, its
    return roots, status, out


def density(roots, window, shape, degrees=None, status=None, skip_mask=0, out=None, stream=None):
    """Count roots into an int32 [height, width] image over the half-open
    window (x0, x1, y0, y1); row 0 holds the lowest imaginary parts.  Counts
    are added to ``out`` when given (a new zeroed image otherwise)."""
    _check(roots, "roots", torch.complex128)
    if roots.dim() != 2:
        raise ValueError("roots must be 2-D [dmax, n]")
    dmax, n = roots.shape
    x0, x1, y0, y1 = (float(v) for v in window)
    width, height = (int(v) for v in shape)
    if out is None:
        out = torch.zeros((height, width), dtype=torch.int32, device=roots.device)
    _check(out, "out", torch.int32, (height, width), device=roots.device)
    if degrees is not None:
        _check(degrees, "degrees", torch.int32, (n,), device=roots.device)
    if status is not None:
        _check(status, "status", torch.int32, (n,), device=roots.device)
    with torch.cuda.device(roots.device):
        rc = lib().pr_density(_ptr(roots), _ptr(degrees), _ptr(status), skip_mask & 0xFFFFFFFF, n,
                              dmax, x0, x1, y0, y1, width, height, _ptr(out), _stream(stream))
    if rc != PR_OK:
        raise ProotsError(rc, "pr_density")
    return out


def density_sorted_workspace(n: int, dmax: int, width: int, height: int) -> int:
    """Bytes of device workspace ``density_sorted`` needs (0: none)."""
    b = lib().pr_density_sorted_workspace(int(n), int(dmax), int(width), int(height))
    if b < 0:
        raise ProotsError(int(b), "pr_density_sorted_workspace")
    return int(b)


def density_sorted(roots, window, shape, degrees=None, status=None, skip_mask=0, out=None,
                   workspace=None, stream=None):
    """``density`` through image tiles counted on chip (pr_density_sorted):
    the same image bit for bit, faster for roots spread over the image.
    ``workspace`` is a uint8 GPU tensor of at least
    ``density_sorted_workspace(n, dmax, width, height)`` bytes (a new one
    when None)."""
    _check(roots, "roots", torch.complex128)
    if roots.dim() != 2:
        raise ValueError("roots must be 2-D [dmax, n]")
    dmax, n = roots.shape
    x0, x1, y0, y1 = (float(v) for v in window)
    width, height = (int(v) for v in shape)
    if out is None:
        out = torch.zeros((height, width), dtype=torch.int32, device=roots.device)
    _check(out, "out", torch.int32, (height, width), device=roots.device)
    if degrees is not None:
        _check(degrees, "degrees", torch.int32, (n,), device=roots.device)
    if status is not None:
        _check(status, "status", torch.int32, (n,), device=roots.device)
    if workspace is None:
        need = density_sorted_workspace(n, dmax, width, height) if n > 0 else 0
        workspace = torch.empty((max(need, 1),), dtype=torch.uint8, device=roots.device)
    _check(workspace, "workspace", torch.uint8, device=roots.device)
    with torch.cuda.device(roots.device):
        rc = lib().pr_density_sorted(_ptr(roots), _ptr(degrees), _ptr(status),
                                     skip_mask & 0xFFFFFFFF, n, dmax, x0, x1, y0, y1, width, height,
                                     _ptr(out), _ptr(workspace), workspace.numel(), _stream(stream))
    if rc != PR_OK:
        raise ProotsError(rc, "pr_density_sorted")
    return out


NOALLOC_SCRATCH_BYTES = 1 << 26   # the static per-GPU array of pr_density_sorted_noalloc


def density_sorted_noalloc(roots, window, shape, degrees=None, status=None, skip_mask=0,
                           out=None, stream=None):
    """``density_sorted`` through the allocation-free entry point
    (pr_density_sorted_noalloc): the library's static per-GPU scratch array
    serves as the workspace, so the call allocates nothing (``out`` must then
    be given by callers that cannot allocate).  Batches needing more than
    NOALLOC_SCRATCH_BYTES raise ProotsError(PR_ERR_NO_MEMORY); calls that
    overlap on one GPU race."""
    _check(roots, "roots", torch.complex128)
    if roots.dim() != 2:
        raise ValueError("roots must be 2-D [dmax, n]")
    dmax, n = roots.shape
    x0, x1, y0, y1 = (float(v) for v in window)
    width, height = (int(v) for v in shape)
    if out is None:
        out = torch.zeros((height, width), dtype=torch.int32, device=roots.device)
    _check(out, "out", torch.int32, (height, width), device=roots.device)
    if degrees is not None:
        _check(degrees, "degrees", torch.int32, (n,), device=roots.device)
    if status is not None:
        _check(status, "status", torch.int32, (n,), device=roots.device)
    with torch.cuda.device(roots.device):
        rc = lib().pr_density_sorted_noalloc(_ptr(roots), _ptr(degrees), _ptr(status),
                                             skip_mask & 0xFFFFFFFF, n, dmax, x0, x1, y0, y1, width,
                                             height, _ptr(out), _stream(stream))
    if rc != PR_OK:
        raise ProotsError(rc, "pr_density_sorted_noalloc")
    return out


def backward(coeffs, roots, grad_roots, degrees=None, status=None, grad_coeffs=None, stream=None):
    """Coefficient cotangents from root cotangents (PyTorch's convention
    dL/dRe + i dL/dIm).  ``status`` (int32 [n]) is read and SINGULAR_DERIV is
    or-ed into it in place; a zero status is used when it is None.  Returns
    ``(grad_coeffs complex128 [dmax+1, n], status)``."""
    _check(coeffs, "coeffs", torch.complex128)
    dmax = coeffs.shape[0] - 1
    n = coeffs.shape[1]
    _check(roots, "roots", torch.complex128, (dmax, n), device=coeffs.device)
    _check(grad_roots, "grad_roots", torch.complex128, (dmax, n), device=coeffs.device)
    if degrees is not None:
        _check(degrees, "degrees", torch.int32, (n,), device=coeffs.device)
    if status is None:
        status = torch.zeros((n,), dtype=torch.int32, device=coeffs.device)
    _check(status, "status", torch.int32, (n,), device=coeffs.device)
    if grad_coeffs is None:
        grad_coeffs = torch.empty_like(coeffs)
    _check(grad_coeffs, "grad_coeffs", torch.complex128, (dmax + 1, n), device=coeffs.device)
    with torch.cuda.device(coeffs.device):
        rc = lib().pr_backward(_ptr(coeffs), _ptr(degrees), _ptr(roots), _ptr(grad_roots), n, dmax,
                               _ptr(grad_coeffs), _ptr(status), _stream(stream))
    if rc != PR_OK:
        raise ProotsError(rc, "pr_backward")
    return grad_coeffs, status


def l2fit_nodes(nr: int, nt: int):
    """Quadrature nodes w_q (complex, [nr*nt]) and weights ([nr*nt], sum pi)
    on the unit disk at which to sample f for ``l2fit`` (host arrays)."""
    import numpy as np
    nodes = np.empty(2 * nr * nt, dtype=np.float64)
    weights = np.empty(nr * nt, dtype=np.float64)
    rc = lib().pr_l2fit_nodes(nr, nt, nodes.ctypes.data, weights.ctypes.data)
    if rc != PR_OK:
        raise ProotsError(rc, "pr_l2fit_nodes")
    return nodes.view(np.complex128), weights


def l2fit(samples, degree: int, nr: int, nt: int, coeffs=None, stream=None):
    """Least-squares polynomial approximation (Sec. II-A) on each disk:
    ``samples`` complex128 [nr*nt, n] (f at the ``l2fit_nodes`` of each
    disk) -> coefficients complex128 [degree+1, n] in the disk's local
    variable."""
    _check(samples, "samples", torch.complex128, (nr * nt, samples.shape[1]))
    n = samples.shape[1]
    if coeffs is None:
        coeffs = torch.empty((degree + 1, n), dtype=torch.complex128, device=samples.device)
    _check(coeffs, "coeffs", torch.complex128, (degree + 1, n), device=samples.device)
    with torch.cuda.device(samples.device):
        rc = lib().pr_l2fit(_ptr(samples), n, degree, nr, nt, _ptr(coeffs), _stream(stream))
    if rc != PR_OK:
        raise ProotsError(rc, "pr_l2fit")
    return coeffs


def density_local(roots, centers, radii, window, shape, rmax2=1.0, degrees=None, status=None,
                  skip_mask=0, out=None, stream=None):
    """``density`` for roots in local disk coordinates: root w of polynomial
    i counts iff |w|^2 < rmax2, at z = centers[i] + radii[i] * w."""
    _check(roots, "roots", torch.complex128)
    dmax, n = roots.shape
    _check(centers, "centers", torch.complex128, (n,), device=roots.device)
    _check(radii, "radii", torch.float64, (n,), device=roots.device)
    x0, x1, y0, y1 = (float(v) for v in window)
    width, height = (int(v) for v in shape)
    if out is None:
        out = torch.zeros((height, width), dtype=torch.int32, device=roots.device)
    _check(out, "out", torch.int32, (height, width), device=roots.device)
    if degrees is not None:
        _check(degrees, "degrees", torch.int32, (n,), device=roots.device)
    if status is not None:
        _check(status, "status", torch.int32, (n,), device=roots.device)
    with torch.cuda.device(roots.device):
        rc = lib().pr_density_local(_ptr(roots), _ptr(degrees), _ptr(status), skip_mask & 0xFFFFFFFF,
                                    n, dmax, _ptr(centers), _ptr(radii), float(rmax2), x0, x1, y0,
                                    y1, width, height, _ptr(out), _stream(stream))
    if rc != PR_OK:
        raise ProotsError(rc, "pr_density_local")
    return out
