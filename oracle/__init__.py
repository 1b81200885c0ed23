"""Plain FP64 CPU oracle for the batched polynomial-root path.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  It shares
no code with the HIP path.

The arithmetic lives in ``oracle.c`` (plain C99 complex doubles, dense
storage, -O2 -ffp-contract=off).  This module compiles it with gcc on first
use when the shared library is missing, and wraps it for numpy arrays.

What each function follows in arXiv 2507.02164:
  solve     -- Sec. II-B (companion matrix, Alg. 1 single-shift QR iteration)
               and Sec. II-C (the Givens rotations whose product gives each
               step's QR factorisation; the step itself is formed with dense
               matrix products), with a
               convergence test and exceptional shift where the paper has a
               fixed iteration count (``fixed_t`` reproduces Alg. 2), and,
               with ``FLAG_WILKINSON_SHIFT``, Wilkinson's shift (the
               eigenvalue of the trailing 2 x 2 block nearest its bottom
               entry) in place of Alg. 1's bottom-right entry; with
               ``FLAG_QUADRATIC_START`` the first step of each polynomial is
               shifted by the root nearest 0 of b0 + b1 z + b2 z^2.
  density   -- Sec. III, roots converted to pixel coordinates and counted.
  backward  -- not in the paper: the implicit-function derivative
               dr/da_k = -r^k / p'(r) of a simple root.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

ST_BAD_DEGREE = 0x1
ST_NONFINITE = 0x2
ST_ZERO_LEADING = 0x4
ST_NOT_CONVERGED = 0x8
ST_SINGULAR_DERIV = 0x20

FLAG_NO_EXCEPTIONAL_SHIFT = 0x1
FLAG_WILKINSON_SHIFT = 0x8
FLAG_QUADRATIC_START = 0x10

_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain IEEE doubles)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_solve.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, P, P, P, ctypes.c_int,
                                     ctypes.c_uint, ctypes.c_int, ctypes.c_int]
        lib.oracle_solve.restype = None
        lib.oracle_density.argtypes = [P, P, P, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int, ctypes.c_int, P]
        lib.oracle_density.restype = None
        lib.oracle_density_local.argtypes = [P, P, P, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int,
                                             P, P, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_int, ctypes.c_int, P]
        lib.oracle_density_local.restype = None
        lib.oracle_backward.argtypes = [P, P, P, P, ctypes.c_int64, ctypes.c_int, P, P, ctypes.c_int]
        lib.oracle_backward.restype = None
        lib.oracle_givens.argtypes = [P, P, P, P]
        lib.oracle_givens.restype = None
        lib.oracle_qr_step.argtypes = [ctypes.c_int, P, P]
        lib.oracle_qr_step.restype = None
        lib.oracle_wilkinson_shift.argtypes = [P, P, P, P, P]
        lib.oracle_wilkinson_shift.restype = None
        lib.oracle_quadratic_start.argtypes = [P, P, P, P]
        lib.oracle_quadratic_start.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c128(x, shape=None):
    a = np.ascontiguousarray(x, dtype=np.complex128)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _degrees(degrees, n):
    if degrees is None:
        return None
    d = np.ascontiguousarray(degrees, dtype=np.int32)
    if d.shape != (n,):
        raise ValueError("degrees must have shape (n,)")
    return d


def max_threads() -> int:
    return _load().oracle_max_threads()


def solve(coeffs, degrees=None, *, cap: int = 30, flags: int = 0, fixed_t: int = 0,
          nthreads: int = 0, return_iters: bool = False):
    """Roots of each column of ``coeffs`` ([dmax+1, n] complex, row k = a_k).

    Returns ``(roots [dmax, n] complex128 in deflation order, NaN beyond the
    degree; status [n] uint32)`` and, with ``return_iters``, the QR steps per
    level ``[dmax-1, n]`` (row m-2 = level m)."""
    coeffs = _c128(coeffs)
    if coeffs.ndim != 2 or not (2 <= coeffs.shape[0] <= 7):
        raise ValueError("coeffs must be [dmax+1, n] with 1 <= dmax <= 6")
    dmax = coeffs.shape[0] - 1
    n = coeffs.shape[1]
    deg = _degrees(degrees, n)
    roots = np.empty((dmax, n), dtype=np.complex128)
    status = np.zeros(n, dtype=np.uint32)
    iters = np.zeros((max(dmax - 1, 0), n), dtype=np.int32)
    _load().oracle_solve(_ptr(coeffs), _ptr(deg), n, dmax, _ptr(roots), _ptr(status),
                         _ptr(iters) if dmax > 1 else None, cap, flags, fixed_t, nthreads)
    if return_iters:
        return roots, status, iters
    return roots, status


def density(roots, window, shape, degrees=None, status=None, skip_mask: int = 0, out=None):
    """Count roots per pixel.  ``window`` = (x0, x1, y0, y1), half-open;
    ``shape`` = (width, height); result int32 [height, width], row 0 = lowest
    imaginary part.  Counts are added to ``out`` when given."""
    roots = _c128(roots)
    dmax, n = roots.shape
    x0, x1, y0, y1 = (float(v) for v in window)
    width, height = (int(v) for v in shape)
    if out is None:
        out = np.zeros((height, width), dtype=np.int32)
    assert out.dtype == np.int32 and out.shape == (height, width) and out.flags.c_contiguous
    deg = _degrees(degrees, n)
    st = None if status is None else np.ascontiguousarray(status, dtype=np.uint32)
    _load().oracle_density(_ptr(roots), _ptr(deg), _ptr(st), skip_mask, n, dmax,
                           x0, x1, y0, y1, width, height, _ptr(out))
    return out


def density_local(roots, centers, radii, window, shape, rmax2=1.0, degrees=None, status=None,
                  skip_mask: int = 0, out=None):
    """``density`` for roots in local disk coordinates w: a root counts iff
    |w|^2 < rmax2, placed at centers[i] + radii[i] * w."""
    roots = _c128(roots)
    dmax, n = roots.shape
    centers = _c128(centers, (n,))
    radii = np.ascontiguousarray(radii, dtype=np.float64)
    x0, x1, y0, y1 = (float(v) for v in window)
    width, height = (int(v) for v in shape)
    if out is None:
        out = np.zeros((height, width), dtype=np.int32)
    deg = _degrees(degrees, n)
    st = None if status is None else np.ascontiguousarray(status, dtype=np.uint32)
    _load().oracle_density_local(_ptr(roots), _ptr(deg), _ptr(st), skip_mask, n, dmax,
                                 _ptr(centers), _ptr(radii), float(rmax2), x0, x1, y0, y1,
                                 width, height, _ptr(out))
    return out


def l2_nodes(nr: int, nt: int):
    """Product quadrature on the unit disk (Sec. II-A inner product):
    nr Gauss-Legendre radii (numpy's rule mapped to [0, 1], weight r dr) times
    nt equally spaced angles.  Returns (nodes complex [nr*nt], weights)."""
    x, w = np.polynomial.legendre.leggauss(nr)
    r = 0.5 * (x + 1.0)
    wr = 0.5 * w * r
    th = 2.0 * np.pi * np.arange(nt) / nt
    nodes = (r[:, None] * np.exp(1j * th)[None, :]).ravel()
    weights = np.repeat(wr * (2.0 * np.pi / nt), nt)
    return nodes, weights


def l2fit(samples, nodes, weights, degree):
    """Sec. II-A: coefficients a of the polynomial p(w) = sum_k a_k w^k that
    minimises ||f - p|| for <g, h> = integral over the unit disk of g conj(h),
    from the normal equations G a = b with G_jk = <w^j, w^k> and
    b_j = <f, w^j>, both by the given quadrature (G is assembled in full and
    solved, not assumed diagonal).  samples [Q, n] -> coefficients
    [degree+1, n]."""
    samples = np.asarray(samples, dtype=np.complex128)
    V = nodes[None, :] ** np.arange(degree + 1)[:, None]             # [deg+1, Q]: w^j
    G = (V * weights[None, :]) @ V.conj().T                          # <w^j, w^k> = sum w_q^j conj(w_q^k)
    # G_jk = <z^j, z^k> = integral z^j conj(z)^k: row j, column k
    B = (V.conj() * weights[None, :]) @ samples                      # b_j = sum f conj(w^j)
    return np.linalg.solve(G.T, B)                                    # sum_k G_kj a_k = b_j


def backward(coeffs, roots, grad_roots, degrees=None, status=None, nthreads: int = 0):
    """Cotangent of the coefficients given root cotangents (PyTorch's
    convention dL/dRe + i dL/dIm).  Returns ``(grad_coeffs [dmax+1, n],
    status)`` with SINGULAR_DERIV or-ed in."""
    coeffs = _c128(coeffs)
    dmax = coeffs.shape[0] - 1
    n = coeffs.shape[1]
    roots = _c128(roots, (dmax, n))
    grad_roots = _c128(grad_roots, (dmax, n))
    deg = _degrees(degrees, n)
    st = np.zeros(n, dtype=np.uint32) if status is None else np.array(status, dtype=np.uint32, copy=True)
    grad = np.empty((dmax + 1, n), dtype=np.complex128)
    _load().oracle_backward(_ptr(coeffs), _ptr(deg), _ptr(roots), _ptr(grad_roots), n, dmax,
                            _ptr(grad), _ptr(st), nthreads)
    return grad, st


def givens(a: complex, b: complex):
    """(c, s) of the Sec. II-C rotation for the pair (a, b)."""
    A = np.array([a.real, a.imag]); B = np.array([b.real, b.imag])
    C = np.zeros(2); S = np.zeros(2)
    _load().oracle_givens(_ptr(A), _ptr(B), _ptr(C), _ptr(S))
    return complex(C[0], C[1]), complex(S[0], S[1])


def wilkinson_shift(a: complex, b: complex, c: complex, e: complex) -> complex:
    """Eigenvalue of [[a, b], [c, e]] nearest e (the shift taken with
    ``FLAG_WILKINSON_SHIFT`` instead of Alg. 1's bottom-right entry)."""
    v = [np.array([z.real, z.imag]) for z in (complex(a), complex(b), complex(c), complex(e))]
    mu = np.zeros(2)
    _load().oracle_wilkinson_shift(*(_ptr(x) for x in v), _ptr(mu))
    return complex(mu[0], mu[1])


def quadratic_start(b0: complex, b1: complex, b2: complex):
    """The root nearest 0 of b0 + b1 z + b2 z^2 and whether it is defined
    (the first shift taken with ``FLAG_QUADRATIC_START``)."""
    v = [np.array([z.real, z.imag]) for z in (complex(b0), complex(b1), complex(b2))]
    z = np.zeros(2)
    ok = _load().oracle_quadratic_start(*(_ptr(x) for x in v), _ptr(z))
    return complex(z[0], z[1]), bool(ok)


def qr_step(H, shift: complex):
    """One shifted QR step (Alg. 1 body: A - sI = QR with Q from the Sec.
    II-C rotations, A <- RQ + sI by dense products) on a dense square
    complex matrix; returns the new matrix."""
    H = np.array(H, dtype=np.complex128, copy=True, order="C")
    m = H.shape[0]
    assert H.shape == (m, m) and 1 <= m <= 6
    s = np.array([shift.real, shift.imag])
    _load().oracle_qr_step(m, _ptr(H), _ptr(s))
    return H
