"""Seeded synthetic inputs for the polynomial-root path.

Shared by the tests (GPU path and oracle alike), the smoke check and the
benchmark.  Nothing here computes roots, pixels or gradients: it only draws
coefficients (or builds them by expanding a product of linear factors) with
numpy's ``default_rng(seed)`` in a fixed draw order.

Layout of every coefficient array: complex128 ``[dmax + 1, n]`` with row k
holding a_k of p(z) = sum_k a_k z^k (structure of arrays), ``dmax = 6``.

Recipes (each a synthetic stand-in; the paper names no dataset):
  gaussian    monic degree 6, a_0..a_5 standard complex normal
              (Re, Im i.i.d. N(0, 1/2)).
  parametric  4096 x 4096 grid (g x g in general) of monic degree-6
              polynomials a_k = c_k + t1 d_k + t2 e_k, with c, d, e standard
              complex normal and (t1, t2) the grid's cell centres over
              [-1, 1]^2; polynomial j*g + i has t1 = centre i, t2 = centre j.
  mixed       degrees uniform over 2..6, leading coefficient 1, the others
              with modulus 10^U(-2, 2) and phase U(0, 2 pi); rows above the
              degree are zero.
  known_roots degree 6 from roots uniform by area in 0.5 < |z| < 2 with
              minimum pairwise gap >= 0.05 (whole-set rejection), product
              expanded in extended precision and rounded to FP64; targets
              are the roots plus 1e-2 standard complex normal noise.
  clustered   degree 6 from 3 roots within radius 1e-3 of a centre uniform
              in the unit disk plus 3 roots uniform in the unit disk,
              expanded in extended precision and rounded to FP64.
"""
from __future__ import annotations

import numpy as np

DMAX = 6
SQRT_HALF = np.sqrt(0.5)


def _par_cols(n: int, fn, min_chunk: int = 1 << 19) -> None:
    """Run fn(s, e) over column ranges that cover [0, n), on a thread pool
    (numpy's elementwise routines release the interpreter lock).  Only
    deterministic elementwise work goes through here -- never a random
    draw -- so every value is the one a single whole-array call gives."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    workers = min(16, os.cpu_count() or 1)
    if n <= min_chunk or workers == 1:
        fn(0, n)
        return
    step = max(min_chunk, -(-n // (4 * workers)))
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda s: fn(s, min(n, s + step)), range(0, n, step)))


def _cn(rng, shape):
    x = rng.standard_normal((2,) + tuple(shape))
    return (x[0] + 1j * x[1]) * SQRT_HALF


def gaussian(n: int, seed: int = 0) -> np.ndarray:
    """[7, n] complex128: monic degree 6, a_0..a_5 ~ CN(0, 1)."""
    rng = np.random.default_rng(seed)
    a = np.empty((DMAX + 1, n), dtype=np.complex128)
    a[:DMAX] = _cn(rng, (DMAX, n))
    a[DMAX] = 1.0
    return a


def grid_centres(g: int) -> np.ndarray:
    """Cell centres of g equal cells over [-1, 1]: -1 + (2i + 1) / g."""
    return -1.0 + (2.0 * np.arange(g, dtype=np.float64) + 1.0) / g


def parametric(g: int = 4096, seed: int = 0, rows: slice | None = None) -> np.ndarray:
    """[7, g*g] complex128 (or the grid rows ``rows`` only): a_k = c_k +
    t1 d_k + t2 e_k, t1 along a grid row, t2 across rows, a_6 = 1."""
    rng = np.random.default_rng(seed)
    c = _cn(rng, (DMAX,))
    d = _cn(rng, (DMAX,))
    e = _cn(rng, (DMAX,))
    t = grid_centres(g)
    jr = np.arange(g) if rows is None else np.arange(g)[rows]
    t1 = np.tile(t, jr.size)                 # column index i varies fastest
    t2 = np.repeat(t[jr], g)
    n = t1.size
    a = np.empty((DMAX + 1, n), dtype=np.complex128)
    for k in range(DMAX):
        # separate multiply and add: numpy does not fuse them
        a[k] = c[k] + t1 * d[k] + t2 * e[k]
    a[DMAX] = 1.0
    return a


def mixed(n: int, seed: int = 0):
    """(coeffs [7, n], degrees [n] int32): degrees 2..6, monic, other
    moduli log-uniform over [1e-2, 1e2], phases uniform."""
    rng = np.random.default_rng(seed)
    deg = rng.integers(2, DMAX + 1, n).astype(np.int32)
    lmag = rng.uniform(-2.0, 2.0, (DMAX, n))
    ph = rng.uniform(0.0, 2.0 * np.pi, (DMAX, n))
    a = np.zeros((DMAX + 1, n), dtype=np.complex128)
    k = np.arange(DMAX + 1)[:, None]

    def fill(s, e):
        blk = a[:, s:e]
        p = ph[:, s:e]
        blk[:DMAX] = 10.0 ** lmag[:, s:e] * (np.cos(p) + 1j * np.sin(p))
        dd = deg[None, s:e]
        blk[k > dd] = 0.0
        blk[k == dd] = 1.0

    _par_cols(n, fill)
    return a, deg


def expand_roots(roots: np.ndarray) -> np.ndarray:
    """Coefficients [d+1, n] (row k = a_k, a_d = 1) of prod_j (z - r_j),
    expanded in x87 extended precision and rounded once to complex128.
    ``roots`` is [d, n]."""
    roots = np.asarray(roots)
    d, n = roots.shape
    out = np.empty((d + 1, n), dtype=np.complex128)

    def expand(s, e):
        r = roots[:, s:e].astype(np.clongdouble)
        c = np.zeros((d + 1, e - s), dtype=np.clongdouble)
        c[0] = 1.0                             # c[k] = coefficient of z^k so far (degree 0)
        for j in range(d):
            # multiply current polynomial by (z - r_j)
            shifted = np.zeros_like(c)
            shifted[1:] = c[:-1]
            c = shifted - r[j][None, :] * c
        out[:, s:e] = c.astype(np.complex128)

    _par_cols(n, expand)
    return out


def _uniform_disk(rng, shape, rmin2=0.0, rmax2=1.0):
    rad = np.sqrt(rng.uniform(rmin2, rmax2, shape))
    ang = rng.uniform(0.0, 2.0 * np.pi, shape)
    return rad * (np.cos(ang) + 1j * np.sin(ang))


def known_roots(n: int, seed: int = 0, min_gap: float = 0.05):
    """(coeffs [7, n], roots [6, n], targets [6, n])."""
    rng = np.random.default_rng(seed)
    roots = _uniform_disk(rng, (DMAX, n), 0.25, 4.0)
    bad = np.arange(n)
    while bad.size:
        r = roots[:, bad]
        gap = np.full(bad.size, np.inf)
        for i in range(DMAX):
            for j in range(i + 1, DMAX):
                gap = np.minimum(gap, np.abs(r[i] - r[j]))
        bad = bad[gap < min_gap]
        if bad.size:
            roots[:, bad] = _uniform_disk(rng, (DMAX, bad.size), 0.25, 4.0)
    coeffs = expand_roots(roots)
    targets = roots + 1e-2 * _cn(rng, (DMAX, n))
    return coeffs, roots, targets


def clustered(n: int, seed: int = 0, radius: float = 1e-3):
    """(coeffs [7, n], roots [6, n]): rows 0..2 a cluster, rows 3..5 isolated."""
    rng = np.random.default_rng(seed)
    centre = _uniform_disk(rng, (n,))
    offs = radius * _uniform_disk(rng, (3, n))
    iso = _uniform_disk(rng, (3, n))
    roots = np.concatenate([centre[None, :] + offs, iso], axis=0)
    return expand_roots(roots), roots


def cotangents(n: int, seed: int = 1, dmax: int = DMAX) -> np.ndarray:
    """[dmax, n] complex128 root cotangents ~ CN(0, 1) (for timing backward)."""
    rng = np.random.default_rng(seed)
    return _cn(rng, (dmax, n))


# Named configurations: full sizes and the windows they are binned over.
PARAMETRIC_WINDOW = (-16.0 / 3.0, 16.0 / 3.0, -3.0, 3.0)      # 1920 x 1080, square pixels
CLUSTERED_WINDOW = (-20.0 / 9.0, 20.0 / 9.0, -1.25, 1.25)     # 1920 x 1080, square pixels
GAUSSIAN_WINDOW = (-3.0, 3.0, -3.0, 3.0)                       # 256 x 256

CONFIGS = {
    "gaussian": dict(n=65536, window=GAUSSIAN_WINDOW, shape=(256, 256)),
    "parametric": dict(g=4096, n=4096 * 4096, window=PARAMETRIC_WINDOW, shape=(1920, 1080)),
    "mixed": dict(n=64 * 2 ** 20),
    "known_roots": dict(n=4 * 2 ** 20),
    "clustered": dict(n=16 * 2 ** 20, window=CLUSTERED_WINDOW, shape=(1920, 1080)),
}
