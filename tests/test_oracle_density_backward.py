"""Pins of the oracle's density binning and root adjoint (CPU only).

Density (Sec. III, roots converted to pixel coordinates and counted):
brute force in plain Python on small inputs, hand-built bin-edge cases, and
the total count.

Backward (implicit-function derivative of a simple root, not in the paper):
closed forms for degrees 1 and 2, central finite differences of the forward
solve with the root assignment frozen, the product form of p'(r), and the
singular-derivative flag on an exact double root.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
import workloads
from rootmatch import match


def _brute_density(roots, degrees, status, skip_mask, window, shape):
    x0, x1, y0, y1 = window
    W, H = shape
    sx = W / (x1 - x0)
    sy = H / (y1 - y0)
    hist = [[0] * W for _ in range(H)]
    dmax, n = roots.shape
    for i in range(n):
        if status is not None and (int(status[i]) & skip_mask):
            continue
        d = dmax if degrees is None else min(int(degrees[i]), dmax)
        for k in range(d):
            z = complex(roots[k, i])
            u = (z.real - x0) * sx
            v = (z.imag - y0) * sy
            if 0.0 <= u < W and 0.0 <= v < H:       # False for NaN
                hist[math.floor(v)][math.floor(u)] += 1
    return np.array(hist, dtype=np.int32)


def test_density_brute_force():
    rng = np.random.default_rng(0)
    n = 700
    roots = (rng.uniform(-1.3, 1.3, (6, n)) + 1j * rng.uniform(-1.2, 1.2, (6, n)))
    roots[rng.random((6, n)) < 0.02] = np.nan
    roots[0, :5] = np.inf
    deg = rng.integers(0, 8, n).astype(np.int32)
    st = rng.integers(0, 64, n).astype(np.uint32)
    window = (-1.0, 1.0, -0.75, 1.0)
    for shape in [(37, 23), (64, 64), (5, 1)]:
        for degrees, status, skip in [(None, None, 0), (deg, st, 0x9), (deg, None, 0)]:
            got = oracle.density(roots, window, shape, degrees, status, skip)
            want = _brute_density(roots, degrees, status, skip, window, shape)
            assert np.array_equal(got, want)


def test_density_edges():
    window = (-2.0, 2.0, -1.0, 1.0)
    shape = (4, 2)                                  # pixels 1.0 wide, 1.0 tall
    pts = np.array([
        -2.0 - 1.0j,          # exact lower-left corner -> (row 0, col 0)
        2.0 + 0.0j,           # re == x1 -> dropped (half-open)
        1.999999 + 0.999999j, # last pixel (row 1, col 3)
        0.0 + 1.0j,           # im == y1 -> dropped
        np.nan + 0.0j,        # NaN -> dropped
        -0.5 - 0.25j,         # row 0, col 1
    ])
    roots = pts[:, None].T.copy()                   # [6, 1] as one degree-6 polynomial
    got = oracle.density(roots.T.reshape(6, 1), window, shape)
    want = np.zeros((2, 4), dtype=np.int32)
    want[0, 0] = 1
    want[1, 3] = 1
    want[0, 1] = 1
    assert np.array_equal(got, want)
    assert got.sum() == 3


def test_density_accumulates_and_counts():
    a = workloads.gaussian(4096, seed=3)
    roots, st = oracle.solve(a)
    win = workloads.GAUSSIAN_WINDOW
    h1 = oracle.density(roots, win, (256, 256))
    inside = ((roots.real >= -3) & (roots.real < 3) & (roots.imag >= -3) & (roots.imag < 3)).sum()
    assert h1.sum() == inside
    h2 = oracle.density(roots, win, (256, 256), out=h1.copy())
    assert np.array_equal(h2, 2 * h1)


def test_backward_degree_one_closed_form():
    """r = -a0/a1: dr/da0 = -1/a1, dr/da1 = a0/a1^2; cotangent conj(dr/da) g."""
    rng = np.random.default_rng(1)
    n = 200
    a0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    a1 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    g = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    coeffs = np.stack([a0, a1])
    roots = (-a0 / a1)[None, :]
    grad, st = oracle.backward(coeffs, roots, g[None, :])
    assert np.all(st == 0)
    np.testing.assert_allclose(grad[0], np.conj(-1 / a1) * g, rtol=1e-13)
    np.testing.assert_allclose(grad[1], np.conj(a0 / a1 ** 2) * g, rtol=1e-13)


def test_backward_quadratic_closed_form():
    """Roots of z^2 + b1 z + b0 from the quadratic formula; derivatives of
    the formula by central differences in extended precision."""
    rng = np.random.default_rng(2)
    n = 100
    b0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    b1 = rng.standard_normal(n) + 1j * rng.standard_normal(n)

    def qroots(b0, b1):
        b0 = np.asarray(b0, dtype=np.clongdouble)
        b1 = np.asarray(b1, dtype=np.clongdouble)
        disc = np.sqrt(b1 * b1 - 4 * b0)
        return np.stack([(-b1 + disc) / 2, (-b1 - disc) / 2])

    r = qroots(b0, b1).astype(np.complex128)
    g = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    coeffs = np.stack([b0, b1, np.ones(n)])
    grad, st = oracle.backward(coeffs, r, g)
    # L = sum_j Re(conj(g_j) r_j): dL/dRe a + i dL/dIm a, by central differences
    h = 1e-7
    for k, (bb0, bb1) in enumerate([(1, 0), (0, 1)]):
        fd = np.zeros(n, dtype=np.complex128)
        for unit in (1.0, 1j):
            rp = qroots(b0 + h * unit * bb0, b1 + h * unit * bb1)
            rm = qroots(b0 - h * unit * bb0, b1 - h * unit * bb1)
            dL = (np.real(np.conj(g) * rp) - np.real(np.conj(g) * rm)).sum(axis=0) / (2 * h)
            fd += unit * dL.astype(np.float64)
        np.testing.assert_allclose(grad[k], fd, rtol=1e-6, atol=1e-8)
    assert np.all(grad[2] == grad[2])                 # finite


def _fd_grad(coeffs, weights, h=1e-6):
    """Central differences of L(a) = sum_j Re(conj(w_j) r_j(a)) through the
    oracle's forward, root assignment frozen to the unperturbed roots."""
    r0, _ = oracle.solve(coeffs)
    dmax1, n = coeffs.shape
    fd = np.zeros((dmax1, n), dtype=np.complex128)
    for k in range(dmax1):
        for unit in (1.0, 1j):
            cp = coeffs.copy(); cp[k] += h * unit
            cm = coeffs.copy(); cm[k] -= h * unit
            rp = match(oracle.solve(cp)[0], r0)
            rm = match(oracle.solve(cm)[0], r0)
            dL = (np.real(np.conj(weights) * rp) - np.real(np.conj(weights) * rm)).sum(axis=0) / (2 * h)
            fd[k] += unit * dL
    return r0, fd


def test_backward_matches_finite_differences():
    """Central differences at h = 1e-6 and 2e-6 combined by one Richardson
    step (the plain central difference has an h^2 truncation error of up to
    3e-5 relative on these roots)."""
    coeffs, true_roots, targets = workloads.known_roots(64, seed=4)
    rng = np.random.default_rng(5)
    w = rng.standard_normal((6, 64)) + 1j * rng.standard_normal((6, 64))
    r0, fd1 = _fd_grad(coeffs, w, 1e-6)
    _, fd2 = _fd_grad(coeffs, w, 2e-6)
    fd = (4 * fd1 - fd2) / 3
    grad, st = oracle.backward(coeffs, r0, w)
    assert np.all(st == 0)
    err = np.abs(grad - fd).max(axis=0) / np.abs(grad).max(axis=0)
    assert err.max() < 1e-6


def test_backward_product_form():
    """p'(r_j) = a_d prod_{l != j} (r_j - r_l) gives the same gradient."""
    a = workloads.gaussian(500, seed=6)
    a[6] = 1.5 - 0.5j
    roots, st = oracle.solve(a)
    rng = np.random.default_rng(7)
    g = rng.standard_normal((6, 500)) + 1j * rng.standard_normal((6, 500))
    grad, st2 = oracle.backward(a, roots, g)
    want = np.zeros((7, 500), dtype=np.complex128)
    for j in range(6):
        dp = a[6].copy()
        for l in range(6):
            if l != j:
                dp = dp * (roots[j] - roots[l])
        for k in range(7):
            want[k] += np.conj(-roots[j] ** k / dp) * g[j]
    np.testing.assert_allclose(grad, want, rtol=1e-9, atol=1e-12 * np.abs(want).max())


def test_backward_singular_and_invalid():
    # p = (z - 1)^2 (z - 2): p'(1) = 0 exactly
    coeffs = np.array([[-2.0], [5.0], [-4.0], [1.0]], dtype=np.complex128)
    roots = np.array([[1.0], [1.0], [2.0]], dtype=np.complex128)
    g = np.ones((3, 1), dtype=np.complex128)
    grad, st = oracle.backward(coeffs, roots, g, status=np.zeros(1, np.uint32))
    assert st[0] == oracle.ST_SINGULAR_DERIV
    # only the simple root contributes: dr/da_k = -2^k / p'(2), p'(2) = 1
    np.testing.assert_allclose(grad[:, 0], [-(2.0 ** k) for k in range(4)])
    # invalid polynomials get zero gradient
    st_in = np.array([oracle.ST_NONFINITE], dtype=np.uint32)
    grad, st = oracle.backward(coeffs, roots, g, status=st_in)
    assert np.all(grad == 0) and st[0] == oracle.ST_NONFINITE
    # rows above the degree are zero
    c, deg = workloads.mixed(50, seed=1)
    r, s = oracle.solve(c, deg)
    gg = np.ones((6, 50), dtype=np.complex128)
    grad, st = oracle.backward(c, np.nan_to_num(r), gg, deg, s)
    for i in range(50):
        assert np.all(grad[deg[i] + 1:, i] == 0)
