"""Pins of the oracle's optional Wilkinson shift (FLAG_WILKINSON_SHIFT), on
CPU, against facts independent of the oracle:

  * the shift is the eigenvalue of the trailing 2 x 2 block nearest its
    bottom entry -- checked against LAPACK's eigenvalues (numpy.linalg.eigvals);
  * special blocks whose eigenvalues are known in closed form;
  * one QR step with that shift on a 2 x 2 matrix makes its subdiagonal
    negligible (an exact shift deflates at once), so every quadratic deflates
    after exactly one step, with the closed-form roots;
  * known roots and Vieta's identities hold with the flag as without it (the
    exact Gaussian-rational lattice pin of the solve runs with it as well);
  * z^d - c: for d >= 3 the trailing block is [[0, 0], [1, 0]], whose shift is
    0 as for the bottom entry, so the exceptional shift is still what breaks
    the stall; for d = 2 the shift is a root and no exceptional shift is used.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from rootmatch import match, rel_err

W = oracle.FLAG_WILKINSON_SHIFT


def _rand_c(rng, n, scale=1.0):
    return scale * (rng.standard_normal(n) + 1j * rng.standard_normal(n))


@pytest.mark.parametrize("scale", [1e-3, 1.0, 1e3])
def test_shift_is_nearest_eigenvalue(scale):
    rng = np.random.default_rng(21)
    n = 2000
    a, b, c, e = (_rand_c(rng, n, scale) for _ in range(4))
    for i in range(n):
        lam = np.linalg.eigvals(np.array([[a[i], b[i]], [c[i], e[i]]]))
        d0, d1 = np.abs(lam - e[i])
        near = lam[0] if d0 <= d1 else lam[1]
        mu = oracle.wilkinson_shift(a[i], b[i], c[i], e[i])
        size = np.abs(lam).max() + scale
        gap = abs(d0 - d1) / size
        if gap > 1e-6:      # a clear nearest eigenvalue
            assert abs(mu - near) <= 1e-12 * size, (i, mu, lam)
        else:               # (near-)tie: either eigenvalue is a valid choice
            assert np.abs(lam - mu).min() <= 1e-9 * size


def test_shift_special_blocks():
    # triangular blocks: eigenvalues a and e, the nearer to e is e itself
    for a, b, e in [(1 + 2j, 3.0, -0.5j), (4.0, 0.0, 4.0), (0.0, 1e300, 1.0)]:
        assert oracle.wilkinson_shift(a, b, 0.0, e) == e
        assert oracle.wilkinson_shift(a, 0.0, b, e) == e
    # zero block: double eigenvalue 0
    assert oracle.wilkinson_shift(0, 0, 0, 0) == 0
    # [[0, q], [1, 0]]: eigenvalues +-sqrt(q), equidistant from 0
    for q in (4.0, -9.0, 2j, 1 + 1j):
        mu = oracle.wilkinson_shift(0, q, 1, 0)
        assert abs(mu * mu - q) <= 1e-15 * abs(q)
    # [[2, 1], [1, 2]]: eigenvalues 1 and 3, equidistant from e = 2
    mu = oracle.wilkinson_shift(2, 1, 1, 2)
    assert min(abs(mu - 1), abs(mu - 3)) <= 1e-15
    # [[a, 1], [eps, e]]: the nearer eigenvalue is e - eps/(a - e) + O(eps^2)
    a, e, eps = 3.0 + 1j, 0.5 - 2j, 1e-9
    mu = oracle.wilkinson_shift(a, 1.0, eps, e)
    assert abs(mu - (e - eps / (a - e))) <= 1e-17 + 4 * eps ** 2


def test_exact_shift_deflates_a_2x2_in_one_step():
    rng = np.random.default_rng(22)
    for _ in range(500):
        H = np.array([[complex(*rng.standard_normal(2)), complex(*rng.standard_normal(2))],
                      [complex(*rng.standard_normal(2)), complex(*rng.standard_normal(2))]])
        mu = oracle.wilkinson_shift(H[0, 0], H[0, 1], H[1, 0], H[1, 1])
        H1 = oracle.qr_step(H, mu)
        assert abs(H1[1, 0]) <= 1e-13 * np.abs(H).max()
        # the step is a similarity: the eigenvalues are kept
        ev0 = np.sort_complex(np.linalg.eigvals(H))
        ev1 = np.sort_complex(np.linalg.eigvals(H1))
        assert np.abs(ev0 - ev1).max() <= 1e-12 * np.abs(H).max()


def test_quadratics_deflate_in_one_step():
    rng = np.random.default_rng(3)
    n = 5000
    b0, b1 = _rand_c(rng, n), _rand_c(rng, n)
    disc = np.sqrt(b1 * b1 - 4 * b0)
    q1, q2 = -(b1 + disc) / 2, -(b1 - disc) / 2
    q = np.where(np.abs(q1) >= np.abs(q2), q1, q2)
    truth = np.stack([q, b0 / q])
    roots, st, its = oracle.solve(np.stack([b0, b1, np.ones(n)]), flags=W, return_iters=True)
    assert np.all(st == 0)
    assert np.all(its[0] == 1)
    m = match(roots, truth)
    sep = np.abs(truth[0] - truth[1]) / np.maximum(np.abs(truth).max(axis=0), 1)
    ok = sep > 1e-3
    assert ok.mean() > 0.99
    assert rel_err(m[:, ok], truth[:, ok]).max() < 1e-12


def test_known_roots_and_vieta_with_the_shift():
    # known roots (annulus 0.5 < |z| < 2, gaps >= 0.05; coefficients rounded
    # to FP64 once, which alone moves the roots by up to ~1e-12 relative)
    a, truth, _ = workloads.known_roots(4000, seed=23)
    roots, st = oracle.solve(a, flags=W)
    assert np.all(st == 0)
    m = match(roots, truth)
    assert rel_err(m, truth).max() < 1e-10
    # Vieta: sum of roots = -b5 (a6 = 1), product = b0
    g = workloads.gaussian(5000, seed=24)
    roots, st = oracle.solve(g, flags=W)
    assert np.all(st == 0)
    scale = np.abs(roots).sum(axis=0)
    assert np.all(np.abs(roots.sum(axis=0) + g[5]) <= 64 * 2.0 ** -53 * scale)
    prod = np.prod(roots, axis=0)
    assert np.all(np.abs(prod - g[0]) <= 1e-12 * np.prod(np.abs(roots) + 1, axis=0))


def test_fewer_steps_than_the_bottom_entry_shift():
    """Wilkinson's shift converges at least as fast on average at every
    level, and the last level (a 2 x 2 block) always takes one step."""
    a = workloads.gaussian(20000, seed=25)
    _, s0, it0 = oracle.solve(a, return_iters=True)
    _, s1, it1 = oracle.solve(a, flags=W, return_iters=True)
    assert np.all(s0 == 0) and np.all(s1 == 0)
    assert np.all(it1.mean(axis=1) <= it0.mean(axis=1))
    assert np.all(it1[0] == 1)
    assert it1.max() < it0.max()


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("c", [1.0, -1.0, 1j, 2.0])
def test_roots_of_c_with_the_shift(d, c):
    coeffs = np.zeros((d + 1, 1), dtype=np.complex128)
    coeffs[0] = -c
    coeffs[d] = 1.0
    truth = (c ** (1.0 / d)) * np.exp(2j * np.pi * np.arange(d) / d)
    roots, st, its = oracle.solve(coeffs, flags=W, return_iters=True)
    assert st[0] == 0
    m = match(roots, truth[:, None])
    assert np.abs(m[:, 0] - truth).max() < 1e-14 * 4
    roots, st, its = oracle.solve(coeffs, flags=W | oracle.FLAG_NO_EXCEPTIONAL_SHIFT,
                                  return_iters=True)
    if d == 2:
        assert st[0] == 0 and its[0, 0] == 1
    else:
        assert st[0] & oracle.ST_NOT_CONVERGED


def _cabs1(z):
    return abs(z.real) + abs(z.imag)


def _step_by_step(a, flags, cap=30):
    """The level loop of Alg. 1 driven from Python through the oracle's
    separately pinned pieces (one QR step, Wilkinson's shift, the quadratic
    start), with the shift chosen as the readings state: the 10th and 20th
    step of a level take the bottom-right entry plus cabs1(subdiagonal)
    (0.75 + 0.5i) whatever the rule, the polynomial's first step the
    quadratic start (when defined), every other step the rule's shift.
    Monic degree-6 a [7].  Returns (roots in deflation order, steps per
    level, number of exceptional steps where Wilkinson's shift differed
    from the bottom entry)."""
    d = 6
    b = a[:d].astype(np.complex128)
    H = np.zeros((d, d), dtype=np.complex128)
    H[0, :] = -b[::-1]
    for i in range(d - 1):
        H[i + 1, i] = 1.0
    eig = np.zeros(d, dtype=np.complex128)
    its_all = np.zeros(d - 1, dtype=np.int32)
    moved = 0
    for m in range(d, 1, -1):
        its = 0
        while True:
            hsub = H[m - 1, m - 2]
            if _cabs1(hsub) <= 2.0 ** -52 * (_cabs1(H[m - 1, m - 1]) + _cabs1(H[m - 2, m - 2])):
                break
            if its == cap:
                break
            e = H[m - 1, m - 1]
            s = e
            if flags & W:
                s = oracle.wilkinson_shift(H[m - 2, m - 2], H[m - 2, m - 1], hsub, e)
            if (flags & oracle.FLAG_QUADRATIC_START) and m == d and its == 0:
                z, ok = oracle.quadratic_start(b[0], b[1], b[2])
                if ok:
                    s = z
            if its in (10, 20):
                moved += int((flags & W) != 0 and s != e)
                s = e + _cabs1(hsub) * (0.75 + 0.5j)
            H[:m, :m] = oracle.qr_step(H[:m, :m], s)
            its += 1
        its_all[m - 2] = its
        eig[m - 1] = H[m - 1, m - 1]
    eig[0] = H[0, 0]
    return eig, its_all, moved


@pytest.mark.parametrize("flags", [0, W, W | oracle.FLAG_QUADRATIC_START])
def test_exceptional_step_takes_the_bottom_entry_under_either_rule(flags):
    """Reading R5: on the 10th and 20th step of a level the shift is the
    bottom-right entry moved off by cabs1(h[m-1][m-2]) (0.75 + 0.5i), under
    Alg. 1's shift and under Wilkinson's alike.  Triple root clusters take
    such steps; the batched solve must follow the step-by-step driver bit
    for bit, including polynomials where Wilkinson's shift at that step
    differs from the bottom entry."""
    coeffs, _ = workloads.clustered(3000, seed=5)
    _, _, its = oracle.solve(coeffs, flags=flags, return_iters=True)
    pick = np.nonzero(its.max(axis=0) >= 11)[0][:24]
    assert pick.size >= 8, "too few polynomials reach an exceptional step"
    roots, st, its = oracle.solve(coeffs[:, pick], flags=flags, return_iters=True)
    moved = 0
    for j, i in enumerate(pick):
        eig, its_py, mv = _step_by_step(coeffs[:, i], flags)
        moved += mv
        np.testing.assert_array_equal(its[:, j], its_py)
        np.testing.assert_array_equal(roots[:, j], eig)
    if flags & W:
        assert moved > 0
