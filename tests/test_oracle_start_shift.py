"""Pins of the oracle's optional first shift (FLAG_QUADRATIC_START): the
very first QR step of a polynomial is shifted by the root nearest 0 of
b0 + b1 z + b2 z^2 (b the monic coefficients), on CPU, against facts
independent of the oracle:

  * the start equals the smallest-modulus root from LAPACK (numpy.roots of
    the quadratic) at several scales, the linear closed form -b0/b1 when
    b2 == 0, and is undefined for a constant;
  * degree-2 polynomials: the start is an exact root, so their one level
    deflates after one step even under Alg. 1's shift otherwise;
  * known roots, the exact Gaussian-rational lattice and Vieta's identities
    hold with the flag;
  * it lowers the steps of the top level on average (the point of it), and
    z^d - c (b1 = b2 = 0 for d >= 3, no start) still needs the exceptional
    shift;
  * the fixed-T mode (Alg. 2 literally) ignores it.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads
from rootmatch import match, rel_err

W, Q = oracle.FLAG_WILKINSON_SHIFT, oracle.FLAG_QUADRATIC_START


def _rand_c(rng, n, scale=1.0):
    return scale * (rng.standard_normal(n) + 1j * rng.standard_normal(n))


@pytest.mark.parametrize("scale", [1e-4, 1.0, 1e4])
def test_start_is_the_smallest_root_of_the_quadratic(scale):
    rng = np.random.default_rng(41)
    b0, b1, b2 = _rand_c(rng, 3000, scale ** 2), _rand_c(rng, 3000, scale), _rand_c(rng, 3000)
    for i in range(b0.size):
        z, ok = oracle.quadratic_start(b0[i], b1[i], b2[i])
        r = np.roots([b2[i], b1[i], b0[i]])
        m = np.abs(r)
        assert ok
        if abs(m[0] - m[1]) > 1e-6 * m.max():      # a clear smaller root
            near = r[np.argmin(m)]
            assert abs(z - near) <= 1e-12 * m.max(), (i, z, r)
        else:                                        # tie: either root
            assert np.abs(r - z).min() <= 1e-9 * m.max()


def test_start_special_cases():
    # linear: -b0/b1
    for b0, b1 in [(3.0, 2.0), (1 + 1j, -0.5j), (-2.0, 1e-3)]:
        z, ok = oracle.quadratic_start(b0, b1, 0.0)
        assert ok and abs(z - (-b0 / b1)) <= 1e-15 * abs(b0 / b1)
    # a constant has no root
    assert oracle.quadratic_start(1.0, 0.0, 0.0)[1] is False
    # z^2 and z (b0 = 0): the root 0
    assert oracle.quadratic_start(0.0, 0.0, 1.0) == (0j, True)
    assert oracle.quadratic_start(0.0, 2.0, 1.0) == (0j, True)
    # (z - 1)(z - 2) and (z - 3i)^2
    assert oracle.quadratic_start(2.0, -3.0, 1.0) == (1 + 0j, True)
    z, ok = oracle.quadratic_start(-9.0, -6j, 1.0)
    assert ok and abs(z - 3j) <= 1e-15 * 3


def test_quadratics_one_step_even_with_alg1_shift_afterwards():
    rng = np.random.default_rng(42)
    n = 5000
    b0, b1 = _rand_c(rng, n), _rand_c(rng, n)
    a = np.stack([b0, b1, np.ones(n)])
    for flags in (Q, W | Q):
        roots, st, its = oracle.solve(a, flags=flags, return_iters=True)
        assert np.all(st == 0)
        assert np.all(its[0] == 1)
    # without the start Alg. 1's shift needs several steps
    _, _, its0 = oracle.solve(a, return_iters=True)
    assert its0[0].mean() > 3


def _lattice_poly(rts):
    c = [(Fraction(1), Fraction(0))]
    for (pr, pi) in rts:
        new = [(Fraction(0), Fraction(0)) for _ in range(len(c) + 1)]
        for k, (cr, ci) in enumerate(c):
            nr, ni = new[k + 1]
            new[k + 1] = (nr + cr, ni + ci)
            nr, ni = new[k]
            new[k] = (nr - (pr * cr - pi * ci), ni - (pr * ci + pi * cr))
        c = new
    return [complex(float(cr), float(ci)) for (cr, ci) in c]


def test_known_roots_lattice_and_vieta():
    rng = np.random.default_rng(43)
    n = 300
    for d in (3, 6):
        coeffs = np.zeros((d + 1, n), dtype=np.complex128)
        truth = np.zeros((d, n), dtype=np.complex128)
        for i in range(n):
            pts = set()
            while len(pts) < d:
                pts.add((int(rng.integers(-8, 9)), int(rng.integers(-8, 9))))
            rts = [(Fraction(p, 4), Fraction(q, 4)) for (p, q) in sorted(pts)]
            coeffs[:, i] = _lattice_poly(rts)
            truth[:, i] = [complex(float(p), float(q)) for (p, q) in rts]
        roots, st = oracle.solve(coeffs, flags=W | Q)
        assert np.all(st == 0)
        assert np.abs(match(roots, truth) - truth).max() < 1e-9
    a, truth, _ = workloads.known_roots(4000, seed=44)
    roots, st = oracle.solve(a, flags=W | Q)
    assert np.all(st == 0)
    assert rel_err(match(roots, truth), truth).max() < 1e-10
    g = workloads.gaussian(5000, seed=45)
    roots, st = oracle.solve(g, flags=W | Q)
    assert np.all(st == 0)
    scale = np.abs(roots).sum(axis=0)
    assert np.all(np.abs(roots.sum(axis=0) + g[5]) <= 64 * 2.0 ** -53 * scale)


def test_fewer_top_level_steps():
    a = workloads.gaussian(20000, seed=46)
    _, s1, it1 = oracle.solve(a, flags=W, return_iters=True)
    _, s2, it2 = oracle.solve(a, flags=W | Q, return_iters=True)
    assert np.all(s1 == 0) and np.all(s2 == 0)
    assert it2[4].mean() < it1[4].mean() - 0.5
    assert it2.sum(axis=0).mean() < it1.sum(axis=0).mean()


@pytest.mark.parametrize("d", [2, 3, 6])
def test_roots_of_c(d):
    c = 2.0 + 1j
    coeffs = np.zeros((d + 1, 1), dtype=np.complex128)
    coeffs[0] = -c
    coeffs[d] = 1.0
    truth = (c ** (1.0 / d)) * np.exp(2j * np.pi * np.arange(d) / d)
    roots, st, its = oracle.solve(coeffs, flags=W | Q, return_iters=True)
    assert st[0] == 0
    assert np.abs(match(roots, truth[:, None])[:, 0] - truth).max() < 1e-14 * 4
    _, st, its = oracle.solve(coeffs, flags=W | Q | oracle.FLAG_NO_EXCEPTIONAL_SHIFT,
                              return_iters=True)
    if d == 2:
        assert st[0] == 0 and its[0, 0] == 1
    else:
        assert st[0] & oracle.ST_NOT_CONVERGED


def test_fixed_t_ignores_the_start():
    a = workloads.gaussian(2000, seed=47)
    r0, s0, i0 = oracle.solve(a, fixed_t=10, return_iters=True)
    r1, s1, i1 = oracle.solve(a, fixed_t=10, flags=W | Q, return_iters=True)
    assert np.array_equal(r0.view(np.int64), r1.view(np.int64))
    assert np.array_equal(s0, s1) and np.array_equal(i0, i1)
