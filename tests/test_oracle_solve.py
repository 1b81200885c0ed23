"""Pins of the oracle's solve against facts fixed by mathematics or the
paper, independent of the oracle itself (runs on CPU).

Each test names what it pins:
  * exactly known roots (Gaussian-rational lattice, exact coefficients),
  * the quadratic closed form, degree 1, z^d and z^d - c,
  * Vieta's identities,
  * an independent iteration (Durand-Kerner in extended precision),
  * third-party eigen/root solvers (mpmath at 50 digits, LAPACK via
    numpy.roots),
  * one QR step against a Householder QR factorisation (numpy), which pins
    the Sec. II-C rotation convention, the two passes and the shift,
  * the Appendix's Hessenberg invariant,
  * the Sec. II-C Givens equation,
  * the fixed-T mode against the step and cycle counts the paper prints
    (Alg. 2, Table III, Sec. IV-A), stored in tests/golden.
"""
from __future__ import annotations

import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads
from rootmatch import match, rel_err

U64 = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _poly_from_roots_exact(roots):
    """Exact coefficients (a_0..a_d, a_d = 1) of prod (z - r) for Gaussian
    rationals r = (p + q i) / 4, as Python Fractions (re, im)."""
    c = [(Fraction(1), Fraction(0))]
    for (pr, pi) in roots:
        new = [(Fraction(0), Fraction(0)) for _ in range(len(c) + 1)]
        for k, (cr, ci) in enumerate(c):
            # z * c_k z^k
            nr, ni = new[k + 1]
            new[k + 1] = (nr + cr, ni + ci)
            # -r * c_k z^k
            nr, ni = new[k]
            new[k] = (nr - (pr * cr - pi * ci), ni - (pr * ci + pi * cr))
        c = new
    return c


@pytest.mark.parametrize("flags", [0, oracle.FLAG_WILKINSON_SHIFT])
def test_known_roots_lattice(flags):
    """Roots on the lattice (p + q i)/4, |p|, |q| <= 8, distinct: the
    expanded coefficients are exact in FP64, so the true roots are known.
    Error bound: first-order perturbation |dr| <= C u ||b||^2 sum|r|^k / |p'(r)|
    (QR on the companion matrix is backward stable in the matrix, which
    puts a backward error of order u ||b||^2 on the coefficients)."""
    rng = np.random.default_rng(7)
    n = 300
    for d in (2, 3, 4, 5, 6):
        coeffs = np.zeros((d + 1, n), dtype=np.complex128)
        truth = np.zeros((d, n), dtype=np.complex128)
        for i in range(n):
            pts = set()
            while len(pts) < d:
                pts.add((int(rng.integers(-8, 9)), int(rng.integers(-8, 9))))
            rts = [(Fraction(p, 4), Fraction(q, 4)) for (p, q) in sorted(pts)]
            c = _poly_from_roots_exact(rts)
            for k, (cr, ci) in enumerate(c):
                fr, fi = float(cr), float(ci)
                assert Fraction(fr) == cr and Fraction(fi) == ci      # exact in FP64
                coeffs[k, i] = complex(fr, fi)
            truth[:, i] = [complex(float(p), float(q)) for (p, q) in rts]
        roots, st = oracle.solve(coeffs, flags=flags)
        assert np.all(st == 0)
        m = match(roots, truth)
        bnorm = np.abs(coeffs[:d]).max(axis=0)
        # |p'(r_j)| = prod_{l != j} |r_j - r_l| exactly (monic)
        dp = np.ones((d, n))
        for j in range(d):
            for l in range(d):
                if l != j:
                    dp[j] *= np.abs(truth[j] - truth[l])
        powsum = sum(np.abs(truth) ** k for k in range(d + 1))
        bound = 64 * d * U64 * (1 + bnorm) ** 2 * powsum / dp
        err = np.abs(m - truth)
        assert np.all(err <= bound), (d, float((err / bound).max()))
        assert err.max() < 1e-9


def test_quadratic_closed_form():
    rng = np.random.default_rng(3)
    n = 5000
    b0 = (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    b1 = (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    disc = np.sqrt(b1 * b1 - 4 * b0)
    q1 = -(b1 + disc) / 2
    q2 = -(b1 - disc) / 2
    q = np.where(np.abs(q1) >= np.abs(q2), q1, q2)
    truth = np.stack([q, b0 / q])
    coeffs = np.stack([b0, b1, np.ones(n)])
    roots, st = oracle.solve(coeffs)
    assert np.all(st == 0)
    m = match(roots, truth)
    sep = np.abs(truth[0] - truth[1]) / np.maximum(np.abs(truth).max(axis=0), 1)
    ok = sep > 1e-3
    assert ok.mean() > 0.99
    assert rel_err(m[:, ok], truth[:, ok]).max() < 1e-12


def test_degree_one_exact():
    rng = np.random.default_rng(4)
    a0 = rng.standard_normal(1000) + 1j * rng.standard_normal(1000)
    # monic: r = -a0 exactly
    roots, st = oracle.solve(np.stack([a0, np.ones(1000)]))
    assert np.all(st == 0)
    assert np.array_equal(roots[0], -a0)
    # general leading coefficient: r = -a0/a1 to within rounding of one division
    a1 = rng.standard_normal(1000) + 1j * rng.standard_normal(1000)
    roots, st = oracle.solve(np.stack([a0, a1]))
    assert rel_err(roots[0], -a0 / a1).max() < 4 * U64 * 4


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6])
def test_monomial_exact_zero(d):
    """z^d: every root is exactly 0 and every level deflates after one step."""
    coeffs = np.zeros((d + 1, 3), dtype=np.complex128)
    coeffs[d] = [1.0, 2.5, -1j]
    roots, st, its = oracle.solve(coeffs, return_iters=True)
    assert np.all(st == 0)
    assert np.all(roots == 0)
    assert np.all(its[: d - 1] == 1)


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("c", [1.0, -1.0, 1j, 2.0])
def test_roots_of_c(d, c):
    """z^d - c: roots c^(1/d) e^(2 pi i k / d).  The pure Rayleigh shift
    stalls here (every shift is 0), so this pins the exceptional shift, and
    with it switched off the level must hit the cap and be flagged."""
    coeffs = np.zeros((d + 1, 1), dtype=np.complex128)
    coeffs[0] = -c
    coeffs[d] = 1.0
    truth = (c ** (1.0 / d)) * np.exp(2j * np.pi * np.arange(d) / d)
    roots, st = oracle.solve(coeffs)
    assert st[0] == 0
    m = match(roots, truth[:, None])
    assert np.abs(m[:, 0] - truth).max() < 1e-14 * 4
    roots, st = oracle.solve(coeffs, flags=oracle.FLAG_NO_EXCEPTIONAL_SHIFT)
    assert st[0] & oracle.ST_NOT_CONVERGED


def test_vieta():
    """Sum of roots = -b_{d-1} (the trace, which every similarity step keeps)
    and product = (-1)^d b_0."""
    a = workloads.gaussian(20000, seed=11)
    roots, st = oracle.solve(a)
    assert np.all(st == 0)
    scale = np.abs(roots).sum(axis=0)
    assert np.all(np.abs(roots.sum(axis=0) + a[5]) <= 64 * U64 * scale)
    prod = np.prod(roots, axis=0)
    assert np.median(rel_err(prod, a[0])) < 1e-14
    assert np.quantile(rel_err(prod, a[0]), 0.999) < 1e-10


def _durand_kerner(coeffs_ld, iters=500):
    """Weierstrass / Durand-Kerner simultaneous iteration in x87 extended
    precision, started from (0.4 + 0.9i)^j; monic coefficients [d+1, n]."""
    d = coeffs_ld.shape[0] - 1
    n = coeffs_ld.shape[1]
    z = np.array([(np.clongdouble(0.4 + 0.9j)) ** j for j in range(d)], dtype=np.clongdouble)
    z = np.repeat(z[:, None], n, axis=1)
    for _ in range(iters):
        for j in range(d):
            p = np.ones(n, dtype=np.clongdouble)
            for k in range(d - 1, -1, -1):
                p = p * z[j] + coeffs_ld[k]
            den = np.ones(n, dtype=np.clongdouble)
            for l in range(d):
                if l != j:
                    den = den * (z[j] - z[l])
            z[j] = z[j] - p / den
    return z


@pytest.mark.parametrize("d", [2, 3, 4])
def test_durand_kerner_extended(d):
    rng = np.random.default_rng(20 + d)
    n = 300
    a = (rng.standard_normal((d, n)) + 1j * rng.standard_normal((d, n))) * np.sqrt(0.5)
    coeffs = np.concatenate([a, np.ones((1, n))])
    z = _durand_kerner(coeffs.astype(np.clongdouble))
    truth = z.astype(np.complex128)
    roots, st = oracle.solve(coeffs)
    assert np.all(st == 0)
    m = match(roots, truth)
    err = rel_err(m, truth, floor=1e-3)
    assert np.median(err) < 1e-15
    assert np.quantile(err, 0.99) < 1e-12


def test_mpmath_polyroots():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    a = workloads.gaussian(40, seed=5)
    roots, st = oracle.solve(a)
    truth = np.zeros((6, 40), dtype=np.complex128)
    for i in range(40):
        cs = [mpmath.mpc(complex(a[k, i])) for k in range(6, -1, -1)]
        rs = mpmath.polyroots(cs, maxsteps=200, extraprec=200)
        truth[:, i] = [complex(r) for r in rs]
    m = match(roots, truth)
    assert rel_err(m, truth).max() < 1e-12
    # mixed degree, log-uniform moduli
    c, deg = workloads.mixed(40, seed=6)
    roots, st = oracle.solve(c, deg)
    for i in range(40):
        d = int(deg[i])
        cs = [mpmath.mpc(complex(c[k, i])) for k in range(d, -1, -1)]
        rs = np.array([complex(r) for r in mpmath.polyroots(cs, maxsteps=400, extraprec=400)])
        mm = match(roots[:d, i:i + 1], rs[:, None])[:, 0]
        assert rel_err(mm, rs).max() < 1e-10, (i, d)


def test_numpy_roots_agree():
    a = workloads.gaussian(1000, seed=9)
    roots, st = oracle.solve(a)
    truth = np.stack([np.roots(a[::-1, i]) for i in range(1000)], axis=1)
    m = match(roots, truth)
    assert np.quantile(rel_err(m, truth), 0.999) < 1e-11


def _hessenberg(rng, m):
    H = (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    return np.triu(H, -1)


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6])
def test_qr_step_matches_householder_qr(m):
    """Alg. 1 body: A - sI = QR, A <- RQ + sI.  numpy's Householder QR gives
    Q, R up to a diagonal unitary D; the Sec. II-C rotations fix it: each
    rotation leaves a real non-negative diagonal entry rho in R (rows
    0..m-2) and each has determinant |c|^2 + |s|^2 = 1, so det Q = 1."""
    rng = np.random.default_rng(100 + m)
    for _ in range(20):
        H = _hessenberg(rng, m)
        s = complex(rng.standard_normal(), rng.standard_normal())
        Q, R = np.linalg.qr(H - s * np.eye(m))
        ph = np.ones(m, dtype=np.complex128)
        for k in range(m - 1):
            ph[k] = R[k, k] / abs(R[k, k])
        ph[m - 1] = 1.0
        ph[m - 1] = 1.0 / (np.linalg.det(Q) * np.prod(ph))
        Qn = Q * ph[None, :]                      # Q D
        Rn = np.conj(ph)[:, None] * R             # D^H R
        expect = Rn @ Qn + s * np.eye(m)
        got = oracle.qr_step(H, s)
        assert np.abs(got - expect).max() < 1e-13 * np.abs(H).max() * m
        # Appendix: the step keeps the matrix upper Hessenberg, exactly.
        assert np.all(np.tril(got, -2) == 0)


def test_hessenberg_invariant_through_solve():
    """Many steps in a row keep every below-subdiagonal entry exactly zero."""
    rng = np.random.default_rng(1)
    H = _hessenberg(rng, 6)
    for k in range(60):
        H = oracle.qr_step(H, H[5, 5])
        assert np.all(np.tril(H, -2) == 0)


def test_givens_equation():
    """Sec. II-C: [[c, s], [-conj(s), conj(c)]] (a, b)^T = (sqrt(|a|^2+|b|^2), 0)^T
    with a unitary matrix."""
    rng = np.random.default_rng(2)
    for _ in range(200):
        a = complex(*rng.standard_normal(2)) * 10 ** rng.uniform(-3, 3)
        b = complex(*rng.standard_normal(2)) * 10 ** rng.uniform(-3, 3)
        c, s = oracle.givens(a, b)
        G = np.array([[c, s], [-np.conj(s), np.conj(c)]])
        out = G @ np.array([a, b])
        rho = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
        assert abs(out[0] - rho) <= 4 * U64 * rho and abs(out[1]) <= 4 * U64 * rho
        assert np.abs(G @ G.conj().T - np.eye(2)).max() < 8 * U64
    c, s = oracle.givens(0j, 0j)
    assert (c, s) == (1, 0)


def test_fixed_t_counts_match_paper():
    """Alg. 2 runs exactly T steps per level, (n-1) T in all; Sec. IV-A
    counts 2m - 2 pipeline passes per step, n (n - 1) T per polynomial.
    The values are the paper's (Table III: n = 6, T = 10)."""
    with open(os.path.join(GOLDEN, "paper_fixed_T.json")) as f:
        g = json.load(f)
    n, T = g["n"], g["T"]
    a = workloads.gaussian(64, seed=0)
    roots, st, its = oracle.solve(a, fixed_t=T, return_iters=True)
    assert np.all(its == T)
    assert np.all(its.sum(axis=0) == g["qr_steps_per_poly"])
    passes = sum((2 * m - 2) * its[m - 2] for m in range(2, n + 1))
    assert np.all(passes == g["pipeline_cycles_per_poly"])
    # Ten steps per level already give roots close to the converged ones
    # for most polynomials (the paper's fixed budget).
    ref, _ = oracle.solve(a)
    err = rel_err(match(roots, ref), ref)
    assert np.median(err) < 1e-6


def test_validation_status():
    coeffs = workloads.gaussian(6, seed=1)
    deg = np.array([6, 0, 7, 6, 6, 3], dtype=np.int32)
    coeffs[2, 3] = np.nan
    coeffs[6, 4] = 0.0
    roots, st = oracle.solve(coeffs, deg)
    assert st[0] == 0 and st[5] == 0
    assert st[1] == oracle.ST_BAD_DEGREE and st[2] == oracle.ST_BAD_DEGREE
    assert st[3] == oracle.ST_NONFINITE
    assert st[4] == oracle.ST_ZERO_LEADING
    for i in (1, 2, 3, 4):
        assert np.all(np.isnan(roots[:, i]))
    # rows beyond the degree are NaN; rows above the degree in coeffs are ignored
    assert np.all(np.isnan(roots[3:, 5])) and np.all(np.isfinite(roots[:3, 5]))
    r3, _ = oracle.solve(coeffs[:4, 5:6])
    assert np.array_equal(np.sort_complex(r3[:, 0]), np.sort_complex(roots[:3, 5]))


def test_non_monic_scaling():
    """Scaling every coefficient by the same nonzero factor leaves the roots
    unchanged (up to the rounding of the normalisation)."""
    a = workloads.gaussian(2000, seed=12)
    r1, _ = oracle.solve(a)
    r2, _ = oracle.solve(a * (0.3 - 2.1j))
    assert np.quantile(rel_err(match(r2, r1), r1), 0.999) < 1e-11


def test_mixed_degree_batch_equals_per_degree():
    c, deg = workloads.mixed(3000, seed=2)
    roots, st = oracle.solve(c, deg)
    for d in range(2, 7):
        cols = np.nonzero(deg == d)[0]
        r, s = oracle.solve(c[: d + 1, cols])
        assert np.array_equal(r, roots[:d, cols], equal_nan=True)
        assert np.all(np.isnan(roots[d:, cols]))
