"""Pins of the L2 approximation front-end (Sec. II-A) on the CPU: the
oracle's fit against closed forms and the paper's printed example, and the
library's host-side quadrature nodes against numpy's Gauss-Legendre rule."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _f(z, c=0.3):
    return 1.0 / (1.0 - c * z)


def test_fit_is_taylor_truncation():
    """With the area measure the monomials are orthogonal on the unit disk,
    so the L2 projection of an analytic f is its Taylor truncation:
    1/(1 - 0.3 z) -> a_k = 0.3^k."""
    nodes, w = oracle.l2_nodes(16, 32)
    a = oracle.l2fit(_f(nodes)[:, None], nodes, w, 6)[:, 0]
    np.testing.assert_allclose(a, 0.3 ** np.arange(7), rtol=1e-13, atol=1e-15)


def test_gram_matrix_is_diagonal_pi_over_j_plus_1():
    nodes, w = oracle.l2_nodes(8, 16)
    V = nodes[None, :] ** np.arange(7)[:, None]
    G = (V * w[None, :]) @ V.conj().T
    np.testing.assert_allclose(G, np.diag(np.pi / (np.arange(7) + 1)), atol=1e-14)
    assert abs(w.sum() - np.pi) < 1e-14


def test_paper_example_bounds():
    """Sec. II-A's example: the degree-6 approximation of 1/(1 - 0.3z) is
    within 7.3e-4 of f on the unit disk (measured: 0.3^7 / 0.7 = 3.1e-4, the
    tail at z = 1 -- the error is analytic, so its maximum is on the circle),
    and within 1e-14 on the disk of radius 1e-2."""
    g = json.load(open(os.path.join(GOLDEN, "paper_l2_example.json")))
    c, n = g["pole_factor"], g["degree"]
    nodes, w = oracle.l2_nodes(16, 32)
    a = oracle.l2fit(_f(nodes, c)[:, None], nodes, w, n)[:, 0]
    circle = np.exp(2j * np.pi * np.arange(4096) / 4096)
    err = np.abs(_f(circle, c) - np.polyval(a[::-1], circle)).max()
    assert err <= g["unit_disk_sup_error_bound"]
    assert abs(err - c ** (n + 1) / (1 - c)) < 1e-12
    # small disk: w = z / rho, f(rho w) sampled at the same nodes
    rho = g["small_disk_radius"]
    a_s = oracle.l2fit(_f(rho * nodes, c)[:, None], nodes, w, n)[:, 0]
    zz = rho * circle
    err_s = np.abs(_f(zz, c) - np.polyval(a_s[::-1], circle)).max()
    assert err_s <= g["small_disk_sup_error_bound"]


def test_polynomial_f_is_recovered_exactly():
    rng = np.random.default_rng(0)
    coef = rng.standard_normal(5) + 1j * rng.standard_normal(5)   # degree 4
    nodes, w = oracle.l2_nodes(8, 16)
    a = oracle.l2fit(np.polyval(coef[::-1], nodes)[:, None], nodes, w, 6)[:, 0]
    np.testing.assert_allclose(a[:5], coef, atol=1e-13)
    assert np.abs(a[5:]).max() < 1e-13


def test_library_nodes_match_numpy_gauss_legendre():
    """pr_l2fit_nodes is a host call: its rule equals numpy's."""
    import paper_2507_02164_amd as pr
    for nr, nt in [(1, 1), (3, 7), (8, 16), (16, 32), (64, 256)]:
        n1, w1 = pr.l2fit_nodes(nr, nt)
        n2, w2 = oracle.l2_nodes(nr, nt)
        np.testing.assert_allclose(n1, n2, atol=2e-15)
        # numpy's rule itself drifts to ~1e-12 relative at 64 nodes (against
        # a 40-digit reference the library's weights are the closer ones)
        np.testing.assert_allclose(w1, w2, rtol=1e-11)
        assert abs(w1.sum() - np.pi) < 1e-12
        # the rule integrates |w|^(2j) exactly over the disk for j < nr:
        # integral = pi / (j + 1)
        for j in range(min(nr, 20)):
            assert abs((w1 * np.abs(n1) ** (2 * j)).sum() - np.pi / (j + 1)) < 1e-13
    with pytest.raises(pr.ProotsError):
        pr.l2fit_nodes(0, 4)
    with pytest.raises(pr.ProotsError):
        pr.l2fit_nodes(4, 257)


def test_fit_is_linear_and_least_squares():
    """The fit is linear in f, and it is the minimiser: every perturbation of
    the coefficients raises the (quadrature) L2 error, with the residual
    orthogonal to each monomial up to degree n."""
    rng = np.random.default_rng(4)
    nodes, w = oracle.l2_nodes(8, 16)
    f1 = np.exp(1.3 * nodes) * np.cos(nodes - 0.2j)
    f2 = 1.0 / (nodes - 1.7 + 0.4j)
    al, be = 0.3 - 1.1j, -2.0 + 0.5j
    F = np.stack([f1, f2, al * f1 + be * f2], axis=1)
    a = oracle.l2fit(F, nodes, w, 5)
    np.testing.assert_allclose(a[:, 2], al * a[:, 0] + be * a[:, 1], atol=1e-13)
    V = nodes[None, :] ** np.arange(6)[:, None]
    for col in range(3):
        resid = F[:, col] - a[:, col] @ V
        inner = (V.conj() * w[None, :]) @ resid
        assert np.abs(inner).max() < 1e-13
        e0 = (w * np.abs(resid) ** 2).sum()
        for _ in range(20):
            da = 1e-3 * (rng.standard_normal(6) + 1j * rng.standard_normal(6))
            e1 = (w * np.abs(F[:, col] - (a[:, col] + da) @ V) ** 2).sum()
            assert e1 > e0


def test_density_local_brute_force():
    rng = np.random.default_rng(5)
    n, dmax = 300, 4
    w = rng.uniform(-1.2, 1.2, (dmax, n)) + 1j * rng.uniform(-1.2, 1.2, (dmax, n))
    w[1, ::7] = np.nan
    c = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    rho = rng.uniform(0.01, 0.3, n)
    deg = rng.integers(0, dmax + 1, n)
    st = np.where(rng.random(n) < 0.1, 8, 0).astype(np.uint32)
    W, H, win = 37, 23, (-1.1, 1.2, -0.9, 1.0)
    for rmax2 in (1.0, 0.6):
        img = oracle.density_local(w, c, rho, win, (W, H), rmax2, deg, st, skip_mask=8)
        ref = np.zeros((H, W), dtype=np.int64)
        for i in range(n):
            if st[i] & 8:
                continue
            for k in range(deg[i]):
                x = w[k, i]
                if not (x.real * x.real + x.imag * x.imag < rmax2):
                    continue
                zr = c[i].real + rho[i] * x.real
                zi = c[i].imag + rho[i] * x.imag
                u = (zr - win[0]) * (W / (win[1] - win[0]))
                v = (zi - win[2]) * (H / (win[3] - win[2]))
                if 0 <= u < W and 0 <= v < H:
                    ref[int(v), int(u)] += 1
        assert np.array_equal(img, ref) and ref.sum() > 50
