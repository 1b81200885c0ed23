"""The seeded input recipes produce what they state (CPU only)."""
from __future__ import annotations

import numpy as np

import workloads


def test_gaussian_recipe():
    a = workloads.gaussian(200000, seed=0)
    assert a.shape == (7, 200000) and a.dtype == np.complex128
    assert np.all(a[6] == 1)
    assert abs(np.mean(np.abs(a[:6]) ** 2) - 1.0) < 0.01
    assert abs(np.mean(a[:6].real)) < 0.01 and abs(np.var(a[:6].real) - 0.5) < 0.01
    assert np.array_equal(a, workloads.gaussian(200000, seed=0))
    assert not np.array_equal(a, workloads.gaussian(200000, seed=1))


def test_parametric_recipe():
    g = 64
    a = workloads.parametric(g, seed=0)
    assert a.shape == (7, g * g)
    rng = np.random.default_rng(0)
    x = [rng.standard_normal((2, 6)) for _ in range(3)]
    c, d, e = [(v[0] + 1j * v[1]) * np.sqrt(0.5) for v in x]
    t = -1 + (2 * np.arange(g) + 1) / g
    for (i, j) in [(0, 0), (5, 9), (63, 63), (17, 0)]:
        p = j * g + i
        np.testing.assert_array_equal(a[:6, p], c + t[i] * d + t[j] * e)
    assert np.all(a[6] == 1)
    # a row slice is the same data
    rows = workloads.parametric(g, seed=0, rows=slice(10, 12))
    np.testing.assert_array_equal(rows, a[:, 10 * g:12 * g])
    assert abs(t).max() < 1 and np.isclose(t[1] - t[0], 2 / g)


def test_mixed_recipe():
    a, deg = workloads.mixed(100000, seed=0)
    assert set(np.unique(deg)) == {2, 3, 4, 5, 6}
    assert np.all(np.abs(np.bincount(deg)[2:] / 1e5 - 0.2) < 0.01)
    k = np.arange(7)[:, None]
    assert np.all(a[k > deg] == 0)
    assert np.all(a[k == deg] == 1)
    mag = np.abs(a[k < deg])
    assert mag.min() >= 1e-2 * (1 - 1e-12) and mag.max() <= 1e2 * (1 + 1e-12)
    lm = np.log10(mag)
    assert abs(lm.mean()) < 0.02


def test_expand_roots_matches_numpy_poly():
    rng = np.random.default_rng(1)
    r = rng.standard_normal((4, 10)) + 1j * rng.standard_normal((4, 10))
    c = workloads.expand_roots(r)
    for i in range(10):
        np.testing.assert_allclose(c[::-1, i], np.poly(r[:, i]), rtol=1e-13, atol=1e-13)


def test_known_roots_recipe():
    coeffs, roots, targets = workloads.known_roots(20000, seed=0)
    mod = np.abs(roots)
    assert mod.min() > 0.5 and mod.max() < 2.0
    gap = np.full(20000, np.inf)
    for i in range(6):
        for j in range(i + 1, 6):
            gap = np.minimum(gap, np.abs(roots[i] - roots[j]))
    assert gap.min() >= 0.05
    assert np.all(coeffs[6] == 1)
    assert abs(np.abs(targets - roots).std() - 1e-2 * 0.6) < 3e-3


def test_clustered_recipe():
    coeffs, roots = workloads.clustered(10000, seed=0)
    c = roots[:3].mean(axis=0)
    assert np.abs(roots[:3] - c[None]).max() <= 2e-3
    assert np.abs(roots).max() <= 1 + 1e-3
    assert np.all(coeffs[6] == 1)
