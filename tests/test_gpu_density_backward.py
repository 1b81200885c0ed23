"""GPU parity of pr_density (bit-exact) and pr_backward against the oracle.

Both sides bin / differentiate the same root array, which the oracle
computed, so neither side ever consumes the other's output.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from gpuutil import rel_condition, to_dev, to_host
from rootmatch import match, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pr = pytest.importorskip("paper_2507_02164_amd")


def _density(roots, window, shape, degrees=None, status=None, skip=0, out=None):
    h = pr.density(to_dev(roots), window, shape,
                   None if degrees is None else to_dev(degrees),
                   None if status is None else to_dev(status.astype(np.int32)), skip,
                   None if out is None else to_dev(out))
    torch.cuda.synchronize()
    return to_host(h)


def test_density_gaussian_256():
    a = workloads.gaussian(65536, seed=0)
    ref, st = oracle.solve(a)
    win, shape = workloads.GAUSSIAN_WINDOW, (256, 256)
    assert np.array_equal(_density(ref, win, shape), oracle.density(ref, win, shape))


def test_density_parametric_1080p():
    a = workloads.parametric(512, seed=0)
    ref, st = oracle.solve(a)
    win, shape = workloads.PARAMETRIC_WINDOW, (1920, 1080)
    got = _density(ref, win, shape)
    want = oracle.density(ref, win, shape)
    assert np.array_equal(got, want)
    assert want.sum() > 0.9 * ref.size


def test_density_masks_degrees_accumulate():
    a, deg = workloads.mixed(40000, seed=1)
    ref, st = oracle.solve(a, deg)
    rng = np.random.default_rng(0)
    st = st | (rng.integers(0, 4, 40000).astype(np.uint32) << 3)   # random flag bits
    win, shape = (-3.0, 3.0, -2.0, 2.0), (300, 200)
    base = rng.integers(0, 5, (200, 300)).astype(np.int32)
    for skip in (0, pr.ST_NOT_CONVERGED, pr.ST_NOT_CONVERGED | pr.ST_POLISH_UNCONVERGED):
        got = _density(ref, win, shape, deg, st, skip, out=base)
        want = oracle.density(ref, win, shape, deg, st, skip, out=base.copy())
        assert np.array_equal(got, want)


def test_density_bin_edges():
    """Roots exactly on pixel edges, window edges, NaN and Inf."""
    win = (-2.0, 2.0, -1.0, 1.0)
    shape = (64, 32)
    xs = np.linspace(-2.0, 2.0, 65)          # every pixel edge, including x1
    ys = np.linspace(-1.0, 1.0, 33)
    X, Y = np.meshgrid(xs, ys)
    pts = (X + 1j * Y).ravel()
    extra = np.array([np.nan, np.inf, -np.inf, complex(np.nan, 0.5), complex(0.5, np.inf),
                      np.nextafter(2.0, 0) + 0j, -2.0 + np.nextafter(1.0, 0) * 1j])
    pts = np.concatenate([pts, extra])
    pad = (-len(pts)) % 6
    pts = np.concatenate([pts, np.full(pad, np.nan)])
    roots = pts.reshape(6, -1)
    got = _density(roots, win, shape)
    want = oracle.density(roots, win, shape)
    assert np.array_equal(got, want)


def test_density_empty():
    r = np.zeros((6, 0), dtype=np.complex128)
    assert _density(r, (-1, 1, -1, 1), (8, 8)).sum() == 0


def test_backward_against_oracle():
    coeffs, true_roots, targets = workloads.known_roots(50000, seed=0)
    ref, st = oracle.solve(coeffs)
    g = 2.0 * (ref - targets)
    got, gst = pr.backward(to_dev(coeffs), to_dev(ref), to_dev(g))
    want, wst = oracle.backward(coeffs, ref, g)
    got = to_host(got)
    scale = np.abs(want).max(axis=0)
    err = np.abs(got - want).max(axis=0) / scale
    assert err.max() < 1e-10
    assert np.all(to_host(gst) == 0)


def test_backward_mixed_and_flags():
    a, deg = workloads.mixed(20000, seed=2)
    ref, st = oracle.solve(a, deg)
    g = workloads.cotangents(20000, seed=3)
    st = st.copy()
    st[:10] |= oracle.ST_NONFINITE
    got, gst = pr.backward(to_dev(a), to_dev(np.nan_to_num(ref)), to_dev(g), to_dev(deg),
                           to_dev(st.astype(np.int32)))
    want, wst = oracle.backward(a, np.nan_to_num(ref), g, deg, st)
    got = to_host(got)
    scale = np.maximum(np.abs(want).max(axis=0), 1e-300)
    assert (np.abs(got - want).max(axis=0) / scale).max() < 1e-10
    assert np.array_equal(to_host(gst).astype(np.uint32), wst)
    assert np.all(got[:, :10] == 0)


def test_backward_singular_root():
    coeffs = np.zeros((7, 1), dtype=np.complex128)
    coeffs[:4, 0] = [-2.0, 5.0, -4.0, 1.0]        # (z-1)^2 (z-2)
    deg = np.array([3], dtype=np.int32)
    roots = np.full((6, 1), np.nan, dtype=np.complex128)
    roots[:3, 0] = [1.0, 1.0, 2.0]
    g = np.ones((6, 1), dtype=np.complex128)
    got, st = pr.backward(to_dev(coeffs), to_dev(roots), to_dev(g), to_dev(deg),
                          to_dev(np.zeros(1, np.int32)))
    want, wst = oracle.backward(coeffs, roots, g, deg, np.zeros(1, np.uint32))
    assert to_host(st)[0] == pr.ST_SINGULAR_DERIV == wst[0]
    np.testing.assert_allclose(to_host(got), want, rtol=1e-14)


def test_autograd_matches_finite_differences():
    """L = sum |r - t|^2 with the assignment to the generating roots frozen;
    gradient of the GPU forward by central differences (h = 1e-6 and 2e-6,
    one Richardson step) within 1e-6 relative."""
    n = 256
    coeffs, true_roots, targets = workloads.known_roots(n, seed=11)
    c = to_dev(coeffs).requires_grad_(True)
    roots, status = pr.RootsFn.apply(c, None, "fp64")
    r0 = to_host(roots)
    perm_r = match(r0, true_roots)
    # targets aligned to the solver's root order
    tgt = np.empty_like(targets)
    for i in range(n):
        for j in range(6):
            k = int(np.argmin(np.abs(true_roots[:, i] - r0[j, i])))
            tgt[j, i] = targets[k, i]
    T = to_dev(tgt)
    loss = (roots - T).abs().pow(2).sum()
    loss.backward()
    grad = to_host(c.grad)

    def L(cc):
        r, _ = pr.solve(to_dev(cc))
        r = match(to_host(r), r0)
        return (np.abs(r - tgt) ** 2).sum(axis=0)

    def fd(h):
        out = np.zeros((7, n), dtype=np.complex128)
        for k in range(7):
            for unit in (1.0, 1j):
                cp = coeffs.copy(); cp[k] += h * unit
                cm = coeffs.copy(); cm[k] -= h * unit
                out[k] += unit * (L(cp) - L(cm)) / (2 * h)
        return out

    f1, f2 = fd(1e-6), fd(2e-6)
    est = (4 * f1 - f2) / 3
    err = np.abs(grad - est).max(axis=0) / np.abs(grad).max(axis=0)
    assert err.max() < 1e-6


def test_gradcheck_tiny():
    coeffs, _, _ = workloads.known_roots(4, seed=3)
    c = to_dev(coeffs).requires_grad_(True)

    def f(x):
        return pr.roots(x)

    assert torch.autograd.gradcheck(f, (c,), eps=1e-7, atol=1e-6, rtol=1e-5)


@pytest.mark.parametrize("n", [0, 1, 127, 128, 129, 1000])
def test_backward_bad_degrees_and_ragged_sizes(n):
    # degrees outside 1..dmax leave the gradient zero and the status as it
    # was, whatever rows the coefficient array holds for them
    rng = np.random.default_rng(11 + n)
    a = workloads.gaussian(max(n, 1), seed=5)[:, :n]
    ref, st = oracle.solve(a) if n else (np.zeros((6, 0), np.complex128), np.zeros(0, np.uint32))
    deg = np.full(n, 6, dtype=np.int32)
    bad = rng.random(n) < 0.3
    deg[bad] = rng.choice(np.array([-3, 0, 7, 100], dtype=np.int32), size=int(bad.sum()))
    g = workloads.cotangents(max(n, 1), seed=6)[:, :n]
    r = np.nan_to_num(ref)
    got, gst = pr.backward(to_dev(a), to_dev(r), to_dev(g), to_dev(deg),
                           to_dev(st.astype(np.int32)))
    want, wst = oracle.backward(a, r, g, deg, st)
    got = to_host(got)
    assert got.shape == (7, n)
    assert np.all(got[:, bad] == 0) and np.all(want[:, bad] == 0)
    assert np.array_equal(to_host(gst).astype(np.uint32), wst)
    if (~bad).any():
        scale = np.abs(want[:, ~bad]).max(axis=0)
        assert (np.abs(got[:, ~bad] - want[:, ~bad]).max(axis=0) / scale).max() < 1e-10
