"""GPU parity of pr_density_sorted, the tile-sorted density path (Sec. III:
roots converted to pixel coordinates and counted).

Its contract is exact: the image pr_density makes from the same roots, bit
for bit, which the oracle's binning pins -- over spread and clustered roots,
degree arrays, status skip masks, NaN and out-of-window roots, bin edges,
accumulation into a non-zero image, ragged and empty batches, tiles whose
roots need several segments, images beyond the tiled path's size (counted
directly), and the workspace errors.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from gpuutil import to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pr = pytest.importorskip("paper_2507_02164_amd")


def _both(roots, win, shape, degrees=None, status=None, skip=0, out=None):
    """(sorted image, direct image) of the same device roots."""
    r = roots if isinstance(roots, torch.Tensor) else to_dev(roots)
    d = None if degrees is None else (degrees if isinstance(degrees, torch.Tensor)
                                      else to_dev(degrees))
    s = None if status is None else (status if isinstance(status, torch.Tensor)
                                     else to_dev(status))
    o1 = None if out is None else to_dev(out)
    o2 = None if out is None else to_dev(out)
    h1 = pr.density_sorted(r, win, shape, d, s, skip, out=o1)
    h2 = pr.density(r, win, shape, d, s, skip, out=o2)
    torch.cuda.synchronize()
    return to_host(h1), to_host(h2)


def _oracle_roots(n, seed):
    a = workloads.gaussian(n, seed=seed)
    ref, _ = oracle.solve(a, flags=oracle.FLAG_WILKINSON_SHIFT | oracle.FLAG_QUADRATIC_START)
    return ref


@pytest.mark.parametrize("shape", [(256, 256), (1920, 1080), (640, 480)])
def test_spread_roots_match_direct_and_oracle(shape):
    roots = _oracle_roots(65536, 0)
    win = workloads.GAUSSIAN_WINDOW
    h1, h2 = _both(roots, win, shape)
    want = oracle.density(roots, win, shape)
    assert np.array_equal(h1, want)
    assert np.array_equal(h2, want)
    assert h1.sum() > 0.9 * roots.size


def test_parametric_slice_1080p():
    a = workloads.parametric(4096, seed=0, rows=slice(1024, 1040))
    roots, _ = oracle.solve(a, flags=oracle.FLAG_WILKINSON_SHIFT | oracle.FLAG_QUADRATIC_START)
    win, shape = workloads.PARAMETRIC_WINDOW, (1920, 1080)
    h1, _ = _both(roots, win, shape)
    assert np.array_equal(h1, oracle.density(roots, win, shape))


@pytest.mark.parametrize("dmax", [1, 2, 3, 4, 5, 6])
def test_degrees_status_and_masks(dmax):
    rng = np.random.default_rng(40 + dmax)
    n = 30000
    roots = (rng.standard_normal((dmax, n)) + 1j * rng.standard_normal((dmax, n))) * 1.2
    deg = rng.integers(-1, dmax + 2, n).astype(np.int32)          # some out of range
    st = rng.integers(0, 4, n).astype(np.uint32) << 3              # NOT_CONVERGED / POLISH bits
    roots[rng.random((dmax, n)) < 0.01] = np.nan
    roots[rng.random((dmax, n)) < 0.01] = complex(np.inf, 0.0)
    win, shape = (-3.0, 3.0, -2.0, 2.5), (300, 200)
    for skip in (0, 0x8, 0x18):
        h1, h2 = _both(roots, win, shape, deg, st.astype(np.int32), skip)
        want = oracle.density(roots, win, shape, deg, st, skip)
        assert np.array_equal(h1, want), skip
        assert np.array_equal(h2, want), skip


def test_bin_edges_and_accumulate():
    """Roots exactly on the window's edges (the lower ones count, the upper
    ones do not) and on pixel edges, counted into an image that already
    holds counts."""
    win, shape = (-2.0, 2.0, -1.0, 1.0), (64, 32)
    xs = np.array([-2.0, 2.0, 0.0, -2.0 + 4.0 / 64, np.nextafter(2.0, 0.0), -1.0, 1.0, 0.5])
    ys = np.array([-1.0, 1.0, 0.0, np.nextafter(1.0, 0.0), -1.0, -1.0 + 2.0 / 32, 0.25, -0.75])
    z = (xs[:, None] + 1j * ys[None, :]).ravel()
    n = z.size // 2 * 2
    roots = z[:n].reshape(2, n // 2)
    prior = np.random.default_rng(5).integers(0, 100, (32, 64)).astype(np.int32)
    h1, h2 = _both(roots, win, shape, out=prior)
    want = oracle.density(roots, win, shape, out=prior.copy())
    assert np.array_equal(h1, want) and np.array_equal(h2, want)


@pytest.mark.parametrize("n", [0, 1, 7, 1023, 1024, 1025, 5000])
def test_ragged_and_empty(n):
    roots = _oracle_roots(max(n, 1), n)[:, :n]
    win, shape = workloads.GAUSSIAN_WINDOW, (256, 256)
    h1, h2 = _both(np.ascontiguousarray(roots), win, shape)
    assert np.array_equal(h1, h2)
    assert np.array_equal(h1, oracle.density(roots, win, shape))


def test_dense_tile_split_into_segments():
    """Every root of 200k polynomials on a few pixels of one tile: the tile's
    list is longer than a segment, so several blocks share the tile and its
    partial images are summed."""
    n = 200_000
    rng = np.random.default_rng(7)
    roots = np.empty((6, n), dtype=np.complex128)
    pts = np.array([0.1 + 0.1j, 0.1001 + 0.1j, -0.2 + 0.05j, 0.3 - 0.01j])
    roots[:] = pts[rng.integers(0, 4, (6, n))]
    roots[0, ::3] = rng.uniform(-3, 3, n // 3 + (n % 3 > 0)) + 1j * rng.uniform(-3, 3, n // 3 + (n % 3 > 0))
    win, shape = workloads.GAUSSIAN_WINDOW, (1920, 1080)
    h1, h2 = _both(roots, win, shape)
    assert np.array_equal(h1, h2)
    assert h1.max() > 200_000


def test_large_image_counts_directly():
    """Images beyond 2^24 pixels need no workspace and are counted by the
    direct kernel: still the same image."""
    assert pr.density_sorted_workspace(65536, 6, 8192, 4096) == 0
    roots = _oracle_roots(65536, 3)
    win, shape = workloads.GAUSSIAN_WINDOW, (8192, 4096)
    h1, h2 = _both(roots, win, shape)
    assert np.array_equal(h1, h2)


def test_workspace_errors():
    roots = to_dev(_oracle_roots(4096, 4))
    win, shape = workloads.GAUSSIAN_WINDOW, (256, 256)
    need = pr.density_sorted_workspace(4096, 6, 256, 256)
    assert need > 0
    small = torch.empty((need - 1,), dtype=torch.uint8, device=roots.device)
    with pytest.raises(pr.ProotsError) as e:
        pr.density_sorted(roots, win, shape, workspace=small)
    assert e.value.code == pr.PR_ERR_NO_MEMORY
    big = torch.empty((need + 512,), dtype=torch.uint8, device=roots.device)
    with pytest.raises(pr.ProotsError) as e:
        pr.density_sorted(roots, win, shape, workspace=big[16:])
    assert e.value.code == pr.PR_ERR_INVALID_ARG
    # a workspace reused across calls of different sizes (its contents on
    # entry do not matter)
    ws = torch.empty((pr.density_sorted_workspace(65536, 6, 1920, 1080),), dtype=torch.uint8,
                     device=roots.device)
    big_roots = to_dev(_oracle_roots(65536, 5))
    win2, shape2 = workloads.GAUSSIAN_WINDOW, (1920, 1080)
    for r in (big_roots, roots, big_roots[:, :1000].contiguous()):
        a = pr.density_sorted(r, win2, shape2, workspace=ws)
        b = pr.density(r, win2, shape2)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


def test_full_size_spread_roots():
    """16Mi Gaussian degree-6 polynomials (100M roots) at 1920 x 1080: the
    GPU's own roots binned both ways, bit for bit, and against the oracle's
    binning of the same root array."""
    n = 16 * 2 ** 20
    a = to_dev(workloads.gaussian(n, seed=0))
    r, st = pr.solve(a, None, "fp32_polish")
    del a
    win, shape = workloads.GAUSSIAN_WINDOW, (1920, 1080)
    h1 = pr.density_sorted(r, win, shape, status=st)
    h2 = pr.density(r, win, shape, status=st)
    torch.cuda.synchronize()
    assert torch.equal(h1, h2)
    want = oracle.density(to_host(r), win, shape)
    assert np.array_equal(to_host(h1), want)
