"""GPU parity of pr_solve_bin, the one-launch solve + density path (Sec. III:
roots go straight to pixel counts).

Its contract is exact: the roots and status of pr_solve, and the image
pr_density makes from them, bit for bit -- with the roots stored or not,
in both precision forms and both launch layouts.  The image is also checked
against the oracle's binning of the same root array.
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

SKIP_ALL = 0x1F  # every flag a solve can set


def _bits(t):
    """Bit pattern of a complex128 tensor (NaN payloads included)."""
    return to_host(torch.view_as_real(t).contiguous().view(torch.int64))


def _case(name):
    if name == "gaussian":
        return workloads.gaussian(65536, seed=0), None, workloads.GAUSSIAN_WINDOW, (256, 256)
    if name == "parametric":
        a = workloads.parametric(4096, seed=0, rows=slice(1024, 1040))   # 65,536 polys
        return a, None, workloads.PARAMETRIC_WINDOW, (1920, 1080)
    if name == "mixed":
        a, deg = workloads.mixed(100_000, seed=2)
        return a, deg, (-10.0, 10.0, -10.0, 10.0), (640, 480)
    if name == "clustered":
        a, _ = workloads.clustered(65536, seed=3)
        return a, None, workloads.CLUSTERED_WINDOW, (1920, 1080)
    raise KeyError(name)


def _compare(a, deg, win, shape, precision, skip, **kw):
    ad = to_dev(a)
    dd = None if deg is None else to_dev(deg)
    kw.setdefault("max_iter_per_level", 30)
    r1, s1 = pr.solve(ad, dd, precision, **kw)
    h1 = pr.density(r1, win, shape, dd, s1, skip)
    r2, s2, h2 = pr.solve_bin(ad, win, shape, dd, precision, skip_mask=skip, **kw)
    r3, s3, h3 = pr.solve_bin(ad, win, shape, dd, precision, skip_mask=skip, store_roots=False,
                              **kw)
    torch.cuda.synchronize()
    assert r3 is None
    assert np.array_equal(_bits(r1), _bits(r2))
    assert np.array_equal(to_host(s1), to_host(s2))
    assert np.array_equal(to_host(s1), to_host(s3))
    img = to_host(h1)
    assert np.array_equal(img, to_host(h2))
    assert np.array_equal(img, to_host(h3))
    # the same image from the oracle's binning of the GPU's root array
    want = oracle.density(to_host(r1), win, shape, deg, to_host(s1).astype(np.uint32), skip)
    assert np.array_equal(img, want)
    return img, to_host(s1)


@pytest.mark.parametrize("precision", ["fp64", "fp32_polish"])
@pytest.mark.parametrize("name", ["gaussian", "parametric", "mixed", "clustered"])
def test_fused_equals_solve_then_density(name, precision):
    a, deg, win, shape = _case(name)
    skip = SKIP_ALL if name == "clustered" else 0
    img, st = _compare(a, deg, win, shape, precision, skip)
    n_roots = a.shape[1] * 6 if deg is None else int(np.clip(deg, 0, 6).sum())
    assert 0 < img.sum() <= n_roots
    if name == "clustered" and precision == "fp32_polish":
        assert (st != 0).any()          # the skip mask was exercised


@pytest.mark.parametrize("precision", ["fp64", "fp32_polish"])
@pytest.mark.parametrize("name", ["gaussian", "clustered", "mixed"])
def test_fused_with_run_ahead(name, precision):
    """Lanes running ahead, in the index-order layout (and for mixed degrees
    also in the sliced one): the same contract.  FP64 with the roots stored
    takes the pixels from the stored roots at the end; without them it keeps
    them in registers."""
    a, deg, win, shape = _case(name)
    skip = SKIP_ALL if name == "clustered" else 0
    _compare(a, deg, win, shape, precision, skip, tile=-1, grid_blocks=0,
             flags=pr.FLAG_RUN_AHEAD)
    if deg is not None:
        _compare(a, deg, win, shape, precision, skip, tile=512, grid_blocks=0,
                 flags=pr.FLAG_RUN_AHEAD)


@pytest.mark.parametrize("precision", ["fp64", "fp32_polish"])
def test_fused_mixed_flat_layout_and_fixed_steps(precision):
    a, deg, win, shape = _case("mixed")
    _compare(a, deg, win, shape, precision, 0, tile=-1)
    _compare(a, deg, win, shape, precision, 0, max_iter_per_level=10,
             flags=pr.FLAG_FIXED_STEPS)


@pytest.mark.parametrize("precision", ["fp64", "fp32_polish"])
def test_fused_invalid_polynomials_ragged_and_accumulate(precision):
    rng = np.random.default_rng(7)
    for n in (1, 63, 65, 257, 3001):
        a = workloads.gaussian(n, seed=n)
        deg = rng.integers(-1, 9, n).astype(np.int32)
        a[2, :: 11] = np.nan
        a[6, 3:: 13] = 0.0
        win, shape = (-2.5, 2.0, -1.5, 2.5), (97, 61)
        for skip in (0, pr.ST_NOT_CONVERGED | pr.ST_POLISH_UNCONVERGED):
            _compare(a, deg, win, shape, precision, skip)
    # counts are added to the given image
    a = workloads.gaussian(5000, seed=9)
    base = rng.integers(0, 3, (50, 40)).astype(np.int32)
    win, shape = (-2.0, 2.0, -2.0, 2.0), (40, 50)
    out = to_dev(base)
    roots, st, out = pr.solve_bin(to_dev(a), win, shape, None, precision, out=out)
    want = oracle.density(to_host(roots), win, shape, None, None, 0, out=base.copy())
    assert np.array_equal(to_host(out), want)


def test_fused_empty_and_errors():
    c = torch.zeros((7, 0), dtype=torch.complex128, device="cuda")
    r, s, h = pr.solve_bin(c, (-1, 1, -1, 1), (8, 8))
    assert r.shape == (6, 0) and s.shape == (0,) and int(h.sum()) == 0
    with pytest.raises(pr.ProotsError):
        pr.solve_bin(to_dev(workloads.gaussian(10)), (1, -1, -1, 1), (8, 8))


@pytest.mark.parametrize("precision", ["fp64", "fp32_polish"])
def test_chunked_accumulation_without_roots(precision):
    """Video-rate use: consecutive chunks counted into one image, no root
    array anywhere; equals the image of the whole batch."""
    a = workloads.parametric(4096, seed=0, rows=slice(2000, 2016))    # 65,536 polys
    win, shape = workloads.PARAMETRIC_WINDOW, (1920, 1080)
    whole, st_whole = _compare(a, None, win, shape, precision, 0)
    img = torch.zeros((shape[1], shape[0]), dtype=torch.int32, device="cuda")
    bounds = [0, 1000, 20000, 20001, 65536]
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        chunk = to_dev(np.ascontiguousarray(a[:, lo:hi]))
        r, st, _ = pr.solve_bin(chunk, win, shape, None, precision, out=img, store_roots=False,
                                max_iter_per_level=30)
        assert r is None
        assert np.array_equal(to_host(st), st_whole[lo:hi])
    assert np.array_equal(to_host(img), whole)
