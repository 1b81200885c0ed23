"""Binning counts every root once whatever the pattern of equal pixels.

The density kernel and the solve kernels' binning epilogue add one atomic
per run of consecutive lanes that hold the same pixel.  These cases put
crafted pixel patterns under that merge -- one pixel for a whole batch,
alternating pixels, runs broken by out-of-window and NaN roots, runs that
cross wave boundaries, skipped lanes and ragged batches -- and hold the
image to the oracle's binning bit for bit (Sec. III: each root adds one to
its pixel).
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

WIN = (-2.0, 2.0, -1.0, 1.0)
SHAPE = (40, 20)          # width, height: pixels of 0.1 x 0.1


def _centre(p):
    """Complex point at the centre of pixel index p (row-major)."""
    u, v = p % SHAPE[0], p // SHAPE[0]
    return complex(WIN[0] + (u + 0.5) * 0.1, WIN[2] + (v + 0.5) * 0.1)


def _runs(rng, n, pixels):
    """Runs of random lengths 1..70 over a few pixels, with out-of-window and
    NaN roots mixed in as their own runs."""
    out = np.empty(n, dtype=np.complex128)
    i = 0
    while i < n:
        ln = int(rng.integers(1, 71))
        kind = rng.integers(0, 8)
        if kind == 0:
            z = complex(WIN[1] + 1.0, 0.0)            # right of the window
        elif kind == 1:
            z = complex(np.nan, 0.0)
        else:
            z = _centre(int(rng.choice(pixels)))
        out[i:i + ln] = z
        i += ln
    return out


@pytest.mark.parametrize("n", [1, 63, 64, 65, 64 * 5 + 37, 4096 + 11])
def test_density_pixel_patterns(n):
    rng = np.random.default_rng(n)
    dmax = 4
    roots = np.empty((dmax, n), dtype=np.complex128)
    roots[0] = _centre(123)                                   # one pixel throughout
    roots[1] = np.where(np.arange(n) % 2 == 0, _centre(5), _centre(6))   # alternating
    roots[2] = _runs(rng, n, [7, 8, 9])                       # runs, repeats apart
    roots[3] = _centre(int(rng.integers(0, SHAPE[0] * SHAPE[1])))
    roots[3, rng.random(n) < 0.3] = complex(0.0, np.inf)      # holes in a long run
    degrees = rng.integers(1, dmax + 1, n).astype(np.int32)
    status = np.where(rng.random(n) < 0.2, pr.ST_NOT_CONVERGED, 0).astype(np.uint32)
    for deg, st, skip in ((None, None, 0), (degrees, None, 0), (degrees, status, pr.ST_NOT_CONVERGED)):
        got = pr.density(to_dev(roots), WIN, SHAPE, None if deg is None else to_dev(deg),
                         None if st is None else to_dev(st.astype(np.int32)), skip)
        torch.cuda.synchronize()
        want = oracle.density(roots, WIN, SHAPE, deg, st, skip)
        assert np.array_equal(to_host(got), want), (n, skip)
    # the whole first row lands on one pixel: a run across every wave
    assert oracle.density(roots[:1], WIN, SHAPE)[123 // SHAPE[0], 123 % SHAPE[0]] == n


@pytest.mark.parametrize("form,flags", [("fp32_polish", 0), ("fp32_polish", "ahead"),
                                        ("fp32_polish", "paired"), ("fp64", 0), ("fp64", "ahead")])
def test_solve_bin_runs_of_identical_polynomials(form, flags):
    """Blocks of identical polynomials put identical roots on neighbouring
    lanes (runs within and across waves); the one-launch image equals the
    oracle's binning of the returned roots (two polynomials per lane is an
    FP32 + polish layout only)."""
    fl = {0: 0, "ahead": pr.FLAG_RUN_AHEAD, "paired": pr.FLAG_PAIRED_LANES}[flags]
    rng = np.random.default_rng(7)
    base = workloads.gaussian(40, seed=11)
    cols, n = [], 0
    while n < 64 * 7 + 13:
        ln = int(rng.integers(1, 100))
        cols.append(np.repeat(base[:, rng.integers(0, 40)][:, None], ln, axis=1))
        n += ln
    a = np.concatenate(cols, axis=1)[:, :64 * 7 + 13].copy()
    win, shape = workloads.GAUSSIAN_WINDOW, (64, 64)
    r, s, h = pr.solve_bin(to_dev(a), win, shape, None, form, flags=fl)
    torch.cuda.synchronize()
    want = oracle.density(to_host(r), win, shape, None, to_host(s).astype(np.uint32), 0)
    assert np.array_equal(to_host(h), want)
    assert want.sum() > 0
