"""GPU parity of pr_solve's default shift rule -- Wilkinson's shift (the
eigenvalue of the trailing 2 x 2 block nearest its bottom entry), the first
step of each polynomial shifted by the root nearest 0 of b0 + b1 z + b2 z^2
-- against the oracle with FLAG_WILKINSON_SHIFT | FLAG_QUADRATIC_START (run
on an MI355X); PR_FLAG_RAYLEIGH_SHIFT selects Alg. 1's bottom-entry shift,
which the other solve tests pin.

The kernels evaluate the shifts without the oracle's divisions (see their
definitions in the solve kernel), so the two sides round differently and
exact per-level step counts are not pinned; their distribution is, and the
roots are held to the same bounds as with Alg. 1's shift."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from gpuutil import parity_bound, rel_condition, to_dev, to_host
from rootmatch import match, match_mixed, rel_err, valid_mask

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pr = pytest.importorskip("paper_2507_02164_amd")

W = oracle.FLAG_WILKINSON_SHIFT | oracle.FLAG_QUADRATIC_START
R = pr.FLAG_RAYLEIGH_SHIFT


def _solve(a, deg=None, precision="fp64", **kw):
    kw.setdefault("max_iter_per_level", 30)
    out = pr.solve(to_dev(a), None if deg is None else to_dev(deg), precision, **kw)
    torch.cuda.synchronize()
    return tuple(to_host(t) for t in out)


def _parity(got, st, a, deg, ref, ref_st, floor=1e-10):
    dmax, n = ref.shape
    m = match(got, ref) if deg is None else match_mixed(got, ref, deg)
    valid = valid_mask(dmax, deg, n)
    err = rel_err(m, ref)
    bound = parity_bound(rel_condition(a, ref, deg), floor)
    check = valid & (ref_st == 0)[None, :] & ((st & pr.ST_POLISH_UNCONVERGED) == 0)[None, :]
    bad = check & ~(err <= bound)
    assert not bad.any(), f"{bad.sum()} roots out of bound, worst {err[bad].max():.3e}"
    assert np.all(np.isnan(got[~valid]))


@pytest.mark.parametrize("precision", ["fp64", "fp32_polish"])
def test_gaussian_parity_and_steps(precision):
    a = workloads.gaussian(65536, seed=31)
    ref, ref_st, oit = oracle.solve(a, flags=W, return_iters=True)
    got, st, it = _solve(a, None, precision, iter_counts=True)
    assert np.all(ref_st == 0)
    assert (st & pr.ST_NOT_CONVERGED).sum() == 0
    assert (st & pr.ST_POLISH_UNCONVERGED).mean() < 1e-3
    _parity(got, st, a, None, ref, ref_st)
    if precision == "fp64":
        assert (it == oit).mean() > 0.95
        assert np.abs(it.mean(axis=1) - oit.mean(axis=1)).max() < 0.05
        assert (it[0] == 1).mean() > 0.999
    # fewer steps per level than with the bottom-entry shift, on the GPU too
    _, _, it0 = _solve(a, None, precision, flags=R, iter_counts=True)
    assert np.all(it.mean(axis=1) <= it0.mean(axis=1))


def test_parametric_slice_fp32_polish():
    a = np.ascontiguousarray(workloads.parametric(4096, seed=0)[:, 7_000_000:7_000_000 + 65536])
    ref, ref_st = oracle.solve(a, flags=W)
    got, st = _solve(a, None, "fp32_polish")
    _parity(got, st, a, None, ref, ref_st)
    assert (st & pr.ST_POLISH_UNCONVERGED).mean() < 1e-3


@pytest.mark.parametrize("precision", ["fp64", "fp32_polish"])
def test_mixed_degrees(precision):
    a, deg = workloads.mixed(100_000, seed=32)
    ref, ref_st, oit = oracle.solve(a, deg, flags=W, return_iters=True)
    for tile in (-1, 512):
        got, st, it = _solve(a, deg, precision, tile=tile, iter_counts=True)
        _parity(got, st, a, deg, ref, ref_st, floor=1e-10 if precision == "fp64" else 1e-8)
        if precision == "fp64":
            # every lane takes the quadratic start at its own top level: the
            # step counts of each degree's top level follow the oracle's
            for d in range(2, 7):
                sel = deg == d
                assert abs(it[d - 2, sel].mean() - oit[d - 2, sel].mean()) < 0.05, d
                assert (it[:, sel] == oit[:, sel]).mean() > 0.95, d


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6])
def test_roots_of_c(d):
    c = 2.0 + 1j
    a = np.zeros((7, 4), dtype=np.complex128)
    a[0] = -c
    a[d] = 1.0
    deg = np.full(4, d, dtype=np.int32)
    truth = (c ** (1.0 / d)) * np.exp(2j * np.pi * np.arange(d) / d)
    for precision in ("fp64", "fp32_polish"):
        got, st, it = _solve(a, deg, precision, iter_counts=True)
        assert np.all(st == 0)
        m = match(got[:d], np.repeat(truth[:, None], 4, axis=1))
        assert np.abs(m - truth[:, None]).max() < 1e-13
        if d == 2:
            assert np.all(it[0] == 1)


def test_large_entries_take_the_bottom_entry_shift():
    """Six roots of modulus about 2^9 (inside the range the FP32 form leaves
    unscaled): companion entries reach 2^54, so where the FP32 Wilkinson
    shift overflows the step must take the bottom entry instead.  Nothing may
    stall, and the result must be as good as with Alg. 1's shift throughout:
    the same share of polynomials flagged (these roots have no minimum gap,
    so FP32 + polish flags some either way) and the known roots elsewhere."""
    rng = np.random.default_rng(33)
    n = 4096
    roots = 512.0 * np.exp(2j * np.pi * rng.random((6, n))) * (1 + 0.5 * rng.random((6, n)))
    a = workloads.expand_roots(roots)
    for precision in ("fp64", "fp32_polish"):
        got, st = _solve(a, None, precision)
        _, st0 = _solve(a, None, precision, flags=R)
        assert not (st & pr.ST_NOT_CONVERGED).any()
        ok = (st & pr.ST_POLISH_UNCONVERGED) == 0
        ok0 = (st0 & pr.ST_POLISH_UNCONVERGED) == 0
        assert ok.mean() >= ok0.mean() - 0.005
        if precision == "fp64":
            assert ok.all()
        m = match(got, roots)
        assert rel_err(m[:, ok], roots[:, ok]).max() < 1e-9


def test_fixed_steps_take_the_bottom_entry_shift():
    """Alg. 2 literally: PR_FLAG_FIXED_STEPS shifts by the bottom entry
    whether or not PR_FLAG_RAYLEIGH_SHIFT is given (bit-identical), as the
    oracle's fixed-T mode does."""
    a = workloads.gaussian(8192, seed=34)
    T = 10
    ref, ref_st, oit = oracle.solve(a, fixed_t=T, return_iters=True)
    got, st, it = _solve(a, None, "fp64", flags=pr.FLAG_FIXED_STEPS, max_iter_per_level=T,
                         iter_counts=True)
    got1, st1 = _solve(a, None, "fp64", flags=pr.FLAG_FIXED_STEPS | R, max_iter_per_level=T)
    assert np.array_equal(np.ascontiguousarray(got).view(np.int64),
                          np.ascontiguousarray(got1).view(np.int64))
    assert np.array_equal(st, st1)
    assert np.all(it == T) and np.all(oit == T)
    _parity(got, st, a, None, ref, ref_st)


@pytest.mark.parametrize("precision", ["fp64", "fp32_polish"])
def test_solve_bin_with_the_default_shift(precision):
    a = workloads.gaussian(65536, seed=35)
    win, shape = workloads.GAUSSIAN_WINDOW, (256, 256)
    ad = to_dev(a)
    r1, s1 = pr.solve(ad, None, precision)
    r2, s2, h2 = pr.solve_bin(ad, win, shape, None, precision)
    torch.cuda.synchronize()
    b1 = to_host(torch.view_as_real(r1).contiguous().view(torch.int64))
    b2 = to_host(torch.view_as_real(r2).contiguous().view(torch.int64))
    assert np.array_equal(b1, b2) and np.array_equal(to_host(s1), to_host(s2))
    want = oracle.density(to_host(r1), win, shape, None, to_host(s1).astype(np.uint32), 0)
    assert np.array_equal(to_host(h2), want)
