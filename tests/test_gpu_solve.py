"""GPU parity of pr_solve against the oracle (run on an MI355X).

Roots are compared after the optimal assignment per polynomial.  FP64 form:
relative error <= 1e-10, or, for a root whose relative condition number
kappa makes 1e-10 unreachable in FP64, <= 1e3 kappa u (the rounding floor
both sides share).  FP32 + FP64-polish form: every root of a polynomial
without POLISH_UNCONVERGED within the same bound; flagged polynomials are
counted and bounded separately.
"""
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

# the oracle with the library's default shift rule (Wilkinson's shift, the
# first step from the quadratic start); tests of Alg. 1's shift pass
# PR_FLAG_RAYLEIGH_SHIFT to the library and no flag to the oracle
OW = oracle.FLAG_WILKINSON_SHIFT | oracle.FLAG_QUADRATIC_START


def _solve(a, deg=None, precision="fp64", **kw):
    kw.setdefault("max_iter_per_level", 30)   # the oracle's cap
    out = pr.solve(to_dev(a), None if deg is None else to_dev(deg), precision, **kw)
    torch.cuda.synchronize()
    return tuple(to_host(t) for t in out)


def _check_roots(got, st, a, deg, ref, ref_st, floor=1e-10, flagged_ok=False):
    """Assert parity; returns (max relative error over checked roots,
    fraction of polynomials flagged)."""
    dmax, n = ref.shape
    m = match(got, ref) if deg is None else match_mixed(got, ref, deg)
    valid = valid_mask(dmax, deg, n)
    kappa = rel_condition(a, ref, deg)
    err = rel_err(m, ref)
    bound = parity_bound(kappa, floor)
    ok_poly = (ref_st == 0)
    flagged = (st & pr.ST_POLISH_UNCONVERGED) != 0
    check = valid & ok_poly[None, :]
    if flagged_ok:
        check &= ~flagged[None, :]
    bad = check & ~(err <= bound)
    assert not bad.any(), (f"{bad.sum()} roots out of bound; worst err {err[bad].max():.3e} "
                           f"kappa {kappa[bad][np.argmax(err[bad])]:.3e}")
    # rows beyond the degree are NaN
    assert np.all(np.isnan(got[~valid]))
    return float(err[check].max()), float(flagged.mean())


# the two shift rules: (library flags, oracle flags).  "alg1" is Alg. 1's
# own shift, the bottom-right entry of the active block; "default" is the
# library's default rule (Wilkinson's shift and the quadratic start).
RULES = {"default": (0, OW), "alg1": (pr.FLAG_RAYLEIGH_SHIFT, 0)}


@pytest.mark.parametrize("rule", ["default", "alg1"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_polish"])
def test_gaussian_full(precision, rule):
    """65,536 monic degree-6 polynomials with standard complex normal
    coefficients, every root, under either shift rule (the oracle taking
    the same rule)."""
    gflags, oflags = RULES[rule]
    a = workloads.gaussian(65536, seed=0)
    ref, ref_st = oracle.solve(a, flags=oflags)
    got, st = _solve(a, None, precision, flags=gflags)
    assert np.all(ref_st == 0)
    if precision == "fp64":
        assert np.all(st == 0)
    else:
        assert np.all((st & ~pr.ST_POLISH_UNCONVERGED) == 0)
    worst, flagged = _check_roots(got, st, a, None, ref, ref_st, flagged_ok=precision != "fp64")
    print(f"\n{precision} {rule}: worst rel err {worst:.3e}, flagged {flagged:.2e}")
    assert flagged < 1e-3
    assert worst < 1e-10


def _grid(source):
    if source == "grid256":       # the parametric family on a 256 x 256 grid
        return workloads.parametric(256, seed=0)
    # 16 rows (65,536 polynomials) of the full 4096 x 4096 grid
    return workloads.parametric(4096, seed=0, rows=slice(2040, 2056))


@pytest.mark.parametrize("rule", ["default", "alg1"])
@pytest.mark.parametrize("source", ["grid256", "slice4096"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_polish"])
def test_parametric_grid(precision, source, rule):
    gflags, oflags = RULES[rule]
    a = _grid(source)
    ref, ref_st = oracle.solve(a, flags=oflags)
    got, st = _solve(a, None, precision, flags=gflags)
    assert np.all(ref_st == 0)
    assert np.all((st & ~pr.ST_POLISH_UNCONVERGED) == 0)
    worst, flagged = _check_roots(got, st, a, None, ref, ref_st, flagged_ok=precision != "fp64")
    print(f"\n{precision} {source} {rule}: worst rel err {worst:.3e}, flagged {flagged:.2e}")
    assert flagged < 1e-3
    if precision == "fp64":
        assert flagged == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32_polish"])
def test_mixed_degree(precision):
    """Degrees 2..6 in one batch, log-uniform moduli; FP32 + polish within
    1e-8 of the FP64 oracle on every polynomial."""
    a, deg = workloads.mixed(50000, seed=3)
    ref, ref_st = oracle.solve(a, deg, flags=OW)
    got, st = _solve(a, deg, precision)
    floor = 1e-10 if precision == "fp64" else 1e-8
    worst, flagged = _check_roots(got, st, a, deg, ref, ref_st, floor=floor,
                                  flagged_ok=precision != "fp64")
    print(f"\n{precision}: worst {worst:.3e} flagged {flagged:.2e}")
    assert flagged < 1e-2


def test_known_roots_against_truth():
    coeffs, roots, _ = workloads.known_roots(20000, seed=0)
    got, st = _solve(coeffs, None, "fp64")
    assert np.all(st == 0)
    m = match(got, roots)
    kappa = rel_condition(coeffs, roots)
    err = rel_err(m, roots)
    # the generating roots are exact only up to the rounding of the expanded
    # coefficients (relative u per coefficient), hence a kappa-scaled bound
    assert np.all(err <= np.maximum(1e-12, 64 * kappa * 2.0 ** -53))


def test_clustered_classes():
    """Three roots within 1e-3 of each other: FP64 resolves the cluster to
    the rounding floor kappa u; the isolated roots and the cluster centroid
    stay within 1e-9.  FP32 + polish flags (nearly) every cluster."""
    coeffs, roots = workloads.clustered(8192, seed=0)
    ref, ref_st = oracle.solve(coeffs, flags=OW)
    got, st = _solve(coeffs, None, "fp64")
    kappa = rel_condition(coeffs, ref)
    m = match(got, ref)
    err = rel_err(m, ref)
    assert np.all(err <= parity_bound(kappa, 1e-9, c=1e4))
    g32, s32 = _solve(coeffs, None, "fp32_polish")
    flagged = (s32 & pr.ST_POLISH_UNCONVERGED) != 0
    assert flagged.mean() > 0.5
    ok = ~flagged
    if ok.any():
        e32 = rel_err(match(g32[:, ok], ref[:, ok]), ref[:, ok])
        assert np.all(e32 <= parity_bound(kappa[:, ok], 1e-9, c=1e4))


@pytest.mark.parametrize("n", [1, 7, 255, 257, 1000])
def test_ragged_sizes(n):
    a = workloads.gaussian(n, seed=n)
    ref, _ = oracle.solve(a, flags=OW)
    for precision in ("fp64", "fp32_polish"):
        got, st = _solve(a, None, precision)
        assert got.shape == (6, n)
        assert rel_err(match(got, ref), ref).max() < 1e-10


@pytest.mark.parametrize("dmax", [1, 2, 3, 4, 5])
def test_smaller_dmax(dmax):
    rng = np.random.default_rng(dmax)
    n = 3000
    a = (rng.standard_normal((dmax + 1, n)) + 1j * rng.standard_normal((dmax + 1, n))) / np.sqrt(2)
    deg = rng.integers(1, dmax + 1, n).astype(np.int32)
    ref, ref_st = oracle.solve(a, deg, flags=OW)
    for precision in ("fp64", "fp32_polish"):
        got, st = _solve(a, deg, precision)
        assert np.array_equal(st & 0x7, ref_st & 0x7)
        _check_roots(got, st, a, deg, ref, ref_st, floor=1e-9, flagged_ok=precision != "fp64")


def test_invalid_inputs_and_flags():
    a = workloads.gaussian(8, seed=1)
    deg = np.array([6, 0, 7, 6, 6, 1, -3, 6], dtype=np.int32)
    a[2, 3] = np.nan
    a[6, 4] = 0.0
    a[1, 7] = np.inf
    ref, ref_st = oracle.solve(a, deg, flags=OW)
    for precision in ("fp64", "fp32_polish"):
        got, st = _solve(a, deg, precision)
        np.testing.assert_array_equal(st.astype(np.uint32) & 0x7, ref_st)
        for i in (1, 2, 3, 4, 6, 7):
            assert np.all(np.isnan(got[:, i]))
        assert abs(got[0, 5] - ref[0, 5]) <= 4e-16 * abs(ref[0, 5])
        assert np.all(np.isnan(got[1:, 5]))


def test_special_polynomials():
    cols = []
    for d in range(2, 7):
        z = np.zeros(7, dtype=np.complex128); z[d] = 1.0          # z^d
        cols.append(z)
        for c in (1.0, -1.0, 1j, 2.0):
            w = np.zeros(7, dtype=np.complex128); w[0] = -c; w[d] = 1.0   # z^d - c
            cols.append(w)
    a = np.stack(cols, axis=1)
    deg = np.array([int(np.nonzero(a[:, i])[0].max()) for i in range(a.shape[1])], dtype=np.int32)
    ref, ref_st = oracle.solve(a, deg, flags=OW)
    got, st = _solve(a, deg, "fp64")
    assert np.all(st == 0) and np.all(ref_st == 0)
    m = match_mixed(got, ref, deg)
    v = valid_mask(6, deg, a.shape[1])
    assert np.abs(m - ref)[v].max() < 1e-14 * 4
    # with the exceptional shift off, z^d - c stalls and is flagged: with
    # Alg. 1's shift at every degree, with Wilkinson's (the default) from
    # degree 3 on (its 2 x 2 block [[0, 0], [1, 0]] gives the same shift 0)
    for gflags, oflags in ((pr.FLAG_RAYLEIGH_SHIFT, 0), (0, OW)):
        got, st = _solve(a, deg, "fp64", flags=pr.FLAG_NO_EXCEPTIONAL_SHIFT | gflags)
        _, ost = oracle.solve(a, deg, flags=oracle.FLAG_NO_EXCEPTIONAL_SHIFT | oflags)
        np.testing.assert_array_equal(st.astype(np.uint32) & pr.ST_NOT_CONVERGED,
                                      ost & pr.ST_NOT_CONVERGED)
        assert (st & pr.ST_NOT_CONVERGED).sum() > 0
    # a cap of one step per level flags (nearly) everything, host-forced
    g = workloads.gaussian(512, seed=2)
    got, st = _solve(g, None, "fp64", max_iter_per_level=1)
    assert ((st & pr.ST_NOT_CONVERGED) != 0).mean() > 0.9


def test_non_monic():
    a = workloads.gaussian(20000, seed=4) * (0.3 - 2.1j)
    ref, _ = oracle.solve(a, flags=OW)
    for precision in ("fp64", "fp32_polish"):
        got, st = _solve(a, None, precision)
        _check_roots(got, st, a, None, ref, np.zeros(a.shape[1], np.uint32),
                     flagged_ok=precision != "fp64")


def test_vieta_trace_on_gpu():
    """Sum of the roots equals -a_5 (monic) up to rounding, converged or not."""
    a = workloads.gaussian(65536, seed=7)
    got, st = _solve(a, None, "fp64", max_iter_per_level=3)
    s = got.sum(axis=0)
    scale = np.abs(got).sum(axis=0)
    assert np.all(np.abs(s + a[5]) <= 64 * 2.0 ** -53 * scale)


def test_iteration_counts_distribution():
    """Alg. 1's shift (PR_FLAG_RAYLEIGH_SHIFT): exact per-level counts depend
    on rounding (parity unpinned); their distribution must match the
    oracle's, and z^d deflates in one step.  The default shift's counts are
    checked with its own tests."""
    a = workloads.gaussian(65536, seed=0)
    _, _, oit = oracle.solve(a, return_iters=True)
    got, st, it = _solve(a, None, "fp64", iter_counts=True, flags=pr.FLAG_RAYLEIGH_SHIFT)
    assert it.shape == (5, 65536)
    assert np.abs(it.mean(axis=1) - oit.mean(axis=1)).max() < 0.05 * oit.mean(axis=1).max()
    assert (it == oit).mean() > 0.9
    z = np.zeros((7, 4), dtype=np.complex128); z[6] = 1.0
    for flags in (pr.FLAG_RAYLEIGH_SHIFT, 0):
        _, _, zit = _solve(z, None, "fp64", iter_counts=True, flags=flags)
        assert np.all(zit == 1)


def test_deterministic():
    a = workloads.gaussian(65536, seed=5)
    for precision in ("fp64", "fp32_polish"):
        r1, s1 = _solve(a, None, precision)
        r2, s2 = _solve(a, None, precision)
        assert np.array_equal(r1, r2, equal_nan=True) and np.array_equal(s1, s2)


def test_stream_and_out_buffers():
    a = workloads.gaussian(4096, seed=6)
    ref, _ = oracle.solve(a, flags=OW)
    s = torch.cuda.Stream()
    ca = to_dev(a)
    roots = torch.empty((6, 4096), dtype=torch.complex128, device=ca.device)
    status = torch.empty((4096,), dtype=torch.int32, device=ca.device)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        pr.solve(ca, None, "fp64", roots=roots, status=status)
    s.synchronize()
    assert rel_err(match(to_host(roots), ref), ref).max() < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32_polish"])
def test_tiled_equals_flat(precision):
    """Degree-sorted tiles only regroup the lanes: every lane's arithmetic is
    its own, so roots, status and step counts are bit-identical to the
    index-order launch, for any tile size and grid."""
    a, deg = workloads.mixed(30000, seed=8)
    deg = deg.copy()
    deg[::997] = 0          # invalid degrees mixed in
    deg[5::1009] = 7
    flat = _solve(a, deg, precision, tile=-1, iter_counts=True)
    # grid 0: one wave per (tile, slice); > 0: persistent waves walking the tiles
    for tile, grid in [(64, 0), (100, 0), (512, 0), (1000, 0), (4096, 0), (100, 3), (2048, 64),
                       (4096, 1), (1000, 7), (2048, 100000)]:
        got = _solve(a, deg, precision, tile=tile, grid_blocks=grid, iter_counts=True)
        for x, y in zip(got, flat):
            assert np.array_equal(x, y, equal_nan=True), (tile, grid)
    ref, ref_st = oracle.solve(a, deg, flags=OW)
    np.testing.assert_array_equal(flat[1].astype(np.uint32) & 0x7, ref_st & 0x7)


@pytest.mark.parametrize("n", [1, 64, 127, 128, 129, 5000, 65536])
def test_paired_lanes_match_the_oracle(n):
    """PR_FLAG_PAIRED_LANES packs two polynomials into each lane.  Each
    polynomial's arithmetic is the same, but the compiler fuses multiply-adds
    differently in the two kernels, so the roots are held to the oracle's
    bounds (not to the one-per-lane kernel's bits); status and the one-launch
    image follow the oracle's rules on the kernel's own roots, for ragged
    batches and smaller dmax too."""
    a = workloads.gaussian(n, seed=40 + n)
    ref, ref_st = oracle.solve(a, flags=OW)
    got, st, it = _solve(a, None, "fp32_polish", iter_counts=True, flags=pr.FLAG_PAIRED_LANES)
    _, st1, it1 = _solve(a, None, "fp32_polish", iter_counts=True)
    assert np.all((st & ~pr.ST_POLISH_UNCONVERGED) == 0)
    _check_roots(got, st, a, None, ref, ref_st, flagged_ok=True)
    assert (it == it1).mean() > 0.95
    win, shape = workloads.GAUSSIAN_WINDOW, (256, 256)
    ad = to_dev(a)
    r2, s2, h2 = pr.solve_bin(ad, win, shape, None, "fp32_polish", flags=pr.FLAG_PAIRED_LANES)
    torch.cuda.synchronize()
    want = oracle.density(to_host(r2), win, shape, None, to_host(s2).astype(np.uint32), 0)
    assert np.array_equal(to_host(h2), want)
    rng = np.random.default_rng(n)
    b = (rng.standard_normal((5, n)) + 1j * rng.standard_normal((5, n))) / np.sqrt(2)
    deg = rng.integers(0, 6, n).astype(np.int32)          # 0 and 5 (> dmax 4): invalid
    deg[0] = 4
    ref, ref_st = oracle.solve(b, deg, flags=OW)
    got, st = _solve(b, deg, "fp32_polish", tile=-1, flags=pr.FLAG_PAIRED_LANES)
    assert np.array_equal(st & 0x7, ref_st & 0x7)
    _check_roots(got, st, b, deg, ref, ref_st, floor=1e-9, flagged_ok=True)


def _ahead_source(source, n):
    """(coeffs, degrees or None, solve keywords) of a run-ahead case."""
    if source == "gaussian":
        return workloads.gaussian(n, seed=61), None, {}
    if source == "clustered":
        return workloads.clustered(n, seed=62)[0], None, {}
    if source == "grid":
        return workloads.parametric(4096, seed=0, rows=slice(1000, 1000 + n // 4096)), None, {}
    a, deg = workloads.mixed(n, seed=63)
    return a, deg, {"tile": 512 if source == "mixed_sliced" else -1, "grid_blocks": 0}


@pytest.mark.parametrize("rule", ["default", "alg1"])
@pytest.mark.parametrize("source", ["gaussian", "clustered", "grid", "mixed_sliced", "mixed_flat"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_polish"])
def test_run_ahead_matches_the_oracle(precision, source, rule):
    """PR_FLAG_RUN_AHEAD lets the lanes one level below the wave's level
    step inside its trips.  Every lane takes the same tests, shifts and
    steps as without it, only earlier: roots are held to the oracle's
    bounds, status to the oracle's status, and the per-level step counts
    agree with the lock-step launch's (rounding may move a deflation test by
    a step now and then)."""
    gflags, oflags = RULES[rule]
    n = 16384 if source == "clustered" else 65536
    a, deg, kw = _ahead_source(source, n)
    ref, ref_st = oracle.solve(a, deg, flags=oflags)
    got, st, it = _solve(a, deg, precision, iter_counts=True, flags=gflags | pr.FLAG_RUN_AHEAD, **kw)
    _, st0, it0 = _solve(a, deg, precision, iter_counts=True, flags=gflags, **kw)
    nc = (st & pr.ST_NOT_CONVERGED) != 0
    ref_nc = (ref_st & oracle.ST_NOT_CONVERGED) != 0
    assert nc.sum() <= ref_nc.sum() + max(2, n // 20000)
    ok = ~nc & ~ref_nc
    floor = 1e-10 if deg is None else 1e-9
    sel = np.flatnonzero(ok)
    worst, flagged = _check_roots(got[:, sel], st[sel], a[:, sel], None if deg is None else deg[sel],
                                  ref[:, sel], ref_st[sel], floor=floor,
                                  flagged_ok=precision != "fp64")
    same = (it == it0).all(axis=0).mean()
    flagged0 = ((st0 & pr.ST_POLISH_UNCONVERGED) != 0).mean()
    print(f"\n{precision} {source} {rule}: worst rel err {worst:.3e}, flagged {flagged:.2e} "
          f"(lock-step {flagged0:.2e}), not converged {nc.sum()} (oracle {ref_nc.sum()}), "
          f"step counts as lock-step {same:.4f}")
    # FP32 sweeps leave a triple cluster to the polish, which flags it (its
    # roots are then checked by the clustered-class tests); elsewhere flags
    # are rare, and run-ahead flags no more than lock-step does
    assert flagged <= flagged0 + 1e-3
    if source != "clustered":
        assert flagged < 1e-3
    assert same > (0.98 if precision == "fp64" else 0.9)


@pytest.mark.parametrize("dmax", [4, 5])
def test_run_ahead_smaller_dmax(dmax):
    """Batches whose dmax is below 6: run-ahead trips from level 4 up only."""
    rng = np.random.default_rng(90 + dmax)
    n = 20000
    b = (rng.standard_normal((dmax + 1, n)) + 1j * rng.standard_normal((dmax + 1, n))) / np.sqrt(2)
    deg = rng.integers(2, dmax + 1, n).astype(np.int32)
    ref, ref_st = oracle.solve(b, deg, flags=OW)
    for precision in ("fp64", "fp32_polish"):
        for tile in (-1, 256):
            got, st = _solve(b, deg, precision, tile=tile, grid_blocks=0, flags=pr.FLAG_RUN_AHEAD)
            assert np.array_equal(st & 0x7, ref_st & 0x7)
            _check_roots(got, st, b, deg, ref, ref_st, floor=1e-9, flagged_ok=precision != "fp64")


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 4097])
def test_run_ahead_ragged_degrees_and_fixed_steps(n):
    """Run-ahead on ragged batches with every degree 0..dmax+1 (invalid
    ones flagged, rows beyond the degree NaN), in index order and in
    degree-sorted tiles (of 128, and of 100: slices that straddle several
    degrees and a partial last slice per tile), in both forms, and in
    fixed-step mode (exactly T steps per level, as without it)."""
    rng = np.random.default_rng(70 + n)
    b = (rng.standard_normal((7, n)) + 1j * rng.standard_normal((7, n))) / np.sqrt(2)
    deg = rng.integers(0, 8, n).astype(np.int32)
    deg[0] = 6
    ref, ref_st = oracle.solve(b, deg, flags=OW)
    for precision in ("fp64", "fp32_polish"):
        for tile in (-1, 128, 100):
            got, st = _solve(b, deg, precision, tile=tile, grid_blocks=0, flags=pr.FLAG_RUN_AHEAD)
            assert np.array_equal(st & 0x7, ref_st & 0x7)
            _check_roots(got, st, b, deg, ref, ref_st, floor=1e-9, flagged_ok=precision != "fp64")
    a = workloads.gaussian(n, seed=80 + n)
    T = 10
    for precision in ("fp64", "fp32_polish"):
        got, st, it = _solve(a, None, precision, flags=pr.FLAG_FIXED_STEPS | pr.FLAG_RUN_AHEAD,
                             max_iter_per_level=T, iter_counts=True)
        ref0, _, it0 = _solve(a, None, precision, flags=pr.FLAG_FIXED_STEPS,
                              max_iter_per_level=T, iter_counts=True)
        assert np.all(it == T) and np.all(it0 == T)
        assert np.all((st & pr.ST_NOT_CONVERGED) == 0)
        if precision == "fp64":
            # T steps need not converge a level, so the diagonal entries
            # read off at the end are only as close as the rounding of two
            # schedules of the same steps lets them be
            err = rel_err(match(got, ref0), ref0)
            assert (err <= 1e-6).mean() > 0.99


def test_tile_argument_validation():
    a = to_dev(workloads.gaussian(16, seed=0))
    d = to_dev(np.full(16, 6, dtype=np.int32))
    for bad in (dict(tile=-2), dict(tile=4097), dict(grid_blocks=-1)):
        with pytest.raises(pr.ProotsError):
            pr.solve(a, d, "fp64", **bad)


@pytest.mark.parametrize("precision", ["fp64", "fp32_polish"])
def test_fixed_steps_mode_matches_oracle_and_paper_counts(precision):
    """Alg. 2 literally: T steps per level, (n-1) T = 50 in all for n = 6,
    T = 10 (Table III); roots agree with the oracle's fixed-T mode."""
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_fixed_T.json")))
    T = g["T"]
    a = workloads.gaussian(8192, seed=12)
    ref, ref_st, ref_it = oracle.solve(a, fixed_t=T, return_iters=True)
    got, st, it = _solve(a, None, precision, flags=pr.FLAG_FIXED_STEPS, max_iter_per_level=T,
                         iter_counts=True)
    assert np.all(it == T) and np.all(it.sum(axis=0) == g["qr_steps_per_poly"])
    assert np.all((st & pr.ST_NOT_CONVERGED) == 0)
    # the converged roots (Alg. 1's shift, convergence test): a polynomial
    # whose T steps per level sufficed has its fixed-T roots within the
    # rounding floor of them
    conv, conv_st = oracle.solve(a)
    assert np.all(conv_st == 0)
    kappa = rel_condition(a, conv)
    settled = np.all(rel_err(match(ref, conv), conv) <= parity_bound(kappa), axis=0)
    assert settled.mean() > 0.9
    if precision == "fp64":
        err = rel_err(match(got, ref), ref)
        # on those, the GPU's fixed-T roots agree with the oracle's fixed-T
        # roots root by root; the others stopped mid-convergence, where the
        # two sides' rounding takes them apart
        assert np.all(err[:, settled] <= parity_bound(kappa[:, settled])), \
            err[:, settled].max()
        assert np.median(err) < 1e-14
        print(f"\nfixed T: {settled.mean():.4f} settled, max rel err {err[:, settled].max():.2e}")
    else:
        # the polish takes the fixed-T FP32 roots to the converged roots
        ok = (st & pr.ST_POLISH_UNCONVERGED) == 0
        err = rel_err(match(got[:, ok], conv[:, ok]), conv[:, ok])
        assert ok.mean() > 0.95
        assert np.all(err <= parity_bound(kappa[:, ok])), err.max()
        print(f"\nfixed T + polish: {ok.mean():.4f} unflagged, max rel err {err.max():.2e}")


def _scaled_lattice(e, n=512, seed=0):
    """n degree-6 polynomials whose roots are distinct dyadic lattice points
    times 2^e; the expanded coefficients are exact doubles."""
    rng = np.random.default_rng(seed)
    base = (rng.integers(-8, 9, (6, n)) + 1j * rng.integers(-8, 9, (6, n))) / 8.0
    base[:, :] += (np.arange(6)[:, None] - 2.5) * 3.0        # keep the six apart
    roots = base * 2.0 ** e
    a = np.zeros((7, n), dtype=np.complex128)
    a[0] = 1.0
    for k in range(6):                                        # multiply by (z - r_k)
        nxt = np.zeros_like(a)
        nxt[1:] = a[:-1]
        nxt -= a * roots[k][None, :]
        a = nxt
    return a, roots


@pytest.mark.parametrize("precision,exps", [("fp32_polish", (-60, -20, -12, 12, 20, 60)),
                                            ("fp64", (-150, -40, 40, 150))])
def test_roots_far_from_unit_scale(precision, exps):
    """Roots of modulus 2^e far outside the sweeps' comfortable range: the
    power-of-two change of variable solves them like any other (the roots
    come back exactly rescaled), where unscaled sweeps overflow or lose
    them.  Checked against the exact roots: the oracle solves the unscaled
    companion matrix, whose first row then spans 2^e .. 2^(6e), and loses
    accuracy with that imbalance (1.8e-11 at 2^9, no digits at 2^60)."""
    for e in exps:
        a, roots = _scaled_lattice(e, seed=e & 0xFF)
        for flags in (0, pr.FLAG_RUN_AHEAD):
            got, st = _solve(a, None, precision, flags=flags)
            assert np.all(st == 0), (e, flags, np.unique(st))
            err = rel_err(match(got, roots), roots)
            assert err.max() < 1e-12, (e, flags, err.max())
