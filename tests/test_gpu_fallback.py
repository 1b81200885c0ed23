"""GPU tests of PR_FLAG_FP64_FALLBACK: FP32 + polish results flagged
NOT_CONVERGED or POLISH_UNCONVERGED are replaced by the FP64 form's, exactly
(bit for bit, with PR_ST_RESOLVED_FP64 added); everything else is left as the
FP32 form computed it.  With binning, the image is the one pr_density makes
from the final roots and status."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from gpuutil import to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pr = pytest.importorskip("paper_2507_02164_amd")

FB = pr.ST_NOT_CONVERGED | pr.ST_POLISH_UNCONVERGED


def _bits(t):
    return to_host(torch.view_as_real(t).contiguous().view(torch.int64))


def _case(name):
    if name == "clustered":            # nearly every FP32 result flagged
        a, _ = workloads.clustered(65536, seed=5)
        return a, None, workloads.CLUSTERED_WINDOW, (1920, 1080)
    if name == "known":                # a few in ten thousand flagged
        a = workloads.known_roots(200_000, seed=5)[0]
        return a, None, (-2.5, 2.5, -2.5, 2.5), (800, 800)
    if name == "mixed":                # degrees: the fallback's own degree sort
        a, deg = workloads.mixed(200_000, seed=5)
        a = a.copy()
        # a few polynomials with a double root: FP32 + polish flags them
        k = np.arange(0, 200_000, 997)
        deg[k] = 4
        a[:, k] = 0.0
        a[0, k], a[1, k], a[2, k], a[3, k], a[4, k] = 1.0, -4.0, 6.0, -4.0, 1.0   # (z - 1)^4
        return a, deg, (-10.0, 10.0, -10.0, 10.0), (640, 480)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["clustered", "known", "mixed"])
def test_fallback_replaces_exactly_the_flagged(name):
    a, deg, win, shape = _case(name)
    ad = to_dev(np.ascontiguousarray(a))
    dd = None if deg is None else to_dev(deg)
    kw = dict(max_iter_per_level=30)
    r0, s0 = pr.solve(ad, dd, "fp32_polish", **kw)
    # the fallback's second launch steps its lanes in lock-step, as the
    # index-order FP64 launch does (any run-ahead the tuner picks for the
    # first launch does not carry over)
    r64, s64, it64 = pr.solve(ad, dd, "fp64", iter_counts=True, tile=-1, grid_blocks=0, **kw)
    rf, sf, itf = pr.solve(ad, dd, "fp32_polish", flags=pr.FLAG_FP64_FALLBACK, iter_counts=True,
                           **kw)
    torch.cuda.synchronize()
    s0, s64, sf = (to_host(x).astype(np.uint32) for x in (s0, s64, sf))
    flagged = (s0 & FB) != 0
    assert flagged.any()
    b0, b64, bf = _bits(r0), _bits(r64), _bits(rf)
    assert np.array_equal(bf[:, ~flagged], b0[:, ~flagged])
    assert np.array_equal(sf[~flagged], s0[~flagged])
    assert np.array_equal(bf[:, flagged], b64[:, flagged])
    assert np.array_equal(sf[flagged], s64[flagged] | pr.ST_RESOLVED_FP64)
    assert np.array_equal(to_host(itf)[:, flagged], to_host(it64)[:, flagged])
    # what is left flagged after the fallback is what FP64 itself flags
    assert ((sf & FB) != 0).sum() == ((s64[flagged] & FB) != 0).sum()


@pytest.mark.parametrize("name", ["clustered", "mixed"])
def test_fallback_after_a_run_ahead_launch(name):
    """The first launch with lanes running ahead, the fallback in lock-step:
    unflagged results are the run-ahead launch's, flagged ones the
    lock-step FP64 solve's, bit for bit."""
    a, deg, _, _ = _case(name)
    ad = to_dev(np.ascontiguousarray(a))
    dd = None if deg is None else to_dev(deg)
    lay = dict(max_iter_per_level=30, tile=-1 if deg is None else 512, grid_blocks=0)
    r0, s0 = pr.solve(ad, dd, "fp32_polish", flags=pr.FLAG_RUN_AHEAD, **lay)
    r64, s64 = pr.solve(ad, dd, "fp64", max_iter_per_level=30, tile=-1, grid_blocks=0)
    rf, sf = pr.solve(ad, dd, "fp32_polish", flags=pr.FLAG_RUN_AHEAD | pr.FLAG_FP64_FALLBACK, **lay)
    torch.cuda.synchronize()
    s0, s64, sf = (to_host(x).astype(np.uint32) for x in (s0, s64, sf))
    flagged = (s0 & FB) != 0
    assert flagged.any()
    b0, b64, bf = _bits(r0), _bits(r64), _bits(rf)
    assert np.array_equal(bf[:, ~flagged], b0[:, ~flagged])
    assert np.array_equal(bf[:, flagged], b64[:, flagged])
    assert np.array_equal(sf[flagged], s64[flagged] | pr.ST_RESOLVED_FP64)


@pytest.mark.parametrize("store", [True, False])
@pytest.mark.parametrize("name", ["clustered", "known", "mixed"])
def test_fallback_with_binning(name, store):
    a, deg, win, shape = _case(name)
    ad = to_dev(np.ascontiguousarray(a))
    dd = None if deg is None else to_dev(deg)
    kw = dict(max_iter_per_level=30, flags=pr.FLAG_FP64_FALLBACK)
    rf, sf = pr.solve(ad, dd, "fp32_polish", **kw)
    for skip in (0, FB, pr.ST_RESOLVED_FP64):
        want = pr.density(rf, win, shape, dd, sf, skip)
        r2, s2, h2 = pr.solve_bin(ad, win, shape, dd, "fp32_polish", skip_mask=skip,
                                  store_roots=store, **kw)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(s2), to_host(sf))
        if store:
            assert np.array_equal(_bits(r2), _bits(rf))
        img = to_host(h2)
        assert np.array_equal(img, to_host(want))
        assert np.array_equal(img, oracle.density(to_host(rf), win, shape, deg,
                                                  to_host(sf).astype(np.uint32), skip))


def test_fallback_flag_is_a_no_op_for_fp64():
    a = workloads.gaussian(20000, seed=3)
    ad = to_dev(a)
    r1, s1 = pr.solve(ad, None, "fp64")
    r2, s2 = pr.solve(ad, None, "fp64", flags=pr.FLAG_FP64_FALLBACK)
    torch.cuda.synchronize()
    assert np.array_equal(_bits(r1), _bits(r2)) and np.array_equal(to_host(s1), to_host(s2))
