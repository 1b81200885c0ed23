"""GPU test of pr_density_sorted_noalloc, the allocation-free variant of
pr_density_sorted for callers that cannot allocate: called through the C
ABI twice in a row -- the second time with a smaller batch, another window
and image -- each result checked against pr_density_sorted with a
caller-supplied workspace (the same image bit for bit, as integer counts
must be), and a batch beyond the static scratch array refused.
"""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import workloads
from gpuutil import to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pr = pytest.importorskip("paper_2507_02164_amd")


def _spread_roots(n, seed):
    """Root arrays of the shape the solver returns: [6, n] complex128 with a
    Gaussian spread (the distribution of random polynomials' roots)."""
    rng = np.random.default_rng(seed)
    r = (rng.standard_normal((6, n)) + 1j * rng.standard_normal((6, n))) * 0.9
    r[:, ::97] = np.nan                 # a few polynomials without roots
    return r


def _noalloc(roots, win, shape, status=None, skip=0):
    """pr_density_sorted_noalloc straight through the C ABI."""
    dmax, n = roots.shape
    width, height = shape
    out = torch.zeros((height, width), dtype=torch.int32, device=roots.device)
    rc = pr.lib().pr_density_sorted_noalloc(
        ctypes.c_void_p(roots.data_ptr()), None,
        None if status is None else ctypes.c_void_p(status.data_ptr()), skip, n, dmax,
        *(float(v) for v in win), width, height, ctypes.c_void_p(out.data_ptr()),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, out


def test_two_calls_in_a_row_match_the_workspace_path():
    cases = [(600_000, 11, workloads.GAUSSIAN_WINDOW, (1920, 1080)),
             (70_000, 12, (-2.0, 2.5, -1.5, 1.0), (640, 480))]
    for n, seed, win, shape in cases:
        need = pr.density_sorted_workspace(n, 6, *shape)
        assert 0 < need <= pr.NOALLOC_SCRATCH_BYTES
        r = to_dev(_spread_roots(n, seed))
        st = torch.from_numpy((np.arange(n) % 5 == 0).astype(np.int32) << 3).to(r.device)
        rc, got = _noalloc(r, win, shape, st, 0x8)
        assert rc == pr.PR_OK
        want = pr.density_sorted(r, win, shape, status=st, skip_mask=0x8)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (n, int((got != want).sum()))
        assert int(got.sum()) > 0


def test_refuses_a_batch_beyond_the_scratch_array():
    n = 4 * 2 ** 20
    assert pr.density_sorted_workspace(n, 6, 1920, 1080) > pr.NOALLOC_SCRATCH_BYTES
    r = torch.zeros((6, n), dtype=torch.complex128, device="cuda")
    rc, out = _noalloc(r, workloads.GAUSSIAN_WINDOW, (1920, 1080))
    assert rc == pr.PR_ERR_NO_MEMORY
    torch.cuda.synchronize()
    assert int(out.sum()) == 0
