"""The captured path replays bit-identically to eager launches (several
replays, eager work in between, and after new inputs are copied in)."""
from __future__ import annotations

import numpy as np
import pytest

import workloads
from gpuutil import to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pr = pytest.importorskip("paper_2507_02164_amd")


def _eager(c, d, prec, win, shape, cot):
    r, st = pr.solve(c, d, prec)
    h = pr.density(r, win, shape, d, st)
    g, st2 = pr.backward(c, r, cot, d, st.clone())
    torch.cuda.synchronize()
    return [to_host(x) for x in (r, st2, h, g)]


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("precision", ["fp32_polish", "fp64"])
@pytest.mark.parametrize("mixed", [False, True])
def test_graph_replay_matches_eager(precision, mixed, fused):
    from paper_2507_02164_amd.graph import PathGraph
    n = 50000
    if mixed:
        a, deg = workloads.mixed(n, seed=1)
        d = to_dev(deg)
    else:
        a = workloads.gaussian(n, seed=1)
        d = None
    win, shape = (-3.0, 3.0, -3.0, 3.0), (300, 200)
    c = to_dev(a)
    cot = to_dev(workloads.cotangents(n, seed=2))
    want = _eager(c, d, precision, win, shape, cot)
    g = PathGraph(c, d, precision, win, shape, cot, fused=fused)
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        got = [to_host(x) for x in (g.roots, g.status, g.hist, g.grad_coeffs)]
        for x, y in zip(got, want):
            assert np.array_equal(x, y, equal_nan=True), rep
        # the program's own eager work between replays
        z = torch.randn((512, 512), device=c.device)
        (z @ z).sum().item()
        pr.solve(c, d, precision)
        torch.cuda.synchronize()
    # a new batch of the same shape: copy it in and replay
    a2 = workloads.gaussian(n, seed=9) if not mixed else workloads.mixed(n, seed=9)[0]
    c.copy_(to_dev(a2))
    torch.cuda.synchronize()
    want2 = _eager(c, d, precision, win, shape, cot)
    g.replay()
    torch.cuda.synchronize()
    got2 = [to_host(x) for x in (g.roots, g.status, g.hist, g.grad_coeffs)]
    for x, y in zip(got2, want2):
        assert np.array_equal(x, y, equal_nan=True)
