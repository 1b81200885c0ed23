"""The whole path -- solve, density image, backward -- captured once into a
HIP graph and replayed.

Every launch the library makes is a plain kernel launch on the caller's
stream (no memset nodes: the image is cleared by a fill kernel), so the
calls capture into one graph whose replay re-runs them on whatever the
captured buffers hold.  With ``fused`` (the default) solve and density are
one launch (pr_solve_bin); otherwise two.  To solve a new batch of the same
shape, copy it into ``coeffs`` (and ``degrees`` / ``cotangents``) and replay.
"""
from __future__ import annotations

import torch

from . import _capi


class PathGraph:
    def __init__(self, coeffs, degrees=None, precision="fp32_polish", window=None, shape=None,
                 cotangents=None, skip_mask=0, fused=True, **solve_opts):
        self.coeffs = coeffs
        self.degrees = degrees
        self.precision = precision
        self.window = window
        self.shape = shape
        self.cotangents = cotangents
        self.skip_mask = skip_mask
        self.fused = fused
        self.solve_opts = solve_opts
        dmax = coeffs.shape[0] - 1
        n = coeffs.shape[1]
        dev = coeffs.device
        self.roots = torch.empty((dmax, n), dtype=torch.complex128, device=dev)
        self.status = torch.empty((n,), dtype=torch.int32, device=dev)
        self.hist = None
        if window is not None:
            self.hist = torch.zeros((shape[1], shape[0]), dtype=torch.int32, device=dev)
        self.grad_coeffs = torch.empty_like(coeffs) if cotangents is not None else None
        self.graph = torch.cuda.CUDAGraph()
        # one eager pass on a side stream first (lazy initialisation happens
        # outside the capture), then the capture itself
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            self._step()
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize(dev)
        with torch.cuda.graph(self.graph):
            self._step()

    def _step(self):
        if self.hist is not None and self.fused:
            self.hist.zero_()
            _capi.solve_bin(self.coeffs, self.window, self.shape, self.degrees, self.precision,
                            skip_mask=self.skip_mask, out=self.hist, roots=self.roots,
                            status=self.status, **self.solve_opts)
        else:
            _capi.solve(self.coeffs, self.degrees, self.precision, roots=self.roots,
                        status=self.status, **self.solve_opts)
        if self.hist is not None and not self.fused:
            self.hist.zero_()
            _capi.density(self.roots, self.window, self.shape, self.degrees, self.status,
                          self.skip_mask, out=self.hist)
        if self.grad_coeffs is not None:
            _capi.backward(self.coeffs, self.roots, self.cotangents, self.degrees, self.status,
                           grad_coeffs=self.grad_coeffs)

    def replay(self):
        self.graph.replay()
        return self.roots, self.status, self.hist, self.grad_coeffs
