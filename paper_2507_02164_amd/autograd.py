"""torch.autograd.Function over pr_solve / pr_backward."""
from __future__ import annotations

import torch

from . import _capi


class RootsFn(torch.autograd.Function):
    """roots, status = RootsFn.apply(coeffs, degrees, precision)

    Forward: pr_solve.  Backward: pr_backward, the implicit-function adjoint
    dr/da_k = -r^k / p'(r) in PyTorch's complex convention (the cotangent of
    a holomorphic map is conj(derivative) times the output cotangent).
    Rows of ``roots`` beyond a polynomial's degree are NaN and receive no
    gradient."""

    @staticmethod
    def forward(ctx, coeffs, degrees=None, precision="fp64"):
        roots, status = _capi.solve(coeffs, degrees, precision)
        ctx.save_for_backward(coeffs, roots, status, degrees)
        ctx.mark_non_differentiable(status)
        return roots, status

    @staticmethod
    def backward(ctx, grad_roots, grad_status):
        coeffs, roots, status, degrees = ctx.saved_tensors
        if grad_roots is None:
            return None, None, None
        g = grad_roots.contiguous()
        if g.dtype != torch.complex128:
            g = g.to(torch.complex128)
        grad, _ = _capi.backward(coeffs, roots, g, degrees, status.clone())
        return grad, None, None


def roots(coeffs, degrees=None, precision="fp64"):
    """Differentiable roots (status is dropped; use RootsFn.apply for it)."""
    return RootsFn.apply(coeffs, degrees, precision)[0]
