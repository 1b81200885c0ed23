"""Helpers shared by the GPU parity tests (test side only)."""
from __future__ import annotations

import numpy as np

U64 = 2.0 ** -53


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev())


def to_host(t):
    return t.detach().cpu().numpy()


def rel_condition(coeffs, roots, degrees=None):
    """Relative condition number of each root of p(z) = sum_k a_k z^k
    under relative perturbations of the coefficients:
    kappa_j = sum_k |a_k| |r_j|^k / (|r_j| |p'(r_j)|), [dmax, n]."""
    dmax1, n = coeffs.shape
    dmax = dmax1 - 1
    deg = np.full(n, dmax) if degrees is None else np.asarray(degrees)
    kk = np.arange(dmax1)[:, None]
    a = np.where(kk <= deg[None, :], coeffs, 0)
    out = np.full(roots.shape, np.inf)
    for j in range(dmax):
        r = roots[j]
        pw = [np.ones(n, dtype=np.complex128)]
        for k in range(dmax):
            pw.append(pw[-1] * r)
        num = sum(np.abs(a[k]) * np.abs(pw[k]) for k in range(dmax1))
        dp = sum(k * a[k] * pw[k - 1] for k in range(1, dmax1))
        with np.errstate(divide="ignore", invalid="ignore"):
            out[j] = num / (np.abs(r) * np.abs(dp))
    return out


def parity_bound(kappa, floor=1e-10, c=1e3):
    """Relative tolerance for a root computed twice in FP64 with different
    rounding: max(floor, c * kappa * u).  Well-conditioned roots get the
    floor; for the rest the FP64 rounding floor itself scales with kappa."""
    return np.maximum(floor, c * kappa * U64)


def deriv_condition(coeffs, roots, degrees=None):
    """Condition number of evaluating p'(r_j) by any backward-stable sum:
    sum_{k>=1} k |a_k| |r_j|^(k-1) / |p'(r_j)|, [dmax, n].  Two evaluations
    with different rounding differ by up to about this times u relative, and
    so do the adjoint terms -r^k / p'(r) built on them."""
    dmax1, n = coeffs.shape
    dmax = dmax1 - 1
    deg = np.full(n, dmax) if degrees is None else np.asarray(degrees)
    kk = np.arange(dmax1)[:, None]
    a = np.where(kk <= deg[None, :], coeffs, 0)
    out = np.full(roots.shape, np.inf)
    for j in range(dmax):
        r = roots[j]
        pw = [np.ones(n, dtype=np.complex128)]
        for k in range(dmax):
            pw.append(pw[-1] * r)
        num = sum(k * np.abs(a[k]) * np.abs(pw[k - 1]) for k in range(1, dmax1))
        dp = sum(k * a[k] * pw[k - 1] for k in range(1, dmax1))
        with np.errstate(divide="ignore", invalid="ignore"):
            out[j] = num / np.abs(dp)
    return out
