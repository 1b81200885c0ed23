"""Root-set comparison helpers for tests.

The order in which roots come out is not part of the result, so two root
sets are compared after the optimal assignment: per polynomial, the
permutation of the tested roots that minimises the sum of squared distances
to the reference roots, found by brute force over all d! <= 720 orderings
(ties go to the lexicographically first permutation).
"""
from __future__ import annotations

import itertools

import numpy as np

_PERMS = {d: np.array(list(itertools.permutations(range(d))), dtype=np.int64) for d in range(1, 7)}


def match(test: np.ndarray, ref: np.ndarray, chunk: int = 2048) -> np.ndarray:
    """Reorder each column of ``test`` ([d, n]) to best match ``ref``."""
    test = np.asarray(test)
    ref = np.asarray(ref)
    d, n = ref.shape
    assert test.shape == (d, n)
    if d == 1:
        return test.copy()
    P = _PERMS[d]
    out = np.empty_like(test)
    cols = np.arange(d)[None, :]
    for s in range(0, n, chunk):
        t = test[:, s:s + chunk]
        r = ref[:, s:s + chunk]
        cost = np.abs(t[:, None, :] - r[None, :, :]) ** 2          # [i_test, j_ref, c]
        cost = np.where(np.isnan(cost), np.inf, cost)
        tot = cost[P, cols, :].sum(axis=1)                          # [perm, c]
        best = np.argmin(tot, axis=0)
        idx = P[best].T                                             # [d, c]
        out[:, s:s + chunk] = np.take_along_axis(t, idx, axis=0)
    return out


def match_mixed(test, ref, degrees):
    """As ``match`` for mixed degrees: only rows k < degree are compared;
    rows beyond keep their values."""
    out = np.array(test, copy=True)
    degrees = np.asarray(degrees)
    for d in np.unique(degrees):
        d = int(d)
        if d < 1 or d > ref.shape[0]:
            continue
        cols = np.nonzero(degrees == d)[0]
        out[:d, cols] = match(test[:d, cols], ref[:d, cols])
    return out


def rel_err(test, ref, floor: float = 0.0):
    """|test - ref| / max(|ref|, floor), elementwise."""
    den = np.maximum(np.abs(ref), floor)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.abs(test - ref) / den


def valid_mask(dmax: int, degrees, n: int):
    """[dmax, n] bool: row k < degree of column."""
    if degrees is None:
        return np.ones((dmax, n), dtype=bool)
    return np.arange(dmax)[:, None] < np.asarray(degrees)[None, :]


def match_nearest(test, ref, chunk: int = 1 << 19):
    """Like ``match`` for large batches.  Per polynomial, each reference
    root is paired with its nearest tested root; where these pairings form a
    permutation, that permutation is used (each root's distance is then the
    smallest any pairing could give it, so a bound that holds for all of
    them proves the two sets agree root by root); the other polynomials go
    through the brute-force ``match``.  Returns (reordered test, number of
    polynomials that needed the brute force)."""
    test = np.asarray(test)
    ref = np.asarray(ref)
    d, n = ref.shape
    assert test.shape == (d, n)
    if d == 1:
        return test.copy(), 0
    out = np.empty_like(test)
    full = (1 << d) - 1
    fallback = 0
    for s in range(0, n, chunk):
        t = test[:, s:s + chunk]
        r = ref[:, s:s + chunk]
        dist = np.abs(t[:, None, :] - r[None, :, :])               # [i_test, j_ref, c]
        dist = np.where(np.isnan(dist), np.inf, dist)
        near = np.argmin(dist, axis=0)                              # [j_ref, c]
        mask = np.bitwise_or.reduce(np.left_shift(1, near), axis=0)
        perm = mask == full
        out[:, s:s + chunk] = np.take_along_axis(t, near, axis=0)
        bad = np.nonzero(~perm)[0]
        if bad.size:
            fallback += bad.size
            out[:, s + bad] = match(t[:, bad], r[:, bad])
    return out, fallback


def match_mixed_nearest(test, ref, degrees):
    """``match_nearest`` for mixed degrees (rows k < degree compared; rows
    beyond keep their values).  Returns (reordered test, fallback count)."""
    out = np.array(test, copy=True)
    degrees = np.asarray(degrees)
    fallback = 0
    for d in np.unique(degrees):
        d = int(d)
        if d < 1 or d > ref.shape[0]:
            continue
        cols = np.nonzero(degrees == d)[0]
        m, fb = match_nearest(test[:d, cols], ref[:d, cols])
        out[:d, cols] = m
        fallback += fb
    return out, fallback
