"""Greedy nearest-neighbour sort of the systems (Alg. 1, "The Sorting Algorithm", Sec. 4.1).

Oracle (test infrastructure only).

Alg. 1 starts at the first system, then repeatedly appends the not-yet-visited system whose
parameter matrix is closest, in Frobenius norm, to that of the system appended last.

Readings taken where the paper is loose:
* The running minimum starts at +infinity (the paper's "a large number, e.g. 1000" would leave
  the choice undefined once every distance exceeds 1000).
* Candidates are scanned in ascending original index with a strict "<", so ties go to the
  lowest index. If no candidate has a finite distance, the lowest remaining index is taken.
* The comparison uses the squared distance (the square root is monotone, so the order is the
  same). The squared distance is defined as the exact sum over all entries of the squares of the
  FP64 differences fl(a_i[p] - a_j[p]), rounded once to FP64. Each square is split exactly into
  two doubles (Dekker's product with Veltkamp splitting) and ``math.fsum`` returns the correctly
  rounded sum, so the value does not depend on any summation order.
"""
from __future__ import annotations

import math

import numpy as np

_SPLIT = 134217729.0  # 2**27 + 1, Veltkamp splitting constant for FP64


def _exact_squares(d: np.ndarray):
    """Return (hi, lo) with hi + lo == d*d exactly (Dekker's product; no overflow assumed)."""
    hi = d * d
    c = _SPLIT * d
    dh = c - (c - d)
    dl = d - dh
    lo = ((dh * dh - hi) + 2.0 * (dh * dl)) + dl * dl
    return hi, lo


def sq_distance(pi: np.ndarray, pj: np.ndarray) -> float:
    """Squared Frobenius distance between two parameter matrices, correctly rounded (see module doc)."""
    d = np.asarray(pi, dtype=np.float64).ravel() - np.asarray(pj, dtype=np.float64).ravel()
    if not np.all(np.isfinite(d)):
        return math.inf if not np.any(np.isnan(d)) else math.nan
    hi, lo = _exact_squares(d)
    return math.fsum(np.concatenate([hi, lo]).tolist())


def greedy_sort(params: np.ndarray, start: int = 0, return_dist: bool = False):
    """Alg. 1 on an (N, p) array of flattened parameter matrices.

    Returns the visiting order (int64 array, first element ``start``) and, with ``return_dist``,
    the squared distance of every step (entry 0 is 0.0).
    """
    params = np.asarray(params, dtype=np.float64)
    N = params.shape[0]
    if N == 0:
        order = np.zeros(0, dtype=np.int64)
        return (order, np.zeros(0)) if return_dist else order
    if not 0 <= start < N:
        raise ValueError("start out of range")
    remaining = [j for j in range(N) if j != start]      # seq_0 with the start removed
    order = [start]                                       # seq_mat
    dists = [0.0]
    cur = start
    for _ in range(N - 1):
        best = math.inf
        jmin = None
        for j in remaining:
            dj = sq_distance(params[cur], params[j])
            if dj < best:
                best, jmin = dj, j
        if jmin is None:
            jmin = remaining[0]
            best = sq_distance(params[cur], params[jmin])
        remaining.remove(jmin)
        order.append(jmin)
        dists.append(best)
        cur = jmin
    order = np.asarray(order, dtype=np.int64)
    return (order, np.asarray(dists)) if return_dist else order
