"""Greedy nearest-neighbour ordering of the systems (Alg. 1, Sec. 4.1).

Oracle (test infrastructure only).

What Alg. 1 computes: the order begins with a chosen first system; after that, each position is
filled by the system, among those not placed yet, whose parameter matrix lies nearest in the
Frobenius norm to the parameter matrix of the system placed just before it.

Readings taken where the paper is loose:
* The paper seeds its running minimum with a finite constant; here nothing is compared against a
  constant, so the choice is defined even when every distance is large.
* Ties go to the lowest original index. NaN distances never win; when no candidate has a finite
  distance, the lowest unplaced index is taken.
* Squared distances are compared (the square root is monotone). The squared distance is defined
  as the exact sum, over all entries, of the squares of the FP64 differences fl(a_i[p] - a_j[p]),
  rounded once to FP64. Each square is split exactly into two doubles (Dekker's product with
  Veltkamp splitting) and ``math.fsum`` returns the correctly rounded sum, so the value does not
  depend on any summation order.
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


def _nearest_unplaced(row: list, placed: np.ndarray) -> int:
    """Index of the smallest entry of ``row`` among the unplaced indices (lowest index on ties,
    NaN never chosen; the lowest unplaced index when none is finite or below +inf)."""
    best_i, best_d = -1, math.inf
    for i, d in enumerate(row):
        if placed[i]:
            continue
        if best_i < 0 and not (d < math.inf):
            continue
        if best_i < 0 or d < best_d:
            best_i, best_d = i, d
    if best_i < 0:
        best_i = int(np.flatnonzero(~placed)[0])
    return best_i


def greedy_sort(params: np.ndarray, start: int = 0, return_dist: bool = False):
    """Greedy nearest-neighbour order (Alg. 1) of an (N, p) array of flattened parameter matrices.

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
    placed = np.zeros(N, dtype=bool)
    placed[start] = True
    order = np.empty(N, dtype=np.int64)
    step_d2 = np.zeros(N)
    order[0] = start
    for t in range(1, N):
        prev = int(order[t - 1])
        # distances from the system placed last to every system (placed ones are skipped)
        row = [math.nan if placed[i] else sq_distance(params[prev], params[i]) for i in range(N)]
        nxt = _nearest_unplaced(row, placed)
        placed[nxt] = True
        order[t] = nxt
        step_d2[t] = row[nxt]
    return (order, step_d2) if return_dist else order
