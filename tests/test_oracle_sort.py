"""Pins of the oracle sort (Alg. 1): exact rational brute force, hand cases, invariants."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import greedy_sort, sq_distance


def exact_sq_distance(pi, pj):
    """Sum of squares of the FP64-rounded differences, exactly in rationals, rounded once."""
    d = np.asarray(pi, dtype=np.float64) - np.asarray(pj, dtype=np.float64)
    return float(sum(Fraction(float(t)) ** 2 for t in d))


def brute_greedy(P, start=0):
    N = len(P)
    D = [[exact_sq_distance(P[i], P[j]) for j in range(N)] for i in range(N)]
    order = [start]
    left = sorted(set(range(N)) - {start})
    while left:
        cur = order[-1]
        best = min(D[cur][j] for j in left)
        nxt = min(j for j in left if D[cur][j] == best)
        order.append(nxt)
        left.remove(nxt)
    return order


def test_sq_distance_is_exact():
    rng = np.random.default_rng(1)
    for trial in range(60):
        p = rng.integers(1, 40)
        scale = 10.0 ** rng.integers(-5, 6, size=p)
        a = rng.standard_normal(p) * scale
        b = a + rng.standard_normal(p) * scale * 10.0 ** rng.integers(-12, 1)
        assert sq_distance(a, b) == exact_sq_distance(a, b)


@pytest.mark.parametrize("seed", range(12))
def test_greedy_matches_exact_bruteforce(seed):
    rng = np.random.default_rng(100 + seed)
    N = int(rng.integers(1, 9))
    p = int(rng.integers(1, 17))
    P = rng.standard_normal((N, p)) * np.exp(rng.standard_normal((1, p)))
    if seed % 3 == 0 and N > 2:       # plant exact duplicates: ties must go to the lowest index
        P[N - 1] = P[1]
    start = int(rng.integers(0, N))
    order = greedy_sort(P, start=start)
    assert list(order) == brute_greedy(P, start)


def test_hand_cases_one_dimensional():
    pts = np.array([[0.0], [5.0], [1.0], [3.0], [10.0]])
    assert list(greedy_sort(pts)) == [0, 2, 3, 1, 4]
    # exact tie from the start: both neighbours at distance 1, lowest index wins
    assert list(greedy_sort(np.array([[0.0], [1.0], [-1.0]]))) == [0, 1, 2]
    # every distance far above 1000: the running minimum must start at +infinity
    assert list(greedy_sort(np.array([[0.0], [5000.0], [3000.0]]))) == [0, 2, 1]


def test_invariants_and_step_distances():
    rng = np.random.default_rng(7)
    P = rng.standard_normal((9, 5))
    order, d = greedy_sort(P, return_dist=True)
    assert order[0] == 0 and sorted(order) == list(range(9)) and order.dtype == np.int64
    assert d[0] == 0.0
    for t in range(1, 9):
        cur = order[t - 1]
        left = [j for j in range(9) if j not in order[:t]]
        assert d[t] == min(exact_sq_distance(P[cur], P[j]) for j in left)


def test_degenerate_sizes():
    assert list(greedy_sort(np.zeros((0, 3)))) == []
    assert list(greedy_sort(np.zeros((1, 3)))) == [0]
    assert list(greedy_sort(np.zeros((4, 2)))) == [0, 1, 2, 3]     # all tied
    with pytest.raises(ValueError):
        greedy_sort(np.zeros((2, 2)), start=2)
