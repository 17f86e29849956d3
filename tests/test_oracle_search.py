"""Pins for the oracle of Alg. 1 (first collision-free motion).

Hand-worked cases follow the algorithm's two loops by hand; the randomised check
compares the loop-by-loop oracle with a closed characterisation of its answer (the
free motion that is least in the lexicographic order (loop, rank), computed with
numpy's lexsort), including tied and NaN proxy values.
"""
import math

import numpy as np
import pytest

from oracle import search


def test_second_loop_hand_case():
    # first loop: m1 (d_hat 0.02) and m2 (0.05) are checked and collide; the second loop
    # visits m0 (0.001) before m3 (0.0) and m0 is free
    d_hat = [0.001, 0.02, 0.05, 0.0]
    d = [0.1, -0.1, 0.003, 0.2]
    assert search.first_free(d, 0.01, d_hat) == (0, 3, 4, 2)
    assert search.visiting_order(d_hat, 0.01) == [1, 2, 0, 3]


def test_first_loop_hand_case():
    # m1 is the first motion with d_hat > eps and it is free: one exact check, two proxies
    assert search.first_free([0.5, 0.02, 0.5], 0.01, [0.0, 0.5, 0.3]) == (1, 1, 2, 2)


def test_plain_search_and_none_free():
    assert search.first_free([-1.0, 0.005, 0.3], 0.01) == (2, 3, 0, 0)
    assert search.first_free([-1.0, 0.01, 0.0], 0.01) == (-1, 3, 0, 0)           # d = eps is not free
    assert search.first_free([-1.0, 0.01, 0.0], 0.01, [0.2, 0.0, -0.3]) == (-1, 3, 3, 1)


def test_ties_keep_given_order_and_nan_last():
    d_hat = [0.0, float("nan"), 0.0, -0.5, 0.0]
    assert search.visiting_order(d_hat, 0.01) == [0, 2, 4, 3, 1]
    assert search.first_free([-1, 1, -1, -1, 1], 0.01, d_hat) == (4, 3, 5, 0)


@pytest.mark.parametrize("seed", range(20))
def test_answer_matches_lexicographic_characterisation(seed):
    g = np.random.default_rng(seed)
    M = int(g.integers(1, 60))
    eps = 0.01
    d = g.choice([-0.05, 0.0, 0.005, 0.01, 0.02, 0.3], size=M, p=[0.35, 0.1, 0.1, 0.05, 0.1, 0.3])
    d_hat = g.choice([-0.1, 0.0, 0.01, 0.015, 0.2, np.nan], size=M)                  # many ties
    got = search.first_free(list(d), eps, list(d_hat))
    key = np.where(np.isnan(d_hat), -np.inf, d_hat)
    loop = np.where(key > eps, 0, 1)
    rank = np.where(loop == 0, np.arange(M), -key)      # loop 1: given order; loop 2: d_hat descending
    order = np.lexsort((np.arange(M), rank, loop))       # last key is primary
    free = [m for m in order if d[m] > eps]
    n_first = int(np.sum(loop == 0))
    if free:
        ans = free[0]
        pos = int(np.where(order == ans)[0][0])
        n_nn = ans + 1 if loop[ans] == 0 else M
        assert got == (ans, pos + 1, n_nn, n_first)
    else:
        assert got == (-1, M, M, n_first)
    assert search.visiting_order(list(d_hat), eps) == [int(m) for m in order]
