"""Pins of the oracle's Equation (8) upper bound (Lemma 4 with p_max = 1):
the smallest, over the greedy prefixes S_i* (i = 0..k), of the prefix's
coverage plus the k largest marginal coverages given the prefix.

* It bounds the optimum: brute force over all C(n, k) seed sets never covers
  more than it (Lemma 4 follows from submodularity of coverage).
* It is no looser than Lemma 5's closed form Lambda(S_k*) / (1 - (1-1/k)^k).
* It is never below greedy's own coverage, and equals the optimum where the
  optimum is known exactly: k = 1 (the best single vertex), and pools that
  greedy covers completely.
* The HyperIM_BRR loop with it stops no later than with the closed form and
  returns a spread lower bound that still holds (the estimate of its seeds
  on the independent pool R2 stays above sigma_l on the tiny workload).
"""
import itertools

import numpy as np
import pytest

import hypergen
import oracle
from test_oracle_greedy import _cov, _random_pool


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("k", [1, 2, 3])
def test_eq8_bounds_the_optimum_and_the_closed_form(seed, k):
    n, theta = 9, 40
    sets, off, mem = _random_pool(300 + seed, n, theta, 4)
    seeds, gains = oracle.greedy(n, off, mem, k)
    ub = oracle.upper_eq8(n, off, mem, seeds)
    opt = max(_cov(sets, S) for S in itertools.combinations(range(n), k))
    lam = int(gains.sum())
    assert opt <= ub
    assert lam <= ub
    assert ub <= lam / (1 - (1 - 1 / k) ** k) + 1e-9
    if k == 1:
        assert ub == opt == lam


def test_eq8_exact_when_greedy_covers_everything():
    # four disjoint pairs of sets, each pair hit by one vertex: k = 4 covers all
    sets = [[0, 5], [0, 6], [1, 5], [1, 7], [2, 8], [2, 6], [3, 7], [3, 8]]
    off = np.zeros(len(sets) + 1, np.uint64)
    off[1:] = np.cumsum([len(s) for s in sets])
    mem = np.array([u for s in sets for u in s], np.uint32)
    seeds, gains = oracle.greedy(9, off, mem, 4)
    assert int(gains.sum()) == len(sets)
    assert oracle.upper_eq8(9, off, mem, seeds) == len(sets)


@pytest.mark.parametrize("seed", range(6))
def test_eq8_on_larger_random_pools(seed):
    n, theta, k = 60, 400, 8
    sets, off, mem = _random_pool(700 + seed, n, theta, 7)
    seeds, gains = oracle.greedy(n, off, mem, k)
    ub = oracle.upper_eq8(n, off, mem, seeds)
    lam = int(gains.sum())
    assert lam <= ub <= lam / (1 - (1 - 1 / k) ** k) + 1e-9
    # the i = 0 term alone: the k largest single-vertex coverages
    cnt = np.bincount(mem, minlength=n)
    assert ub <= int(np.sort(cnt)[::-1][:k].sum())


def test_brr_loop_with_eq8_stops_no_later_and_stays_valid():
    w = hypergen.workload("tiny")
    o = oracle.Graph(w.build(), w.model, w.p)
    o.stratify()
    a = o.select_seeds(w.k, w.eps, w.ell, bound=0)
    b = o.select_seeds(w.k, w.eps, w.ell, bound=1)
    assert a["rounds"] <= b["rounds"]
    assert a["sigma_l"] <= a["spread"]
    assert a["lambda_u"] >= a["lambda1"]
    if a["rounds"] == b["rounds"]:
        assert a["sigma_u"] <= b["sigma_u"] + 1e-9
