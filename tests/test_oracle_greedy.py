"""Pins of the oracle's greedy max coverage (Algorithm 1, Equations (1)-(2)).

* Every chosen seed maximises the marginal coverage of Equation (2),
  recomputed from scratch with Python sets, ties broken toward the smallest id.
* Brute force over all C(n,k) seed sets: greedy's coverage is at least
  (1 - (1 - 1/k)^k) of the optimum (the classical max-coverage guarantee).
* Special cases: k = 1 picks the most frequent vertex; once every set is
  covered the remaining seeds are the smallest unchosen ids.
"""
import itertools

import numpy as np
import pytest

import oracle


def _random_pool(seed, n, theta, max_size):
    rng = np.random.default_rng(seed)
    sets = []
    for _ in range(theta):
        s = int(rng.integers(1, max_size + 1))
        # skewed membership so coverage differs a lot between vertices
        w = 1.0 / np.arange(1, n + 1) ** 0.8
        sets.append(sorted(rng.choice(n, size=min(s, n), replace=False, p=w / w.sum()).tolist()))
    off = np.zeros(theta + 1, np.uint64)
    off[1:] = np.cumsum([len(s) for s in sets])
    mem = np.array([u for s in sets for u in s], np.uint32)
    return sets, off, mem


def _cov(sets, S):
    S = set(S)
    return sum(1 for s in sets if S.intersection(s))


@pytest.mark.parametrize("seed", range(12))
def test_each_seed_maximises_marginal_coverage(seed):
    n, theta, k = 25, 80, 6
    sets, off, mem = _random_pool(seed, n, theta, 6)
    seeds, gains = oracle.greedy(n, off, mem, k)
    chosen = []
    for i in range(k):
        base = _cov(sets, chosen)
        marg = [(-1 if v in chosen else _cov(sets, chosen + [v]) - base) for v in range(n)]
        best = max(marg)
        assert seeds[i] == marg.index(best)          # lowest id among the maxima
        assert gains[i] == best
        chosen.append(int(seeds[i]))
    assert int(gains.sum()) == _cov(sets, chosen) == oracle.coverage(n, off, mem, seeds)


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_greedy_guarantee_against_brute_force(seed, k):
    n, theta = 9, 40
    sets, off, mem = _random_pool(100 + seed, n, theta, 4)
    seeds, gains = oracle.greedy(n, off, mem, k)
    opt = max(_cov(sets, S) for S in itertools.combinations(range(n), k))
    assert int(gains.sum()) >= (1 - (1 - 1 / k) ** k) * opt - 1e-9
    assert int(gains.sum()) <= opt


def test_k1_is_most_frequent_lowest_id():
    sets = [[0, 3], [3, 4], [1, 4], [2]]
    off = np.array([0, 2, 4, 6, 7], np.uint64)
    mem = np.array([u for s in sets for u in s], np.uint32)
    seeds, gains = oracle.greedy(5, off, mem, 1)
    assert list(seeds) == [3] and list(gains) == [2]      # 3 and 4 tie at 2 -> 3


def test_exhaustion_picks_smallest_unchosen():
    sets = [[4], [4], [2, 4]]
    off = np.array([0, 1, 2, 4], np.uint64)
    mem = np.array([4, 4, 2, 4], np.uint32)
    seeds, gains = oracle.greedy(6, off, mem, 4)
    assert list(seeds) == [4, 0, 1, 2] and list(gains) == [3, 0, 0, 0]


def test_theta_prefix_only():
    sets, off, mem = _random_pool(7, 20, 50, 5)
    s_full, _ = oracle.greedy(20, off, mem, 3, theta=50)
    s_pre, g_pre = oracle.greedy(20, off[:21], mem[:int(off[20])], 3)
    s_pre2, g_pre2 = oracle.greedy(20, off, mem, 3, theta=20)
    assert np.array_equal(s_pre, s_pre2) and np.array_equal(g_pre, g_pre2)


def test_invalid_k():
    off = np.array([0, 1], np.uint64)
    mem = np.array([0], np.uint32)
    with pytest.raises(ValueError):
        oracle.greedy(3, off, mem, 0)
    with pytest.raises(ValueError):
        oracle.greedy(3, off, mem, 4)
