"""Pins of the oracle's spread estimator and the full HyperIM_BRR loop.

* Equation (1): n * Lambda_R(S) / theta is unbiased for the expected influence
  of S, checked against the exact influence from enumerating every live-edge
  world (forward reachability from S, the cascade of Section 2.1).
* The stratified (systematic) roots give lower estimator variance than iid
  uniform roots (F-test).
* The full loop on the tiny workload: its R2 spread estimate agrees with a
  forward independent-cascade Monte Carlo on the explicit channel graph
  (numpy coins, not Philox) within 10% relative.
* Greedy on a large pool reaches >= (1 - 1/e - eps) of the exact optimum on an
  enumerable hypergraph.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import breadth_first_order

import hypergen
import oracle

ALWAYS = 0xFFFFFFFF
EDGES = [[0, 1, 2], [2, 3], [3, 4], [1, 4], [4, 5, 1]]     # 18 channels


def _channels(hg):
    out = []
    for e in range(hg.m):
        mem = hg.he_mem[hg.he_off[e]:hg.he_off[e + 1]]
        for u in mem:
            for v in mem:
                if v != u:
                    out.append((int(u), int(v)))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def _probs(g):
    thr = g.arrays()["thr"]
    return np.array([1.0 if t == ALWAYS else int(t) / 2 ** 32 for t in thr])


def _exact_spread_all(hg, pv, seedsets):
    """Exact expected influence of each seed set by enumerating all worlds."""
    ch = _channels(hg)
    C = len(ch)
    worlds = np.arange(1 << C, dtype=np.int64)
    live = ((worlds[:, None] >> np.arange(C)) & 1).astype(bool)
    p = pv[ch[:, 1]]
    pr = np.prod(np.where(live, p, 1 - p), axis=1)
    out = []
    for S in seedsets:
        act = np.zeros((len(worlds), hg.n), bool)
        act[:, list(S)] = True
        for _ in range(hg.n):
            for c in range(C):
                u, v = ch[c]
                act[:, v] |= live[:, c] & act[:, u]
        out.append(float(pr @ act.sum(axis=1)))
    return out


@pytest.mark.slow
def test_estimator_unbiased_for_fixed_seed_set():
    hg = hypergen.from_lists(6, EDGES)
    g = oracle.Graph(hg, 0, 0.35)
    g.stratify()
    S = [1, 3]
    exact = _exact_spread_all(hg, _probs(g), [S])[0]
    theta, reps = 256, 300
    est = []
    for s in range(reps):
        off, mem, _ = g.generate(s, 0, 0, 0, theta)
        est.append(hg.n * oracle.coverage(hg.n, off, mem, S) / theta)
    est = np.array(est)
    z = (est.mean() - exact) / (est.std(ddof=1) / np.sqrt(reps))
    assert abs(z) < 4.5, (est.mean(), exact)


@pytest.mark.slow
def test_stratified_roots_reduce_variance():
    hg = hypergen.tiny_hypergraph(31, 300, 450, 2, 5)
    g = oracle.Graph(hg, 0, 0.03)
    g.stratify()
    S = list(range(20))
    theta, reps = 512, 300
    rng = np.random.default_rng(0)
    strat, iid = [], []
    for s in range(reps):
        off, mem, _ = g.generate(s, 0, 0, 0, theta)
        strat.append(oracle.coverage(hg.n, off, mem, S))
        roots = rng.integers(0, hg.n, size=theta).astype(np.uint32)
        off, mem, _ = g.generate(s, 0, 0, 0, theta, roots=roots)
        iid.append(oracle.coverage(hg.n, off, mem, S))
    from scipy.stats import f
    v1, v2 = np.var(strat, ddof=1), np.var(iid, ddof=1)
    assert v1 < v2
    assert f.cdf(v1 / v2, reps - 1, reps - 1) < 0.01
    assert abs(np.mean(strat) - np.mean(iid)) < 4 * np.sqrt(v2 / reps + v1 / reps)


def _forward_mc_spread(hg, pv, S, worlds, rng):
    ch = _channels(hg)
    p = pv[ch[:, 1]]
    tot = 0
    for _ in range(worlds):
        live = rng.random(len(ch)) < p
        A = sp.csr_matrix((np.ones(int(live.sum())), (ch[live, 0], ch[live, 1])), shape=(hg.n, hg.n))
        reach = set()
        for s in S:
            if s in reach:
                continue
            reach.update(breadth_first_order(A, s, directed=True, return_predecessors=False).tolist())
        tot += len(reach)
    return tot / worlds


@pytest.mark.slow
def test_tiny_workload_spread_estimate_matches_forward_monte_carlo():
    w = hypergen.workload("tiny")
    hg = w.build()
    g = oracle.Graph(hg, w.model, w.p)
    g.stratify()
    r = g.select_seeds(w.k, w.eps, w.ell, theta_fixed=1 << 13)
    truth = _forward_mc_spread(hg, _probs(g), [int(x) for x in r["seeds"]], 1500,
                               np.random.default_rng(1))
    assert r["spread"] == pytest.approx(truth, rel=0.1)
    # R1's estimate is biased upward by selection, never below R2's by much
    assert hg.n * r["lambda1"] / r["theta"] >= 0.95 * r["spread"]


@pytest.mark.slow
def test_brr_loop_stops_by_ratio_and_spread_matches():
    w = hypergen.workload("tiny")
    hg = w.build()
    g = oracle.Graph(hg, w.model, w.p)
    g.stratify()
    r = g.select_seeds(w.k, w.eps, w.ell)
    assert r["rounds"] >= 1 and r["theta"] >= 256
    t = 1 - 1 / np.e
    assert r["sigma_l"] / r["sigma_u"] >= t - w.eps or r["rounds"] == r["i_max"]
    assert r["sigma_l"] <= r["spread"] <= r["sigma_u"]


@pytest.mark.slow
def test_greedy_reaches_guarantee_against_exact_optimum():
    hg = hypergen.from_lists(6, EDGES)
    g = oracle.Graph(hg, 0, 0.35)
    g.stratify()
    k, eps = 2, 0.1
    r = g.select_seeds(k, eps, 1.0, theta_fixed=1 << 14)
    sets = list(itertools.combinations(range(6), k))
    ex = _exact_spread_all(hg, _probs(g), sets + [tuple(int(x) for x in r["seeds"])])
    opt = max(ex[:-1])
    assert ex[-1] >= (1 - 1 / np.e - eps) * opt
