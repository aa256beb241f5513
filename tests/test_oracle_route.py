"""Pins of the oracle's division of the RR sets into R1 and R2 (Section 4.1,
"Division of the RR sets"), independent of the oracle's own code.

* Tables: the small layers (|L_i| < alpha |A(v)| for 1 <= i <= beta, with
  alpha = F_cnt / T_cnt and beta = L_cnt / |V| recomputed from Python-built
  layers in exact integers), the R1 vertices, their forced members, and the
  two root lists as the stratum-ordered subsequences of P.
* Roots: pool 0 draws only R1 vertices, pool 1 only the others, each vertex
  T / n_pool times per ladder block up to one.
* R1 sets: the vertices with a live path into the root or into any of its
  forced members, with coins from an independent Philox and scipy BFS.
* Bias (documented, reading R25): the R2 estimate n Lambda_R2({s}) / theta
  converges to n times the mean, over the R2 vertices only, of
  Pr[s in RR(v)] (exact enumeration), which differs from the spread.
* Inert and rejected cases, switching off, and re-stratifying (which keeps
  the division).
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import breadth_first_order

import hypergen
import oracle
from conftest import independent_coins
from test_oracle_layered import _layers_python
from test_oracle_rr import ALWAYS, TINY_EDGES, _channels, _enumerate_inclusion_f64, _tiny_thresholds_as_probs


def _division_python(hg):
    """(R1 flag per vertex, forced members per vertex) from Python layers."""
    lay = _layers_python(hg)
    Fc = sum(len(ls[0]) for ls in lay if ls)
    Tc = sum(sum(len(x) for x in ls) for ls in lay)
    Lc = sum(len(ls) for ls in lay)
    ilim = Lc // hg.n
    forced = []
    for ls in lay:
        deg = sum(len(x) for x in ls)
        f = []
        for i, layer in enumerate(ls):
            if i >= ilim:
                break
            if len(layer) * Tc < Fc * deg:
                f.extend(layer)
        forced.append(f)
    return [bool(f) for f in forced], forced


CASES = {
    "tiny": lambda: hypergen.workload("tiny").build(),
    "small_a": lambda: hypergen.tiny_hypergraph(3, 80, 120, 2, 7),
    "small_b": lambda: hypergen.tiny_hypergraph(8, 150, 90, 2, 9, allow_singletons=True),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_division_tables_match_python(case):
    hg = CASES[case]()
    g = oracle.Graph(hg, 0, 0.1)
    st = g.stratify()
    r1, forced = _division_python(hg)
    n1 = g.route()
    assert n1 == sum(r1)
    assert 0 < n1 < hg.n   # the division is not inert on these graphs
    rP, f_off, f_mem = g.route_tables()
    P = st["P"]
    assert list(rP[:n1]) == [v for v in P if r1[v]]
    assert list(rP[n1:]) == [v for v in P if not r1[v]]
    for v in range(hg.n):
        assert list(f_mem[f_off[v]:f_off[v + 1]]) == forced[v], v


def test_roots_by_pool():
    hg = CASES["small_a"]()
    g = oracle.Graph(hg, 0, 0.1)
    g.stratify()
    r1, _ = _division_python(hg)
    n1 = g.route()
    sizes = {0: n1, 1: hg.n - n1}
    for pool in (0, 1):
        for lo, T in ((0, 256), (256, 256), (512, 512)):
            roots = [g.root(4, 1, pool, j) for j in range(lo, lo + T)]
            assert all(r1[r] == (pool == 0) for r in roots)
            cnt = np.bincount(roots, minlength=hg.n)
            mine = np.array([v for v in range(hg.n) if r1[v] == (pool == 0)])
            q = T / sizes[pool]
            assert cnt[mine].min() >= np.floor(q) and cnt[mine].max() <= np.ceil(q)


def _reach_to_any(n, src, dst, starts):
    A = sp.csr_matrix((np.ones(len(src)), (dst, src)), shape=(n, n))
    seen = set()
    for s in starts:
        seen.update(int(x) for x in breadth_first_order(A, s, directed=True, return_predecessors=False))
    return np.array(sorted(seen), np.uint32)


@pytest.mark.parametrize("model,p", [(0, 0.2), (5, 0.2), (1, 0.0)])
def test_r1_sets_are_closures_from_root_and_forced(model, p, torch_philox):
    hg = CASES["small_a"]()
    g = oracle.Graph(hg, model, p)
    g.stratify()
    _, forced = _division_python(hg)
    g.route()
    thr = g.arrays()["thr"]
    ch = _channels(hg)
    seed, inst = 6, 1
    for pool in (0, 1):
        for j in range(0, 120):
            root = g.root(seed, inst, pool, j)
            got = g.rr_set(seed, inst, pool, j)
            starts = [root] + (forced[root] if pool == 0 else [])
            assert set(starts) <= set(got.tolist())
            if model == 5:
                continue   # gap models: the stream words are pinned elsewhere
            coins = independent_coins(torch_philox, seed, inst, pool, j, ch[:, 0], ch[:, 3], ch[:, 1])
            t = thr[ch[:, 3]].astype(np.uint64)
            live = (t == ALWAYS) | (coins.astype(np.uint64) < t)
            ref = _reach_to_any(hg.n, ch[live, 2], ch[live, 3], starts)
            assert np.array_equal(got, ref), (pool, j)


@pytest.mark.slow
def test_r2_estimate_is_biased_toward_the_r2_vertices():
    hg = hypergen.from_lists(6, TINY_EDGES)
    g = oracle.Graph(hg, 0, 0.35)
    g.stratify()
    r1, _ = _division_python(hg)
    n1 = g.route()
    assert 0 < n1 < 6
    pv = _tiny_thresholds_as_probs(g)
    incl = np.array([_enumerate_inclusion_f64(hg, pv, root) for root in range(6)])   # incl[root, u]
    v2 = [v for v in range(6) if not r1[v]]
    N = 16384   # a ladder boundary: every block whole, so each R2 vertex is a root N / n2 times
    off, mem, roots = g.generate(2, 0, 1, 0, N)
    assert set(roots.tolist()) <= set(v2)
    worst = 0.0
    for s in range(6):
        sigma = incl[:, s].sum()                     # spread of {s}: sum over roots of Pr[s in RR(root)]
        biased = 6 * incl[v2, s].mean()              # what n Lambda_R2 / theta converges to
        cover = sum(1 for i in range(N) if s in set(mem[off[i]:off[i + 1]].tolist()))
        est = 6 * cover / N
        q = biased / 6
        se = 6 * np.sqrt(q * (1 - q) / N)
        assert abs(est - biased) < 5 * se + 1e-12, (s, est, biased)
        worst = max(worst, abs(biased - sigma) / sigma)
    assert worst > 0.05   # the division moves the estimate away from the spread


def test_inert_rejected_off_and_restratify():
    # a graph whose every vertex has the same layer structure: no small layer
    hg = hypergen.from_lists(4, [[0, 1, 2, 3]])
    g = oracle.Graph(hg, 0, 0.3)
    g.stratify()
    plain = [g.root(0, 0, pool, j) for pool in (0, 1) for j in range(64)]
    assert g.route() in (0, 4)
    assert [g.root(0, 0, pool, j) for pool in (0, 1) for j in range(64)] == plain
    for model in (2, 3, 4):
        h = oracle.Graph(CASES["small_a"](), model, 0.1)
        h.stratify()
        with pytest.raises(oracle.OracleError):
            h.route()
    unstrat = oracle.Graph(CASES["small_a"](), 0, 0.1)
    with pytest.raises(oracle.OracleError):
        unstrat.route()
    g2 = oracle.Graph(CASES["small_a"](), 0, 0.1)
    g2.stratify()
    base = [g2.root(1, 0, 0, j) for j in range(200)]
    sets = [g2.rr_set(1, 0, 0, j) for j in range(50)]
    g2.route()
    assert [g2.root(1, 0, 0, j) for j in range(200)] != base
    g2.route(False)
    assert [g2.root(1, 0, 0, j) for j in range(200)] == base
    assert all(np.array_equal(a, g2.rr_set(1, 0, 0, j)) for j, a in enumerate(sets))
    g2.route()
    routed = [g2.root(1, 0, 0, j) for j in range(200)]
    g2.stratify()   # new strata: the division is rebuilt (the same strata give the same one)
    assert [g2.root(1, 0, 0, j) for j in range(200)] == routed
