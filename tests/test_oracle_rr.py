"""Pins of the oracle's RR sets against what the paper and mathematics fix.

* Live-world reachability: every coin recomputed with an independent Philox
  implementation (PyTorch's engine), the live channels assembled into a sparse
  matrix and the RR set taken as the set of vertices reaching the root
  (scipy breadth-first search on the reversed live graph) -- a different
  traversal from the oracle's queue, so this also pins order independence.
* Exact enumeration of every live-edge world on tiny hypergraphs (<= 20
  channels): inclusion probabilities Pr[u in RR(r)] (Equation (1)'s
  reverse-reachability reading) and the equivalence with the weighted clique
  graph G_w whose pair probability is 1 - (1 - p_v)^w(u,v) (Section 2.1).
* Special cases: p = 1 gives connected components; p = 0 gives {root}.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import breadth_first_order, connected_components

import hypergen
import oracle
from conftest import independent_coins

ALWAYS = 0xFFFFFFFF


def _channels(hg):
    """All channels (he, pos_u, u, v): u at position pos_u of he, v another member."""
    out = []
    for e in range(hg.m):
        mem = hg.he_mem[hg.he_off[e]:hg.he_off[e + 1]]
        for pu, u in enumerate(mem):
            for v in mem:
                if v != u:
                    out.append((e, pu, int(u), int(v)))
    return np.array(out, dtype=np.int64).reshape(-1, 4)


def _reach_to(n, src, dst, root):
    """Vertices with a directed path src->...->dst ending at root."""
    if len(src) == 0:
        return np.array([root])
    A = sp.csr_matrix((np.ones(len(src)), (dst, src)), shape=(n, n))   # reversed edges v->u
    order = breadth_first_order(A, root, directed=True, return_predecessors=False)
    return np.sort(order)


@pytest.mark.parametrize("case", ["small", "tiny_workload"])
def test_rr_sets_equal_live_world_reachability(case, torch_philox):
    if case == "small":
        hg = hypergen.tiny_hypergraph(21, 60, 80, 2, 6)
        p, ids, seed, inst = 0.3, range(0, 300), 5, 2
    else:
        w = hypergen.workload("tiny")
        hg = w.build()
        p, ids, seed, inst = w.p, list(range(0, 12)) + [1000, 5000], 0, 0
    g = oracle.Graph(hg, 0, p)
    g.stratify()
    thr = g.arrays()["thr"]
    ch = _channels(hg)
    for pool in (0, 1):
        for j in ids:
            root = g.root(seed, inst, pool, j)
            coins = independent_coins(torch_philox, seed, inst, pool, j, ch[:, 0], ch[:, 3], ch[:, 1])
            t = thr[ch[:, 3]].astype(np.uint64)
            live = (t == ALWAYS) | (coins.astype(np.uint64) < t)
            ref = _reach_to(hg.n, ch[live, 2], ch[live, 3], root)
            got = g.rr_set(seed, inst, pool, j)
            assert np.array_equal(got, ref), (pool, j)


def test_p_one_gives_connected_components():
    hg = hypergen.tiny_hypergraph(4, 200, 120, 1, 4, allow_singletons=True)
    g = oracle.Graph(hg, 0, 1.0)
    g.stratify()
    sizes = np.diff(hg.he_off.astype(np.int64))
    owner = np.repeat(np.arange(hg.m), sizes)
    B = sp.csr_matrix((np.ones(hg.nnz), (hg.he_mem.astype(np.int64), hg.n + owner)),
                      shape=(hg.n + hg.m, hg.n + hg.m))
    _, lab = connected_components(B, directed=False)
    for j in range(512):
        r = g.root(1, 0, 0, j)
        comp = np.nonzero(lab[:hg.n] == lab[r])[0]
        assert np.array_equal(g.rr_set(1, 0, 0, j), comp)


def test_p_zero_and_isolated_give_root_only():
    hg = hypergen.tiny_hypergraph(4, 50, 40)
    g = oracle.Graph(hg, 0, 0.0)
    g.stratify()
    for j in range(300):
        assert list(g.rr_set(0, 0, 1, j)) == [g.root(0, 0, 1, j)]
    g2 = oracle.Graph(hypergen.from_lists(5, [[1], [], [3]]), 0, 1.0)
    g2.stratify()
    for j in range(20):
        assert list(g2.rr_set(0, 0, 0, j)) == [g2.root(0, 0, 0, j)]


# ---------------------------------------------------------------------------
# exact enumeration on tiny hypergraphs
# ---------------------------------------------------------------------------
TINY_EDGES = [[0, 1, 2], [2, 3], [3, 4], [1, 4], [4, 5, 1]]   # 6+2+2+2+6 = 18 channels


def _enumerate_inclusion(hg, pv, root):
    """Exact Pr[u in RR(root)] over all 2^C live-edge worlds (Fractions)."""
    ch = _channels(hg)
    C = len(ch)
    probs = [Fraction(pv[int(v)]) for v in ch[:, 3]]
    incl = [Fraction(0)] * hg.n
    for bits in range(1 << C):
        pr = Fraction(1)
        for c in range(C):
            pr *= probs[c] if (bits >> c) & 1 else 1 - probs[c]
        live = [c for c in range(C) if (bits >> c) & 1]
        reach = {root}
        grow = True
        while grow:
            grow = False
            for c in live:
                u, v = int(ch[c, 2]), int(ch[c, 3])
                if v in reach and u not in reach:
                    reach.add(u)
                    grow = True
        for u in reach:
            incl[u] += pr
    return incl


def _clique_inclusion(n, edges, pv, root):
    """Same probabilities on G_w: one channel per ordered pair (u,v) of
    co-members, live with 1 - (1 - p_v)^w(u,v)."""
    w = {}
    for e in edges:
        for u in e:
            for v in e:
                if u != v:
                    w[(u, v)] = w.get((u, v), 0) + 1
    pairs = sorted(w)
    pe = [1 - (1 - Fraction(pv[v])) ** w[(u, v)] for (u, v) in pairs]
    incl = [Fraction(0)] * n
    for bits in range(1 << len(pairs)):
        pr = Fraction(1)
        for c in range(len(pairs)):
            pr *= pe[c] if (bits >> c) & 1 else 1 - pe[c]
        reach = {root}
        grow = True
        while grow:
            grow = False
            for c in range(len(pairs)):
                if (bits >> c) & 1:
                    u, v = pairs[c]
                    if v in reach and u not in reach:
                        reach.add(u)
                        grow = True
        for u in reach:
            incl[u] += pr
    return incl


def _enumerate_inclusion_f64(hg, pv, root):
    """Pr[u in RR(root)] over all live-edge worlds, vectorised in float64."""
    ch = _channels(hg)
    C = len(ch)
    worlds = np.arange(1 << C, dtype=np.int64)
    live = ((worlds[:, None] >> np.arange(C)) & 1).astype(bool)
    p = np.array([float(pv[int(v)]) for v in ch[:, 3]])
    pr = np.prod(np.where(live, p, 1 - p), axis=1)
    reach = np.zeros((len(worlds), hg.n), bool)
    reach[:, root] = True
    for _ in range(hg.n):
        for c in range(C):
            u, v = int(ch[c, 2]), int(ch[c, 3])
            reach[:, u] |= live[:, c] & reach[:, v]
    return pr @ reach


def _tiny_thresholds_as_probs(g):
    thr = g.arrays()["thr"]
    return [Fraction(1) if t == ALWAYS else Fraction(int(t), 2 ** 32) for t in thr]


@pytest.mark.slow
def test_exact_inclusion_and_clique_equivalence():
    edges = [[0, 1, 2], [2, 3], [1, 2], [3, 0]]      # pair (1,2) has weight 2; 10 channels
    hg = hypergen.from_lists(4, edges)
    g = oracle.Graph(hg, 0, 0.3)
    g.stratify()
    pv = _tiny_thresholds_as_probs(g)
    for root in range(4):
        a = _enumerate_inclusion(hg, pv, root)
        b = _clique_inclusion(4, edges, pv, root)
        assert a == b                        # algebraic identity, exact


@pytest.mark.slow
@pytest.mark.parametrize("model,p", [(0, 0.35), (1, 0.0)])
def test_oracle_inclusion_frequencies_match_exact(model, p):
    hg = hypergen.from_lists(6, TINY_EDGES)
    g = oracle.Graph(hg, model, p)
    g.stratify()
    pv = _tiny_thresholds_as_probs(g)
    N = 20000
    for root in (0, 4):
        exact = _enumerate_inclusion_f64(hg, pv, root)
        off, mem, _ = g.generate(3, 1, 0, 0, N, roots=np.full(N, root, np.uint32))
        freq = np.bincount(mem, minlength=6) / N
        for u in range(6):
            q = float(exact[u])
            if q < 1e-9 or q > 1 - 1e-9:
                assert freq[u] == round(q)
            else:
                z = (freq[u] - q) / np.sqrt(q * (1 - q) / N)
                assert abs(z) < 5, (root, u, freq[u], q)
