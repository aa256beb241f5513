"""Pins of the oracle's graph build, thresholds, sample-set layers, strata and
stratified roots, against independent computations (numpy transposes,
networkx clique expansion, exact rational arithmetic, counting)."""
from fractions import Fraction

import networkx as nx
import numpy as np
import pytest

import hypergen
import oracle

ALWAYS = 0xFFFFFFFF


def _random_hg(seed, n=40, m=60, lo=1, hi=6, dup_edges=10):
    """Random hypergraph with some repeated hyperedges (so weights w > 1 occur)."""
    rng = np.random.default_rng(seed)
    edges = []
    for _ in range(m):
        s = int(rng.integers(lo, hi + 1))
        edges.append(list(rng.choice(n, size=min(s, n), replace=False)))
    for _ in range(dup_edges):
        e = list(edges[int(rng.integers(0, m))])
        rng.shuffle(e)
        edges.append(e)
    return hypergen.from_lists(n, edges)


def test_incidence_lists_match_numpy_transpose():
    hg = hypergen.tiny_hypergraph(3, 300, 500, 1, 7)
    g = oracle.Graph(hg, 0, 0.1)
    a = g.arrays()
    sizes = np.diff(hg.he_off.astype(np.int64))
    owner = np.repeat(np.arange(hg.m), sizes)
    order = np.lexsort((owner, hg.he_mem))
    ref_v_he = owner[order]
    ref_v_off = np.concatenate([[0], np.cumsum(np.bincount(hg.he_mem, minlength=hg.n))])
    assert np.array_equal(a["v_off"], ref_v_off)
    assert np.array_equal(a["v_he"], ref_v_he)
    ref_c = np.bincount(hg.he_mem, weights=np.repeat(sizes - 1, sizes), minlength=hg.n)
    assert np.array_equal(a["c"], ref_c.astype(np.uint64))


@pytest.mark.parametrize("p,expect", [(0.5, 2 ** 31), (0.25, 2 ** 30), (1.0, ALWAYS), (2.0, ALWAYS),
                                      (0.0, 0), (2.0 ** -32, 1), (0.75, 3 * 2 ** 30)])
def test_constant_threshold_closed_form(p, expect):
    hg = hypergen.from_lists(3, [[0, 1, 2]])
    thr = oracle.Graph(hg, 0, p).arrays()["thr"]
    assert list(thr) == [expect] * 3


def test_constant_threshold_exact_rational():
    for p in np.random.default_rng(1).random(200).astype(np.float32):
        hg = hypergen.from_lists(2, [[0, 1]])
        thr = int(oracle.Graph(hg, 0, float(p)).arrays()["thr"][0])
        exact = Fraction(float(p)) * 2 ** 32       # float32 value is exact in a Fraction
        assert thr == int(exact)                    # floor of a positive rational


def test_weighted_cascade_threshold_exact_rational():
    hg = hypergen.tiny_hypergraph(9, 400, 900, 1, 12)
    a = oracle.Graph(hg, 1).arrays()
    for v in range(hg.n):
        c = int(a["c"][v])
        if c == 0:
            assert a["thr"][v] == 0
            continue
        pv = np.float32(1.0 / c)       # correctly rounded double, then float32
        if pv >= 1:
            assert a["thr"][v] == ALWAYS
        else:
            assert int(a["thr"][v]) == int(Fraction(float(pv)) * 2 ** 32)


@pytest.mark.parametrize("edges,n,model,p", [
    ([[0, 5]], 5, 0, 0.1),              # id >= n
    ([[0, 1, 0]], 3, 0, 0.1),           # duplicate member
    ([[0, 1]], 3, 0, float("nan")),     # NaN p
    ([[0, 1]], 3, 0, -0.5),             # negative p
    ([[0, 1]], 3, 7, 0.1),              # unknown model
    ([[0, 1]], 3, 2, float("nan")),     # NaN p under LT
])
def test_invalid_inputs_rejected(edges, n, model, p):
    with pytest.raises(oracle.OracleError):
        oracle.Graph(hypergen.from_lists(n, edges), model, p)


def test_unsorted_offsets_rejected():
    hg = hypergen.Hypergraph(3, np.array([0, 2, 1], np.uint32), np.array([0, 1], np.uint32))
    with pytest.raises(oracle.OracleError):
        oracle.Graph(hg, 0, 0.1)


def test_empty_and_singleton_hyperedges_are_legal():
    hg = hypergen.from_lists(4, [[], [2], [0, 1]])
    g = oracle.Graph(hg, 1)
    a = g.arrays()
    assert list(a["c"]) == [1, 1, 0, 0]
    st = g.stratify()
    assert list(st["l"]) == [1, 1, 0, 0]


@pytest.mark.parametrize("seed", range(6))
def test_layers_against_explicit_clique_graph(seed):
    """Section 3.1.1: layers of A(v) by edge weight of G_w; built here with
    networkx from the clique expansion of every hyperedge."""
    hg = _random_hg(seed)
    G = nx.Graph()
    G.add_nodes_from(range(hg.n))
    for e in hg.edges():
        e = [int(x) for x in e]
        for a in range(len(e)):
            for b in range(a + 1, len(e)):
                u, v = e[a], e[b]
                if G.has_edge(u, v):
                    G[u][v]["w"] += 1
                else:
                    G.add_edge(u, v, w=1)
    g = oracle.Graph(hg, 0, 0.1)
    st = g.stratify()
    for v in range(hg.n):
        ws = [G[v][u]["w"] for u in G.neighbors(v)]
        assert st["deg"][v] == len(ws) == G.degree(v)
        assert st["l"][v] == len(set(ws))
        assert st["top"][v] == (ws.count(max(ws)) if ws else 0)
        lv = len(set(ws))
        expect_s = 0 if lv == 0 else min(7, lv.bit_length())
        assert st["stratum"][v] == expect_s
    # P sorted by (stratum, id); B = stratum boundaries
    ref_P = np.lexsort((np.arange(hg.n), st["stratum"]))
    assert np.array_equal(st["P"], ref_P)
    counts = np.bincount(st["stratum"], minlength=8)
    assert np.array_equal(st["B"], np.concatenate([[0], np.cumsum(counts)]))
    # Section 4.1 statistics and Theorem 2's theta(l*)
    assert st["alpha"] == pytest.approx(st["top"].sum() / st["deg"].sum(), rel=1e-15)
    assert st["beta"] == pytest.approx(st["l"].sum() / hg.n, rel=1e-15)
    l = st["l"][st["l"] > 0].astype(np.float64)
    assert st["theta_l"] == pytest.approx(float(np.sum(l / np.log(l + 1))) / hg.n, rel=1e-12)


def test_strata_saturate_at_seven():
    # vertex 0 shares 1..130 hyperedges with distinct partners -> 130 distinct weights
    edges = []
    for u in range(1, 131):
        edges += [[0, u]] * u
    hg = hypergen.from_lists(131, edges)
    st = oracle.Graph(hg, 0, 0.1).stratify()
    assert st["l"][0] == 130
    assert st["stratum"][0] == 7 and 130 .bit_length() == 8


def test_ladder_blocks():
    blk = []
    import ctypes as C
    for j in [0, 1, 255, 256, 511, 512, 1023, 1024, 2 ** 20 - 1, 2 ** 20]:
        b, J, T = C.c_uint32(), C.c_uint64(), C.c_uint64()
        oracle.lib().orc_block_of(j, 8, C.byref(b), C.byref(J), C.byref(T))
        blk.append((j, b.value, J.value, T.value))
    for j, b, J, T in blk:
        assert J <= j < J + T
        if b == 0:
            assert (J, T) == (0, 256)
        else:
            assert J == T == 256 << (b - 1)


@pytest.mark.parametrize("n", [1, 7, 300, 1000])
def test_root_quotas_and_counts(n):
    """Systematic proportional allocation: inside every ladder block, each
    vertex is a root floor(T/n) or ceil(T/n) times and each stratum receives
    within one of T N_h / n roots."""
    hg = hypergen.tiny_hypergraph(n, n, 2 * n, 1, 5, allow_singletons=True)
    g = oracle.Graph(hg, 0, 0.1)
    st = g.stratify()
    strat = st["stratum"]
    for pool in (0, 1):
        for b, (J, T) in enumerate([(0, 256), (256, 256), (512, 512), (1024, 1024), (2048, 2048)]):
            roots = np.array([g.root(9, 4, pool, J + t) for t in range(T)])
            cnt = np.bincount(roots, minlength=n)
            assert cnt.min() >= T // n and cnt.max() <= -(-T // n)
            assert cnt.sum() == T
            q = np.bincount(strat[roots], minlength=8)
            Nh = np.bincount(strat, minlength=8)
            assert np.all(np.abs(q - T * Nh / n) < 1.0 + 1e-9)
            # ids of one stratum are contiguous and ascending in P order
            pos_in_P = np.argsort(st["P"])[roots]
            assert np.all(np.diff(pos_in_P) >= 0)


def test_root_inclusion_probability_is_T_over_n():
    """With T < n, each vertex is a root in a block with probability exactly
    T/n over the block's random offset (checked by a z-test over seeds)."""
    n = 10
    hg = hypergen.tiny_hypergraph(2, n, 20)
    g = oracle.Graph(hg, 0, 0.1)
    g.stratify()
    trials, T = 6000, 4                      # qlog = 2: block 0 holds ids 0..3
    counts = np.zeros(n)
    for s in range(trials):
        roots = [g.root(s, 0, 0, t, qlog=2) for t in range(T)]
        assert len(set(roots)) == T          # T <= n: no vertex twice in a block
        counts[roots] += 1
    p = T / n
    z = (counts - trials * p) / np.sqrt(trials * p * (1 - p))
    assert np.all(np.abs(z) < 5)
