"""GPU parity of the linear-threshold model (Section 2.1, LT bullet, in its
live-edge form): the walk kernel through the C ABI against the oracle, bit
for bit -- roots, RR sets (ascending members), and the whole HyperIM_BRR
query (seeds, gains, theta, rounds, Lambda1, Lambda2, Lambda_u).  Cases cover
the LDS and global visited bitmaps (|V| above 32768), capped weights, p = 0
and p = 1, isolated vertices, high RR ids, the plain form, and a generation
call that mixes LT and IC graphs."""
import sys

import numpy as np
import pytest

import hypergen
import oracle

pytestmark = pytest.mark.gpu

LT_CONST, LT_WC = 2, 3


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hy():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_01911_amd as hy
    hy.load_library()
    return hy


def _path(n):
    return hypergen.from_lists(n, [[i, i + 1] for i in range(n - 1)])


CASES = {
    "tiny_lt": lambda: (hypergen.workload("tiny_lt").build(), LT_WC, 0.0),
    "small_const_015": lambda: (hypergen.tiny_hypergraph(31, 60, 80, 2, 6), LT_CONST, 0.15),
    "small_const_capped": lambda: (hypergen.tiny_hypergraph(32, 60, 80, 2, 6), LT_CONST, 0.6),
    "singletons_wc": lambda: (hypergen.tiny_hypergraph(5, 300, 500, 1, 8, allow_singletons=True), LT_WC, 0.0),
    "p_one_star": lambda: (hypergen.from_lists(7, [[0, i] for i in range(1, 6)] + [[6]]), LT_CONST, 1.0),
    "p_zero": lambda: (hypergen.tiny_hypergraph(4, 50, 40), LT_CONST, 0.0),
    "one_vertex": lambda: (hypergen.from_lists(1, [[0], []]), LT_WC, 0.0),
    "path_40000": lambda: (_path(40000), LT_WC, 0.0),
    # a hub in 9999 hyperedges: the channel search takes several 64-way rounds
    "hub_lt": lambda: (hypergen.from_lists(10001, [[0, i, i + 1] for i in range(1, 10000)]), LT_WC, 0.0),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_lt_rr_sets_bit_exact(hy, case):
    _flush(f"[gpu] LT rr sets case={case}")
    hg, model, p = CASES[case]()
    g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, model, p)
    o = oracle.Graph(hg, model, p)
    a, b = g.read(strata=False), o.arrays()
    for k in ("v_off", "v_he", "thr", "c"):
        assert np.array_equal(a[k], b[k]), k
    g.stratify()
    o.stratify()
    for pool_tag, (lo, hi) in [(0, (0, 1500)), (1, (200, 700)), (0, ((1 << 33) - 100, (1 << 33) + 100))]:
        pool = hy.Pool(g)
        hy.generate_rr(g, 7, 3, pool_tag, lo, hi, pool)
        off, mem, roots = pool.read()
        roff, rmem, rroots = o.generate(7, 3, pool_tag, lo, hi)
        assert np.array_equal(roots, rroots)
        assert np.array_equal(off, roff)
        assert np.array_equal(mem, rmem)
    if case == "path_40000":
        assert np.diff(off).max() > 2   # walks go on past their first step (global bitmaps: |V| > 32768)


def test_lt_mid_sets_sampled_and_select_seeds_match_oracle(hy):
    """mid_lt (|V| = 1e5, global visited bitmaps): a generation call's sets
    and the whole query, in the persistent and the plain form, for both upper
    bounds."""
    _flush("[gpu] LT mid")
    w = hypergen.workload("mid_lt")
    hg = w.build()
    g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, w.model, w.p)
    o = oracle.Graph(hg, w.model, w.p)
    g.stratify()
    o.stratify()
    pool = hy.Pool(g)
    hy.generate_rr(g, w.philox_seed, 0, 0, 0, 4096, pool)
    off, mem, roots = pool.read()
    roff, rmem, rroots = o.generate(w.philox_seed, 0, 0, 0, 4096)
    assert np.array_equal(roots, rroots) and np.array_equal(off, roff) and np.array_equal(mem, rmem)
    for bound in (0, 1):
        ro = o.select_seeds(w.k, w.eps, w.ell, seed=w.philox_seed, bound=bound)
        for form in (0, 1):
            r = hy.select_seeds(g, w.k, w.eps, w.ell, seed=w.philox_seed, form=form, bound=bound)
            for key in ("rounds", "theta", "lambda1", "lambda2", "entries1", "entries2", "i_max", "lambda_u"):
                assert r[key] == ro[key], (bound, form, key, r[key], ro[key])
            assert np.array_equal(r["seeds"], ro["seeds"]) and np.array_equal(r["gains"], ro["gains"])
            assert r["sigma_l"] == pytest.approx(ro["sigma_l"], rel=1e-12)
            assert r["sigma_u"] == pytest.approx(ro["sigma_u"], rel=1e-12)


def test_lt_tiny_select_seeds_matches_oracle(hy):
    _flush("[gpu] LT tiny select")
    w = hypergen.workload("tiny_lt")
    hg = w.build()
    g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, w.model, w.p)
    o = oracle.Graph(hg, w.model, w.p)
    g.stratify()
    o.stratify()
    r = hy.select_seeds(g, w.k, w.eps, w.ell)
    ro = o.select_seeds(w.k, w.eps, w.ell)
    for key in ("rounds", "theta", "lambda1", "lambda2", "entries1", "entries2", "lambda_u"):
        assert r[key] == ro[key], key
    assert np.array_equal(r["seeds"], ro["seeds"]) and np.array_equal(r["gains"], ro["gains"])


def test_lt_and_ic_graphs_in_one_generation_call(hy):
    """Tasks of an LT graph and an IC graph in one call run in separate launch
    groups; every pool equals the oracle's."""
    _flush("[gpu] LT + IC in one call")
    hg = hypergen.tiny_hypergraph(41, 2000, 3000, 2, 6)
    graphs = []
    for model, p in ((LT_WC, 0.0), (0, 0.1), (LT_CONST, 0.05)):
        g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, model, p)
        g.stratify()
        o = oracle.Graph(hg, model, p)
        o.stratify()
        graphs.append((g, o))
    tasks, pools = [], []
    for i, (g, o) in enumerate(graphs):
        for tag in (0, 1):
            pl = hy.Pool(g)
            pools.append((pl, o, tag, i))
            tasks.append(dict(graph=g, pool=pl, seed=3, instance=i, pool_tag=tag, id_begin=0, id_end=1000))
    hy.generate_rr_batch(tasks)
    for pl, o, tag, i in pools:
        off, mem, roots = pl.read()
        roff, rmem, rroots = o.generate(3, i, tag, 0, 1000)
        assert np.array_equal(roots, rroots) and np.array_equal(off, roff) and np.array_equal(mem, rmem), (i, tag)


def test_lt_graph_rejects_unknown_model(hy):
    hg = hypergen.from_lists(3, [[0, 1]])
    with pytest.raises(hy.HyperIMError):
        hy.build_graph(hg.n, hg.he_off, hg.he_mem, 7, 0.1)
    with pytest.raises(hy.HyperIMError):
        hy.build_graph(hg.n, hg.he_off, hg.he_mem, LT_CONST, float("nan"))


def test_lt_query_batched_with_ic_query_matches_alone_and_oracle(hy):
    """A batch (shared launch groups per round) holding an LT query and an IC
    query on the same hypergraph: each result equals the query alone, and
    the LT one the oracle's."""
    _flush("[gpu] LT + IC batch")
    w = hypergen.workload("tiny_lt")
    hg = w.build()
    g_lt = hy.build_graph(hg.n, hg.he_off, hg.he_mem, LT_WC, 0.0)
    g_ic = hy.build_graph(hg.n, hg.he_off, hg.he_mem, 0, 0.05)
    for g in (g_lt, g_ic):
        g.stratify()
    qs = [dict(graph=g_lt, k=w.k, eps=w.eps, ell=w.ell, seed=0, instance=0),
          dict(graph=g_ic, k=w.k, eps=w.eps, ell=w.ell, seed=0, instance=1)]
    rs = hy.select_seeds_batch(qs)
    for q, r in zip(qs, rs):
        a = hy.select_seeds(q["graph"], q["k"], q["eps"], q["ell"], seed=q["seed"], instance=q["instance"])
        assert np.array_equal(a["seeds"], r["seeds"]) and np.array_equal(a["gains"], r["gains"])
        assert a["theta"] == r["theta"] and a["lambda2"] == r["lambda2"]
    o = oracle.Graph(hg, LT_WC, 0.0)
    o.stratify()
    ro = o.select_seeds(w.k, w.eps, w.ell, seed=0, instance=0)
    assert np.array_equal(rs[0]["seeds"], ro["seeds"]) and rs[0]["theta"] == ro["theta"]


def test_large_lt_sampled_sets_exact(hy):
    """large_lt (|V| = 1e6, |HE| = 2e6) as the benchmark runs it: both pools'
    ids [0, 4096) in one generation call; sampled ids, including the longest
    walks, regenerated one by one by the oracle, equal the library's sets and
    roots."""
    import concurrent.futures as cf
    import os
    _flush("[gpu] large_lt: generating the hypergraph")
    w = hypergen.workload("large_lt")
    hg = w.build()
    g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, w.model, w.p)
    g.stratify()
    ids = 4096
    pools = {tag: hy.Pool(g) for tag in (0, 1)}
    hy.generate_rr_batch([dict(graph=g, pool=pools[tag], seed=w.philox_seed, instance=0, pool_tag=tag,
                               id_begin=0, id_end=ids) for tag in (0, 1)])
    _flush("[gpu] large_lt: oracle graph and strata (about a minute)")
    o = oracle.Graph(hg, w.model, w.p)
    o.stratify()
    rng = np.random.default_rng(17)
    checks = []
    for tag in (0, 1):
        off, mem, roots = pools[tag].read()
        sizes = np.diff(off)
        big = [int(j) for j in np.argsort(sizes, kind="stable")[-4:]]
        pick = big + [int(j) for j in rng.choice(ids, size=12, replace=False) if int(j) not in big]
        for j in pick:
            checks.append((tag, j, mem[off[j]:off[j + 1]].copy(), int(roots[j])))
    threads = max(1, min(len(checks), int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        ref = list(ex.map(lambda c: (o.rr_set(w.philox_seed, 0, c[0], c[1]), o.root(w.philox_seed, 0, c[0], c[1])),
                          checks))
    for (tag, j, got, root), (want, wroot) in zip(checks, ref):
        assert root == wroot, (tag, j)
        assert np.array_equal(got, want), (tag, j, got.size, want.size)
