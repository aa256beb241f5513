"""GPU parity of the independent cascade drawn by geometric gaps (models 5
and 6): per (RR id, hyperedge, target) stream the kernels skip the dead
member positions with one Philox word per gap, and must reproduce the
oracle's sets bit for bit -- roots, RR sets (ascending members), and whole
HyperIM_BRR queries.  Cases cover the LDS and global visited bitmaps (|V|
above 32768), hyperedges long enough for many Philox blocks per stream,
p = 0 and p = 1, singleton and empty hyperedges, high RR ids, heavy vertices
split over a wave and over several waves of the grid-wide phase, sets
deferred to that phase almost at once (tiny budget), the plain form, and a
generation call that mixes coin and gap graphs."""
import sys

import numpy as np
import pytest

import hypergen
import oracle
from test_gpu_parity import _chain_with_hubs

pytestmark = pytest.mark.gpu

GAPS_CONST, GAPS_WC = 5, 6


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


CASES = {
    "tiny_gaps": lambda: (hypergen.workload("tiny_gaps").build(), GAPS_CONST, 0.05),
    "small_p03": lambda: (hypergen.tiny_hypergraph(21, 60, 80, 2, 6), GAPS_CONST, 0.3),
    "singletons_wc": lambda: (hypergen.tiny_hypergraph(5, 300, 500, 1, 8, allow_singletons=True), GAPS_WC, 0.0),
    "p_one": lambda: (hypergen.tiny_hypergraph(4, 200, 120, 1, 4, allow_singletons=True), GAPS_CONST, 1.0),
    "p_zero": lambda: (hypergen.tiny_hypergraph(4, 50, 40), GAPS_CONST, 0.0),
    "empty_edges": lambda: (hypergen.from_lists(6, [[], [2], [0, 1], [], [3, 4, 5], [1, 5]]), GAPS_CONST, 0.5),
    "one_vertex": lambda: (hypergen.from_lists(1, [[0], []]), GAPS_WC, 0.0),
    # streams of 1500 positions: many Philox blocks and long gaps per stream
    "big_edge": lambda: (hypergen.from_lists(3000, [list(range(0, 3000, 2)), list(range(1, 3000, 3)),
                                                     list(range(5, 1200))]), GAPS_CONST, 0.002),
    # a hub in 9999 hyperedges: its incidences are split over the wave
    "hub": lambda: (hypergen.from_lists(10001, [[0, i, i + 1] for i in range(1, 10000)]), GAPS_CONST, 0.2),
    "chain_hubs_40000": lambda: (_chain_with_hubs(), GAPS_CONST, 0.75),
}


def _same_sets(hy, g, o, seed, instance, pool_tag, lo, hi):
    pool = hy.Pool(g)
    hy.generate_rr(g, seed, instance, pool_tag, lo, hi, pool)
    off, mem, roots = pool.read()
    roff, rmem, rroots = o.generate(seed, instance, pool_tag, lo, hi)
    assert np.array_equal(roots, rroots)
    assert np.array_equal(off, roff)
    assert np.array_equal(mem, rmem)
    return off, mem, roots


@pytest.mark.parametrize("case", sorted(CASES))
def test_gap_rr_sets_bit_exact(hy, case):
    _flush(f"[gpu] gap sampler rr sets case={case}")
    hg, model, p = CASES[case]()
    g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, model, p)
    o = oracle.Graph(hg, model, p)
    a, b = g.read(strata=False), o.arrays()
    for k in ("v_off", "v_he", "thr", "c"):
        assert np.array_equal(a[k], b[k]), k
    g.stratify()
    o.stratify()
    for pool_tag, (lo, hi) in [(0, (0, 700)), (1, (150, 450)), (0, ((1 << 33) - 64, (1 << 33) + 64))]:
        off, mem, roots = _same_sets(hy, g, o, 7, 3, pool_tag, lo, hi)
    if case == "p_one":   # every co-member is live: sets are whole components
        assert off[-1] > hi - lo
    if case == "p_zero":
        assert np.array_equal(np.diff(off), np.ones(hi - lo, np.int64))


def test_gap_sets_deferred_to_grid_phase_bit_exact(hy):
    """Sets deferred to the grid-wide phase almost at once (tiny budget and
    heavy threshold, 16-incidence chunks): the gap streams of items shared
    by several waves, continuation levels and heavy chunks."""
    _flush("[gpu] gap sampler grid-wide phase")
    hg = _chain_with_hubs()
    g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, GAPS_CONST, 0.75)
    o = oracle.Graph(hg, GAPS_CONST, 0.75)
    g.stratify()
    o.stratify()
    g.set_tuning(budget=8, heavy=8, chunk=16, seg=16, steps_per_sync=3)
    for pool_tag, (lo, hi) in [(0, (0, 600)), (1, (100, 400))]:
        off, _, _ = _same_sets(hy, g, o, 5, 2, pool_tag, lo, hi)
        assert off[-1] > 5 * (hi - lo)   # the sets are not trivial


def test_gap_queries_match_oracle(hy):
    """tiny_gaps and mid_gaps (|V| = 1e5, global bitmaps, weighted cascade):
    a generation call's sets and the whole query in the persistent and the
    plain form, for both upper bounds."""
    for name in ("tiny_gaps", "mid_gaps"):
        _flush(f"[gpu] gap sampler query {name}")
        w = hypergen.workload(name)
        hg = w.build()
        g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, w.model, w.p)
        o = oracle.Graph(hg, w.model, w.p)
        g.stratify()
        o.stratify()
        _same_sets(hy, g, o, w.philox_seed, 0, 1, 0, 4096)
        for bound in (0, 1):
            ro = o.select_seeds(w.k, w.eps, w.ell, seed=w.philox_seed, bound=bound)
            for form in (0, 1):
                r = hy.select_seeds(g, w.k, w.eps, w.ell, seed=w.philox_seed, form=form, bound=bound)
                for key in ("rounds", "theta", "lambda1", "lambda2", "entries1", "entries2", "lambda_u"):
                    assert r[key] == ro[key], (name, bound, form, key, r[key], ro[key])
                assert np.array_equal(r["seeds"], ro["seeds"]) and np.array_equal(r["gains"], ro["gains"])


def test_gap_and_coin_graphs_in_one_generation_call(hy):
    """Tasks of gap graphs and coin graphs in one call run in separate launch
    groups; every pool equals the oracle's."""
    _flush("[gpu] gap + coin graphs in one call")
    hg = hypergen.tiny_hypergraph(61, 3000, 4000, 2, 6)
    graphs = []
    for model, p in ((GAPS_CONST, 0.1), (0, 0.1), (GAPS_WC, 0.0)):
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
            tasks.append(dict(graph=g, pool=pl, seed=4, instance=i, pool_tag=tag, id_begin=0, id_end=1200))
    hy.generate_rr_batch(tasks)
    for pl, o, tag, i in pools:
        off, mem, roots = pl.read()
        roff, rmem, rroots = o.generate(4, i, tag, 0, 1200)
        assert np.array_equal(roots, rroots) and np.array_equal(off, roff) and np.array_equal(mem, rmem), (i, tag)


def test_gap_graph_rejects_nan_and_unknown_model(hy):
    hg = hypergen.from_lists(3, [[0, 1]])
    with pytest.raises(hy.HyperIMError):
        hy.build_graph(hg.n, hg.he_off, hg.he_mem, 7, 0.1)
    with pytest.raises(hy.HyperIMError):
        hy.build_graph(hg.n, hg.he_off, hg.he_mem, GAPS_CONST, float("nan"))
    with pytest.raises(hy.HyperIMError):
        hy.build_graph(hg.n, hg.he_off, hg.he_mem, GAPS_CONST, -0.5)


def test_large_gaps_sampled_sets_under_stored_tuning_exact(hy):
    """The launch configuration the benchmark times on large_gaps (|V| = 1e6,
    |HE| = 2e6, giant sets of ~1e5 members): its stored tuning, both pools'
    ids [0, 4096) in one generation call.  Sampled ids, including the largest
    sets, regenerated one by one by the oracle (each id depends only on its
    key), equal the library's sets and roots."""
    import concurrent.futures as cf
    import os
    from paper_2406_01911_amd import autotune
    _flush("[gpu] large_gaps: generating the hypergraph")
    w = hypergen.workload("large_gaps")
    hg = w.build()
    g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, w.model, w.p)
    g.stratify()
    tuning = autotune.load("large_gaps")
    assert tuning is not None
    g.set_tuning(**tuning)
    _flush(f"[gpu] large_gaps: tuning {tuning}")
    ids = 4096
    pools = {tag: hy.Pool(g) for tag in (0, 1)}
    _flush(f"[gpu] large_gaps: both pools [0, {ids}) under the stored tuning")
    hy.generate_rr_batch([dict(graph=g, pool=pools[tag], seed=w.philox_seed, instance=0, pool_tag=tag,
                               id_begin=0, id_end=ids) for tag in (0, 1)])
    _flush("[gpu] large_gaps: oracle graph and strata (about a minute)")
    o = oracle.Graph(hg, w.model, w.p)
    o.stratify()
    rng = np.random.default_rng(13)
    checks = []
    for tag in (0, 1):
        off, mem, roots = pools[tag].read()
        sizes = np.diff(off)
        assert sizes.max() > 50_000   # giant sets are generated and checked
        big = [int(j) for j in np.argsort(sizes, kind="stable")[-3:]]
        pick = big + [int(j) for j in rng.choice(ids, size=5, replace=False) if int(j) not in big]
        for j in pick:
            checks.append((tag, j, mem[off[j]:off[j + 1]].copy(), int(roots[j])))
    _flush(f"[gpu] large_gaps: {len(checks)} sampled ids on the CPU")
    threads = max(1, min(len(checks), int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        ref = list(ex.map(lambda c: (o.rr_set(w.philox_seed, 0, c[0], c[1]), o.root(w.philox_seed, 0, c[0], c[1])),
                          checks))
    for (tag, j, got, root), (want, wroot) in zip(checks, ref):
        assert root == wroot, (tag, j)
        assert np.array_equal(got, want), (tag, j, got.size, want.size)
