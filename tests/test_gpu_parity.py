"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs.  Integer and index work must be bit-exact: graph
arrays, strata, roots, every RR set (ascending members), greedy seeds and
gains, coverage counts, the doubling loop's theta / rounds / Lambda1 / Lambda2.
Floating statistics (alpha, beta, theta(l*)) agree to 1e-12 relative (device
log and summation order differ only in the last bits)."""
import os
import sys

import numpy as np
import pytest

import hypergen
import oracle

pytestmark = pytest.mark.gpu


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


def _pair(hy, hg, model, p):
    g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, model, p)
    o = oracle.Graph(hg, model, p)
    return g, o


def _check_graph(g, o):
    a, b = g.read(strata=False), o.arrays()
    for k in ("v_off", "v_he", "thr", "c"):
        assert np.array_equal(a[k], b[k]), k


def hy_n(info):
    return int(info["B"][-1])


def _check_strata(g, o):
    info = g.stratify()
    st = o.stratify()
    a = g.read()
    for k in ("l", "deg", "top", "stratum", "P"):
        assert np.array_equal(a[k], st[k]), k
    assert np.array_equal(info["B"], st["B"])
    assert info["alpha"] == pytest.approx(st["alpha"], rel=1e-12)
    assert info["beta"] == pytest.approx(st["beta"], rel=1e-12)
    # theta(l*) is a sum of n doubles: the oracle adds them in vertex order, the
    # library groups them by value; recursive summation differs by at most
    # about n * 2^-52 relative
    tol = max(1e-14, hy_n(info) * 2.0 ** -52)
    assert info["theta_l"] == pytest.approx(st["theta_l"], rel=tol)


CASES = {
    "tiny": lambda: (hypergen.workload("tiny").build(), 0, 0.05),
    "small_p03": lambda: (hypergen.tiny_hypergraph(21, 60, 80, 2, 6), 0, 0.3),
    "singletons_wc": lambda: (hypergen.tiny_hypergraph(5, 300, 500, 1, 8, allow_singletons=True), 1, 0.0),
    "p_one": lambda: (hypergen.tiny_hypergraph(4, 200, 120, 1, 4, allow_singletons=True), 0, 1.0),
    "p_zero": lambda: (hypergen.tiny_hypergraph(4, 50, 40), 0, 0.0),
    "empty_edges": lambda: (hypergen.from_lists(6, [[], [2], [0, 1], [], [3, 4, 5], [1, 5]]), 0, 0.5),
    "one_vertex": lambda: (hypergen.from_lists(1, [[0], []]), 0, 0.5),
    "big_edge": lambda: (hypergen.from_lists(3000, [list(range(0, 3000, 2)), list(range(1, 3000, 3)),
                                                     list(range(5, 1200))]), 0, 0.002),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_graph_strata_and_rr_sets_bit_exact(hy, case):
    _flush(f"[gpu] graph/strata/rr case={case}")
    hg, model, p = CASES[case]()
    g, o = _pair(hy, hg, model, p)
    _check_graph(g, o)
    _check_strata(g, o)
    for pool_tag, (a, b) in [(0, (0, 700)), (1, (0, 300))]:
        pool = hy.Pool(g)
        hy.generate_rr(g, 7, 3, pool_tag, a, b, pool)
        off, mem, roots = pool.read()
        roff, rmem, rroots = o.generate(7, 3, pool_tag, a, b)
        assert np.array_equal(roots, rroots)
        assert np.array_equal(off, roff)
        assert np.array_equal(mem, rmem)


def _chain_with_hubs(n=40000, hubs=12, per_hub=40, seed=17):
    """A path {i, i+1} over n vertices (long thin traversals) plus hubs that
    sit in many 3-member hyperedges (heavy vertices for small chunk sizes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    edges = [[i, i + 1] for i in range(n - 1)]
    for h in rng.choice(n, size=hubs, replace=False):
        for _ in range(per_hub):
            a, b = rng.choice(n, size=2, replace=False)
            if h not in (a, b):
                edges.append([int(h), int(a), int(b)])
    return hypergen.from_lists(n, edges)


@pytest.mark.parametrize("prefilter", [1 << 30, 1])
def test_grid_phase_chains_bit_exact(hy, prefilter):
    """Sets deferred to the grid-wide phase almost at once (tiny budget and
    heavy threshold, 16-incidence chunks): thin traversals many levels deep,
    expanded by shared items, continuation and heavy chunks, must equal the
    oracle's sets member for member."""
    _flush(f"[gpu] grid-wide phase chains prefilter={prefilter}")
    hg = _chain_with_hubs()
    g, o = _pair(hy, hg, 0, 0.75)
    g.stratify()
    o.stratify()
    g.set_tuning(budget=8, heavy=8, chunk=16, seg=16, prefilter_min=prefilter, steps_per_sync=3)
    for pool_tag, (a, b) in [(0, (0, 600)), (1, (100, 400))]:
        pool = hy.Pool(g)
        hy.generate_rr(g, 5, 2, pool_tag, a, b, pool)
        off, mem, roots = pool.read()
        roff, rmem, rroots = o.generate(5, 2, pool_tag, a, b)
        assert np.array_equal(roots, rroots)
        assert np.array_equal(off, roff)
        assert np.array_equal(mem, rmem)
        assert off[-1] > 5 * (b - a)   # the sets are not trivial


@pytest.mark.parametrize("case", sorted(CASES))
def test_bundled_mode_bit_exact(hy, case):
    """Sets grown in bundles of 64, bit-parallel over the sets (forced here by
    a members-per-set threshold of 1, which also starts a graph not seen yet
    in bundled mode), appended over two calls, equal the oracle's."""
    _flush(f"[gpu] bundled case={case}")
    hg, model, p = CASES[case]()
    g, o = _pair(hy, hg, model, p)
    g.stratify()
    o.stratify()
    g.set_tuning(ms_min=1)
    for pool_tag, (a, b) in [(0, (0, 2048 + 333)), (1, (100, 2048 + 100 + 130))]:
        pool = hy.Pool(g)
        hy.generate_rr(g, 7, 3, pool_tag, a, b, pool)
        hy.generate_rr(g, 7, 3, pool_tag, b, b + 200, pool)
        off, mem, roots = pool.read()
        roff, rmem, rroots = o.generate(7, 3, pool_tag, a, b + 200)
        assert np.array_equal(roots, rroots)
        assert np.array_equal(off, roff)
        assert np.array_equal(mem, rmem)


def test_bundled_select_matches_oracle(hy):
    _flush("[gpu] bundled select tiny / mid rr sets")
    w = hypergen.workload("tiny")
    hg = w.build()
    g, o = _pair(hy, hg, w.model, w.p)
    g.stratify()
    o.stratify()
    g.set_tuning(ms_min=1)
    hy.select_seeds(g, w.k, w.eps, w.ell)        # learns the members per set
    r = hy.select_seeds(g, w.k, w.eps, w.ell)
    ro = o.select_seeds(w.k, w.eps, w.ell)
    for key in ("rounds", "theta", "lambda1", "lambda2", "entries1", "entries2"):
        assert r[key] == ro[key], key
    assert np.array_equal(r["seeds"], ro["seeds"]) and np.array_equal(r["gains"], ro["gains"])
    wm = hypergen.workload("mid")
    hm = wm.build()
    gm, om = _pair(hy, hm, wm.model, wm.p)
    gm.stratify()
    om.stratify()
    gm.set_tuning(ms_min=1)
    pool = hy.Pool(gm)
    hy.generate_rr(gm, 0, 0, 0, 0, 2048 + 952, pool)
    off, mem, roots = pool.read()
    roff, rmem, rroots = om.generate(0, 0, 0, 0, 3000)
    assert np.array_equal(off, roff) and np.array_equal(mem, rmem) and np.array_equal(roots, rroots)


def test_append_across_ladder_blocks(hy):
    _flush("[gpu] append across ladder blocks")
    hg = hypergen.workload("tiny").build()
    g, o = _pair(hy, hg, 0, 0.05)
    g.stratify()
    o.stratify()
    pool = hy.Pool(g)
    for a, b in [(0, 100), (100, 256), (256, 700), (700, 1500)]:
        hy.generate_rr(g, 11, 0, 1, a, b, pool)
    off, mem, roots = pool.read()
    roff, rmem, rroots = o.generate(11, 0, 1, 0, 1500)
    assert np.array_equal(off, roff) and np.array_equal(mem, rmem) and np.array_equal(roots, rroots)
    # a pool only grows at its end, with its own key
    with pytest.raises(hy.HyperIMError):
        hy.generate_rr(g, 11, 0, 1, 1600, 1700, pool)
    with pytest.raises(hy.HyperIMError):
        hy.generate_rr(g, 12, 0, 1, 1500, 1600, pool)


def test_offset_start_and_high_ids(hy):
    _flush("[gpu] high ids")
    hg = hypergen.tiny_hypergraph(21, 60, 80, 2, 6)
    g, o = _pair(hy, hg, 0, 0.3)
    g.stratify()
    o.stratify()
    for a in [5000, (1 << 32) - 100, (1 << 38) + 12345]:
        pool = hy.Pool(g)
        hy.generate_rr(g, 99, 5, 0, a, a + 200, pool)
        off, mem, roots = pool.read()
        roff, rmem, rroots = o.generate(99, 5, 0, a, a + 200)
        assert np.array_equal(off, roff) and np.array_equal(mem, rmem) and np.array_equal(roots, rroots)


def test_mid_workload_rr_sets_bit_exact(hy):
    _flush("[gpu] mid workload rr sets")
    w = hypergen.workload("mid")
    hg = w.build()
    g, o = _pair(hy, hg, w.model, w.p)
    _check_graph(g, o)
    _check_strata(g, o)
    pool = hy.Pool(g)
    hy.generate_rr(g, 0, 0, 0, 0, 3000, pool)
    off, mem, roots = pool.read()
    roff, rmem, rroots = o.generate(0, 0, 0, 0, 3000)
    assert np.array_equal(off, roff) and np.array_equal(mem, rmem) and np.array_equal(roots, rroots)


@pytest.mark.parametrize("case", ["tiny", "small_p03", "singletons_wc"])
def test_greedy_and_coverage_bit_exact(hy, case):
    _flush(f"[gpu] greedy case={case}")
    hg, model, p = CASES[case]()
    g, o = _pair(hy, hg, model, p)
    g.stratify()
    o.stratify()
    pool = hy.Pool(g)
    hy.generate_rr(g, 1, 0, 0, 0, 2048, pool)
    off, mem, _ = pool.read()
    for k in (1, 5, min(40, hg.n)):
        for theta in (2048, 1000):
            s, gn = hy.greedy(g, pool, theta, k)
            rs, rg = oracle.greedy(hg.n, off, mem, k, theta=theta)
            assert np.array_equal(s, rs) and np.array_equal(gn, rg), (k, theta)
            assert hy.coverage(g, pool, theta, s) == oracle.coverage(hg.n, off, mem, s, theta=theta)


def test_greedy_graph_replays(hy):
    """The k greedy rounds run as one captured graph, replayed with new
    arguments: thetas of one grid shape reuse it, with eager work (coverage,
    generation into another pool) between the replays; every replay must
    equal the oracle."""
    _flush("[gpu] greedy graph replays")
    hg, model, p = CASES["small_p03"]()
    g, o = _pair(hy, hg, model, p)
    g.stratify()
    pool = hy.Pool(g)
    other = hy.Pool(g)
    hy.generate_rr(g, 3, 1, 0, 0, 2048, pool)
    off, mem, _ = pool.read()
    k = min(12, hg.n)
    for i, theta in enumerate((2048, 1900, 2048, 1800, 2048)):
        s, gn = hy.greedy(g, pool, theta, k)
        rs, rg = oracle.greedy(hg.n, off, mem, k, theta=theta)
        assert np.array_equal(s, rs) and np.array_equal(gn, rg), (i, theta)
        assert hy.coverage(g, pool, theta, s) == oracle.coverage(hg.n, off, mem, s, theta=theta)
        hy.generate_rr(g, 5, 0, 1, 256 * i, 256 * (i + 1), other)


def test_select_seeds_tiny_matches_oracle(hy):
    _flush("[gpu] select tiny")
    w = hypergen.workload("tiny")
    hg = w.build()
    g, o = _pair(hy, hg, w.model, w.p)
    g.stratify()
    o.stratify()
    for form in (0, 1):
        r = hy.select_seeds(g, w.k, w.eps, w.ell, form=form)
        ro = o.select_seeds(w.k, w.eps, w.ell)
        for key in ("rounds", "theta", "lambda1", "lambda2", "entries1", "entries2", "i_max"):
            assert r[key] == ro[key], key
        assert np.array_equal(r["seeds"], ro["seeds"]) and np.array_equal(r["gains"], ro["gains"])
        assert r["sigma_l"] == pytest.approx(ro["sigma_l"], rel=1e-12)
        assert r["sigma_u"] == pytest.approx(ro["sigma_u"], rel=1e-12)
    rf = hy.select_seeds(g, w.k, w.eps, w.ell, theta_fixed=4096)
    rof = o.select_seeds(w.k, w.eps, w.ell, theta_fixed=4096)
    assert np.array_equal(rf["seeds"], rof["seeds"]) and rf["lambda2"] == rof["lambda2"]


def test_select_seeds_mid_matches_oracle(hy):
    _flush("[gpu] select mid")
    w = hypergen.workload("mid")
    hg = w.build()
    g, o = _pair(hy, hg, w.model, w.p)
    g.stratify()
    o.stratify()
    r = hy.select_seeds(g, w.k, w.eps, w.ell, flags=hy.FLAG_INCIDENCES)
    ro = o.select_seeds(w.k, w.eps, w.ell)
    for key in ("rounds", "theta", "lambda1", "lambda2", "entries1", "entries2"):
        assert r[key] == ro[key], key
    assert np.array_equal(r["seeds"], ro["seeds"]) and np.array_equal(r["gains"], ro["gains"])
    assert r["incidences"] > 0


def test_plain_and_persistent_forms_identical(hy):
    _flush("[gpu] plain vs persistent")
    w = hypergen.workload("mid")
    hg = w.build()
    g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, w.model, w.p)
    g.stratify()
    a = hy.select_seeds(g, w.k, w.eps, w.ell, form=0, theta_fixed=8192)
    b = hy.select_seeds(g, w.k, w.eps, w.ell, form=1, theta_fixed=8192)
    c = hy.select_seeds(g, w.k, w.eps, w.ell, form=0, theta_fixed=8192)
    for x in (b, c):
        assert np.array_equal(a["seeds"], x["seeds"]) and np.array_equal(a["gains"], x["gains"])
        assert a["lambda2"] == x["lambda2"] and a["entries1"] == x["entries1"]


def test_invalid_graphs_rejected(hy):
    _flush("[gpu] invalid graphs")
    bad = [
        (5, [[0, 5]]),          # id >= n
        (3, [[0, 1, 0]]),       # duplicate member
    ]
    for n, edges in bad:
        hg = hypergen.from_lists(n, edges)
        with pytest.raises(hy.HyperIMError) as e:
            hy.build_graph(n, hg.he_off, hg.he_mem, 0, 0.1)
        assert e.value.status == hy.EINVAL
    with pytest.raises(hy.HyperIMError) as e:
        hy.build_graph(3, np.array([0, 2, 1], np.uint32), np.array([0, 1], np.uint32), 0, 0.1)
    assert e.value.status == hy.EINVAL
    # a hub whose duplicate is only visible through the bitmap sort path
    edges = [[0, u] for u in range(1, 5001)] + [[0, 7, 0]]
    hg = hypergen.from_lists(5001, edges)
    with pytest.raises(hy.HyperIMError):
        hy.build_graph(5001, hg.he_off, hg.he_mem, 0, 0.1)


def test_state_and_capacity_errors(hy):
    _flush("[gpu] state/capacity")
    import torch
    hg = hypergen.workload("tiny").build()
    g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, 0, 0.05)
    pool = hy.Pool(g)
    with pytest.raises(hy.HyperIMError) as e:
        hy.generate_rr(g, 0, 0, 0, 0, 10, pool)
    assert e.value.status == hy.ESTATE
    g.stratify()
    buf = torch.empty(4096, dtype=torch.uint8, device="cuda")
    small = hy.Pool(g, buf=buf, id_capacity=64)
    with pytest.raises(hy.HyperIMError) as e:
        hy.generate_rr(g, 0, 0, 0, 0, 64, small)
    assert e.value.status == hy.ECAPACITY
    need = small.required()
    assert need > 4096
    big = torch.empty(need, dtype=torch.uint8, device="cuda")
    ok = hy.Pool(g, buf=big, id_capacity=64)
    hy.generate_rr(g, 0, 0, 0, 0, 64, ok)
    o = oracle.Graph(hg, 0, 0.05)
    o.stratify()
    off, mem, roots = ok.read()
    roff, rmem, rroots = o.generate(0, 0, 0, 0, 64)
    assert np.array_equal(off, roff) and np.array_equal(mem, rmem)
    with pytest.raises(hy.HyperIMError):
        hy.greedy(g, ok, 64, 0)
    with pytest.raises(hy.HyperIMError):
        hy.greedy(g, ok, 65, 3)
