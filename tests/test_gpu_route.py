"""GPU parity of the division of the RR sets into R1 and R2 (Section 4.1):
after hyperim_route, pool 0 draws its roots from the vertices with a small
layer and starts each set from the root and those layers' members, pool 1
draws from the other vertices.  The library's roots and RR sets equal the
oracle's bit for bit -- per-set and bundled mode, sets deferred to the
grid-wide phase, LDS and global visited bitmaps, coins and gaps -- and so do
whole HyperIM_BRR queries.  Error and state rules of the entry point."""
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


CASES = {
    "tiny": lambda: (hypergen.workload("tiny").build(), 0, 0.05),
    "small_wc": lambda: (hypergen.tiny_hypergraph(3, 80, 120, 2, 7), 1, 0.0),
    "small_singletons": lambda: (hypergen.tiny_hypergraph(8, 150, 90, 2, 9, allow_singletons=True), 0, 0.3),
    "small_gaps": lambda: (hypergen.tiny_hypergraph(3, 80, 120, 2, 7), 5, 0.2),
    # |V| = 1e5: global visited bitmaps
    "mid_wc": lambda: (hypergen.workload("mid").build(), 1, 0.0),
}


def _routed_pair(hy, hg, model, p):
    g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, model, p)
    o = oracle.Graph(hg, model, p)
    g.stratify()
    o.stratify()
    n1 = g.route()
    assert n1 == o.route()
    return g, o, n1


def _same(hy, g, o, seed, inst, tag, lo, hi):
    pool = hy.Pool(g)
    hy.generate_rr(g, seed, inst, tag, lo, hi, pool)
    off, mem, roots = pool.read()
    roff, rmem, rroots = o.generate(seed, inst, tag, lo, hi)
    assert np.array_equal(roots, rroots)
    assert np.array_equal(off, roff)
    assert np.array_equal(mem, rmem)
    return off, mem, roots


@pytest.mark.parametrize("case", sorted(CASES))
def test_routed_rr_sets_bit_exact(hy, case):
    _flush(f"[gpu] divided RR sets case={case}")
    hg, model, p = CASES[case]()
    g, o, n1 = _routed_pair(hy, hg, model, p)
    assert 0 < n1 < hg.n
    rP, f_off, _ = o.route_tables()
    r1 = set(rP[:n1].tolist())
    for tag, (lo, hi) in [(0, (0, 700)), (1, (0, 700)), (0, (300, 900)), (1, ((1 << 33) - 64, (1 << 33) + 64))]:
        off, mem, roots = _same(hy, g, o, 7, 3, tag, lo, hi)
        assert all((r in r1) == (tag == 0) for r in roots.tolist())


def test_routed_bundled_and_deferred_bit_exact(hy):
    """Bundled mode (forced by a members-per-set threshold of 1) seeds the
    forced members at level 0; a tiny per-set budget sends sets with forced
    members through the grid-wide phase."""
    hg, model, p = CASES["mid_wc"]()
    for tuning in (dict(ms_min=1), dict(budget=8, heavy=8, chunk=16, seg=16, steps_per_sync=3)):
        _flush(f"[gpu] divided RR sets under {tuning}")
        g, o, _ = _routed_pair(hy, hg, model, p)
        g.set_tuning(**tuning)
        for tag in (0, 1):
            _same(hy, g, o, 5, 2, tag, 0, 640)


def test_routed_queries_match_oracle(hy):
    """tiny: the whole query (it stops after one round); mid: one round at a
    fixed theta -- divided, mid's bounds never pass the stop test before
    theta_max (R1's forced members inflate sigma_u about twofold), so the
    whole query would run to the last admissible round."""
    for name, theta in (("tiny", 0), ("mid", 2048)):
        _flush(f"[gpu] divided query {name}")
        w = hypergen.workload(name)
        hg = w.build()
        g, o, n1 = _routed_pair(hy, hg, w.model, w.p)
        assert 0 < n1 < hg.n
        ro = o.select_seeds(w.k, w.eps, w.ell, seed=w.philox_seed, theta_fixed=theta)
        for form in (0, 1):
            r = hy.select_seeds(g, w.k, w.eps, w.ell, seed=w.philox_seed, form=form, theta_fixed=theta)
            for key in ("rounds", "theta", "lambda1", "lambda2", "entries1", "entries2", "lambda_u"):
                assert r[key] == ro[key], (name, form, key, r[key], ro[key])
            assert np.array_equal(r["seeds"], ro["seeds"]) and np.array_equal(r["gains"], ro["gains"])


def test_route_state_rules(hy):
    _flush("[gpu] divided RR sets: state rules")
    hg, model, p = CASES["small_wc"]()
    # linear threshold and the stratified setting are refused
    for m in (2, 3, 4):
        gl = hy.build_graph(hg.n, hg.he_off, hg.he_mem, m, 0.1)
        gl.stratify()
        with pytest.raises(hy.HyperIMError) as e:
            gl.route()
        assert e.value.status == hy.EINVAL
    g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, model, p)
    with pytest.raises(hy.HyperIMError) as e:   # not stratified
        g.route()
    assert e.value.status == hy.ESTATE
    g.stratify()
    o = oracle.Graph(hg, model, p)
    o.stratify()
    g.route()
    g.route(False)   # undone before any set: the plain pools
    _same(hy, g, o, 1, 0, 0, 0, 300)
    with pytest.raises(hy.HyperIMError) as e:   # sets exist now
        g.route()
    assert e.value.status == hy.ESTATE
    # a re-stratified divided graph keeps its division
    g2, o2, _ = _routed_pair(hy, hg, model, p)
    g2.stratify()
    _same(hy, g2, o2, 2, 0, 0, 0, 300)
    # inert: no vertex has a small layer
    hi_ = hypergen.from_lists(4, [[0, 1, 2, 3]])
    g3 = hy.build_graph(hi_.n, hi_.he_off, hi_.he_mem, 0, 0.3)
    o3 = oracle.Graph(hi_, 0, 0.3)
    g3.stratify()
    o3.stratify()
    assert g3.route() == o3.route()
    _same(hy, g3, o3, 0, 0, 0, 0, 64)
