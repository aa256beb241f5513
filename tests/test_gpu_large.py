"""GPU parity at the large workload's full size (|V| = 1e6, |HE| = 2e6,
supercritical: giant RR sets of ~1e5 members).  The oracle cannot run the
whole query there, so the comparison is on quantities it can compute one by
one: every graph and strata array (full), and sampled RR ids -- including
giant sets -- regenerated individually on the CPU (keyed coins make each id
reproducible alone), in the launch configuration the library uses for the
query (both pools in one launch group)."""
import concurrent.futures as cf
import os
import sys

import numpy as np
import pytest

import hypergen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def large():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_01911_amd as hy
    hy.load_library()
    print("[gpu] large workload: generating", flush=True)
    w = hypergen.workload("large")
    hg = w.build()
    g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, w.model, w.p)
    o = oracle.Graph(hg, w.model, w.p)
    return hy, w, hg, g, o


def test_large_graph_and_strata_exact(large):
    hy, w, hg, g, o = large
    print("[gpu] large: graph arrays", flush=True)
    a, b = g.read(strata=False), o.arrays()
    for k in ("v_off", "v_he", "thr", "c"):
        assert np.array_equal(a[k], b[k]), k
    print("[gpu] large: strata (oracle stratify takes ~1 min)", flush=True)
    info = g.stratify()
    st = o.stratify()
    a = g.read()
    for k in ("l", "deg", "top", "stratum", "P"):
        assert np.array_equal(a[k], st[k]), k
    assert np.array_equal(info["B"], st["B"])


def test_large_sampled_rr_sets_exact(large):
    hy, w, hg, g, o = large
    if not o.stratified:
        o.stratify()
    if g.info is None:
        g.stratify()
    theta = 2048
    pools = {}
    for tag in (0, 1):
        print(f"[gpu] large: generating pool {tag}", flush=True)
        pools[tag] = hy.Pool(g)
        hy.generate_rr(g, w.philox_seed, 0, tag, 0, theta, pools[tag])
    rng = np.random.default_rng(7)
    checks = []
    for tag in (0, 1):
        off, mem, roots = pools[tag].read()
        sizes = np.diff(off)
        giant = np.nonzero(sizes > 50_000)[0]
        small = np.nonzero(sizes <= 50_000)[0]
        pick = list(rng.choice(giant, size=min(6, giant.size), replace=False)) + \
            list(rng.choice(small, size=min(10, small.size), replace=False))
        for j in pick:
            checks.append((tag, int(j), mem[off[j]:off[j + 1]].copy(), int(roots[j])))
    print(f"[gpu] large: {len(checks)} sampled ids on the CPU", flush=True)
    threads = max(1, min(len(checks), int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        ref = list(ex.map(lambda c: (o.rr_set(w.philox_seed, 0, c[0], c[1]), o.root(w.philox_seed, 0, c[0], c[1])),
                          checks))
    for (tag, j, got, root), (want, wroot) in zip(checks, ref):
        assert root == wroot, (tag, j)
        assert np.array_equal(got, want), (tag, j, got.size, want.size)


def test_large_bundled_mode_under_stored_tuning_exact(large):
    """The launch configuration the benchmark times on this workload: the
    stored tuning, whose bundled mode grows the sets of a graph that averages
    at least ms_min members per set in bundles of 64 (a graph not seen yet
    starts bundled and learns its members per set from that first group).
    Both pools' ids [0, 6144) in one generation call on a fresh graph handle.
    Sampled ids, including the largest sets, equal the oracle's sets and
    roots."""
    hy, w, hg, g, o = large
    from paper_2406_01911_amd import autotune
    if not o.stratified:
        o.stratify()
    tuning = autotune.load("large")
    assert tuning and tuning["ms_min"] < 0xFFFFFFFF
    g2 = hy.build_graph(hg.n, hg.he_off, hg.he_mem, w.model, w.p)
    g2.stratify()
    g2.set_tuning(**tuning)
    ids = 6144
    pools = {tag: hy.Pool(g2) for tag in (0, 1)}
    print(f"[gpu] large: both pools [0, {ids}) under the stored tuning", flush=True)
    hy.generate_rr_batch([dict(graph=g2, pool=pools[tag], seed=w.philox_seed, instance=0, pool_tag=tag,
                               id_begin=0, id_end=ids) for tag in (0, 1)])
    data = {tag: pools[tag].read() for tag in (0, 1)}
    off0 = data[0][0]
    learned = off0[2048] / 2048.0
    # the sets are large: bundled mode stays on after the first group
    assert learned >= tuning["ms_min"], learned
    rng = np.random.default_rng(11)
    checks = []
    for tag in (0, 1):
        off, mem, roots = data[tag]
        sizes = np.diff(off)
        lo = 2048 if tag == 0 else 0
        bundled = np.arange(lo, ids)
        big = list(bundled[np.argsort(sizes[lo:], kind="stable")[-4:]])
        pick = big + [int(j) for j in rng.choice(bundled, size=4, replace=False) if j not in big]
        if tag == 0:
            pick += [int(j) for j in rng.choice(2048, size=2, replace=False)]
        for j in pick:
            checks.append((tag, int(j), mem[off[j]:off[j + 1]].copy(), int(roots[j])))
    print(f"[gpu] large: {len(checks)} sampled ids on the CPU (learned {learned:.0f} members per set)", flush=True)
    threads = max(1, min(len(checks), int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        ref = list(ex.map(lambda c: (o.rr_set(w.philox_seed, 0, c[0], c[1]), o.root(w.philox_seed, 0, c[0], c[1])),
                          checks))
    for (tag, j, got, root), (want, wroot) in zip(checks, ref):
        assert root == wroot, (tag, j)
        assert np.array_equal(got, want), (tag, j, got.size, want.size)


def test_large_forms_identical_on_a_round(large):
    """Plain per-stratum launches and the persistent launch give the same bytes."""
    hy, w, hg, g, o = large
    if g.info is None:
        g.stratify()
    print("[gpu] large: plain vs persistent on one round", flush=True)
    a = hy.select_seeds(g, w.k, w.eps, w.ell, theta_fixed=1024, form=0)
    b = hy.select_seeds(g, w.k, w.eps, w.ell, theta_fixed=1024, form=1)
    assert np.array_equal(a["seeds"], b["seeds"]) and np.array_equal(a["gains"], b["gains"])
    assert a["lambda2"] == b["lambda2"] and a["entries1"] == b["entries1"] and a["entries2"] == b["entries2"]
