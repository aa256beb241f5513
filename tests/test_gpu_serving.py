"""GPU: the serving loop and the autotuner.  Every query served in the mix
(Poisson arrivals, continuous batching, resident pools shared by queries on
one graph) returns exactly what it returns alone; every tuning candidate
returns the baseline's bytes."""
import sys

import numpy as np
import pytest

import hypergen

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


def test_serving_mix_equals_alone(hy):
    from paper_2406_01911_amd import serving
    _flush("[gpu] serving mix")
    ws = hypergen.serving_workloads(4, n_max=40000, n_min=3000)
    graphs = []
    for w in ws:
        hg = w.build()
        g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, w.model, w.p)
        g.stratify()
        graphs.append(g)
    queries = serving.draw_queries(24, len(graphs), ks=(5, 10, 20), eps=0.3, seed=4)
    arrivals = serving.poisson_arrivals(len(queries), 400.0, seed=4)
    run = serving.serve(graphs, queries, arrivals)
    s = run["summary"]
    assert s["failed"] == 0 and s["queries"] == 24 and s["p50_ms"] <= s["p99_ms"]
    assert s["max_in_flight"] > 1   # queries overlapped
    for i, (q, r) in enumerate(zip(queries, run["results"])):
        a = hy.select_seeds(graphs[q["graph"]], q["k"], q["eps"], q["ell"], seed=q["seed"], instance=q["instance"])
        for key in ("theta", "rounds", "lambda1", "lambda2", "entries1", "entries2"):
            assert a[key] == r[key], (i, key)
        assert np.array_equal(a["seeds"], r["seeds"]) and np.array_equal(a["gains"], r["gains"]), i


def test_autotune_keeps_bytes(hy):
    from paper_2406_01911_amd import autotune
    _flush("[gpu] autotune")
    w = hypergen.workload("tiny")
    hg = w.build()
    g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, w.model, w.p)
    g.stratify()
    base = hy.select_seeds(g, w.k, w.eps, w.ell, theta_fixed=4096)
    space = {"heavy": [8, 1024], "budget": [64, 16384], "chunk": [16, 256], "steps_per_sync": [1, 8]}
    res = autotune.autotune(g, w.k, w.eps, w.ell, theta=4096, space=space, reps=1, sweeps=1)
    assert len(res["trials"]) >= 4 and res["ms_rr"] > 0
    assert g.tuning()["heavy"] == res["tuning"]["heavy"]
    r = hy.select_seeds(g, w.k, w.eps, w.ell, theta_fixed=4096)
    assert np.array_equal(r["seeds"], base["seeds"]) and r["lambda2"] == base["lambda2"]
