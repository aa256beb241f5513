"""GPU parity of the batched and serving forms.

Every query answered in a batch (RR generation of all instances, strata and
both pools in shared launches) or in a serving session (queries joining while
others run, admission by an HBM budget) must return exactly what the same
query returns alone -- seeds, gains, theta, rounds, Lambda1, Lambda2, pool
entries -- and, on inputs the oracle finishes in seconds, exactly what the
oracle returns."""
import sys

import numpy as np
import pytest

import hypergen
import oracle

pytestmark = pytest.mark.gpu

KEYS = ("rounds", "theta", "lambda1", "lambda2", "entries1", "entries2", "i_max")


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


def _same(a, b, what=""):
    for key in KEYS:
        assert a[key] == b[key], (what, key, a[key], b[key])
    assert np.array_equal(a["seeds"], b["seeds"]), what
    assert np.array_equal(a["gains"], b["gains"]), what
    assert a["sigma_l"] == pytest.approx(b["sigma_l"], rel=1e-12)
    assert a["sigma_u"] == pytest.approx(b["sigma_u"], rel=1e-12)


# Small mixed instances: one above 32768 vertices (visited marks in HBM rather
# than LDS), one of WC model, size and probability mix; subcritical so that
# the oracle finishes every query in seconds.
SMALL = [
    # n, m, sizes, model, p, k, eps, seed, instance
    (800, 1600, ("powerlaw", 2.5, 2, 20), 0, 0.03, 5, 0.5, 0, 0),
    (3000, 6000, ("powerlaw", 2.5, 2, 30), 0, 0.02, 10, 0.4, 7, 1),
    (40000, 80000, ("powerlaw", 2.5, 2, 20), 0, 0.01, 20, 0.5, 0, 2),
    (2000, 4000, ("uniform", 2, 6), 1, 0.0, 10, 0.3, 3, 3),
    (1500, 1000, ("powerlaw", 2.2, 2, 100), 0, 0.005, 8, 0.5, 0, 4),
    (1000, 2000, ("uniform", 2, 6), 0, 0.05, 10, 0.5, 0, 5),
]


@pytest.fixture(scope="module")
def small(hy):
    out = []
    for i, (n, m, sizes, model, p, k, eps, seed, inst) in enumerate(SMALL):
        hg = hypergen.make_hypergraph(n, m, sizes, ("uniform",), 500 + i)
        g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, model, p)
        g.stratify()
        out.append(dict(hg=hg, g=g, model=model, p=p, k=k, eps=eps, ell=1.0, seed=seed, instance=inst))
    return out


def _q(c, **over):
    d = dict(graph=c["g"], k=c["k"], eps=c["eps"], ell=c["ell"], seed=c["seed"], instance=c["instance"])
    d.update(over)
    return d


def test_batch_matches_alone_and_oracle(hy, small):
    _flush("[gpu] batch small instances")
    alone = [hy.select_seeds(c["g"], c["k"], c["eps"], c["ell"], seed=c["seed"], instance=c["instance"])
             for c in small]
    for form in (0, 1):
        batch = hy.select_seeds_batch([_q(c) for c in small], form=form)
        for i, (a, b) in enumerate(zip(alone, batch)):
            assert b["status"] == hy.OK
            _same(a, b, f"instance {i} form {form}")
    for i, c in enumerate(small):
        o = oracle.Graph(c["hg"], c["model"], c["p"])
        o.stratify()
        ro = o.select_seeds(c["k"], c["eps"], c["ell"], seed=c["seed"], instance=c["instance"])
        _same(alone[i], ro, f"oracle instance {i}")


def test_generate_ahead_keeps_results(hy, small):
    """Rounds that also generate the ids of later rounds (options.ahead) return
    the same bytes as rounds that generate exactly their own ids."""
    _flush("[gpu] generate ahead")
    for i, c in enumerate(small):
        off = hy.select_seeds(c["g"], c["k"], c["eps"], c["ell"], seed=c["seed"], instance=c["instance"], ahead=1)
        for ahead in (0, 1 << 16):
            r = hy.select_seeds(c["g"], c["k"], c["eps"], c["ell"], seed=c["seed"], instance=c["instance"],
                                ahead=ahead)
            _same(off, r, f"instance {i} ahead {ahead}")
    qs = [_q(c) for c in small]
    for ahead in (1, 1 << 16):
        batch = hy.select_seeds_batch(qs, ahead=ahead)
        for i, (c, b) in enumerate(zip(small, batch)):
            a = hy.select_seeds(c["g"], c["k"], c["eps"], c["ell"], seed=c["seed"], instance=c["instance"], ahead=1)
            _same(a, b, f"batch instance {i} ahead {ahead}")


def test_batch_shared_pools(hy, small):
    _flush("[gpu] batch shared pools")
    c = small[1]
    qs = [_q(c), _q(c, k=3), _q(c, eps=0.2), _q(c, instance=9), _q(small[0])]
    batch = hy.select_seeds_batch(qs)
    for q, b in zip(qs, batch):
        a = hy.select_seeds(q["graph"], q["k"], q["eps"], q["ell"], seed=q["seed"], instance=q["instance"])
        _same(a, b, str((q["k"], q["eps"], q["instance"])))


def test_batch_theta_fixed_and_errors(hy, small):
    _flush("[gpu] batch theta_fixed / errors")
    qs = [_q(c) for c in small[:3]]
    batch = hy.select_seeds_batch(qs, theta_fixed=3000)
    for q, b in zip(qs, batch):
        a = hy.select_seeds(q["graph"], q["k"], q["eps"], q["ell"], seed=q["seed"], instance=q["instance"],
                            theta_fixed=3000)
        _same(a, b)
    with pytest.raises(hy.HyperIMError) as e:
        hy.select_seeds_batch([_q(small[0]), _q(small[1], k=0)])
    assert e.value.status == hy.EINVAL
    # a pool cap that only the largest instance exceeds fails that query alone
    r = hy.select_seeds_batch(qs, theta_fixed=3000, max_entries=20000, raise_on_error=False)
    big = [hy.select_seeds(q["graph"], q["k"], q["eps"], q["ell"], seed=q["seed"], instance=q["instance"],
                           theta_fixed=3000) for q in qs]
    for a, b in zip(big, r):
        if max(a["entries1"], a["entries2"]) > 20000:
            assert b["status"] == hy.ECAPACITY
        else:
            assert b["status"] == hy.OK
            _same(a, b)
    assert hy.workspace_bytes() > 0


def test_session_continuous_batching(hy, small):
    _flush("[gpu] session")
    alone = [hy.select_seeds(c["g"], c["k"], c["eps"], c["ell"], seed=c["seed"], instance=c["instance"])
             for c in small]
    s = hy.Session()
    tickets = {}
    # three queries start, the rest join while those run
    for i in range(3):
        tickets[s.submit(small[i]["g"], small[i]["k"], small[i]["eps"], 1.0, small[i]["seed"],
                         small[i]["instance"])] = i
    st = s.step()
    assert st["admitted"] == 3
    for i in range(3, len(small)):
        tickets[s.submit(small[i]["g"], small[i]["k"], small[i]["eps"], 1.0, small[i]["seed"],
                         small[i]["instance"])] = i
    # a repeat of query 1 reuses its resident pools
    tickets[s.submit(small[1]["g"], small[1]["k"], small[1]["eps"], 1.0, small[1]["seed"],
                     small[1]["instance"])] = 1
    got = {}
    for _ in range(200):
        st = s.step()
        for t in list(tickets):
            r = s.poll(t)
            if r is not None:
                got[t] = (tickets.pop(t), r)
        if not tickets:
            break
    assert not tickets
    for t, (i, r) in got.items():
        _same(alone[i], r, f"session query {i}")
    assert st["finished"] == len(small) + 1
    s.close()


def test_session_budget(hy, small):
    _flush("[gpu] session budget")
    c = small[2]
    alone = hy.select_seeds(c["g"], c["k"], c["eps"], c["ell"], seed=c["seed"], instance=c["instance"])
    # a budget below what is already resident: the query cannot run at all
    s = hy.Session(hbm_budget=1 << 20)
    t = s.submit(c["g"], c["k"], c["eps"], 1.0, c["seed"], c["instance"])
    s.step()
    with pytest.raises(hy.HyperIMError) as e:
        s.poll(t)
    assert e.value.status == hy.ECAPACITY
    s.close()
    # a budget that holds one query at a time: the second waits, both exact
    resident = hy.workspace_bytes()
    s = hy.Session(hbm_budget=resident + (256 << 20))
    t1 = s.submit(c["g"], c["k"], c["eps"], 1.0, c["seed"], c["instance"])
    t2 = s.submit(small[0]["g"], small[0]["k"], small[0]["eps"], 1.0, small[0]["seed"], small[0]["instance"])
    r1 = r2 = None
    for _ in range(200):
        s.step()
        r1 = r1 or s.poll(t1)
        r2 = r2 or s.poll(t2)
        if r1 is not None and r2 is not None:
            break
    _same(alone, r1)
    a0 = hy.select_seeds(small[0]["g"], small[0]["k"], small[0]["eps"], 1.0, seed=small[0]["seed"],
                         instance=small[0]["instance"])
    _same(a0, r2)
    s.close()


@pytest.mark.slow
def test_multi_instance_workload_batch_equals_alone(hy):
    """Eight instances of the 64-instance workload at full size: batched
    (shared launches) and alone give the same bytes."""
    _flush("[gpu] multi-instance workload subset")
    ws = hypergen.multi_instance_workloads(64)[:8]
    gs = []
    for i, w in enumerate(ws):
        hg = w.build()
        g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, w.model, w.p)
        g.stratify()
        gs.append((g, w, i))
    qs = [dict(graph=g, k=w.k, eps=w.eps, ell=w.ell, seed=w.philox_seed, instance=i) for g, w, i in gs]
    batch = hy.select_seeds_batch(qs)
    for (g, w, i), b in zip(gs, batch):
        a = hy.select_seeds(g, w.k, w.eps, w.ell, seed=w.philox_seed, instance=i)
        _flush(f"[gpu]   instance {i}: n={w.n} theta={a['theta']} rounds={a['rounds']}")
        _same(a, b, f"instance {i}")
