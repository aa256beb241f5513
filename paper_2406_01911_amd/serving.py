"""Serving loop over a hyperim session: Poisson arrivals of IM queries over a
pool of resident graphs, continuous batching, latency percentiles.

Queries arrive at the times of a seeded Poisson process of rate `qps`.  The
loop submits every query whose arrival time has passed, then advances the
session by one step (one doubling round of every admitted query, RR
generation shared across them), then collects finished queries.  A query
arriving while others run joins at the next step; admission is by the
session's HBM budget.  Latency = completion time - arrival time, so queueing
counts.  Query i draws its graph and k from the same seeded stream; its
Philox key is (0, graph index), so queries on one graph share resident pools
and reuse their prefix.

    python -m paper_2406_01911_amd.serving --qps 5 --queries 200
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def poisson_arrivals(count: int, qps: float, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of a Poisson process of rate qps, first at its first
    exponential gap."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / qps, size=count))


def draw_queries(count: int, n_graphs: int, ks=(10, 50, 200), eps: float = 0.1, seed: int = 0) -> list:
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    gi = rng.integers(0, n_graphs, size=count)
    kk = rng.choice(np.asarray(ks), size=count)
    return [{"graph": int(a), "k": int(b), "eps": eps, "ell": 1.0, "seed": 0, "instance": int(a)}
            for a, b in zip(gi, kk)]


def latency_summary(lat_s) -> dict:
    """p50 / p99 / mean / max in ms (nearest-rank percentiles)."""
    lat = np.sort(np.asarray(lat_s, dtype=np.float64)) * 1e3
    if lat.size == 0:
        return {"p50_ms": None, "p99_ms": None, "mean_ms": None, "max_ms": None}

    def rank(q):
        return float(lat[max(int(np.ceil(q * lat.size)) - 1, 0)])
    return {"p50_ms": rank(0.50), "p99_ms": rank(0.99), "mean_ms": float(lat.mean()), "max_ms": float(lat[-1])}


def serve(graphs: list, queries: list, arrivals: np.ndarray, hbm_budget: int = 0, stream=None, log=None) -> dict:
    """Run the queries through one session; returns per-query results and the summary."""
    import paper_2406_01911_amd as hy
    n = len(queries)
    sess = hy.Session(hbm_budget=hbm_budget, stream=stream)
    pending = {}
    results = [None] * n
    finish = np.zeros(n)
    nxt, done, steps, max_active, max_resident = 0, 0, 0, 0, 0
    t0 = time.perf_counter()
    while done < n:
        now = time.perf_counter() - t0
        while nxt < n and arrivals[nxt] <= now:
            q = queries[nxt]
            t = sess.submit(graphs[q["graph"]], q["k"], q["eps"], q["ell"], q["seed"], q["instance"])
            pending[t] = nxt
            nxt += 1
        if not pending:
            time.sleep(max(0.0, float(arrivals[nxt]) - now))
            continue
        st = sess.step()
        steps += 1
        max_active = max(max_active, st["active"] + st["waiting"])
        max_resident = max(max_resident, st["bytes_resident"])
        now = time.perf_counter() - t0
        for t in list(pending):
            r = sess.poll(t)
            if r is not None:
                i = pending.pop(t)
                results[i] = r
                finish[i] = now
                done += 1
        if log and steps % 20 == 0:
            log(f"[serving] step {steps}: {done}/{n} done, {len(pending)} in flight, t={now:.1f}s")
    stats = sess.stats()
    sess.close()
    lat = finish - arrivals
    makespan = float(finish.max() - arrivals[0]) if n else 0.0
    out = latency_summary(lat)
    out.update({"queries": n, "qps_offered": n / float(arrivals[-1]) if n else 0.0,
                "qps_served": n / makespan if makespan > 0 else 0.0, "steps": steps,
                "max_in_flight": max_active, "max_resident_bytes": int(max_resident),
                "hbm_budget": int(stats["hbm_budget"]), "failed": int(stats["failed"])})
    return {"summary": out, "results": results, "latency_s": lat}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--qps", type=str, default="5.0",
                    help="arrival rate, or a comma-separated list of rates run one after another "
                         "(a fresh session each, the graphs built once)")
    ap.add_argument("--queries", type=int, default=200)
    ap.add_argument("--graphs", type=int, default=16)
    ap.add_argument("--n-max", type=float, default=5e6)
    ap.add_argument("--n-min", type=float, default=5e4)
    ap.add_argument("--budget-gb", type=float, default=0.0, help="HBM budget (0: device memory less 8 GiB)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--verify", type=int, default=8, help="queries re-run alone and compared")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch  # noqa: F401
    import hypergen
    import paper_2406_01911_amd as hy
    hy.load_library()

    def log(m):
        print(m, file=sys.stderr, flush=True)
    ws = hypergen.serving_workloads(args.graphs, int(args.n_max), int(args.n_min))
    graphs, t0 = [], time.time()
    for i, w in enumerate(ws):
        hg = w.build()
        g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, w.model, w.p)
        g.stratify()
        graphs.append(g)
        log(f"[serving] graph {i}: n={w.n} nnz={int(hg.he_off[-1])} ({time.time() - t0:.1f} s)")
    queries = draw_queries(args.queries, len(graphs), seed=args.seed)
    for qps in [float(x) for x in args.qps.split(",") if x.strip()]:
        log(f"[serving] rate {qps} qps, {args.queries} queries")
        arrivals = poisson_arrivals(args.queries, qps, seed=args.seed)
        run = serve(graphs, queries, arrivals, int(args.budget_gb * 1e9), log=log)
        # a sample re-run alone must give the same bytes
        rng = np.random.Generator(np.random.PCG64(args.seed + 7))
        checked = 0
        for i in rng.choice(len(queries), size=min(args.verify, len(queries)), replace=False):
            q, r = queries[i], run["results"][i]
            a = hy.select_seeds(graphs[q["graph"]], q["k"], q["eps"], q["ell"], seed=q["seed"],
                                instance=q["instance"])
            assert np.array_equal(a["seeds"], r["seeds"]) and np.array_equal(a["gains"], r["gains"]), i
            assert a["theta"] == r["theta"] and a["lambda2"] == r["lambda2"], i
            checked += 1
        line = {"metric": "queries/s", "value": run["summary"]["qps_served"], "unit": "queries/s",
                "latency": {k: run["summary"][k] for k in ("p50_ms", "p99_ms", "mean_ms", "max_ms")},
                "workload": f"{args.graphs} graphs, |V| log-spaced {int(args.n_min)}..{int(args.n_max)}, "
                            f"|HE|=2|V|, sizes power-law(2.1) on [2,1000], uniform members, WC; "
                            f"k in {{10,50,200}}, eps=0.1; Poisson arrivals at {qps} qps, {args.queries} queries",
                "qps_rate": qps, "verified_alone": checked}
        line.update({k: v for k, v in run["summary"].items() if k not in line["latency"]})
        print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
