"""Autotuner for RR generation's execution parameters (hyperim_tuning).

The parameters decide the schedule, never the result: when a set leaves its
wavefront for the grid-wide phase (heavy, budget: per-wave versus
multi-workgroup granularity), how many workgroups per compute unit each phase
launches (blocks_a, blocks_b), how large the grid-wide work items are (chunk,
seg), when visited marks are tested before coins (prefilter_min), how many
supersteps run between host checks (steps_per_sync) and how much staging
memory a launch group may use (stage_mib) and when sets grow in bit-parallel
bundles (ms_min).  The tuner measures one round of
seed selection at a fixed theta for each candidate, by coordinate descent
over a small grid per parameter, and keeps a candidate only if its seeds and
gains equal the baseline's (they must: every schedule gives the same bytes).

    python -m paper_2406_01911_amd.autotune --workload mid

writes tuning/<workload>.json beside this file; Graph.apply_tuning / the
bench's --tuning flag read it back.  `--workload multi` tunes the
64-instance workload: one tuning applied to every graph, each candidate
timed on one batched round of all instances.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_DIR = os.path.join(HERE, "tuning")

SPACE = {
    "heavy": [256, 512, 1024, 2048, 4096],
    "budget": [4096, 8192, 16384, 32768, 65536],
    "chunk": [128, 256, 512, 1024, 2048, 4096],
    "seg": [256, 512, 1024, 2048, 4096, 8192],
    "prefilter_min": [256, 1024, 4096, 16384, 1 << 30],
    "steps_per_sync": [2, 4, 8, 16, 32],
    "blocks_a": [2, 3, 4, 6, 8],
    "blocks_b": [3, 4, 6, 8],
    "ms_min": [1024, 4096, 65536, 0xFFFFFFFF],
    "ms_filter": [1, 4, 6, 8, 12, 16, 24, 40, 65],
}


def _measure(hy, g, k, eps, ell, seed, theta, reps, stream):
    best, out = None, None
    for _ in range(reps):
        r = hy.select_seeds(g, k, eps, ell, seed=seed, theta_fixed=theta, stream=stream)
        t = r["ms_rr"]
        if best is None or t < best:
            best, out = t, r
    return best, out


def autotune(g, k: int, eps: float, ell: float = 1.0, seed: int = 0, theta: int | None = None,
             space: dict | None = None, reps: int = 3, sweeps: int = 2, stream=None, log=None) -> dict:
    """Coordinate descent over `space`; returns {"tuning", "ms_rr", "baseline_ms_rr", "theta", "trials"}.
    The graph keeps the best tuning."""
    import paper_2406_01911_amd as hy
    space = space or SPACE
    if theta is None:
        theta = hy.select_seeds(g, k, eps, ell, seed=seed, stream=stream)["theta"]
    start = g.tuning()
    # warm-up (workspace allocation), then the baseline
    hy.select_seeds(g, k, eps, ell, seed=seed, theta_fixed=theta, stream=stream)
    base_ms, base = _measure(hy, g, k, eps, ell, seed, theta, reps, stream)
    cur, cur_ms = dict(start), base_ms
    trials = [{"tuning": dict(cur), "ms_rr": base_ms}]
    for sweep in range(sweeps):
        improved = False
        for name, values in space.items():
            for v in values:
                if v == cur[name]:
                    continue
                cand = dict(cur)
                cand[name] = v
                if cand["seg"] < cand["chunk"]:
                    continue
                g.set_tuning(**cand)
                ms, r = _measure(hy, g, k, eps, ell, seed, theta, reps, stream)
                same = np.array_equal(r["seeds"], base["seeds"]) and np.array_equal(r["gains"], base["gains"])
                if not same:
                    raise RuntimeError(f"tuning {cand} changed the result")
                trials.append({"tuning": dict(cand), "ms_rr": ms})
                if log:
                    log(f"[autotune] sweep {sweep} {name}={v}: {ms:.2f} ms (best {cur_ms:.2f})")
                if ms < cur_ms * 0.98:
                    cur, cur_ms, improved = cand, ms, True
            g.set_tuning(**cur)
        if not improved:
            break
    g.set_tuning(**cur)
    return {"tuning": cur, "ms_rr": cur_ms, "baseline_ms_rr": base_ms, "theta": theta, "trials": trials}


def _measure_batch(hy, gs, ws, theta, reps, stream):
    """Best RR time of one batched round (all instances, shared launch
    groups) over `reps` runs, and that run's per-query results."""
    best, out = None, None
    qs = [dict(graph=g, k=w.k, eps=w.eps, ell=w.ell, seed=w.philox_seed, instance=i)
          for i, (g, w) in enumerate(zip(gs, ws))]
    for _ in range(reps):
        tot = {}
        rs = hy.select_seeds_batch(qs, theta_fixed=theta, stream=stream, totals=tot)
        t = tot["ms_rr"]
        if best is None or t < best:
            best, out = t, rs
    return best, out


def autotune_batch(gs, ws, theta: int, space: dict | None = None, reps: int = 2, sweeps: int = 1, stream=None,
                   log=None) -> dict:
    """Coordinate descent as `autotune`, for many instances answered in one
    batch: a candidate is applied to every graph and timed on one batched
    round at `theta` sets per pool; it is kept only if every query's seeds
    and gains equal the baseline's."""
    import paper_2406_01911_amd as hy
    space = space or SPACE
    start = gs[0].tuning()
    for g in gs:
        g.set_tuning(**start)
    _measure_batch(hy, gs, ws, theta, 1, stream)   # warm-up
    base_ms, base = _measure_batch(hy, gs, ws, theta, reps, stream)
    cur, cur_ms = dict(start), base_ms
    trials = [{"tuning": dict(cur), "ms_rr": base_ms}]
    for sweep in range(sweeps):
        improved = False
        for name, values in space.items():
            for v in values:
                if v == cur[name]:
                    continue
                cand = dict(cur)
                cand[name] = v
                if cand["seg"] < cand["chunk"]:
                    continue
                for g in gs:
                    g.set_tuning(**cand)
                ms, rs = _measure_batch(hy, gs, ws, theta, reps, stream)
                for a, b in zip(rs, base):
                    if not (np.array_equal(a["seeds"], b["seeds"]) and np.array_equal(a["gains"], b["gains"])):
                        raise RuntimeError(f"tuning {cand} changed a result")
                trials.append({"tuning": dict(cand), "ms_rr": ms})
                if log:
                    log(f"[autotune] sweep {sweep} {name}={v}: {ms:.1f} ms (best {cur_ms:.1f})")
                if ms < cur_ms * 0.98:
                    cur, cur_ms, improved = cand, ms, True
            for g in gs:
                g.set_tuning(**cur)
        if not improved:
            break
    for g in gs:
        g.set_tuning(**cur)
    return {"tuning": cur, "ms_rr": cur_ms, "baseline_ms_rr": base_ms, "theta": theta, "trials": trials}


def tuning_path(workload: str) -> str:
    return os.path.join(TUNING_DIR, f"{workload}.json")


def load(workload: str) -> dict | None:
    """The stored tuning of a workload, or None."""
    p = tuning_path(workload)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        return json.load(f)["tuning"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="mid")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--sweeps", type=int, default=2)
    ap.add_argument("--theta", type=int, default=0, help="RR sets per pool of the measured round (0: the query's)")
    ap.add_argument("--out", default="")
    ap.add_argument("--params", default="", help="comma-separated subset of the parameters to search")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    import torch  # noqa: F401
    import hypergen
    import paper_2406_01911_amd as hy
    hy.load_library()
    t0 = time.time()
    space = {k: v for k, v in SPACE.items() if not args.params or k in args.params.split(",")}
    stored = load(args.workload)
    log = lambda m: print(m, file=sys.stderr, flush=True)   # noqa: E731
    if args.workload == "multi":
        # the 64-instance workload: one tuning for every graph, timed on one
        # batched round
        ws = hypergen.multi_instance_workloads(64)
        gs = []
        for wl in ws:
            hg = wl.build()
            g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, wl.model, wl.p)
            g.stratify()
            if stored:
                g.set_tuning(**stored)
            gs.append(g)
        log(f"[autotune] multi: {len(gs)} graphs built ({time.time() - t0:.1f} s)")
        res = autotune_batch(gs, ws, args.theta or 1024, space=space, reps=args.reps, sweeps=args.sweeps, log=log)
    else:
        w = hypergen.workload(args.workload)
        hg = w.build()
        g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, w.model, w.p)
        g.stratify()
        if stored:
            g.set_tuning(**stored)   # refine the stored result
        res = autotune(g, w.k, w.eps, w.ell, seed=w.philox_seed, theta=args.theta or None, space=space,
                       reps=args.reps, sweeps=args.sweeps, log=log)
    res["workload"] = args.workload
    res["seconds"] = time.time() - t0
    out = args.out or tuning_path(args.workload)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps({k: res[k] for k in ("workload", "tuning", "ms_rr", "baseline_ms_rr", "theta")}), flush=True)


if __name__ == "__main__":
    main()
