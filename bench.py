"""Benchmark of HyperIM's hot path on one MI355X.

One step = one whole query on a device-resident synthetic hypergraph: build
the incidence CSR and thresholds, stratify, then the HyperIM_BRR loop (RR-set
generation for both pools, greedy max coverage, R2 check, doubling) until the
seed set is returned.  Inputs (he_off, he_mem) are already in HBM when the
timed region starts.  The default workload is the large one (|V| = 1e6,
|HE| = 2e6, IC p = 0.01, k = 100) under its stored tuning, with the plain
per-stratum form timed beside it.

Prints one JSON line: RR sets/s (value), incidences/s, coins/s, Philox
blocks/s, time-to-seed-set, the roofline of the dominant RR-generation kernel
(its Philox work against the VALU peak and its algorithmic bytes against
8 TB/s, both per HIP-event-timed launch; `bound` is what the committed
hardware counters show) and the CPU oracle timed on a bounded sample of the
same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOAD_TEXT = {
    "tiny": "|V|=1e3 |HE|=2e3 sizes U[2,6] uniform members, IC p=0.05, k=10 eps=0.5 ell=1",
    "mid": "|V|=1e5 |HE|=2e5 sizes power-law(2.5) on [2,50], Zipf(1.0) members, weighted cascade, "
           "k=50 eps=0.1 ell=1",
    "large": "|V|=1e6 |HE|=2e6 sizes power-law(2.2) on [2,200], Zipf(1.1) members, IC p=0.01, "
             "k=100 eps=0.1 ell=1",
    "multi": "64 instances: |V| log-uniform in [1e4,5e5], |HE|=2|V|, sizes power-law(2.5) on [2,100], "
             "uniform members, IC p~U[0.005,0.05], k~U{10..200}, eps in {0.1,0.2}, ell=1, instance id i",
    "tiny_lt": "the tiny hypergraph under the linear-threshold model, channel weights 1/c(v), k=10 eps=0.5 ell=1",
    "mid_lt": "the mid hypergraph (|V|=1e5 |HE|=2e5 sizes power-law(2.5) on [2,50], Zipf(1.0) members) under "
              "the linear-threshold model, channel weights 1/c(v), k=50 eps=0.1 ell=1",
    "large_lt": "the large hypergraph (|V|=1e6 |HE|=2e6 sizes power-law(2.2) on [2,200], Zipf(1.1) members) "
                "under the linear-threshold model, channel weights 1/c(v), k=100 eps=0.1 ell=1",
    "tiny_layered": "the tiny hypergraph under the stratified setting (per-layer probabilities 1/(i ln(l+1)) "
                    "split over the layer), k=10 eps=0.5 ell=1",
    "mid_layered": "the mid hypergraph (|V|=1e5 |HE|=2e5 sizes power-law(2.5) on [2,50], Zipf(1.0) members) under "
                   "the stratified setting (per-layer probabilities 1/(i ln(l+1)) split over the layer), "
                   "k=50 eps=0.1 ell=1",
    "large_layered": "the large hypergraph (|V|=1e6 |HE|=2e6 sizes power-law(2.2) on [2,200], Zipf(1.1) members) "
                     "under the stratified setting (per-layer probabilities 1/(i ln(l+1)) split over the layer), "
                     "k=100 eps=0.1 ell=1",
    "tiny_gaps": "the tiny workload (IC p=0.05) with live channels drawn by geometric gaps, k=10 eps=0.5 ell=1",
    "mid_gaps": "the mid hypergraph (|V|=1e5 |HE|=2e5 sizes power-law(2.5) on [2,50], Zipf(1.0) members), "
                "weighted cascade with live channels drawn by geometric gaps, k=50 eps=0.1 ell=1",
    "large_gaps": "the large hypergraph (|V|=1e6 |HE|=2e6 sizes power-law(2.2) on [2,200], Zipf(1.1) members), "
                  "IC p=0.01 with live channels drawn by geometric gaps, k=100 eps=0.1 ell=1",
}
LT_WORKLOADS = ("tiny_lt", "mid_lt", "large_lt")
LAYERED_WORKLOADS = ("tiny_layered", "mid_layered", "large_layered")
GAPS_WORKLOADS = ("tiny_gaps", "mid_gaps", "large_gaps")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--form", type=int, default=0, help="0 persistent launch per pool block, 1 plain per stratum")
    ap.add_argument("--plain-steps", type=int, default=-1,
                    help="steps of the plain per-stratum form timed for comparison (-1: 1 on large and multi, "
                         "as many as --steps otherwise)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU-baseline sample time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning", default="stored", choices=["stored", "default"],
                    help="execution parameters: the autotuner's stored result for the workload, or the defaults")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every superstep kernel directly instead of replaying captured batches")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of this many MiB (reference kernel for "
                         "scaling hardware byte counters)")
    return ap.parse_args()


# The VALU peak of MI355X in 32-bit lane operations: 256 compute units x 4
# SIMDs x 16 lanes per clock x 2.4 GHz (the 157.3 TFLOP/s fp32 vector figure
# counts a packed FMA as 4 flops per lane).  One Philox4x32-10 block is 20
# v_mad_u64_u32 and 40 v_xor_b32 in the generated code (key schedule in
# scalar registers); a v_mad_u64_u32 issues in one pass on gfx950 (the
# throughput probe measures 661-684 Gblocks/s, against 655 for one pass and
# 328 for four).
VALU_LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9
PHILOX_XOR, PHILOX_MAD, PHILOX_MAD_PASSES = 40, 20, 1
PHILOX_PEAK_BLOCKS_PER_S = VALU_LANE_OPS_PER_S / (PHILOX_XOR + PHILOX_MAD * PHILOX_MAD_PASSES)

# expansion kernels the line can name as dominant: result fields of their
# time, launches, algorithmic bytes and Philox blocks
KERNELS = {
    "k_rr_light": ("ms_light", None, "bytes_light", "philox_light"),
    "k_expand": ("ms_expand", "expand_launches", "bytes_heavy", None),
    "k_ms_expand": ("ms_bundled", "bundled_launches", "bytes_bundled", "philox_bundled"),
}


def rr_device_sha256() -> str:
    """sha256 of rr.hip's device code: the text before its host-side marker."""
    src = os.path.join(ROOT, "paper_2406_01911_amd", "csrc", "rr.hip")
    with open(src) as f:
        text = f.read()
    return hashlib.sha256(text.split("// ---- host side", 1)[0].encode()).hexdigest()


def kernel_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed hardware-counter
    summary of this workload (FETCH_SIZE + WRITE_SIZE per dispatch, scaled by
    the same counters on a copy of known size); None when there is none or
    when the device code of RR generation (rr.hip up to its host-side part)
    has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("rr_hip_sha256") != rr_device_sha256():
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(hg, w, seconds: float, workload: str, sets_needed: int = 0):
    """The oracle as it stands, on the host cores: RR sets of pool R1 from id 0
    in chunks until about `seconds` of CPU work (build + stratify untimed)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    threads = max(1, min(threads, os.cpu_count() or 1))
    o = oracle.Graph(hg, w.model, w.p)
    o.stratify()
    supercritical = workload in ("large", "large_gaps")   # sets of ~1e5 members
    done, chunk, t0 = 0, 2 * threads if supercritical else 512, time.perf_counter()
    while True:
        o.generate(w.philox_seed, 0, 0, done, done + chunk, nthreads=threads)
        done += chunk
        el = time.perf_counter() - t0
        if el >= seconds or done >= (1 << 22):
            break
        if el < seconds / 4:
            chunk *= 2
    what = (f"RR ids [0, {done}) of pool R1 of the same workload, {el:.1f} s wall, {threads} threads over ids")
    if supercritical:
        what += (f"; an extrapolation: the query draws {sets_needed} sets (both pools), the sample covers "
                 f"the first ids of pool R1")
    return {"value": done / el, "unit": "RR sets/s", "cores": threads, "kind": "oracle", "cpu": cpu_model(),
            "sample": what}


def philox_rate():
    """Measured throughput of the library's Philox4x32-10 block function at
    full occupancy (microbench/philox_rate.hip), blocks/s."""
    import ctypes as C
    path = os.path.join(ROOT, "paper_2406_01911_amd", "microbench", "libphilox_rate.so")
    if not os.path.exists(path):
        return None
    L = C.CDLL(path)
    L.philox_rate.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.POINTER(C.c_double)]
    bps, ms, blocks = C.c_double(), C.c_double(), C.c_double()
    rc = L.philox_rate(2048, 16, 5, C.byref(bps), C.byref(ms), C.byref(blocks))
    if rc != 0:
        return None
    return {"blocks_per_s": bps.value, "ms": ms.value, "blocks": blocks.value}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of RR ids is a design note, not a measured path.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import hypergen
    import paper_2406_01911_amd as hy

    hy.load_library()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    t_gen = time.perf_counter()
    if args.workload == "multi":
        ws = hypergen.multi_instance_workloads(64)
        hgs = []
        for i, wl in enumerate(ws):
            hgs.append(wl.build())
            if i % 16 == 15:
                print(f"[bench] generated {i + 1} of {len(ws)} instances "
                      f"({time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)
    else:
        ws = [hypergen.workload(args.workload)]
        hgs = [ws[0].build()]
    w = ws[0]
    dev = [(torch.from_numpy(h.he_off.view(np.int32)).cuda(), torch.from_numpy(h.he_mem.view(np.int32)).cuda())
           for h in hgs]
    torch.cuda.synchronize()
    print(f"[bench] {args.workload} input generated and resident ({time.perf_counter() - t_gen:.1f} s)",
          file=sys.stderr, flush=True)
    from paper_2406_01911_amd import autotune
    tuning = autotune.load(args.workload) if args.tuning == "stored" else None
    # timed steps: the production path (superstep batches replayed as captured
    # graphs), nothing else
    flags_prod = hy.FLAG_NO_GRAPHS if args.no_graphs else 0
    # one instrumented step after them: every expansion launch timed by events
    # its launch stamps (direct launches: events recorded inside a captured
    # graph do not time against the stream), plus the extra pass that sums the
    # final pools' work (incidences, coins, Philox blocks, algorithmic bytes);
    # the ids, and so the work, are those of every timed step
    flags_inst = hy.FLAG_INCIDENCES | hy.FLAG_KERNEL_TIMES

    def step(form, flags=flags_prod, inputs=dev):
        """One query step: build + stratify every graph, then seed selection
        (one query, or all instances batched; form 1 runs them one by one in
        the plain per-stratum form).  `inputs` holds each graph's (he_off,
        he_mem): device tensors, or host arrays that build_graph copies over."""
        gs = []
        for h, (o, m), wl in zip(hgs, inputs, ws):
            g = hy.build_graph(h.n, o, m, wl.model, wl.p, stream=stream)
            g.stratify(stream=stream)
            if tuning:
                g.set_tuning(**tuning)
            gs.append(g)
        if args.workload != "multi":
            r = hy.select_seeds(gs[0], w.k, w.eps, w.ell, seed=w.philox_seed, form=form, flags=flags,
                                stream=stream)
            return [r], r
        if form == 0:
            tot = {}
            rs = hy.select_seeds_batch([dict(graph=g, k=wl.k, eps=wl.eps, ell=wl.ell, seed=wl.philox_seed,
                                             instance=i) for i, (g, wl) in enumerate(zip(gs, ws))],
                                       flags=flags, stream=stream, totals=tot)
            return rs, tot
        rs = [hy.select_seeds(g, wl.k, wl.eps, wl.ell, seed=wl.philox_seed, instance=i, form=1, flags=flags,
                              stream=stream) for i, (g, wl) in enumerate(zip(gs, ws))]
        tot = {k: sum(r[k] for r in rs) for k in rs[0] if k not in ("seeds", "gains")}
        return rs, tot

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes}), file=sys.stderr, flush=True)
        del src, dst

    px_rate = philox_rate()

    def timed(steps, warmup, form, what):
        for i in range(warmup):
            step(form)
            print(f"[bench] {what}: warm-up step {i + 1} of {warmup} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        out = []
        t0 = time.perf_counter()
        for i in range(steps):
            out.append(step(form))
            print(f"[bench] {what}: step {i + 1} of {steps} done ({time.perf_counter() - t0:.1f} s)",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    steps_out, elapsed = timed(args.steps, args.warmup, args.form, f"form {args.form}")
    results = [r for r, _ in steps_out]
    totals = [t for _, t in steps_out]
    print(f"[bench] {args.steps} steps of form {args.form}: {elapsed:.3f} s", file=sys.stderr, flush=True)
    big = args.workload in ("large", "multi")
    plain_steps = args.plain_steps if args.plain_steps >= 0 else (1 if big else args.steps)
    plain = None
    if plain_steps and args.form == 0:
        # the workspace is warm from the steps above; small workloads still
        # take one plain warm-up step
        pres, pel = timed(plain_steps, 0 if big else 1, 1, "plain form")
        for a, b in zip(pres[-1][0], results[-1]):
            assert np.array_equal(a["seeds"], b["seeds"]) and a["theta"] == b["theta"]
        plain = {"form": "plain per-stratum launches, one query at a time", "steps": plain_steps,
                 "ms_per_step": 1000.0 * pel / plain_steps}
        print(f"[bench] {plain_steps} steps of the plain form: {pel:.3f} s", file=sys.stderr, flush=True)
    last = results[-1]
    mtot = totals[-1]
    for r in results[:-1]:
        for a, b in zip(r, last):
            assert np.array_equal(a["seeds"], b["seeds"]) and a["theta"] == b["theta"]
    # per-kernel times: one instrumented step of the same workload
    inst_res, itot = step(args.form, flags=flags_inst)
    for a, b in zip(inst_res, last):
        assert np.array_equal(a["seeds"], b["seeds"]) and a["theta"] == b["theta"]
    print("[bench] instrumented step done", file=sys.stderr, flush=True)
    # the same step with the input handed over in host memory: build_graph
    # copies it across PCIe inside the step (reported beside the line; the
    # line's value keeps the input resident in HBM)
    host_in = [(h.he_off, h.he_mem) for h in hgs]
    host_steps = 1 if big else min(args.steps, 5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(host_steps):
        hres, _ = step(args.form, inputs=host_in)
    torch.cuda.synchronize()
    host_el = time.perf_counter() - t0
    for a, b in zip(hres, last):
        assert np.array_equal(a["seeds"], b["seeds"]) and a["theta"] == b["theta"]
    print(f"[bench] {host_steps} steps from host input: {host_el:.3f} s", file=sys.stderr, flush=True)

    def mean_total(key):
        return float(np.mean([t[key] for t in totals]))

    ms_per_step = 1000.0 * elapsed / args.steps
    rr_sets_per_step = sum(2 * r["theta"] for r in last)
    value = rr_sets_per_step * args.steps / elapsed
    per_s = args.steps / elapsed
    lt = args.workload in LT_WORKLOADS
    layered = args.workload in LAYERED_WORKLOADS
    gaps = args.workload in GAPS_WORKLOADS
    kernel_bytes = itot["bytes_light"] + itot["bytes_heavy"] + itot["bytes_bundled"]
    # the kernels count the bytes of every expansion they perform; the pools'
    # final prefixes can only hold fewer (sets generated ahead of a round that
    # was not reached are spent work).  A linear-threshold walk reads one
    # channel per step, and the gap sampler reads only the live positions of a
    # hyperedge: their algorithmic bytes are the kernels' own count.
    alg_bytes = kernel_bytes if (lt or layered or gaps) else itot["alg_bytes"]
    assert kernel_bytes >= alg_bytes, (kernel_bytes, alg_bytes)
    # dominant expansion kernel: the largest event-timed share in the
    # instrumented step
    kernels = dict(KERNELS)
    if lt or layered:   # these kernels report through the per-set phase's fields
        kernels = {"k_lt_walk" if lt else "k_layered": kernels.pop("k_rr_light")}
    times = {k: float(itot[f[0]]) for k, f in kernels.items()}
    kern = max(times, key=times.get)
    f_ms, f_launch, f_bytes, f_px = kernels[kern]
    k_ms = times[kern]
    k_launches = itot[f_launch] if f_launch else 1
    k_bytes = itot[f_bytes]
    if f_px is None:
        k_px = itot["philox_drawn"] - itot["philox_light"] - itot["philox_bundled"]
    else:
        k_px = itot[f_px]
    per_launch_s = k_ms * 1e-3 / max(k_launches, 1)
    alg_per_launch = k_bytes / max(k_launches, 1)
    px_per_launch = k_px / max(k_launches, 1)
    hbm_achieved = alg_per_launch / per_launch_s / 1e9 if per_launch_s > 0 else 0.0
    px_achieved = px_per_launch / per_launch_s if per_launch_s > 0 else 0.0
    frac_hbm = hbm_achieved / HBM_PEAK_GBS
    frac_valu = px_achieved / PHILOX_PEAK_BLOCKS_PER_S
    traffic = kernel_traffic(kern, args.workload)
    # bound: counters below the algorithmic bytes mean the bytes come from
    # caches and the integer ALU binds; without counters, the larger fraction
    if traffic is not None:
        bound = "alu" if traffic < alg_per_launch else "hbm"
    else:
        bound = "alu" if frac_valu >= frac_hbm else "hbm"
    if bound == "alu":
        roof = {"bound": "alu", "achieved": px_achieved / 1e9, "peak": PHILOX_PEAK_BLOCKS_PER_S / 1e9,
                "unit": "Gblocks/s (Philox4x32-10 on the VALU)", "frac": frac_valu}
    else:
        roof = {"bound": "hbm", "achieved": hbm_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": frac_hbm}
    roof.update({
        "kernel": kern,
        "timing": "average launch time from events each launch stamps, on one instrumented step of the same "
                  "workload run after the timed steps (direct launches); the timed steps replay captured "
                  "superstep batches",
        "traffic": traffic,
        "frac_hbm": frac_hbm,
        "frac_valu": frac_valu,
        "alg_bytes_per_launch": alg_per_launch,
        "philox_blocks_per_launch": px_per_launch,
        "avg_launch_ms": per_launch_s * 1e3,
        "launches_per_step": k_launches,
        "philox_peak_derivation": f"{VALU_LANE_OPS_PER_S / 1e12:.1f}e12 VALU lane-ops/s / "
                                  f"({PHILOX_XOR} + {PHILOX_MAD} x {PHILOX_MAD_PASSES}) per block",
    })
    if px_rate:
        roof["philox_measured_peak_gblocks_s"] = px_rate["blocks_per_s"] / 1e9
    bfs_ms = mean_total("ms_bfs")
    line = {
        "metric": "RR sets/s",
        "value": value,
        "unit": "RR sets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_TEXT[args.workload]}",
                   "form": "persistent" if args.form == 0 else "plain-per-stratum",
                   "tuning": tuning if tuning else "default",
                   "parallelism": "single-gpu"},
        # channel-model figures (IC); the other models draw per step or per layer
        "incidences_per_s": None if (lt or layered) else itot["incidences"] * per_s,
        "coins_per_s": mtot["philox_drawn"] * per_s if (lt or layered or gaps) else itot["coins"] * per_s,
        "philox_blocks_per_s": {"drawn": mtot["philox_drawn"] * per_s, "per_set_traversal": itot["philox_alg"] * per_s},
        "time_to_seed_set_ms": ms_per_step,
        "theta": [r["theta"] for r in last] if len(last) > 1 else last[0]["theta"],
        "rounds": max(r["rounds"] for r in last),
        "spread": [r["spread"] for r in last] if len(last) > 1 else last[0]["spread"],
        "ms_rr": mean_total("ms_rr"),
        "ms_greedy": mean_total("ms_greedy"),
        "kernels_ms": {k: v for k, v in times.items()},
        "roofline": roof,
        "rr_generation": {
            "kernels": "k_lt_walk" if lt else "k_layered" if layered else
                       "k_rr_light, k_plan, k_expand, k_finish, k_ms_*",
            "achieved_GBps": kernel_bytes / (bfs_ms * 1e-3) / 1e9 if bfs_ms > 0 else 0.0,
            "frac_hbm": kernel_bytes / (bfs_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if bfs_ms > 0 else 0.0,
            "ms": bfs_ms,
            "launches_per_step": totals[-1]["bfs_launches"],
            "superstep_batches": "direct launches" if args.no_graphs else "captured HIP graphs, replayed",
            "deferred_sets": mtot["deferred"],
            "supersteps": mtot["supersteps"],
        },
    }
    line["host_input"] = {
        "what": "the same step with he_off / he_mem handed to build_graph in host memory "
                "(pageable), so the input crosses PCIe inside each step",
        "steps": host_steps,
        "input_bytes": int(sum(h.he_off.nbytes + h.he_mem.nbytes for h in hgs)),
        "ms_per_step": 1000.0 * host_el / host_steps,
        "value": rr_sets_per_step * host_steps / host_el,
    }
    if plain is not None:
        plain["batched_speedup"] = plain["ms_per_step"] / ms_per_step
        line["plain_form"] = plain
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(hgs[0], ws[0], args.cpu_seconds, args.workload,
                                            sets_needed=2 * last[0]["theta"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
