"""Seeded synthetic hypergraphs shaped like the paper's workloads.

This module draws *inputs* only: hyperedge member lists in CSR form
(``he_off[m+1]``, ``he_mem[nnz]``, both uint32) plus the query parameters of
each workload.  It holds none of the method's arithmetic (no coins, no
thresholds, no strata, no RR sets, no greedy), so both the CPU oracle and the
GPU path may consume what it produces.

The paper evaluates on five real hypergraphs (its evaluation section, the
dataset table: email-Eu-full ... coauth-MAG-Geology-full).  None of them is
available here, so the workloads below are synthetic stand-ins that bracket
their sizes: hyperedge sizes follow a discrete truncated power law (or a
uniform law for the tiny case), members are drawn without replacement either
uniformly or by Zipf popularity over a seeded random permutation of vertex
ids (so ids carry no locality).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Hypergraph", "Workload", "WORKLOADS", "workload", "power_law_sizes",
    "uniform_sizes", "draw_members", "make_hypergraph", "tiny_hypergraph",
    "from_lists",
]

MODEL_CONST = 0   # constant channel probability p
MODEL_WC = 1      # weighted cascade: p_v = 1 / (weighted clique in-degree of v)
MODEL_LT_CONST = 2   # linear threshold, channel weight p
MODEL_LT_WC = 3      # linear threshold, channel weight 1 / (weighted clique in-degree of v)
MODEL_LAYERED = 4    # stratified setting: per-layer probabilities of the sample sets
MODEL_GAPS_CONST = 5   # MODEL_CONST's cascade, live channels found by geometric gaps
MODEL_GAPS_WC = 6      # MODEL_WC's cascade, live channels found by geometric gaps


@dataclasses.dataclass
class Hypergraph:
    n: int
    he_off: np.ndarray   # uint32[m+1]
    he_mem: np.ndarray   # uint32[nnz]

    @property
    def m(self) -> int:
        return int(self.he_off.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.he_mem.shape[0])

    def edges(self):
        """Yield each hyperedge's member list (host-side convenience)."""
        for e in range(self.m):
            yield self.he_mem[self.he_off[e]:self.he_off[e + 1]]


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    m: int
    sizes: tuple            # ("uniform", lo, hi) or ("powerlaw", gamma, lo, hi)
    members: tuple          # ("uniform",) or ("zipf", s)
    model: int              # MODEL_CONST .. MODEL_GAPS_WC
    p: float                # used when model == MODEL_CONST
    k: int
    eps: float
    ell: float
    gen_seed: int
    philox_seed: int = 0

    def build(self) -> Hypergraph:
        return make_hypergraph(self.n, self.m, self.sizes, self.members, self.gen_seed)


# The synthetic stand-ins.  "tiny" is small enough for the oracle to run the
# whole query in seconds; "mid" is the single-GPU measurement workload;
# "large" is the supercritical, heavily skewed case.
WORKLOADS = {
    "tiny": Workload("tiny", 1_000, 2_000, ("uniform", 2, 6), ("uniform",),
                     MODEL_CONST, 0.05, 10, 0.5, 1.0, gen_seed=0),
    "mid": Workload("mid", 100_000, 200_000, ("powerlaw", 2.5, 2, 50), ("zipf", 1.0),
                    MODEL_WC, 0.0, 50, 0.1, 1.0, gen_seed=1),
    "large": Workload("large", 1_000_000, 2_000_000, ("powerlaw", 2.2, 2, 200), ("zipf", 1.1),
                      MODEL_CONST, 0.01, 100, 0.1, 1.0, gen_seed=2),
    # the same hypergraphs under the linear-threshold model (weighted cascade
    # weights, the standard LT setting)
    "tiny_lt": Workload("tiny_lt", 1_000, 2_000, ("uniform", 2, 6), ("uniform",),
                        MODEL_LT_WC, 0.0, 10, 0.5, 1.0, gen_seed=0),
    "mid_lt": Workload("mid_lt", 100_000, 200_000, ("powerlaw", 2.5, 2, 50), ("zipf", 1.0),
                       MODEL_LT_WC, 0.0, 50, 0.1, 1.0, gen_seed=1),
    "large_lt": Workload("large_lt", 1_000_000, 2_000_000, ("powerlaw", 2.2, 2, 200), ("zipf", 1.1),
                         MODEL_LT_WC, 0.0, 100, 0.1, 1.0, gen_seed=2),
    # ... and under the stratified setting of the sample-set layers
    "tiny_layered": Workload("tiny_layered", 1_000, 2_000, ("uniform", 2, 6), ("uniform",),
                             MODEL_LAYERED, 0.0, 10, 0.5, 1.0, gen_seed=0),
    "mid_layered": Workload("mid_layered", 100_000, 200_000, ("powerlaw", 2.5, 2, 50), ("zipf", 1.0),
                            MODEL_LAYERED, 0.0, 50, 0.1, 1.0, gen_seed=1),
    "large_layered": Workload("large_layered", 1_000_000, 2_000_000, ("powerlaw", 2.2, 2, 200), ("zipf", 1.1),
                              MODEL_LAYERED, 0.0, 100, 0.1, 1.0, gen_seed=2),
    # ... and the independent cascade of tiny / mid / large with its live
    # channels drawn by geometric gaps instead of one coin per channel
    "tiny_gaps": Workload("tiny_gaps", 1_000, 2_000, ("uniform", 2, 6), ("uniform",),
                          MODEL_GAPS_CONST, 0.05, 10, 0.5, 1.0, gen_seed=0),
    "mid_gaps": Workload("mid_gaps", 100_000, 200_000, ("powerlaw", 2.5, 2, 50), ("zipf", 1.0),
                         MODEL_GAPS_WC, 0.0, 50, 0.1, 1.0, gen_seed=1),
    "large_gaps": Workload("large_gaps", 1_000_000, 2_000_000, ("powerlaw", 2.2, 2, 200), ("zipf", 1.1),
                           MODEL_GAPS_CONST, 0.01, 100, 0.1, 1.0, gen_seed=2),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def multi_instance_workloads(count: int = 64, base_seed: int = 1000):
    """Independent IM instances of mixed size: |V| log-uniform in [1e4, 5e5],
    |HE| = 2|V|, sizes power law (2.5) on [2, 100], uniform members,
    p ~ U[0.005, 0.05], k ~ U{10..200}, eps in {0.1, 0.2}."""
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(base_seed + i))
        n = int(round(math.exp(rng.uniform(math.log(1e4), math.log(5e5)))))
        p = float(np.float32(rng.uniform(0.005, 0.05)))
        k = int(rng.integers(10, 201))
        eps = float(rng.choice([0.1, 0.2]))
        out.append(Workload(f"multi{i}", n, 2 * n, ("powerlaw", 2.5, 2, 100), ("uniform",),
                            MODEL_CONST, p, k, eps, 1.0, gen_seed=base_seed + i))
    return out


def serving_workloads(count: int = 16, n_max: int = 5_000_000, n_min: int = 50_000, base_seed: int = 2000):
    """Graphs of the serving pool: |V| log-spaced from n_max down to n_min,
    |HE| = 2|V|, sizes power law (2.1) on [2, 1000], uniform members, weighted
    cascade.  Query parameters (k in {10, 50, 200}, eps = 0.1) are drawn by
    the serving driver."""
    out = []
    for i in range(count):
        n = int(round(n_max * (n_min / n_max) ** (i / max(count - 1, 1))))
        out.append(Workload(f"serve{i}", n, 2 * n, ("powerlaw", 2.1, 2, 1000), ("uniform",),
                            MODEL_WC, 0.0, 50, 0.1, 1.0, gen_seed=base_seed + i))
    return out


def power_law_sizes(rng: np.random.Generator, m: int, gamma: float, lo: int, hi: int) -> np.ndarray:
    """m sizes from P(s) proportional to s**-gamma on [lo, hi], by inverse CDF
    over the exact probability table."""
    s = np.arange(lo, hi + 1, dtype=np.float64)
    pmf = s ** (-gamma)
    cdf = np.cumsum(pmf)
    cdf /= cdf[-1]
    idx = np.searchsorted(cdf, rng.random(m), side="right")
    idx = np.minimum(idx, len(s) - 1)
    return (lo + idx).astype(np.int64)


def uniform_sizes(rng: np.random.Generator, m: int, lo: int, hi: int) -> np.ndarray:
    return rng.integers(lo, hi + 1, size=m).astype(np.int64)


def _popularity_sampler(rng: np.random.Generator, n: int, members: tuple):
    if members[0] == "uniform":
        return lambda size: rng.integers(0, n, size=size, dtype=np.int64)
    if members[0] == "zipf":
        s = float(members[1])
        w = 1.0 / np.arange(1, n + 1, dtype=np.float64) ** s
        cdf = np.cumsum(w)
        cdf /= cdf[-1]
        perm = rng.permutation(n).astype(np.int64)   # rank -> vertex id

        def draw(size):
            r = np.searchsorted(cdf, rng.random(size), side="right")
            return perm[np.minimum(r, n - 1)]
        return draw
    raise ValueError(members)


def draw_members(rng: np.random.Generator, n: int, sizes: np.ndarray, members: tuple) -> np.ndarray:
    """Members of every hyperedge, without replacement inside a hyperedge
    (a duplicate is redrawn until none remain)."""
    if np.any(sizes > n):
        raise ValueError("hyperedge larger than the vertex set")
    draw = _popularity_sampler(rng, n, members)
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    nnz = int(off[-1])
    seg = np.repeat(np.arange(len(sizes), dtype=np.int64), sizes)
    mem = draw(nnz)
    pos_all = np.arange(nnz, dtype=np.int64)
    active = pos_all                       # positions of hyperedges still to check
    while active.size:
        order = np.lexsort((mem[active], seg[active]))
        idx = active[order]
        sm, ss = mem[idx], seg[idx]
        dup = np.zeros(idx.size, dtype=bool)
        dup[1:] = (sm[1:] == sm[:-1]) & (ss[1:] == ss[:-1])
        if not dup.any():
            break
        pos = idx[dup]
        mem[pos] = draw(len(pos))
        bad = np.zeros(len(sizes), dtype=bool)
        bad[seg[pos]] = True
        active = pos_all[bad[seg]]
    return mem


def make_hypergraph(n: int, m: int, sizes_spec: tuple, members: tuple, seed: int) -> Hypergraph:
    rng = np.random.Generator(np.random.PCG64(seed))
    if sizes_spec[0] == "uniform":
        sizes = uniform_sizes(rng, m, sizes_spec[1], sizes_spec[2])
    elif sizes_spec[0] == "powerlaw":
        sizes = power_law_sizes(rng, m, sizes_spec[1], sizes_spec[2], sizes_spec[3])
    else:
        raise ValueError(sizes_spec)
    mem = draw_members(rng, n, sizes, members)
    off = np.zeros(m + 1, dtype=np.uint64)
    np.cumsum(sizes, out=off[1:])
    if off[-1] >= 2 ** 32:
        raise ValueError("nnz must fit in uint32")
    return Hypergraph(n, off.astype(np.uint32), mem.astype(np.uint32))


def tiny_hypergraph(seed: int, n: int, m: int, lo: int = 2, hi: int = 4,
                    allow_singletons: bool = False) -> Hypergraph:
    """Small random hypergraph for exhaustive checks (uniform sizes and members)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = uniform_sizes(rng, m, 1 if allow_singletons else lo, hi)
    sizes = np.minimum(sizes, n)
    mem = draw_members(rng, n, sizes, ("uniform",))
    off = np.zeros(m + 1, dtype=np.uint32)
    np.cumsum(sizes, out=off[1:])
    return Hypergraph(n, off, mem.astype(np.uint32))


def from_lists(n: int, edges) -> Hypergraph:
    """Hypergraph from an explicit list of member lists (order preserved)."""
    sizes = [len(e) for e in edges]
    off = np.zeros(len(edges) + 1, dtype=np.uint32)
    off[1:] = np.cumsum(sizes) if edges else []
    mem = np.array([u for e in edges for u in e], dtype=np.uint32)
    return Hypergraph(n, off, mem)
