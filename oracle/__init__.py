"""CPU oracle for HyperIM's hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke entry point and the benchmark's CPU-baseline
leg may import this package.  It wraps ``hyperim_oracle.c`` (plain C, built
with gcc into ``liboracle.so`` next to it) through ctypes and shares no code
with the GPU library.

Functions (each cites the passage of the paper it follows in the C source):
  philox(ctr, key)            Philox4x32-10 block (SC'11 definition)
  coin(...)                   the keyed coin of one channel (IC, Section 2.1)
  Graph(hg, model, p)         validated hypergraph + incidence lists + thresholds
                              (model 0/1: IC with constant p / weighted cascade;
                              2/3: the linear-threshold model, live-edge form,
                              with the same thresholds; 4: the stratified
                              setting of Section 3.1.1; 5/6: IC with constant
                              p / weighted cascade drawn by geometric gaps)
  Graph.layers()              stratified setting: A(v) by layers
  Graph.stratify()            sample-set layers (Section 3.1.1), strata, P
  Graph.root(...)             stratified root of an RR id
  Graph.rr_set(...)           one RR set (Algorithm 3 skeleton; under LT the
                              reverse walk of the live-edge form), ascending
  Graph.generate(...)         many RR sets as a CSR (threads over ids)
  greedy(...)                 Algorithm 1
  coverage(...)               Lambda_R(S), Equation (1)
  schedule(...)               theta_max / theta_0 / ladder (Section 4)
  sigma_lower / sigma_upper   Equation (12) / Lemma 5
  Graph.select_seeds(...)     Algorithm 4 (HyperIM_BRR loop)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hyperim_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

EINVAL = -1
ENOMEM = -2
NSTRATA = 8


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (always, when force is set)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        u32p = C.POINTER(C.c_uint32)
        u64p = C.POINTER(C.c_uint64)
        vp = C.c_void_p
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox_batch.argtypes = [C.c_uint64, vp, vp, vp]
        L.orc_coin.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_coin.restype = C.c_uint32
        L.orc_graph_new.argtypes = [C.c_uint32, C.c_uint32, vp, vp, C.c_uint32, C.c_float, C.POINTER(vp)]
        L.orc_graph_free.argtypes = [vp]
        L.orc_graph_export.argtypes = [vp, vp, vp, vp, vp]
        L.orc_stratify.argtypes = [vp]
        L.orc_strata_export.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_block_of.argtypes = [C.c_uint64, C.c_uint32, u32p, u64p, u64p]
        L.orc_block_offset.argtypes = [C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_block_offset.restype = C.c_uint64
        L.orc_root.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32]
        L.orc_root.restype = C.c_uint32
        L.orc_rr_set.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32, vp]
        L.orc_rr_set.restype = C.c_uint32
        L.orc_rr_set_rooted.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32, vp]
        L.orc_rr_set_rooted.restype = C.c_uint32
        L.orc_generate.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64,
                                   C.c_uint32, C.c_uint32, vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]
        L.orc_free.argtypes = [vp]
        L.orc_greedy.argtypes = [C.c_uint32, C.c_uint64, vp, vp, C.c_uint32, vp, vp]
        L.orc_coverage.argtypes = [C.c_uint32, C.c_uint64, vp, vp, C.c_uint32, vp]
        L.orc_coverage.restype = C.c_uint64
        L.orc_make_schedule.argtypes = [C.c_uint32, C.c_uint32, C.c_double, C.c_double, C.c_uint32, vp]
        L.orc_sigma_lower.argtypes = [C.c_double] * 4
        L.orc_sigma_lower.restype = C.c_double
        L.orc_sigma_upper.argtypes = [C.c_double, C.c_uint32, C.c_double, C.c_double, C.c_double]
        L.orc_sigma_upper.restype = C.c_double
        L.orc_select_seeds.argtypes = [vp, C.c_uint32, C.c_double, C.c_double, C.c_uint64, C.c_uint32,
                                       C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint32, vp, vp, vp]
        L.orc_upper_eq8.argtypes = [C.c_uint32, C.c_uint64, vp, vp, C.c_uint32, vp]
        L.orc_upper_eq8.restype = C.c_uint64
        L.orc_sigma_upper_cov.argtypes = [C.c_double] * 4
        L.orc_sigma_upper_cov.restype = C.c_double
        L.orc_layers_export.argtypes = [vp, vp, vp, vp, vp]
        L.orc_route.argtypes = [vp, C.c_int, u32p]
        L.orc_route_export.argtypes = [vp, vp, vp, vp]
        L.orc_gap_draw.argtypes = [C.c_double, C.c_uint32, C.c_uint32]
        L.orc_gap_draw.restype = C.c_uint32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def philox(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def philox_batch(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """Philox4x32-10 of many records: ctr u32[N,4], key u32[N,2] -> u32[N,4]."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32)
    key = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros_like(ctr)
    lib().orc_philox_batch(ctr.shape[0], _p(ctr), _p(key), _p(out))
    return out


def block_of(j: int, qlog: int = 8):
    """Ladder block of RR id j: (b, first id J, size T)."""
    b, J, T = C.c_uint32(0), C.c_uint64(0), C.c_uint64(0)
    lib().orc_block_of(j, qlog, C.byref(b), C.byref(J), C.byref(T))
    return b.value, J.value, T.value


def block_offset(n: int, seed: int, instance: int, pool: int, b: int) -> int:
    """Random offset o_b of ladder block b of a pool."""
    return int(lib().orc_block_offset(n, seed, instance, pool, b))


def coin(seed, instance, pool, j, he, v, pos) -> int:
    return int(lib().orc_coin(seed, instance, pool, j, he, v, pos))


class _Schedule(C.Structure):
    _fields_ = [("delta", C.c_double), ("lnC", C.c_double), ("theta_max", C.c_double),
                ("theta0", C.c_double), ("a", C.c_double), ("theta1", C.c_uint64),
                ("i_max", C.c_uint32)]


class _Result(C.Structure):
    _fields_ = [("rounds", C.c_uint32), ("i_max", C.c_uint32), ("theta", C.c_uint64),
                ("lambda1", C.c_uint64), ("lambda2", C.c_uint64), ("sigma_l", C.c_double),
                ("sigma_u", C.c_double), ("spread", C.c_double), ("theta_max", C.c_double),
                ("entries1", C.c_uint64), ("entries2", C.c_uint64), ("lambda_u", C.c_uint64)]


def schedule(n, k, eps, ell, qlog=8) -> dict:
    s = _Schedule()
    rc = lib().orc_make_schedule(n, k, eps, ell, qlog, C.byref(s))
    if rc:
        raise ValueError("invalid schedule arguments (%d)" % rc)
    return {f: getattr(s, f) for f, _ in _Schedule._fields_}


def sigma_lower(lambda2, a, n, theta) -> float:
    return float(lib().orc_sigma_lower(lambda2, a, n, theta))


def sigma_upper(lambda1, k, a, n, theta) -> float:
    return float(lib().orc_sigma_upper(lambda1, k, a, n, theta))


def sigma_upper_cov(cov_upper, a, n, theta) -> float:
    return float(lib().orc_sigma_upper_cov(cov_upper, a, n, theta))


def upper_eq8(n, off, mem, seeds, theta=None) -> int:
    """Equation (8) (p_max = 1) for greedy seeds in selection order."""
    off = np.ascontiguousarray(off, dtype=np.uint64)
    mem = np.ascontiguousarray(mem, dtype=np.uint32)
    seeds = np.ascontiguousarray(seeds, dtype=np.uint32)
    theta = len(off) - 1 if theta is None else theta
    return int(lib().orc_upper_eq8(n, theta, _p(off), _p(mem if mem.size else np.zeros(1, np.uint32)),
                                   len(seeds), _p(seeds)))


def gap_draw(q: float, x: int, G: int) -> int:
    """Geometric-gap sampler: the gap drawn from word x with G positions left
    (q = 1 - p)."""
    return int(lib().orc_gap_draw(q, x, G))


def greedy(n, off: np.ndarray, mem: np.ndarray, k: int, theta: int | None = None):
    off = np.ascontiguousarray(off, dtype=np.uint64)
    mem = np.ascontiguousarray(mem, dtype=np.uint32)
    theta = len(off) - 1 if theta is None else theta
    seeds = np.zeros(k, dtype=np.uint32)
    gains = np.zeros(k, dtype=np.uint64)
    rc = lib().orc_greedy(n, theta, _p(off), _p(mem if mem.size else np.zeros(1, np.uint32)), k,
                          _p(seeds), _p(gains))
    if rc:
        raise ValueError("greedy failed (%d)" % rc)
    return seeds, gains


def coverage(n, off, mem, seeds, theta=None) -> int:
    off = np.ascontiguousarray(off, dtype=np.uint64)
    mem = np.ascontiguousarray(mem, dtype=np.uint32)
    seeds = np.ascontiguousarray(seeds, dtype=np.uint32)
    theta = len(off) - 1 if theta is None else theta
    return int(lib().orc_coverage(n, theta, _p(off), _p(mem if mem.size else np.zeros(1, np.uint32)),
                                  len(seeds), _p(seeds)))


class OracleError(RuntimeError):
    pass


class Graph:
    """Oracle view of one hypergraph (validated copy, incidence lists,
    thresholds; strata after stratify())."""

    def __init__(self, hg, model: int, p: float = 0.0):
        self.n = int(hg.n)
        self.m = int(hg.m)
        he_off = np.ascontiguousarray(hg.he_off, dtype=np.uint32)
        he_mem = np.ascontiguousarray(hg.he_mem, dtype=np.uint32)
        if he_mem.size == 0:
            he_mem = np.zeros(1, np.uint32)
        h = C.c_void_p()
        rc = lib().orc_graph_new(self.n, self.m, _p(he_off), _p(he_mem), model, C.c_float(p), C.byref(h))
        if rc:
            raise OracleError("orc_graph_new: %d" % rc)
        self._h = h
        self.nnz = int(hg.he_off[-1])
        self.stratified = False

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_graph_free(self._h)
            self._h = None

    def arrays(self):
        v_off = np.zeros(self.n + 1, np.uint32)
        v_he = np.zeros(max(self.nnz, 1), np.uint32)
        thr = np.zeros(max(self.n, 1), np.uint32)
        c = np.zeros(max(self.n, 1), np.uint64)
        lib().orc_graph_export(self._h, _p(v_off), _p(v_he), _p(thr), _p(c))
        return {"v_off": v_off, "v_he": v_he[:self.nnz], "thr": thr[:self.n], "c": c[:self.n]}

    def stratify(self):
        rc = lib().orc_stratify(self._h)
        if rc:
            raise OracleError("orc_stratify: %d" % rc)
        self.stratified = True
        return self.strata()

    def strata(self):
        n = max(self.n, 1)
        out = {k: np.zeros(n, np.uint32) for k in ("l", "deg", "top", "P")}
        out["stratum"] = np.zeros(n, np.uint8)
        B = np.zeros(NSTRATA + 1, np.uint32)
        stats = np.zeros(3, np.float64)
        lib().orc_strata_export(self._h, _p(out["l"]), _p(out["deg"]), _p(out["top"]),
                                _p(out["stratum"]), _p(out["P"]), _p(B), _p(stats))
        out = {k: v[:self.n] for k, v in out.items()}
        out["B"] = B
        out["alpha"], out["beta"], out["theta_l"] = (float(x) for x in stats)
        return out

    def layers(self):
        """Stratified-setting model (or a graph divided by route()): per vertex the members of A(v) layer by
        layer (layer 1 = largest w(v,u)), ascending ids within a layer, as
        (nb_off, nb, ly_off, ly_end): layer i of v is nb[nb_off[v] + ly_end[ly_off[v] + i - 2]
        .. nb_off[v] + ly_end[ly_off[v] + i - 1]) (the first layer starts at nb_off[v])."""
        st = self.strata()
        n = self.n
        nb_off = np.zeros(n + 1, np.uint64)
        ly_off = np.zeros(n + 1, np.uint64)
        nb = np.zeros(max(int(st["deg"].sum()), 1), np.uint32)
        ly_end = np.zeros(max(int(st["l"].sum()), 1), np.uint32)
        rc = lib().orc_layers_export(self._h, _p(nb_off), _p(nb), _p(ly_off), _p(ly_end))
        if rc:
            raise OracleError("orc_layers_export: %d" % rc)
        return nb_off, nb[:int(st["deg"].sum())], ly_off, ly_end[:int(st["l"].sum())]

    def route(self, on: bool = True) -> int:
        """Division of the RR sets into R1 / R2 (Section 4.1), after stratify():
        pool 0 then draws its roots from the vertices with a small layer
        (|L_i| < alpha |A(v)| for some i <= floor(beta)) and its sets start from
        the root and those layers' members; pool 1 draws from the other
        vertices.  Returns the number of R1 vertices (the division is inert
        when that is 0 or n)."""
        n1 = C.c_uint32()
        rc = lib().orc_route(self._h, 1 if on else 0, C.byref(n1))
        if rc:
            raise OracleError("orc_route: %d" % rc)
        return int(n1.value)

    def route_tables(self):
        """(rP, f_off, f_mem) of a divided graph: R1 roots rP[:n1], R2 roots
        rP[n1:], and the forced members of each vertex."""
        n = self.n
        rP = np.zeros(max(n, 1), np.uint32)
        f_off = np.zeros(n + 1, np.uint64)
        nb_total = int(self.strata()["deg"].sum())
        f_mem = np.zeros(max(nb_total, 1), np.uint32)
        rc = lib().orc_route_export(self._h, _p(rP), _p(f_off), _p(f_mem))
        if rc:
            raise OracleError("orc_route_export: %d" % rc)
        return rP[:n], f_off, f_mem[:int(f_off[-1])]

    def root(self, seed, instance, pool, j, qlog=8) -> int:
        return int(lib().orc_root(self._h, seed, instance, pool, j, qlog))

    def rr_set(self, seed, instance, pool, j, qlog=8, root=None) -> np.ndarray:
        out = np.zeros(max(self.n, 1), np.uint32)
        if root is None:
            sz = lib().orc_rr_set(self._h, seed, instance, pool, j, qlog, _p(out))
        else:
            sz = lib().orc_rr_set_rooted(self._h, seed, instance, pool, j, int(root), _p(out))
        return out[:sz].copy()

    def generate(self, seed, instance, pool, id_begin, id_end, qlog=8, nthreads=None, roots=None):
        """RR sets [id_begin, id_end) as (off u64[count+1], mem u32, roots u32)."""
        if nthreads is None:
            nthreads = os.cpu_count() or 1
        o, mm, r = C.c_void_p(), C.c_void_p(), C.c_void_p()
        rin = None
        if roots is not None:
            rin = np.ascontiguousarray(roots, dtype=np.uint32)
        rc = lib().orc_generate(self._h, seed, instance, pool, id_begin, id_end, qlog, nthreads,
                                _p(rin) if rin is not None else None, C.byref(o), C.byref(mm), C.byref(r))
        if rc:
            raise OracleError("orc_generate: %d" % rc)
        count = id_end - id_begin
        off = np.ctypeslib.as_array(C.cast(o, C.POINTER(C.c_uint64)), shape=(count + 1,)).copy()
        total = int(off[-1])
        mem = (np.ctypeslib.as_array(C.cast(mm, C.POINTER(C.c_uint32)), shape=(total,)).copy()
               if total else np.zeros(0, np.uint32))
        rts = (np.ctypeslib.as_array(C.cast(r, C.POINTER(C.c_uint32)), shape=(count,)).copy()
               if count else np.zeros(0, np.uint32))
        for ptr in (o, mm, r):
            lib().orc_free(ptr)
        return off, mem, rts

    def select_seeds(self, k, eps, ell, seed=0, instance=0, qlog=8, theta_fixed=0, nthreads=None, bound=0):
        """Algorithm 4; bound 0 = Equation (8)'s upper bound, 1 = Lemma 5's closed form."""
        if nthreads is None:
            nthreads = os.cpu_count() or 1
        seeds = np.zeros(k, np.uint32)
        gains = np.zeros(k, np.uint64)
        res = _Result()
        rc = lib().orc_select_seeds(self._h, k, eps, ell, seed, instance, qlog, theta_fixed, nthreads, bound,
                                    _p(seeds), _p(gains), C.byref(res))
        if rc:
            raise OracleError("orc_select_seeds: %d" % rc)
        out = {f: getattr(res, f) for f, _ in _Result._fields_}
        out["seeds"] = seeds
        out["gains"] = gains
        return out
