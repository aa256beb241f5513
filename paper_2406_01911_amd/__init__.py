"""Python binding of libhyperim (HyperIM's hot path on MI355X / gfx950).

Argument marshalling only: every step runs in the HIP library through its C
ABI (include/hyperim.h).  PyTorch supplies device memory and streams; it is
imported first so that the library binds to the same HIP runtime as torch.
There is no CPU fallback: if libhyperim.so has not been built, importing the
library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (must load the HIP runtime before libhyperim.so)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhyperim.so")

OK, EINVAL, ENOMEM, ECAPACITY, ESTATE, EHIP = 0, -1, -2, -3, -4, -5
PENDING = 1
MODEL_CONST, MODEL_WC, MODEL_LT_CONST, MODEL_LT_WC, MODEL_LAYERED = 0, 1, 2, 3, 4
MODEL_GAPS_CONST, MODEL_GAPS_WC = 5, 6
NSTRATA = 8
FLAG_INCIDENCES = 1
FLAG_KERNEL_TIMES = 2
FLAG_NO_GRAPHS = 4


class HyperIMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class _Prob(C.Structure):
    _fields_ = [("model", C.c_uint32), ("p", C.c_float)]


class _StrataInfo(C.Structure):
    _fields_ = [("B", C.c_uint32 * (NSTRATA + 1)), ("sum_top", C.c_uint64), ("sum_deg", C.c_uint64),
                ("sum_l", C.c_uint64), ("alpha", C.c_double), ("beta", C.c_double), ("theta_l", C.c_double)]


class _Options(C.Structure):
    _fields_ = [("qlog", C.c_uint32), ("form", C.c_uint32), ("theta_fixed", C.c_uint64),
                ("max_entries", C.c_uint64), ("flags", C.c_uint32), ("ahead", C.c_uint32), ("bound", C.c_uint32)]


class _Result(C.Structure):
    _fields_ = [("rounds", C.c_uint32), ("i_max", C.c_uint32), ("theta", C.c_uint64), ("lambda1", C.c_uint64),
                ("lambda2", C.c_uint64), ("sigma_l", C.c_double), ("sigma_u", C.c_double), ("spread", C.c_double),
                ("theta_max", C.c_double), ("entries1", C.c_uint64), ("entries2", C.c_uint64),
                ("incidences", C.c_uint64), ("ms_rr", C.c_double), ("ms_greedy", C.c_double),
                ("ms_total", C.c_double), ("alg_bytes", C.c_uint64), ("ms_bfs", C.c_double),
                ("bfs_launches", C.c_uint64), ("ms_light", C.c_double), ("ms_heavy", C.c_double),
                ("deferred", C.c_uint64), ("supersteps", C.c_uint64), ("bytes_light", C.c_uint64),
                ("bytes_heavy", C.c_uint64), ("ms_expand", C.c_double), ("expand_launches", C.c_uint64),
                ("philox_drawn", C.c_uint64), ("coins", C.c_uint64), ("philox_alg", C.c_uint64),
                ("philox_bundled", C.c_uint64), ("bytes_bundled", C.c_uint64), ("ms_bundled", C.c_double),
                ("bundled_launches", C.c_uint64), ("philox_light", C.c_uint64), ("lambda_u", C.c_uint64)]


class _Tuning(C.Structure):
    _fields_ = [("heavy", C.c_uint32), ("budget", C.c_uint32), ("chunk", C.c_uint32), ("seg", C.c_uint32),
                ("prefilter_min", C.c_uint32), ("steps_per_sync", C.c_uint32), ("stage_mib", C.c_uint32),
                ("blocks_a", C.c_uint32), ("blocks_b", C.c_uint32), ("ms_min", C.c_uint32),
                ("ms_filter", C.c_uint32)]


class _Query(C.Structure):
    _fields_ = [("graph", C.c_void_p), ("k", C.c_uint32), ("instance", C.c_uint32), ("eps", C.c_double),
                ("ell", C.c_double), ("seed", C.c_uint64)]


class _RRTask(C.Structure):
    _fields_ = [("graph", C.c_void_p), ("pool", C.c_void_p), ("seed", C.c_uint64), ("instance", C.c_uint32),
                ("pool_tag", C.c_uint32), ("id_begin", C.c_uint64), ("id_end", C.c_uint64)]


class _SessionStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("admitted", C.c_uint64), ("finished", C.c_uint64),
                ("failed", C.c_uint64), ("active", C.c_uint32), ("waiting", C.c_uint32), ("steps", C.c_uint64),
                ("ran_last", C.c_uint64), ("bytes_resident", C.c_size_t), ("hbm_budget", C.c_size_t)]


TUNING_FIELDS = ["heavy", "budget", "chunk", "seg", "prefilter_min", "steps_per_sync", "stage_mib", "blocks_a",
                 "blocks_b", "ms_min", "ms_filter"]

EXPORTS = ["hyperim_build_graph", "hyperim_stratify", "hyperim_route", "hyperim_graph_read", "hyperim_pool_create",
           "hyperim_generate_rr", "hyperim_generate_rr_batch", "hyperim_pool_view", "hyperim_pool_read", "hyperim_pool_required",
           "hyperim_pool_reset", "hyperim_greedy", "hyperim_coverage", "hyperim_coverage_noalloc",
           "hyperim_select_seeds",
           "hyperim_select_seeds_batch", "hyperim_session_create", "hyperim_session_submit",
           "hyperim_session_step", "hyperim_session_poll", "hyperim_session_drop", "hyperim_session_stats_get",
           "hyperim_session_free", "hyperim_workspace_info", "hyperim_workspace_release",
           "hyperim_set_tuning", "hyperim_get_tuning",
           "hyperim_pool_free", "hyperim_graph_free", "hyperim_strerror"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhyperim.so (raises if it is missing: no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing; build it with paper_2406_01911_amd/build.py "
                          "(or __graft_entry__.build())")
    L = C.CDLL(path)
    vp, u32, u64, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
    L.hyperim_build_graph.argtypes = [u32, u32, vp, vp, i32, _Prob, vp, C.POINTER(vp)]
    L.hyperim_stratify.argtypes = [vp, vp, C.POINTER(_StrataInfo)]
    L.hyperim_route.argtypes = [vp, u32, vp, C.POINTER(u32)]
    L.hyperim_graph_read.argtypes = [vp] + [vp] * 9 + [i32, vp]
    L.hyperim_pool_create.argtypes = [vp, vp, C.c_size_t, u64, C.POINTER(vp)]
    L.hyperim_generate_rr.argtypes = [vp, u64, u32, u32, u64, u64, vp, vp]
    L.hyperim_generate_rr_batch.argtypes = [C.POINTER(_RRTask), u32, u32, vp]
    L.hyperim_pool_view.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(u64), C.POINTER(u64)]
    L.hyperim_pool_read.argtypes = [vp, vp, vp, vp, i32, vp]
    L.hyperim_pool_required.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.hyperim_pool_reset.argtypes = [vp]
    L.hyperim_greedy.argtypes = [vp, vp, u64, u32, vp, vp, vp]
    L.hyperim_coverage.argtypes = [vp, vp, u64, vp, u32, vp, C.POINTER(u64)]
    L.hyperim_coverage_noalloc.argtypes = [vp, vp, u64, vp, u32, vp, vp]
    L.hyperim_select_seeds.argtypes = [vp, u32, C.c_double, C.c_double, u64, u32, C.POINTER(_Options), vp, vp, vp,
                                       C.POINTER(_Result)]
    L.hyperim_select_seeds_batch.argtypes = [C.POINTER(_Query), u32, C.POINTER(_Options), vp, vp, vp,
                                             C.POINTER(_Result), C.POINTER(i32), C.POINTER(_Result)]
    L.hyperim_session_create.argtypes = [C.c_size_t, C.POINTER(_Options), vp, C.POINTER(vp)]
    L.hyperim_session_submit.argtypes = [vp, C.POINTER(_Query), C.POINTER(u64)]
    L.hyperim_session_step.argtypes = [vp, C.POINTER(_SessionStats)]
    L.hyperim_session_poll.argtypes = [vp, u64, vp, vp, C.POINTER(_Result)]
    L.hyperim_session_drop.argtypes = [vp, vp]
    L.hyperim_session_stats_get.argtypes = [vp, C.POINTER(_SessionStats)]
    L.hyperim_session_free.argtypes = [vp]
    L.hyperim_session_free.restype = None
    L.hyperim_workspace_info.argtypes = [C.POINTER(C.c_size_t)]
    L.hyperim_workspace_release.argtypes = []
    L.hyperim_set_tuning.argtypes = [vp, C.POINTER(_Tuning)]
    L.hyperim_get_tuning.argtypes = [vp, C.POINTER(_Tuning)]
    L.hyperim_pool_free.argtypes = [vp]
    L.hyperim_pool_free.restype = None
    L.hyperim_graph_free.argtypes = [vp]
    L.hyperim_graph_free.restype = None
    L.hyperim_strerror.argtypes = [i32]
    L.hyperim_strerror.restype = C.c_char_p
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        raise HyperIMError(rc, _lib.hyperim_strerror(rc).decode())


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


class Graph:
    """Handle of a device-resident hypergraph (hyperim_build_graph)."""

    def __init__(self, handle, n, m, nnz):
        self._h = handle
        self.n, self.m, self.nnz = n, m, nnz
        self.info = None

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hyperim_graph_free(self._h)
            self._h = None

    # hyperim_stratify
    def stratify(self, stream=None) -> dict:
        info = _StrataInfo()
        _check(_lib.hyperim_stratify(self._h, _stream(stream), C.byref(info)))
        self.info = {"B": np.array(list(info.B), np.uint32), "sum_top": info.sum_top, "sum_deg": info.sum_deg,
                     "sum_l": info.sum_l, "alpha": info.alpha, "beta": info.beta, "theta_l": info.theta_l}
        return self.info

    # hyperim_route
    def route(self, on: bool = True, stream=None) -> int:
        """Division of the RR sets into R1 (pool 0) and R2 (pool 1) of
        Section 4.1 (biased; see hyperim_route); returns the number of R1
        vertices."""
        n1 = C.c_uint32()
        _check(_lib.hyperim_route(self._h, 1 if on else 0, _stream(stream), C.byref(n1)))
        return int(n1.value)

    # hyperim_set_tuning / hyperim_get_tuning
    def set_tuning(self, **kw):
        t = _Tuning()
        for k, v in kw.items():
            if k not in TUNING_FIELDS:
                raise KeyError(k)
            setattr(t, k, int(v))
        _check(_lib.hyperim_set_tuning(self._h, C.byref(t)))
        return self.tuning()

    def tuning(self) -> dict:
        t = _Tuning()
        _check(_lib.hyperim_get_tuning(self._h, C.byref(t)))
        return {k: getattr(t, k) for k in TUNING_FIELDS}

    # hyperim_graph_read
    def read(self, strata: bool = True) -> dict:
        n, nnz = self.n, self.nnz
        out = {"v_off": np.zeros(n + 1, np.uint32), "v_he": np.zeros(max(nnz, 1), np.uint32),
               "thr": np.zeros(n, np.uint32), "c": np.zeros(n, np.uint64)}
        if strata:
            out.update({"l": np.zeros(n, np.uint32), "deg": np.zeros(n, np.uint32), "top": np.zeros(n, np.uint32),
                        "stratum": np.zeros(n, np.uint8), "P": np.zeros(n, np.uint32)})
        keys = ["v_off", "v_he", "thr", "c", "l", "deg", "top", "stratum", "P"]
        _check(_lib.hyperim_graph_read(self._h, *[_ptr(out.get(k)) for k in keys], 0, None))
        out["v_he"] = out["v_he"][:nnz]
        return out


def build_graph(n: int, he_off, he_mem, model: int, p: float = 0.0, stream=None) -> Graph:
    """hyperim_build_graph: he_off/he_mem as numpy (host) or torch cuda tensors (device).
    model: MODEL_CONST / MODEL_WC (independent cascade), MODEL_LT_CONST / MODEL_LT_WC
    (linear threshold), MODEL_LAYERED (stratified setting; p ignored),
    MODEL_GAPS_CONST / MODEL_GAPS_WC (independent cascade with live channels
    drawn by geometric gaps)."""
    load_library()
    on_dev = isinstance(he_off, torch.Tensor) and he_off.is_cuda
    if not on_dev:
        he_off = np.ascontiguousarray(he_off, dtype=np.uint32)
        he_mem = np.ascontiguousarray(he_mem, dtype=np.uint32)
        if he_mem.size == 0:
            he_mem = np.zeros(1, np.uint32)
        m = he_off.shape[0] - 1
        nnz = int(he_off[-1])
    else:
        assert he_off.dtype == torch.int32 and he_mem.dtype == torch.int32, "device arrays are int32 views of uint32"
        m = he_off.shape[0] - 1
        nnz = int(he_off[-1].item()) & 0xFFFFFFFF
    h = C.c_void_p()
    _check(_lib.hyperim_build_graph(n, m, _ptr(he_off), _ptr(he_mem), 1 if on_dev else 0, _Prob(model, p),
                                    _stream(stream), C.byref(h)))
    return Graph(h, n, m, nnz)


class Pool:
    """RR-set pool (hyperim_pool_create); library-owned storage unless buf is given."""

    def __init__(self, g: Graph, buf: torch.Tensor | None = None, id_capacity: int = 0):
        self.g = g
        self._buf = buf
        h = C.c_void_p()
        if buf is None:
            _check(_lib.hyperim_pool_create(g._h, None, 0, 0, C.byref(h)))
        else:
            _check(_lib.hyperim_pool_create(g._h, C.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(),
                                            id_capacity, C.byref(h)))
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hyperim_pool_free(self._h)
            self._h = None

    def view(self):
        off, mem, roots = C.c_void_p(), C.c_void_p(), C.c_void_p()
        b, cnt = C.c_uint64(), C.c_uint64()
        _check(_lib.hyperim_pool_view(self._h, C.byref(off), C.byref(mem), C.byref(roots), C.byref(b),
                                      C.byref(cnt)))
        return {"off": off.value, "mem": mem.value, "roots": roots.value, "id_begin": b.value, "count": cnt.value}

    def read(self, stream=None):
        """(off u64[count+1], mem u32[total], roots u32[count]) as numpy arrays."""
        v = self.view()
        count = v["count"]
        off = np.zeros(count + 1, np.uint64)
        _check(_lib.hyperim_pool_read(self._h, _ptr(off), None, None, 0, _stream(stream)))
        total = int(off[-1])
        mem = np.zeros(max(total, 1), np.uint32)
        roots = np.zeros(max(count, 1), np.uint32)
        _check(_lib.hyperim_pool_read(self._h, None, _ptr(mem), _ptr(roots), 0, _stream(stream)))
        return off, mem[:total], roots[:count]

    def required(self) -> int:
        b = C.c_size_t()
        _check(_lib.hyperim_pool_required(self._h, C.byref(b)))
        return b.value

    def reset(self):
        _check(_lib.hyperim_pool_reset(self._h))


def generate_rr(g: Graph, seed: int, instance: int, pool_tag: int, id_begin: int, id_end: int, pool: Pool,
                stream=None):
    """hyperim_generate_rr: append RR ids [id_begin, id_end) to pool."""
    _check(_lib.hyperim_generate_rr(g._h, seed, instance, pool_tag, id_begin, id_end, pool._h, _stream(stream)))


def generate_rr_batch(tasks, form: int = 0, stream=None):
    """hyperim_generate_rr_batch: tasks is a list of dicts with graph, pool,
    seed, instance, pool_tag, id_begin, id_end; all generated in one call
    (shared launch groups for form 0)."""
    arr = (_RRTask * max(len(tasks), 1))()
    for i, t in enumerate(tasks):
        arr[i] = _RRTask(t["graph"]._h, t["pool"]._h, t.get("seed", 0), t.get("instance", 0), t.get("pool_tag", 0),
                         t["id_begin"], t["id_end"])
    _check(_lib.hyperim_generate_rr_batch(arr, len(tasks), form, _stream(stream)))


def greedy(g: Graph, pool: Pool, theta: int, k: int, stream=None):
    """hyperim_greedy -> (seeds u32[k], gains u64[k])."""
    seeds = np.zeros(k, np.uint32)
    gains = np.zeros(k, np.uint64)
    _check(_lib.hyperim_greedy(g._h, pool._h, theta, k, _stream(stream), _ptr(seeds), _ptr(gains)))
    return seeds, gains


def coverage(g: Graph, pool: Pool, theta: int, seeds, stream=None) -> int:
    """hyperim_coverage: number of the first theta sets meeting the seeds."""
    seeds = np.ascontiguousarray(seeds, dtype=np.uint32)
    out = C.c_uint64()
    _check(_lib.hyperim_coverage(g._h, pool._h, theta, _ptr(seeds) if seeds.size else None, seeds.size,
                                 _stream(stream), C.byref(out)))
    return out.value


def coverage_noalloc(g: Graph, pool: Pool, theta: int, seeds_dev: torch.Tensor, out_dev: torch.Tensor,
                     stream=None) -> None:
    """hyperim_coverage_noalloc: seeds_dev (int32/uint32 device tensor of k
    ids) and out_dev (one 64-bit device word) stay on the device; the call is
    stream-ordered and does not wait."""
    if seeds_dev.dtype not in (torch.int32,) or not seeds_dev.is_cuda or not seeds_dev.is_contiguous():
        raise ValueError("seeds_dev must be a contiguous int32 CUDA tensor")
    if out_dev.dtype != torch.int64 or not out_dev.is_cuda or out_dev.numel() < 1:
        raise ValueError("out_dev must be an int64 CUDA tensor")
    k = seeds_dev.numel()
    _check(_lib.hyperim_coverage_noalloc(g._h, pool._h, theta, C.c_void_p(seeds_dev.data_ptr()) if k else None, k,
                                         _stream(stream), C.c_void_p(out_dev.data_ptr())))


def select_seeds(g: Graph, k: int, eps: float, ell: float, seed: int = 0, instance: int = 0, qlog: int = 0,
                 form: int = 0, theta_fixed: int = 0, max_entries: int = 0, flags: int = 0, stream=None,
                 ahead: int = 0, bound: int = 0) -> dict:
    """hyperim_select_seeds (HyperIM_BRR loop) -> dict with seeds, gains and the result fields.
    ahead: hyperim_options.ahead (0: device default, 1: off)."""
    seeds = np.zeros(k, np.uint32)
    gains = np.zeros(k, np.uint64)
    opt = _Options(qlog, form, theta_fixed, max_entries, flags, ahead, bound)
    res = _Result()
    _check(_lib.hyperim_select_seeds(g._h, k, eps, ell, seed, instance, C.byref(opt), _stream(stream),
                                     _ptr(seeds), _ptr(gains), C.byref(res)))
    out = {f: getattr(res, f) for f, _ in _Result._fields_}
    out["seeds"] = seeds
    out["gains"] = gains
    return out


def _result_dict(res: _Result) -> dict:
    return {f: getattr(res, f) for f, _ in _Result._fields_}


def _query(q) -> _Query:
    """q: dict or tuple (graph, k, eps, ell, seed, instance)."""
    if isinstance(q, dict):
        g, k, eps, ell = q["graph"], q["k"], q["eps"], q.get("ell", 1.0)
        seed, inst = q.get("seed", 0), q.get("instance", 0)
    else:
        g, k, eps, ell, seed, inst = q
    return _Query(g._h, int(k), int(inst), float(eps), float(ell), int(seed))


def select_seeds_batch(queries, qlog: int = 0, form: int = 0, theta_fixed: int = 0, max_entries: int = 0,
                       flags: int = 0, stream=None, raise_on_error: bool = True, totals: dict | None = None,
                       ahead: int = 0, bound: int = 0) -> list:
    """hyperim_select_seeds_batch: queries answered together (shared RR launches).

    Each query is a dict {graph, k, eps, ell, seed, instance}; returns one dict
    per query (seeds, gains, result fields, status).  If `totals` is a dict it
    receives the whole-batch result fields."""
    qs = [_query(q) for q in queries]
    arr = (_Query * max(len(qs), 1))(*qs)
    ks = [q.k for q in qs]
    seeds = np.zeros(max(sum(ks), 1), np.uint32)
    gains = np.zeros(max(sum(ks), 1), np.uint64)
    res = (_Result * max(len(qs), 1))()
    status = (C.c_int * max(len(qs), 1))()
    opt = _Options(qlog, form, theta_fixed, max_entries, flags, ahead, bound)
    tot = _Result()
    rc = _lib.hyperim_select_seeds_batch(arr, len(qs), C.byref(opt), _stream(stream), _ptr(seeds), _ptr(gains),
                                         res, status, C.byref(tot))
    if totals is not None:
        totals.update(_result_dict(tot))
    if raise_on_error:
        _check(rc)
    out, at = [], 0
    for i, k in enumerate(ks):
        d = _result_dict(res[i])
        d["seeds"] = seeds[at:at + k].copy()
        d["gains"] = gains[at:at + k].copy()
        d["status"] = status[i]
        out.append(d)
        at += k
    return out


class Session:
    """Serving session (hyperim_session_*): submit queries at any time, step
    to advance every admitted query by one round, poll for results."""

    def __init__(self, hbm_budget: int = 0, qlog: int = 0, form: int = 0, theta_fixed: int = 0,
                 max_entries: int = 0, flags: int = 0, stream=None, ahead: int = 0, bound: int = 0):
        load_library()
        opt = _Options(qlog, form, theta_fixed, max_entries, flags, ahead, bound)
        h = C.c_void_p()
        _check(_lib.hyperim_session_create(int(hbm_budget), C.byref(opt), _stream(stream), C.byref(h)))
        self._h = h
        self._k = {}
        self._graphs = {}   # keep graphs alive while the session may hold their pools

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hyperim_session_free(self._h)
            self._h = None
            self._graphs = {}

    def submit(self, graph: Graph, k: int, eps: float, ell: float = 1.0, seed: int = 0, instance: int = 0) -> int:
        q = _Query(graph._h, int(k), int(instance), float(eps), float(ell), int(seed))
        t = C.c_uint64()
        _check(_lib.hyperim_session_submit(self._h, C.byref(q), C.byref(t)))
        self._k[t.value] = int(k)
        self._graphs[id(graph)] = graph
        return t.value

    def step(self) -> dict:
        st = _SessionStats()
        _check(_lib.hyperim_session_step(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in _SessionStats._fields_}

    def stats(self) -> dict:
        st = _SessionStats()
        _check(_lib.hyperim_session_stats_get(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in _SessionStats._fields_}

    def poll(self, ticket: int):
        """None while pending; else the result dict (raises on a failed query)."""
        k = self._k[ticket]
        seeds = np.zeros(k, np.uint32)
        gains = np.zeros(k, np.uint64)
        res = _Result()
        rc = _lib.hyperim_session_poll(self._h, ticket, _ptr(seeds), _ptr(gains), C.byref(res))
        if rc == PENDING:
            return None
        del self._k[ticket]
        _check(rc)
        d = _result_dict(res)
        d["seeds"] = seeds
        d["gains"] = gains
        return d

    def drop(self, graph: Graph):
        _check(_lib.hyperim_session_drop(self._h, graph._h))
        self._graphs.pop(id(graph), None)


def workspace_bytes() -> int:
    """hyperim_workspace_info: bytes of the current device's RR workspace."""
    load_library()
    b = C.c_size_t()
    _check(_lib.hyperim_workspace_info(C.byref(b)))
    return b.value


def workspace_release():
    """hyperim_workspace_release: free the current device's RR workspace."""
    load_library()
    _check(_lib.hyperim_workspace_release())
