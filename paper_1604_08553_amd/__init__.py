"""MI355X sampled betweenness centrality (the KADABRA hot path) -- Python binding.

Thin ctypes marshalling over ``libkadabra.so`` (C ABI in ``include/kadabra.h``):
every step of the sampling path runs in the library's HIP kernels, the stopping
statistics in its C++ host code.  PyTorch is optional and only used to hand over
device tensors and HIP streams.  The binding fails loudly when the library has not
been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

__all__ = ["Context", "Graph", "run", "run_batch", "Server", "sample_paths", "hit_counts",
           "hit_counts_noalloc", "edge_hit_counts",
           "KadError", "lib",
           "library_path", "declared_symbols", "omega", "alpha", "default_interval",
           "vertex_diameter", "bound_f", "bound_g", "compute_delta", "topk_lambdas",
           "have_to_stop"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libkadabra.so")
_HEADER = os.path.join(os.path.dirname(_HERE), "include", "kadabra.h")

ALL_NODES, TOPK = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
STOP_OMEGA, STOP_RULE, STOP_FIXED = 0, 1, 2
SCHEDULES = {"adaptive": 0, "rk": 1, "hoeffding": 2}
SEARCHES = {"balanced": 0, "forward": 1}
TARGETS = {"nodes": 0, "edges": 1}
SAMPLE_OVERFLOW, SAMPLE_CAPACITY, SAMPLE_RNG = 1, 2, 4

_STATUS = {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "device error",
           -4: "busy", -5: "buffer too small", -6: "overflow", -7: "random draw rejected",
           -8: "canceled", -9: "internal error"}
EBUSY = -4


class KadError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class _Params(C.Structure):
    _fields_ = [("epsilon", C.c_double), ("delta", C.c_double), ("mode", C.c_uint32),
                ("k", C.c_uint32), ("seed", C.c_uint64), ("check_interval", C.c_uint32),
                ("kernel_batch", C.c_uint32), ("vd_override", C.c_uint32),
                ("schedule", C.c_uint32), ("c", C.c_double), ("balance_eps", C.c_double),
                ("target", C.c_uint32)]


class _Result(C.Structure):
    _fields_ = [("tau", C.c_uint64), ("omega", C.c_uint64), ("alpha", C.c_uint64),
                ("interval", C.c_uint64), ("arcs_scanned", C.c_uint64),
                ("pilot_arcs_scanned", C.c_uint64), ("overflow_samples", C.c_uint64),
                ("vd", C.c_uint32), ("vd_exact", C.c_uint32), ("stop_reason", C.c_uint32),
                ("n", C.c_uint32), ("seconds", C.c_double), ("C", C.c_double),
                ("seconds_setup", C.c_double), ("seconds_pilot", C.c_double),
                ("seconds_delta", C.c_double), ("seconds_main", C.c_double),
                ("count", C.c_void_p), ("bc", C.c_void_p), ("lower", C.c_void_p),
                ("upper", C.c_void_p), ("topk_cap", C.c_uint32), ("topk_len", C.c_uint32),
                ("topk_node", C.c_void_p), ("rank_lo", C.c_void_p), ("rank_hi", C.c_void_p),
                ("items", C.c_uint64)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libkadabra.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with "
                          "`python -m paper_1604_08553_amd.build`")
    L = C.CDLL(_LIB_PATH)
    vp, u32, u64, i32, dbl, st = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int, C.c_double, C.c_int
    sig = {
        "kad_ctx_create": ([i32, u64, vp], st),
        "kad_ctx_destroy": ([vp], st),
        "kad_graph_create": ([vp, u32, u64, i32, vp, vp, vp, vp, i32, vp], st),
        "kad_graph_destroy": ([vp], st),
        "kad_run": ([vp, vp, C.POINTER(_Params), C.POINTER(_Result), vp], st),
        "kad_sample_paths": ([vp, vp, u64, u32, u64, u32, vp, vp, vp, vp, u64, vp, vp, vp], st),
        "kad_hit_counts": ([vp, vp, u64, u32, u64, u64, vp, vp, vp], st),
        "kad_hit_counts_noalloc": ([vp, vp, u64, u32, u64, u64, vp, vp, vp, vp], st),
        "kad_edge_hit_counts": ([vp, vp, u64, u32, u64, u64, vp, vp, vp], st),
        "kad_graph_edge_count": ([vp, vp], st),
        "kad_graph_edge_ids": ([vp, vp], st),
        "kad_omega": ([dbl, dbl, u32, dbl], u64),
        "kad_alpha": ([u64], u64),
        "kad_fixed_samples": ([u32, dbl, dbl, u32, u32, dbl], u64),
        "kad_default_interval": ([u64], u64),
        "kad_vertex_diameter": ([u32, u64, i32, vp, vp, vp, vp, dbl, vp, vp], st),
        "kad_bound_f": ([dbl, dbl, dbl, dbl], dbl),
        "kad_bound_g": ([dbl, dbl, dbl, dbl], dbl),
        "kad_compute_delta": ([u32, vp, u64, u64, vp, vp, dbl, dbl, vp, vp, vp], st),
        "kad_compute_delta_hist": ([u32, vp, u64, u64, u64, dbl, dbl, dbl, dbl, vp, vp, vp, vp,
                                    vp], st),
        "kad_topk_lambdas": ([u32, u32, vp, u64, dbl, vp, vp], st),
        "kad_topk_select": ([u32, u32, vp, vp, vp, u32, vp, vp, vp, vp], st),
        "kad_have_to_stop": ([u32, u32, u32, vp, u64, u64, dbl, vp, vp], st),
        "kad_run_batch": ([vp, u32, vp, vp, vp, vp], st),
        "kad_server_create": ([vp, vp], st),
        "kad_server_submit": ([vp, vp, C.POINTER(_Params), vp], st),
        "kad_server_poll": ([vp, u64, C.POINTER(_Result)], st),
        "kad_server_wait": ([vp, u64, C.POINTER(_Result), dbl], st),
        "kad_server_stats": ([vp, vp, vp, vp], st),
        "kad_server_cancel": ([vp], st),
        "kad_server_destroy": ([vp], st),
        "kad_graph_set_launch": ([vp, u32, u32], st),
        "kad_graph_set_search": ([vp, u32], st),
        "kad_graph_get_search": ([vp, vp], st),
        "kad_graph_get_launch": ([vp, vp, vp], st),
        "kad_autotune": ([vp, vp, u32, vp, vp, vp], st),
        "kad_ctx_set_timing": ([vp, i32], st),
        "kad_ctx_get_timing": ([vp, vp, vp, vp, vp, vp, vp], st),
        "kad_ctx_set_exec": ([vp, u32], st),
        "kad_ctx_set_wide": ([vp, u32, u64], st),
        "kad_ctx_get_wide": ([vp, vp, vp, vp, vp], st),
        "kad_ctx_set_table": ([vp, u32], st),
        "kad_ctx_get_table": ([vp, vp, vp, vp], st),
        "kad_ctx_get_exec": ([vp, vp, vp, vp], st),
        "kad_last_error": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def declared_symbols() -> list:
    """Function names declared in include/kadabra.h."""
    text = open(_HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kad_[a-z0-9_]+)\s*\(", text)))


def _check(rc):
    if rc != 0:
        msg = lib().kad_last_error()
        raise KadError(rc, msg.decode() if msg else "")


def _p(a):
    return None if a is None else a.ctypes.data


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


# ----------------------------------------------------------------------------- objects


EXECS = {"graph": 0, "stream": 1, "plain": 2}


class Context:
    """A HIP device with the library's working memory (``hbm_budget`` bytes, 0 = 90%
    of the free memory)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        h = C.c_void_p()
        _check(lib().kad_ctx_create(device, hbm_budget, C.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib().kad_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timing(self, enable: bool = True):
        _check(lib().kad_ctx_set_timing(self.handle, 1 if enable else 0))

    def set_exec(self, mode: str):
        """How kad_run launches: "graph" (recorded batch chains, the default), "stream"
        (call by call) or "plain" (the plain single-graph path); see kad_ctx_set_exec."""
        _check(lib().kad_ctx_set_exec(self.handle, EXECS[mode]))

    def set_wide(self, slots: int = 0, limbs: int = 0):
        """First-pass wide-count slots and arena limbs (0 = library choice); see
        kad_ctx_set_wide."""
        _check(lib().kad_ctx_set_wide(self.handle, slots, limbs))

    def wide_info(self) -> dict:
        a, c = C.c_uint32(), C.c_uint32()
        b, d = C.c_uint64(), C.c_uint64()
        _check(lib().kad_ctx_get_wide(self.handle, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return {"slots": a.value, "limbs": b.value, "slots2": c.value, "limbs2": d.value}

    def set_table(self, log2_records: int = 0):
        """Sampler slot layout: 0 = library choice, 1 = one record per node, 6..24 = hash
        tables of 2^log2_records records per slot; see kad_ctx_set_table."""
        _check(lib().kad_ctx_set_table(self.handle, log2_records))

    def table_info(self) -> dict:
        b, s_, w = C.c_uint32(), C.c_uint32(), C.c_uint32()
        _check(lib().kad_ctx_get_table(self.handle, C.byref(b), C.byref(s_), C.byref(w)))
        return {"log2_records": b.value, "slots": s_.value, "wide_slots": w.value}

    def exec_info(self) -> dict:
        m, rec, rep = C.c_uint32(), C.c_uint64(), C.c_uint64()
        _check(lib().kad_ctx_get_exec(self.handle, C.byref(m), C.byref(rec), C.byref(rep)))
        name = {v: k for k, v in EXECS.items()}[m.value]
        return {"mode": name, "records": rec.value, "replays": rep.value}

    def timing(self) -> dict:
        """Totals over the event-timed sampler launches (see kad_ctx_get_timing)."""
        v = [C.c_uint64() for _ in range(5)]
        sec = C.c_double()
        _check(lib().kad_ctx_get_timing(self.handle, C.byref(v[0]), C.byref(v[1]), C.byref(sec),
                                        C.byref(v[2]), C.byref(v[3]), C.byref(v[4])))
        return {"launches": v[0].value, "samples": v[1].value, "seconds": sec.value,
                "arcs": v[2].value, "nodes": v[3].value, "hits": v[4].value}


class Graph:
    """A CSR graph registered with a context.

    ``csr`` is any object with ``n, row, col, directed`` (and ``rrow, rcol`` for
    directed graphs), e.g. ``graphgen.CSR``.  With torch tensors on the context's GPU
    pass ``mem="device"``: the library borrows them (keep them alive)."""

    def __init__(self, ctx: Context, csr=None, *, n=None, row=None, col=None, rrow=None,
                 rcol=None, directed=None, mem="host"):
        if csr is not None:
            n, row, col, directed = csr.n, csr.row, csr.col, csr.directed
            rrow = getattr(csr, "rrow", None) if directed else None
            rcol = getattr(csr, "rcol", None) if directed else None
        self.ctx = ctx
        self.n = int(n)
        self.directed = bool(directed)
        h = C.c_void_p()
        if mem == "device":
            self._keep = (row, col, rrow, rcol)
            ptr = lambda t: None if t is None else t.data_ptr()
            arcs = int(col.numel())
            rc = lib().kad_graph_create(ctx.handle, self.n, arcs, 1 if self.directed else 0,
                                        ptr(row), ptr(col), ptr(rrow), ptr(rcol), MEM_DEVICE,
                                        C.byref(h))
        else:
            row, col = _u32(row), _u32(col)
            rrow = None if rrow is None else _u32(rrow)
            rcol = None if rcol is None else _u32(rcol)
            self._keep = (row, col, rrow, rcol)
            arcs = int(col.size)
            rc = lib().kad_graph_create(ctx.handle, self.n, arcs, 1 if self.directed else 0,
                                        _p(row), _p(col), _p(rrow), _p(rcol), MEM_HOST,
                                        C.byref(h))
        _check(rc)
        self.handle = h
        self.arcs = arcs

    def set_launch(self, block: int = 0, small_expansion: int = 0):
        """Sampler launch shape for this graph ((0, 0) = library default)."""
        _check(lib().kad_graph_set_launch(self.handle, block, small_expansion))

    def set_search(self, search: str = "balanced"):
        """How this graph's samples search for paths: "balanced" (section 4's balanced
        bidirectional BFS, the default) or "forward" (a plain BFS from s until t's level)."""
        _check(lib().kad_graph_set_search(self.handle, SEARCHES[search]))

    def search(self) -> str:
        v = C.c_uint32()
        _check(lib().kad_graph_get_search(self.handle, C.byref(v)))
        return {b: a for a, b in SEARCHES.items()}[v.value]

    def edge_count(self) -> int:
        """Edges: arcs (directed) or arcs / 2 (undirected)."""
        v = C.c_uint64()
        _check(lib().kad_graph_edge_count(self.handle, C.byref(v)))
        return v.value

    def edge_ids(self) -> np.ndarray:
        """Edge id of every arc position (kad_graph_edge_ids)."""
        eid = np.zeros(max(self.arcs, 1), dtype=np.uint32)
        _check(lib().kad_graph_edge_ids(self.handle, _p(eid)))
        return eid[:self.arcs]

    def launch(self):
        b, e = C.c_uint32(), C.c_uint32()
        _check(lib().kad_graph_get_launch(self.handle, C.byref(b), C.byref(e)))
        return b.value, e.value

    def autotune(self, samples: int = 0) -> dict:
        """Time every candidate launch shape and keep the fastest (kad_autotune)."""
        b, e, sec = C.c_uint32(), C.c_uint32(), C.c_double()
        _check(lib().kad_autotune(self.ctx.handle, self.handle, samples, C.byref(b), C.byref(e),
                                  C.byref(sec)))
        return {"block": b.value, "small_expansion": e.value, "seconds": sec.value}

    def close(self):
        if getattr(self, "handle", None):
            lib().kad_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


# ----------------------------------------------------------------------------- calls


_SCALARS = ("tau", "omega", "alpha", "interval", "arcs_scanned", "pilot_arcs_scanned",
            "overflow_samples", "vd", "vd_exact", "stop_reason", "seconds", "C",
            "seconds_setup", "seconds_pilot", "seconds_delta", "seconds_main", "items")


def _params(epsilon, delta, mode="all", k=0, seed=1, check_interval=0, kernel_batch=0,
            vd_override=0, c=0.0, balance_eps=0.0, schedule="adaptive", target="nodes"):
    return _Params(epsilon, delta, TOPK if mode == "topk" else ALL_NODES, k, seed,
                   check_interval, kernel_batch, vd_override, SCHEDULES[schedule], c,
                   balance_eps, TARGETS[target])


def _result(n, topk, topk_cap=0, out=None):
    """A kad_result wired to numpy arrays (reusing those in ``out`` when they fit)."""
    prev = out or {}
    arrs = {}
    for name, dt in (("count", np.uint64), ("bc", np.float64), ("lower", np.float64),
                     ("upper", np.float64)):
        a = prev.get(name)
        if a is None or a.shape != (n,) or a.dtype != dt or not a.flags.c_contiguous:
            a = np.empty(n, dtype=dt)
        arrs[name] = a
    cap = topk_cap or (n if topk else 0)
    for name in ("topk_node", "rank_lo", "rank_hi"):
        arrs[name] = np.zeros(max(cap, 1), dtype=np.uint32)
    r = _Result()
    for name, a in arrs.items():
        setattr(r, name, a.ctypes.data)
    r.topk_cap = cap
    return r, arrs


def _collect(r, arrs, topk):
    out = {k: arrs[k] for k in ("count", "bc", "lower", "upper")}
    for name in _SCALARS:
        out[name] = getattr(r, name)
    if topk:
        m = r.topk_len
        for name in ("topk_node", "rank_lo", "rank_hi"):
            out[name] = arrs[name][:m].copy()
    return out


def run(ctx: Context, graph: Graph, epsilon: float, delta: float, mode: str = "all", k: int = 0,
        seed: int = 1, check_interval: int = 0, kernel_batch: int = 0, vd_override: int = 0,
        c: float = 0.0, balance_eps: float = 0.0, topk_cap: int = 0, stream=None,
        out: dict = None, schedule: str = "adaptive", target: str = "nodes") -> dict:
    """The adaptive run (Algorithm 1), or a fixed schedule ("rk", "hoeffding").  Returns
    scalars plus the per-item arrays (per node, or per edge id with target="edges").

    ``out`` may hold preallocated arrays "count" (uint64[n]), "bc", "lower", "upper"
    (float64[n]) to be filled in place (saves page-faulting fresh arrays per call)."""
    p = _params(epsilon, delta, mode, k, seed, check_interval, kernel_batch, vd_override, c,
                balance_eps, schedule, target)
    items = graph.n if target == "nodes" else graph.edge_count()
    r, arrs = _result(items, mode == "topk", topk_cap, out)
    _check(lib().kad_run(ctx.handle, graph.handle, C.byref(p), C.byref(r), _stream(stream)))
    return _collect(r, arrs, mode == "topk")


def run_batch(ctx: Context, graphs, params) -> list:
    """Run queries (graphs[i], params[i]) together through the multi-query engine
    (kad_run_batch).  params[i] is a dict of run()'s keyword arguments (epsilon and
    delta required).  Returns one result dict per query, as run() does; raises on
    the first failing query."""
    m = len(graphs)
    if len(params) != m:
        raise ValueError("one parameter set per graph")
    ps = (_Params * max(m, 1))()
    rs = (_Result * max(m, 1))()
    keep, topk = [], []
    for i, (g, kw) in enumerate(zip(graphs, params)):
        kw = dict(kw)
        cap = kw.pop("topk_cap", 0)
        ps[i] = _params(**kw)
        r, arrs = _result(g.n, kw.get("mode") == "topk", cap)
        rs[i] = r
        keep.append(arrs)
        topk.append(kw.get("mode") == "topk")
    handles = (C.c_void_p * max(m, 1))(*[g.handle for g in graphs])
    status = np.zeros(max(m, 1), dtype=np.int32)
    _check(lib().kad_run_batch(ctx.handle, m, handles, ps, rs, _p(status)))
    return [_collect(rs[i], keep[i], topk[i]) for i in range(m)]


class Server:
    """Continuous-batching server over a context (kad_server_*): queries submitted at
    any time join the running engine; results are identical to run()'s."""

    def __init__(self, ctx: Context):
        h = C.c_void_p()
        _check(lib().kad_server_create(ctx.handle, C.byref(h)))
        self.handle = h
        self.ctx = ctx
        self._pending = {}

    def submit(self, graph: Graph, epsilon: float, delta: float, topk_cap: int = 0, **kw) -> int:
        p = _params(epsilon, delta, **kw)
        t = C.c_uint64()
        _check(lib().kad_server_submit(self.handle, graph.handle, C.byref(p), C.byref(t)))
        self._pending[t.value] = _result(graph.n, kw.get("mode") == "topk", topk_cap) + (
            kw.get("mode") == "topk",)
        return t.value

    def poll(self, ticket: int):
        """The result dict, or None while the query runs."""
        r, arrs, topk = self._pending[ticket]
        rc = lib().kad_server_poll(self.handle, ticket, C.byref(r))
        if rc == EBUSY:
            return None
        del self._pending[ticket]
        _check(rc)
        return _collect(r, arrs, topk)

    def wait(self, ticket: int, timeout: float = -1.0):
        r, arrs, topk = self._pending[ticket]
        rc = lib().kad_server_wait(self.handle, ticket, C.byref(r), float(timeout))
        if rc == EBUSY:
            return None
        del self._pending[ticket]
        _check(rc)
        return _collect(r, arrs, topk)

    def cancel(self):
        """Cancel every query not yet completed (their results report KAD_ECANCELED)."""
        _check(lib().kad_server_cancel(self.handle))

    def stats(self) -> dict:
        v = [C.c_uint64() for _ in range(3)]
        _check(lib().kad_server_stats(self.handle, *[C.byref(x) for x in v]))
        return {"completed": v[0].value, "launches": v[1].value, "samples": v[2].value}

    def close(self):
        if getattr(self, "handle", None):
            lib().kad_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sample_paths(ctx: Context, graph: Graph, seed: int, phase: int, first: int, count: int,
                 stream=None) -> dict:
    """Per-sample trace of ids [first, first+count): s, t, packed paths, arcs, flags."""
    s = np.zeros(count, dtype=np.uint32)
    t = np.zeros(count, dtype=np.uint32)
    off = np.zeros(count + 1, dtype=np.uint64)
    arcs = np.zeros(count, dtype=np.uint64)
    flags = np.zeros(count, dtype=np.uint32)
    cap = max(16, count * 8)
    while True:
        nodes = np.zeros(cap, dtype=np.uint32)
        rc = lib().kad_sample_paths(ctx.handle, graph.handle, seed, phase, first, count, _p(s),
                                    _p(t), _p(off), _p(nodes), cap, _p(arcs), _p(flags),
                                    _stream(stream))
        if rc == -5:
            cap = int(off[count]) + 16
            continue
        _check(rc)
        return {"s": s, "t": t, "path_off": off, "nodes": nodes[:int(off[count])],
                "arcs": arcs, "flags": flags}


def hit_counts(ctx: Context, graph: Graph, seed: int, phase: int, first: int, count: int,
               stream=None):
    """(count[n], arcs scanned) of sample ids [first, first+count)."""
    cnt = np.zeros(graph.n, dtype=np.uint64)
    arcs = C.c_uint64()
    _check(lib().kad_hit_counts(ctx.handle, graph.handle, seed, phase, first, count, _p(cnt),
                                C.byref(arcs), _stream(stream)))
    return cnt, arcs.value


def edge_hit_counts(ctx: Context, graph: Graph, seed: int, phase: int, first: int, count: int,
                    stream=None):
    """(count per edge id, arcs scanned) of sample ids [first, first+count)."""
    cnt = np.zeros(max(graph.edge_count(), 1), dtype=np.uint64)
    arcs = C.c_uint64()
    _check(lib().kad_edge_hit_counts(ctx.handle, graph.handle, seed, phase, first, count, _p(cnt),
                                     C.byref(arcs), _stream(stream)))
    return cnt[:graph.edge_count()], arcs.value


def hit_counts_noalloc(ctx: Context, graph: Graph, seed: int, phase: int, first: int,
                       count: int, count_dev, arcs_dev, flags_dev, stream=None):
    """kad_hit_counts_noalloc: enqueue the hit counts of ids [first, first+count) into
    device tensors (count_dev: 8-byte integers [n], arcs_dev: 8-byte [1], flags_dev: 4-byte
    [1], all accumulated) using only the library's fixed scratch; returns without waiting."""
    _check(lib().kad_hit_counts_noalloc(ctx.handle, graph.handle, seed, phase, first, count,
                                        count_dev.data_ptr(), arcs_dev.data_ptr(),
                                        flags_dev.data_ptr(), _stream(stream)))


# ----------------------------------------------------------------------------- host statistics


def omega(epsilon, delta, vd, c=0.5) -> int:
    return int(lib().kad_omega(epsilon, delta, vd, c))


def fixed_samples(schedule, epsilon, delta, vd, n, c=0.0) -> int:
    """Sample count of a fixed schedule ("rk" or "hoeffding")."""
    return int(lib().kad_fixed_samples(SCHEDULES[schedule], epsilon, delta, vd, n, c))


def alpha(om) -> int:
    return int(lib().kad_alpha(om))


def default_interval(om) -> int:
    return int(lib().kad_default_interval(om))


def vertex_diameter(csr, exact_limit=1e9):
    row, col = _u32(csr.row), _u32(csr.col)
    rrow = _u32(csr.rrow) if csr.directed else None
    rcol = _u32(csr.rcol) if csr.directed else None
    vd, ex = C.c_uint32(), C.c_uint32()
    _check(lib().kad_vertex_diameter(csr.n, int(col.size), 1 if csr.directed else 0, _p(row),
                                     _p(col), _p(rrow), _p(rcol), exact_limit, C.byref(vd),
                                     C.byref(ex)))
    return int(vd.value), bool(ex.value)


def bound_f(bt, L, om, tau) -> float:
    return float(lib().kad_bound_f(bt, L, float(om), float(tau)))


def bound_g(bt, L, om, tau) -> float:
    return float(lib().kad_bound_g(bt, L, float(om), float(tau)))


def compute_delta(count0, alpha_, omega_, lam_l, lam_u, delta, balance_eps=0.001):
    count0 = np.ascontiguousarray(count0, dtype=np.uint64)
    n = count0.size
    ll = np.ascontiguousarray(lam_l, dtype=np.float64)
    lu = np.ascontiguousarray(lam_u, dtype=np.float64)
    Ll, Lu, Cv = np.zeros(n), np.zeros(n), C.c_double()
    _check(lib().kad_compute_delta(n, _p(count0), alpha_, omega_, _p(ll), _p(lu), delta,
                                   balance_eps, _p(Ll), _p(Lu), C.byref(Cv)))
    return Ll, Lu, Cv.value


def compute_delta_hist(hist, alpha_, omega_, lam_l, lam_u, delta, balance_eps=0.001):
    """computeDelta for uniform half-widths from the pilot-count histogram: returns
    (group_of_count, L_l per group, L_u per group, C)."""
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    m = hist.size
    gof = np.zeros(m, dtype=np.uint32)
    Ll, Lu = np.zeros(m), np.zeros(m)
    ng, Cv = C.c_uint32(), C.c_double()
    _check(lib().kad_compute_delta_hist(int(hist.sum()), _p(hist), m - 1, alpha_, omega_, lam_l,
                                        lam_u, delta, balance_eps, _p(gof), _p(Ll), _p(Lu),
                                        C.byref(ng), C.byref(Cv)))
    return gof, Ll[:ng.value], Lu[:ng.value], Cv.value


def topk_lambdas(count0, k, alpha_, epsilon):
    count0 = np.ascontiguousarray(count0, dtype=np.uint64)
    n = count0.size
    ll, lu = np.zeros(n), np.zeros(n)
    _check(lib().kad_topk_lambdas(n, k, _p(count0), alpha_, epsilon, _p(ll), _p(lu)))
    return ll, lu


def topk_select(count, lower, upper, k):
    """The top-k output: nodes whose rank interval reaches the top k, by count descending
    (id ascending), with rank_lo and rank_hi; see kad_topk_select."""
    count = np.ascontiguousarray(count, dtype=np.uint64)
    lo = np.ascontiguousarray(lower, dtype=np.float64)
    hi = np.ascontiguousarray(upper, dtype=np.float64)
    n = count.size
    node, rlo, rhi = (np.zeros(n, dtype=np.uint32) for _ in range(3))
    ln = C.c_uint32()
    _check(lib().kad_topk_select(n, k, _p(count), _p(lo), _p(hi), n, _p(node), _p(rlo), _p(rhi),
                                 C.byref(ln)))
    m = ln.value
    return node[:m].copy(), rlo[:m].copy(), rhi[:m].copy()


def have_to_stop(count, tau, omega_, epsilon, L_l, L_u, mode="all", k=0) -> bool:
    count = np.ascontiguousarray(count, dtype=np.uint64)
    Ll = np.ascontiguousarray(L_l, dtype=np.float64)
    Lu = np.ascontiguousarray(L_u, dtype=np.float64)
    r = lib().kad_have_to_stop(count.size, TOPK if mode == "topk" else ALL_NODES, k,
                               _p(count), tau, omega_, epsilon, _p(Ll), _p(Lu))
    if r < 0:
        _check(r)
    return bool(r)
