"""CPU oracle for the sampled-betweenness hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the bench's ``cpu_baseline``
leg may import this package.  The product (``paper_1604_08553_amd``) never does.

This is a thin ctypes binding over ``kadabra_oracle.c`` (plain C11 + OpenMP,
arbitrary-precision path counts, binary64 statistics built without FMA
contraction).  See that file for the algorithm and the paper passages it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kadabra_oracle.c")
_LIB = os.path.join(_HERE, "libkadabra_oracle.so")

ERRORS = {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "buffer too small",
          -4: "random draw rejected too often"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (C11, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-Wno-unused-function", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class _Graph(C.Structure):
    _fields_ = [("n", C.c_uint32), ("arcs", C.c_uint64), ("directed", C.c_int32),
                ("row", C.c_void_p), ("col", C.c_void_p),
                ("rrow", C.c_void_p), ("rcol", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("epsilon", C.c_double), ("delta", C.c_double), ("mode", C.c_uint32),
                ("k", C.c_uint32), ("seed", C.c_uint64), ("check_interval", C.c_uint64),
                ("vd_override", C.c_uint32), ("c", C.c_double), ("balance_eps", C.c_double),
                ("exact_vd_limit", C.c_double), ("threads", C.c_int32), ("forward", C.c_int32),
                ("edges", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [("tau", C.c_uint64), ("omega", C.c_uint64), ("alpha", C.c_uint64),
                ("interval", C.c_uint64), ("arcs", C.c_uint64), ("pilot_arcs", C.c_uint64),
                ("vd", C.c_uint32), ("stop_rule", C.c_uint32), ("vd_exact", C.c_int32),
                ("C", C.c_double),
                ("count", C.c_void_p), ("bc", C.c_void_p), ("lower", C.c_void_p),
                ("upper", C.c_void_p), ("L_l", C.c_void_p), ("L_u", C.c_void_p),
                ("count0", C.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        vp, u32, u64, i32, dbl = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32, C.c_double
        L.or_philox4x64_10.argtypes = [vp, vp, vp]
        L.or_philox4x64_10.restype = None
        L.or_uniform_below.argtypes = [vp, u32, u64, u64, u32, u32, u64, vp, u32]
        L.or_uniform_below.restype = C.c_int
        L.or_sample_paths.argtypes = [C.POINTER(_Graph), u64, u32, u64, u64, C.c_int, vp, vp, vp,
                                      vp, u64, vp, vp]
        L.or_sample_paths.restype = C.c_int
        L.or_sample_paths_search.argtypes = [C.POINTER(_Graph), u64, u32, u64, u64, C.c_int,
                                             C.c_int, vp, vp, vp, vp, u64, vp, vp]
        L.or_sample_paths_search.restype = C.c_int
        L.or_vertex_diameter.argtypes = [C.POINTER(_Graph), dbl, vp, vp]
        L.or_vertex_diameter.restype = C.c_int
        L.or_omega.argtypes = [dbl, dbl, u32, dbl]
        L.or_omega.restype = u64
        L.or_alpha.argtypes = [u64]
        L.or_alpha.restype = u64
        L.or_default_interval.argtypes = [u64]
        L.or_default_interval.restype = u64
        L.or_f.argtypes = [dbl, dbl, dbl, dbl]
        L.or_f.restype = dbl
        L.or_g.argtypes = [dbl, dbl, dbl, dbl]
        L.or_g.restype = dbl
        L.or_compute_delta.argtypes = [u32, vp, u64, u64, vp, vp, dbl, dbl, vp, vp, vp]
        L.or_compute_delta.restype = C.c_int
        L.or_stop_all.argtypes = [u32, vp, u64, u64, dbl, vp, vp]
        L.or_stop_all.restype = C.c_int
        L.or_stop_topk.argtypes = [u32, u32, vp, u64, u64, dbl, vp, vp]
        L.or_stop_topk.restype = C.c_int
        L.or_topk_lambdas.argtypes = [u32, u32, vp, u64, dbl, vp, vp]
        L.or_topk_lambdas.restype = C.c_int
        L.or_run.argtypes = [C.POINTER(_Graph), C.POINTER(_Params), C.POINTER(_Result)]
        L.or_run.restype = C.c_int
        L.or_rank_intervals.argtypes = [u32, vp, vp, vp, vp]
        L.or_rank_intervals.restype = C.c_int
        L.or_brandes.argtypes = [C.POINTER(_Graph), vp]
        L.or_brandes.restype = C.c_int
        L.or_sigma_st.argtypes = [C.POINTER(_Graph), u32, u32, vp, u32]
        L.or_sigma_st.restype = C.c_int64
        L.or_edge_count.argtypes = [C.POINTER(_Graph)]
        L.or_edge_count.restype = u64
        L.or_edge_ids.argtypes = [C.POINTER(_Graph), vp]
        L.or_edge_ids.restype = C.c_int
        L.or_edge_hits.argtypes = [C.POINTER(_Graph), u64, u32, u64, u64, C.c_int, C.c_int, vp,
                                   vp]
        L.or_edge_hits.restype = C.c_int
        L.or_edge_brandes.argtypes = [C.POINTER(_Graph), vp]
        L.or_edge_brandes.restype = C.c_int
        L.or_omega_edges.argtypes = [dbl, dbl, u32, dbl]
        L.or_omega_edges.restype = u64
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"oracle error {rc}: {ERRORS.get(rc, '?')}")


def _ptr(a):
    return a.ctypes.data if a is not None else None


class Graph:
    """Keeps the numpy CSR arrays alive next to the C struct."""

    def __init__(self, csr):
        self.n = int(csr.n)
        self.row = np.ascontiguousarray(csr.row, dtype=np.uint32)
        self.col = np.ascontiguousarray(csr.col, dtype=np.uint32)
        self.rrow = np.ascontiguousarray(csr.rrow, dtype=np.uint32)
        self.rcol = np.ascontiguousarray(csr.rcol, dtype=np.uint32)
        self.directed = bool(csr.directed)
        self.s = _Graph(self.n, int(self.col.size), 1 if self.directed else 0,
                        _ptr(self.row), _ptr(self.col), _ptr(self.rrow), _ptr(self.rcol))


def as_graph(g) -> Graph:
    return g if isinstance(g, Graph) else Graph(g)


# ---------------------------------------------------------------- primitives

def philox(ctr, key):
    c = np.array(ctr, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return [int(x) for x in out]


def _to_words(x: int, nw: int) -> np.ndarray:
    return np.array([(x >> (64 * j)) & 0xFFFFFFFFFFFFFFFF for j in range(nw)], dtype=np.uint64)


def uniform_below(bound: int, seed: int, i: int, phase: int, purpose: int, step: int) -> int:
    nw = max(1, (bound.bit_length() + 63) // 64)
    b = _to_words(bound, nw)
    out = np.zeros(nw, dtype=np.uint64)
    _check(lib().or_uniform_below(_ptr(b), nw, seed, i, phase, purpose, step, _ptr(out), nw))
    return sum(int(out[j]) << (64 * j) for j in range(nw))


# ---------------------------------------------------------------- sampling

@dataclass
class Samples:
    s: np.ndarray
    t: np.ndarray
    path_off: np.ndarray
    nodes: np.ndarray
    arcs: np.ndarray
    sigma_bits: np.ndarray

    def path(self, k):
        return self.nodes[self.path_off[k]:self.path_off[k + 1]]


def sample_paths(g, seed: int, phase: int, first: int, count: int, threads: int = 0,
                 search: str = "balanced") -> Samples:
    """Sample ids [first, first+count): the balanced bidirectional search of section 4, or
    with search="forward" the plain BFS from s until t's level is done."""
    g = as_graph(g)
    forward = {"balanced": 0, "forward": 1}[search]
    s = np.zeros(count, dtype=np.uint32)
    t = np.zeros(count, dtype=np.uint32)
    off = np.zeros(count + 1, dtype=np.uint64)
    arcs = np.zeros(count, dtype=np.uint64)
    bits = np.zeros(count, dtype=np.uint64)
    cap = max(16, count * 16)
    while True:
        nodes = np.zeros(cap, dtype=np.uint32)
        rc = lib().or_sample_paths_search(C.byref(g.s), seed, phase, first, count, threads,
                                          forward, _ptr(s), _ptr(t), _ptr(off), _ptr(nodes),
                                          cap, _ptr(arcs), _ptr(bits))
        if rc == -3:
            cap *= 4
            continue
        _check(rc)
        return Samples(s, t, off, nodes[:int(off[count])], arcs, bits)


# ---------------------------------------------------------------- schedule / statistics

def vertex_diameter(g, exact_limit: float = 1e9):
    g = as_graph(g)
    vd = np.zeros(1, dtype=np.uint32)
    ex = np.zeros(1, dtype=np.int32)
    _check(lib().or_vertex_diameter(C.byref(g.s), exact_limit, _ptr(vd), _ptr(ex)))
    return int(vd[0]), bool(ex[0])


def omega(lam: float, delta: float, vd: int, c: float = 0.5) -> int:
    return int(lib().or_omega(lam, delta, vd, c))


def alpha(om: int) -> int:
    return int(lib().or_alpha(om))


def default_interval(om: int) -> int:
    return int(lib().or_default_interval(om))


def f(bt, L, om, tau) -> float:
    return float(lib().or_f(bt, L, float(om), float(tau)))


def g(bt, L, om, tau) -> float:
    return float(lib().or_g(bt, L, float(om), float(tau)))


def compute_delta(count0, alpha_, omega_, lam_l, lam_u, delta, eps_bal=0.001):
    count0 = np.ascontiguousarray(count0, dtype=np.uint64)
    n = count0.size
    lam_l = np.ascontiguousarray(lam_l, dtype=np.float64)
    lam_u = np.ascontiguousarray(lam_u, dtype=np.float64)
    Ll = np.zeros(n)
    Lu = np.zeros(n)
    Cv = np.zeros(1)
    _check(lib().or_compute_delta(n, _ptr(count0), alpha_, omega_, _ptr(lam_l), _ptr(lam_u),
                                  delta, eps_bal, _ptr(Ll), _ptr(Lu), _ptr(Cv)))
    return Ll, Lu, float(Cv[0])


def stop_all(count, tau, omega_, lam, Ll, Lu) -> bool:
    count = np.ascontiguousarray(count, dtype=np.uint64)
    r = lib().or_stop_all(count.size, _ptr(count), tau, omega_, lam,
                          _ptr(np.ascontiguousarray(Ll)), _ptr(np.ascontiguousarray(Lu)))
    return bool(r)


def stop_topk(count, k, tau, omega_, lam, Ll, Lu) -> bool:
    count = np.ascontiguousarray(count, dtype=np.uint64)
    r = lib().or_stop_topk(count.size, k, _ptr(count), tau, omega_, lam,
                           _ptr(np.ascontiguousarray(Ll)), _ptr(np.ascontiguousarray(Lu)))
    if r < 0:
        _check(r)
    return bool(r)


def topk_lambdas(count0, k, alpha_, lam):
    count0 = np.ascontiguousarray(count0, dtype=np.uint64)
    n = count0.size
    ll = np.zeros(n)
    lu = np.zeros(n)
    _check(lib().or_topk_lambdas(n, k, _ptr(count0), alpha_, lam, _ptr(ll), _ptr(lu)))
    return ll, lu


def rank_intervals(lower, upper):
    lower = np.ascontiguousarray(lower, dtype=np.float64)
    upper = np.ascontiguousarray(upper, dtype=np.float64)
    n = lower.size
    lo = np.zeros(n, dtype=np.uint32)
    hi = np.zeros(n, dtype=np.uint32)
    _check(lib().or_rank_intervals(n, _ptr(lower), _ptr(upper), _ptr(lo), _ptr(hi)))
    return lo, hi


# ---------------------------------------------------------------- whole run

def run(g, epsilon, delta, mode="all", k=0, seed=1, check_interval=0, vd_override=0, c=0.0,
        balance_eps=0.0, exact_vd_limit=0.0, threads=0, search="balanced",
        target="nodes") -> dict:
    """Algorithm 1 with the batched stopping check; returns a dict of results (per-item
    arrays: one entry per node, or per edge id with target="edges")."""
    g = as_graph(g)
    edges = {"nodes": 0, "edges": 1}[target]
    n = edge_count(g) if edges else g.n
    p = _Params(epsilon, delta, 1 if mode == "topk" else 0, k, seed, check_interval,
                vd_override, c, balance_eps, exact_vd_limit, threads,
                {"balanced": 0, "forward": 1}[search], edges)
    out = {name: np.zeros(n, dtype=np.uint64) for name in ("count", "count0")}
    for name in ("bc", "lower", "upper", "L_l", "L_u"):
        out[name] = np.zeros(n)
    r = _Result()
    for name in ("count", "bc", "lower", "upper", "L_l", "L_u", "count0"):
        setattr(r, name, out[name].ctypes.data)
    _check(lib().or_run(C.byref(g.s), C.byref(p), C.byref(r)))
    for name in ("tau", "omega", "alpha", "interval", "arcs", "pilot_arcs", "vd", "stop_rule",
                 "vd_exact", "C"):
        out[name] = getattr(r, name)
    return out


def brandes(g) -> np.ndarray:
    g = as_graph(g)
    bc = np.zeros(g.n)
    _check(lib().or_brandes(C.byref(g.s), _ptr(bc)))
    return bc


def sigma_st(g, s, t, words=64):
    """(distance, number of shortest s->t paths) by a plain BFS; (-1, 0) if unreachable."""
    g = as_graph(g)
    buf = np.zeros(words, dtype=np.uint64)
    d = int(lib().or_sigma_st(C.byref(g.s), s, t, _ptr(buf), words))
    if d == -2:
        raise RuntimeError("sigma wider than the buffer")
    if d < 0:
        return -1, 0
    return d, sum(int(buf[j]) << (64 * j) for j in range(words))


# ---------------------------------------------------------------- edge betweenness

def edge_count(g) -> int:
    """Edges whose betweenness is estimated: arcs (directed) or arcs / 2 (undirected)."""
    g = as_graph(g)
    return int(lib().or_edge_count(C.byref(g.s)))


def edge_ids(g) -> np.ndarray:
    """Edge id of every arc position (directed: the position; undirected: the rank of the
    edge's u < v arc, shared by both arcs)."""
    g = as_graph(g)
    eid = np.zeros(max(int(g.col.size), 1), dtype=np.uint32)
    _check(lib().or_edge_ids(C.byref(g.s), _ptr(eid)))
    return eid[:int(g.col.size)]


def edge_hits(g, seed: int, phase: int, first: int, count: int, threads: int = 0,
              search: str = "balanced"):
    """(hits per edge id, arcs scanned) of sample ids [first, first+count)."""
    g = as_graph(g)
    cnt = np.zeros(max(edge_count(g), 1), dtype=np.uint64)
    arcs = np.zeros(1, dtype=np.uint64)
    _check(lib().or_edge_hits(C.byref(g.s), seed, phase, first, count, threads,
                              {"balanced": 0, "forward": 1}[search], _ptr(cnt), _ptr(arcs)))
    return cnt[:edge_count(g)], int(arcs[0])


def edge_brandes(g) -> np.ndarray:
    """Exact edge betweenness (ordered-pair normalisation, indexed by edge id)."""
    g = as_graph(g)
    ebc = np.zeros(max(edge_count(g), 1))
    _check(lib().or_edge_brandes(C.byref(g.s), _ptr(ebc)))
    return ebc[:edge_count(g)]


def omega_edges(lam: float, delta: float, vd: int, c: float = 0.5) -> int:
    return int(lib().or_omega_edges(lam, delta, vd, c))
