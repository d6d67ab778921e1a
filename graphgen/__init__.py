"""Seeded synthetic graph generators shared by the CPU oracle, the tests and the bench.

This module only builds inputs: canonical CSR graphs (nodes 0..n-1, rows sorted
ascending, no self-loops, no duplicate arcs; an undirected edge is stored as two
arcs; a directed graph also carries its transpose).  It holds none of the
betweenness method's arithmetic, so both the oracle and the GPU library can take
their inputs from here without sharing any of the method's code.

Random models follow the paper's appendix on random graphs (Chung-Lu:
p_uv = min(1, w_u w_v / W)); the Erdos-Renyi and grid workloads are plain
textbook models.  Every generator is a pure function of its arguments and seed.
Transcendental functions are evaluated with Python's scalar ``math`` (glibc) and
numpy's scalar random distributions, never with numpy's SIMD ufuncs, so the same
seed gives the same CSR on any x86 host of this image.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "CSR", "csr_from_edges", "er_lcc", "chung_lu", "chung_lu_directed",
    "grid", "damaged_grid", "path_graph", "star_graph", "cycle_graph",
    "complete_graph", "complete_bipartite", "disjoint_union", "gnp",
    "hub_layers", "configuration_model", "norros_reittu", "generalized_random_graph",
    "random_model", "batch_family_spec", "batch_graph", "serve_family_spec", "serve_graph", "serve_queries",
    "workload",
]


@dataclass
class CSR:
    """Canonical compressed-sparse-row graph.

    ``row``/``col`` are the out-rows.  For a directed graph ``rrow``/``rcol`` are
    the in-rows (transpose); for an undirected graph they alias ``row``/``col``.
    """
    n: int
    row: np.ndarray            # uint32 [n+1]
    col: np.ndarray            # uint32 [arcs]
    directed: bool
    rrow: np.ndarray = None    # uint32 [n+1]
    rcol: np.ndarray = None    # uint32 [arcs]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def arcs(self) -> int:
        return int(self.col.shape[0])

    def out_degree(self) -> np.ndarray:
        return np.diff(self.row.astype(np.int64))

    def in_degree(self) -> np.ndarray:
        return np.diff(self.rrow.astype(np.int64))

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.uint64(self.n).tobytes())
        h.update(np.uint8(1 if self.directed else 0).tobytes())
        h.update(np.ascontiguousarray(self.row, dtype=np.uint32).tobytes())
        h.update(np.ascontiguousarray(self.col, dtype=np.uint32).tobytes())
        return h.hexdigest()

    def edges(self):
        """Arc list (src, dst) as int64 arrays."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.out_degree())
        return src, self.col.astype(np.int64)


def csr_from_edges(n: int, src, dst, directed: bool, name: str = "", meta=None) -> CSR:
    """Build a canonical CSR from an edge list.

    Self-loops and duplicates are dropped.  For undirected graphs every edge
    {u, v} becomes the two arcs u->v and v->u.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if src.size:
        if src.min() < 0 or dst.min() < 0 or max(src.max(), dst.max()) >= n:
            raise ValueError("edge endpoint out of range")
    keep = src != dst
    src, dst = src[keep], dst[keep]
    if not directed:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
    key = src * np.int64(n) + dst
    key = np.unique(key)                       # sorts and removes duplicates
    s = key // n
    d = key % n
    if key.size >= 2**32:
        raise ValueError("too many arcs for uint32 CSR")
    counts = np.bincount(s, minlength=n)
    row = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row[1:])
    g = CSR(n=n, row=row.astype(np.uint32), col=d.astype(np.uint32),
            directed=directed, name=name, meta=dict(meta or {}))
    if directed:
        tkey = np.unique(d * np.int64(n) + s)
        ts, td = tkey // n, tkey % n
        tc = np.bincount(ts, minlength=n)
        rrow = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(tc, out=rrow[1:])
        g.rrow = rrow.astype(np.uint32)
        g.rcol = td.astype(np.uint32)
    else:
        g.rrow, g.rcol = g.row, g.col
    return g


# ----------------------------------------------------------------------------
# small closed-form graphs (used by the oracle's pins)
# ----------------------------------------------------------------------------

def path_graph(n: int) -> CSR:
    i = np.arange(n - 1)
    return csr_from_edges(n, i, i + 1, False, name=f"path{n}")


def star_graph(n: int) -> CSR:
    """Centre 0 joined to leaves 1..n-1."""
    return csr_from_edges(n, np.zeros(n - 1, dtype=np.int64), np.arange(1, n), False,
                          name=f"star{n}")


def cycle_graph(n: int, directed: bool = True) -> CSR:
    i = np.arange(n)
    return csr_from_edges(n, i, (i + 1) % n, directed, name=f"cycle{n}")


def complete_graph(n: int) -> CSR:
    u, v = np.triu_indices(n, 1)
    return csr_from_edges(n, u, v, False, name=f"K{n}")


def complete_bipartite(a: int, b: int) -> CSR:
    u = np.repeat(np.arange(a), b)
    v = np.tile(np.arange(a, a + b), a)
    return csr_from_edges(a + b, u, v, False, name=f"K{a},{b}")


def disjoint_union(*gs: CSR) -> CSR:
    directed = any(g.directed for g in gs)
    srcs, dsts, off = [], [], 0
    for g in gs:
        s, d = g.edges()
        srcs.append(s + off)
        dsts.append(d + off)
        off += g.n
    return csr_from_edges(off, np.concatenate(srcs), np.concatenate(dsts), directed,
                          name="+".join(g.name for g in gs))


def gnp(n: int, p: float, seed: int, directed: bool = False) -> CSR:
    """Erdos-Renyi G(n, p) by independent coin flips (small n only)."""
    rng = np.random.default_rng(seed)
    if directed:
        m = rng.random((n, n)) < p
        np.fill_diagonal(m, False)
        s, d = np.nonzero(m)
    else:
        u, v = np.triu_indices(n, 1)
        keep = rng.random(u.size) < p
        s, d = u[keep], v[keep]
    return csr_from_edges(n, s, d, directed, name=f"gnp{n}_{p}_{seed}")


def grid(rows: int, cols: int) -> CSR:
    return damaged_grid(rows, cols, 0.0, seed=0)


def damaged_grid(rows: int, cols: int, p_delete: float, seed: int) -> CSR:
    """4-neighbour rows x cols grid; each edge deleted independently with p_delete.

    Node (r, c) has id r*cols + c.  Isolated nodes are kept.
    """
    rng = np.random.default_rng(seed)
    ids = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    hs, hd = ids[:, :-1].ravel(), ids[:, 1:].ravel()
    vs, vd = ids[:-1, :].ravel(), ids[1:, :].ravel()
    s = np.concatenate([hs, vs])
    d = np.concatenate([hd, vd])
    if p_delete > 0:
        keep = rng.random(s.size) >= p_delete
        s, d = s[keep], d[keep]
    return csr_from_edges(rows * cols, s, d, False, name=f"grid{rows}x{cols}_{p_delete}",
                          meta={"rows": rows, "cols": cols, "p_delete": p_delete, "seed": seed})


# ----------------------------------------------------------------------------
# Erdos-Renyi largest connected component
# ----------------------------------------------------------------------------

def er_lcc(n: int = 2000, avg_deg: float = 8.0, seed: int = 1) -> CSR:
    """networkx G(n, avg_deg/(n-1)) with the given seed, restricted to its largest
    connected component, nodes relabelled 0.. in increasing original id."""
    import networkx as nx
    g = nx.gnp_random_graph(n, avg_deg / (n - 1), seed=seed)
    comp = max(nx.connected_components(g), key=len)
    keep = sorted(comp)
    relabel = {v: i for i, v in enumerate(keep)}
    e = np.array([(relabel[u], relabel[v]) for u, v in g.subgraph(keep).edges()],
                 dtype=np.int64).reshape(-1, 2)
    return csr_from_edges(len(keep), e[:, 0], e[:, 1], False,
                          name=f"er{n}_d{avg_deg}_s{seed}_lcc",
                          meta={"model": "gnp-lcc", "n0": n, "avg_deg": avg_deg, "seed": seed})


# ----------------------------------------------------------------------------
# Chung-Lu (rank-1 inhomogeneous random graph, f(x) = min(x, 1))
# ----------------------------------------------------------------------------

def _pareto_profile(n: int, beta: float) -> np.ndarray:
    """Pareto quantiles c_i = ((i+1)/n)^(-1/(beta-1)), descending in i (scalar libm)."""
    e = -1.0 / (beta - 1.0)
    return np.array([math.pow((i + 1) / n, e) for i in range(n)], dtype=np.float64)


def _expected_mean_degree(cout: np.ndarray, cin_sorted_desc: np.ndarray, scale_out: float,
                          scale_in: float, wsum: float) -> float:
    """(1/n) sum_u sum_{v != u} min(1, w_u w_v / W), self pairs ignored (O(n log n)).

    Used only to pick the weight scale; the realised graph is what it is.
    """
    n = cout.size
    wo = cout * scale_out
    wi = cin_sorted_desc * scale_in
    # for each u, the v's with wi_v >= W / wo_u are capped at 1
    thr = wsum / wo
    asc = wi[::-1]
    k = n - np.searchsorted(asc, thr, side="left")          # number of capped v
    suffix = np.concatenate([np.cumsum(wi[::-1])[::-1], [0.0]])
    tail = suffix[np.minimum(k, n)]
    tot = k.astype(np.float64) + wo * tail / wsum
    return math.fsum(tot.tolist()) / n


def _tune_scale(c_out, c_in_sorted, mean_deg, directed):
    """Bisection on the weight scale x_min so that the expected mean degree hits
    ``mean_deg`` (deterministic: fixed 40 iterations)."""
    n = c_out.size
    sum_out = math.fsum(c_out.tolist())
    sum_in = math.fsum(c_in_sorted.tolist())

    def mean_for(x):
        so = x
        si = x * sum_out / sum_in            # equal total weights out and in
        return _expected_mean_degree(c_out, c_in_sorted, so, si, x * sum_out)

    lo, hi = 0.0, mean_deg * n / sum_out * 4.0
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        if mean_for(mid) < mean_deg:
            lo = mid
        else:
            hi = mid
    x = 0.5 * (lo + hi)
    return x, x * sum_out / sum_in, x * sum_out


def _bucket_bounds(w_desc: np.ndarray, ratio: float = 2.0):
    """Split a descending weight array into contiguous index ranges whose weights
    stay within a factor ``ratio`` of the range's first weight."""
    bounds = [0]
    n = w_desc.size
    while bounds[-1] < n:
        start = bounds[-1]
        top = w_desc[start]
        # first index whose weight is < top / ratio
        asc = w_desc[::-1]
        j = n - int(np.searchsorted(asc, top / ratio, side="left"))
        j = max(j, start + 1)
        bounds.append(min(j, n))
    return bounds


def _sample_cells(rng, ncells: int, p: float) -> np.ndarray:
    """Indices of a Bernoulli(p) subset of range(ncells), by geometric gaps."""
    if ncells <= 0 or p <= 0.0:
        return np.zeros(0, dtype=np.int64)
    if p >= 1.0:
        return np.arange(ncells, dtype=np.int64)
    out = []
    pos = -1
    expect = ncells * p
    while True:
        k = int(expect + 6.0 * math.sqrt(expect + 1.0) + 64)
        gaps = rng.geometric(p, size=k).astype(np.int64)
        cs = pos + np.cumsum(gaps)
        cut = int(np.searchsorted(cs, ncells, side="left"))
        out.append(cs[:cut])
        if cut < k:
            break
        pos = int(cs[-1])
        expect = max((ncells - pos) * p, 1.0)
    return np.concatenate(out)


def _chung_lu_arcs(rng, wo, wi, in_order, wsum, directed, model="cl"):
    """Sample pairs (u, v) with independent probability min(1, wo_u wi_v / W).

    ``wo`` is descending by node id; ``in_order`` lists node ids by descending
    in-weight and ``wi`` is the in-weight in that order.  Candidates are drawn per
    pair of weight buckets with the bucket's largest probability and thinned to
    the exact one, so every pair is an independent coin flip.  For undirected
    graphs only u < v pairs are kept (``wo`` is ``wi`` and ``in_order`` is the
    identity).
    """
    bo = _bucket_bounds(wo)
    bi = _bucket_bounds(wi)
    srcs, dsts = [], []
    for a in range(len(bo) - 1):
        a0, a1 = bo[a], bo[a + 1]
        for b in range(len(bi) - 1):
            b0, b1 = bi[b], bi[b + 1]
            if not directed and b0 < a0:
                continue                       # undirected: only bucket pairs with b >= a
            if model == "cl":
                pmax = min(1.0, wo[a0] * wi[b0] / wsum)
            else:  # generalized random graph: x / (1 + x), increasing in x
                x0 = wo[a0] * wi[b0] / wsum
                pmax = x0 / (1.0 + x0)
            nb = b1 - b0
            cells = _sample_cells(rng, (a1 - a0) * nb, pmax)
            if cells.size == 0:
                continue
            u = a0 + cells // nb
            vpos = b0 + cells % nb
            v = in_order[vpos]
            if model == "cl":
                p = np.minimum(1.0, wo[u] * wi[vpos] / wsum)
            else:
                x = wo[u] * wi[vpos] / wsum
                p = x / (1.0 + x)
            acc = rng.random(cells.size) * pmax < p
            if directed:
                acc &= u != v
            else:
                acc &= u < v
            srcs.append(u[acc])
            dsts.append(v[acc])
    if not srcs:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(srcs), np.concatenate(dsts)


def chung_lu(n: int, beta: float, mean_deg: float, seed: int) -> CSR:
    """Undirected Chung-Lu graph with Pareto(beta) expected degrees of mean ``mean_deg``."""
    rng = np.random.default_rng(seed)
    c = _pareto_profile(n, beta)
    scale, _, wsum = _tune_scale(c, c, mean_deg, False)
    w = c * scale
    s, d = _chung_lu_arcs(rng, w, w, np.arange(n, dtype=np.int64), wsum, False)
    return csr_from_edges(n, s, d, False, name=f"cl{n}_b{beta}_d{mean_deg}_s{seed}",
                          meta={"model": "chung-lu", "beta": beta, "mean_deg": mean_deg,
                                "seed": seed, "xmin": scale})


def chung_lu_directed(n: int, beta_out: float, beta_in: float, mean_deg: float,
                      seed: int) -> CSR:
    """Directed Chung-Lu: arc u->v with probability min(1, wo_u wi_v / W).

    Out-weights are Pareto(beta_out) by node id; in-weights Pareto(beta_in) are
    assigned to nodes through a seeded permutation, so in- and out-degree are
    independent.  Both weight sets have the same total W.
    """
    rng = np.random.default_rng(seed)
    co = _pareto_profile(n, beta_out)
    ci = _pareto_profile(n, beta_in)
    perm = rng.permutation(n)               # node perm[j] gets the j-th largest in-weight
    so, si, wsum = _tune_scale(co, ci, mean_deg, True)
    s, d = _chung_lu_arcs(rng, co * so, ci * si, perm.astype(np.int64), wsum, True)
    return csr_from_edges(n, s, d, True,
                          name=f"dcl{n}_bo{beta_out}_bi{beta_in}_d{mean_deg}_s{seed}",
                          meta={"model": "chung-lu-directed", "beta_out": beta_out,
                                "beta_in": beta_in, "mean_deg": mean_deg, "seed": seed})


# ----------------------------------------------------------------------------
# the other random-graph models of the paper's appendix on random graphs
# ----------------------------------------------------------------------------
#
# All are undirected with n Pareto(beta) weights w_v (the quantiles of _pareto_profile)
# scaled to mean weight mean_deg, and M = sum of the weights:
#   * configuration model: node v gets round(w_v) (at least 1) half-edges, one more on a
#     seeded random node if the total is odd, paired by a seeded permutation; self-loops
#     and repeated edges are erased;
#   * Norros-Reittu: {u, v} is an edge with probability 1 - exp(-w_u w_v / M), i.e. when a
#     Poisson(w_u w_v / M) number of parallel edges is at least one.  Drawn exactly without
#     evaluating exp: Poisson(M/2) ordered endpoint pairs, each endpoint independently with
#     probability w/M, give every unordered pair a Poisson(w_u w_v / M) count;
#   * generalized random graph: probability x/(1+x), x = w_u w_v / M (the Chung-Lu sampler
#     with that function);
#   * Chung-Lu (chung_lu above): probability min(1, x), with the weight scale tuned to the
#     realised mean degree.


def _scaled_weights(n: int, beta: float, mean_deg: float) -> np.ndarray:
    c = _pareto_profile(n, beta)
    return c * (mean_deg * n / math.fsum(c.tolist()))


def configuration_model(n: int, beta: float, mean_deg: float, seed: int) -> CSR:
    rng = np.random.default_rng(seed)
    w = _scaled_weights(n, beta, mean_deg)
    deg = np.maximum(1, np.rint(w)).astype(np.int64)
    if int(deg.sum()) % 2 == 1:
        deg[int(rng.integers(0, n))] += 1
    stubs = np.repeat(np.arange(n, dtype=np.int64), deg)
    stubs = stubs[rng.permutation(stubs.size)]
    return csr_from_edges(n, stubs[0::2], stubs[1::2], False,
                          name=f"cm{n}_b{beta}_d{mean_deg}_s{seed}",
                          meta={"model": "configuration", "beta": beta, "mean_deg": mean_deg,
                                "seed": seed})


def norros_reittu(n: int, beta: float, mean_deg: float, seed: int) -> CSR:
    rng = np.random.default_rng(seed)
    w = _scaled_weights(n, beta, mean_deg)
    cum = np.cumsum(w)
    total = float(cum[-1])
    pairs = int(rng.poisson(total / 2.0))
    u = np.searchsorted(cum, rng.random(pairs) * total, side="right")
    v = np.searchsorted(cum, rng.random(pairs) * total, side="right")
    u = np.minimum(u, n - 1)
    v = np.minimum(v, n - 1)
    return csr_from_edges(n, u, v, False, name=f"nr{n}_b{beta}_d{mean_deg}_s{seed}",
                          meta={"model": "norros-reittu", "beta": beta, "mean_deg": mean_deg,
                                "seed": seed})


def generalized_random_graph(n: int, beta: float, mean_deg: float, seed: int) -> CSR:
    rng = np.random.default_rng(seed)
    w = _scaled_weights(n, beta, mean_deg)
    wsum = math.fsum(w.tolist())
    s, d = _chung_lu_arcs(rng, w, w, np.arange(n, dtype=np.int64), wsum, False, model="grg")
    return csr_from_edges(n, s, d, False, name=f"grg{n}_b{beta}_d{mean_deg}_s{seed}",
                          meta={"model": "generalized-random-graph", "beta": beta,
                                "mean_deg": mean_deg, "seed": seed})


RANDOM_MODELS = {"cl": lambda n, b, d, s: chung_lu(n, b, d, s),
                 "cm": configuration_model, "nr": norros_reittu,
                 "grg": generalized_random_graph}


def random_model(model: str, n: int, beta: float, mean_deg: float, seed: int) -> CSR:
    """One of the appendix's random-graph models: "cl", "cm", "nr" or "grg"."""
    return RANDOM_MODELS[model](n, beta, mean_deg, seed)


# ----------------------------------------------------------------------------
# a layered gadget with hub rows
# ----------------------------------------------------------------------------

def hub_layers(seed: int = 21) -> CSR:
    """Directed graph whose touch scans test hub rows by binary search: a regular node
    points to 16 of 64 A hubs and is pointed to by 16 of 64 B hubs; an A hub points to
    20,000 of 50,000 feeder nodes and 3 B hubs; a feeder points to 32 B hubs.  For two
    regular endpoints the s side's second level is 16 A hubs (320K arcs), the t side's
    16 B hubs (400K arcs in), so the A rows are searched for 16 nodes each: 256 (row,
    node) pairs, more than one pass of a workgroup."""
    rng = np.random.default_rng(seed)
    nr, nc, na, nb = 40_000, 50_000, 64, 64
    R0, C0, A0, B0 = 0, nr, nr + nc, nr + nc + na
    n = B0 + nb
    src, dst = [], []
    pick = np.argsort(rng.random((nr, na)), axis=1)[:, :16]
    src.append(np.repeat(np.arange(nr) + R0, 16)); dst.append(pick.ravel() + A0)
    pick = np.argsort(rng.random((nr, nb)), axis=1)[:, :16]
    src.append(pick.ravel() + B0); dst.append(np.repeat(np.arange(nr) + R0, 16))
    for a in range(na):
        tg = rng.choice(nc, 20_000, replace=False) + C0
        src.append(np.full(tg.size, A0 + a)); dst.append(tg)
        bb = rng.choice(nb, 3, replace=False) + B0
        src.append(np.full(3, A0 + a)); dst.append(bb)
    pick = np.argsort(rng.random((nc, nb)), axis=1)[:, :32]
    src.append(np.repeat(np.arange(nc) + C0, 32)); dst.append(pick.ravel() + B0)
    return csr_from_edges(n, np.concatenate(src), np.concatenate(dst), True,
                          name="hub_layers")


# ----------------------------------------------------------------------------
# many-graph family and the named workloads
# ----------------------------------------------------------------------------

def batch_family_spec(i: int) -> dict:
    """Parameters of graph i of the 256-graph family (seed 1000+i)."""
    rng = np.random.default_rng(1000 + i)
    n = int(round(10.0 ** rng.uniform(3.0, 5.0)))
    directed = bool(i % 2 == 1)
    b_out = float(rng.uniform(2.1, 2.8))
    b_in = float(rng.uniform(2.1, 2.8))
    mean_deg = float(rng.uniform(4.0, 30.0))
    return {"n": n, "directed": directed, "beta_out": b_out, "beta_in": b_in,
            "mean_deg": mean_deg, "seed": 1000 + i}


def batch_graph(i: int) -> CSR:
    sp = batch_family_spec(i)
    if sp["directed"]:
        return chung_lu_directed(sp["n"], sp["beta_out"], sp["beta_in"], sp["mean_deg"],
                                 sp["seed"])
    return chung_lu(sp["n"], sp["beta_out"], sp["mean_deg"], sp["seed"])


def serve_family_spec(i: int) -> dict:
    """Graph i (0..29) of the serving set's Chung-Lu graphs: n log-uniform in
    [1e4, 1e6], half directed, exponents in [2.1, 2.8], mean degree 4..30 (seed 2000+i)."""
    rng = np.random.default_rng(2000 + i)
    n = int(round(10.0 ** rng.uniform(4.0, 6.0)))
    directed = bool(i % 2 == 1)
    b_out = float(rng.uniform(2.1, 2.8))
    b_in = float(rng.uniform(2.1, 2.8))
    mean_deg = float(rng.uniform(4.0, 30.0))
    return {"n": n, "directed": directed, "beta_out": b_out, "beta_in": b_in,
            "mean_deg": mean_deg, "seed": 2000 + i}


SERVE_GRAPHS = 33


def serve_graph(i: int) -> CSR:
    """The resident graphs of the serving workload: 0 = er2000, 1 = cl1m,
    2..31 = serve_family_spec(0..29), 32 = grid2000."""
    if i == 0:
        return workload("er2000")
    if i == 1:
        return workload("cl1m")
    if i == 32:
        return workload("grid2000")
    sp = serve_family_spec(i - 2)
    if sp["directed"]:
        return chung_lu_directed(sp["n"], sp["beta_out"], sp["beta_in"], sp["mean_deg"],
                                 sp["seed"])
    return chung_lu(sp["n"], sp["beta_out"], sp["mean_deg"], sp["seed"])


def serve_queries(count: int, rate: float = 20.0, seed: int = 7, graphs: int = 33):
    """Poisson query stream: arrival times (s), graph index, mode, k, epsilon, seed.
    Graph index graphs-1 is the damaged grid; all-nodes or top-k (k in {10, 100}) with
    probability 1/2 each; epsilon uniform in [0.002, 0.02]; delta 0.1; Philox seed =
    query id + 1."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    gi = rng.integers(0, graphs, count)
    topk = rng.random(count) < 0.5
    k = np.where(rng.random(count) < 0.5, 10, 100)
    eps = rng.uniform(0.002, 0.02, count)
    return [{"t": float(t[q]), "graph": int(gi[q]), "mode": "topk" if topk[q] else "all",
             "k": int(k[q]) if topk[q] else 0, "epsilon": float(eps[q]), "delta": 0.1,
             "seed": q + 1} for q in range(count)]


def workload(name: str) -> CSR:
    """Named synthetic workloads.

    * ``er2000``: G(2000, 8/1999) seed 1, largest component (small case).
    * ``cl1m``: undirected Chung-Lu, n=1e6, beta=2.3, mean degree 20, seed 1.
    * ``dcl4m``: directed Chung-Lu, n=4e6, out beta 2.5, in beta 2.1, mean 15, seed 3.
    * ``grid2000``: 2000x2000 grid, 5% edges deleted, seed 5.
    """
    if name == "er2000":
        return er_lcc(2000, 8.0, 1)
    if name == "cl1m":
        return chung_lu(1_000_000, 2.3, 20.0, 1)
    if name == "dcl4m":
        return chung_lu_directed(4_000_000, 2.5, 2.1, 15.0, 3)
    if name == "grid2000":
        return damaged_grid(2000, 2000, 0.05, 5)
    raise KeyError(name)
