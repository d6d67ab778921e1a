"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit for bit.

Sampled paths (s, t, every node, arcs scanned), hit counts, and whole adaptive runs
(tau, counts, interval bounds, top-k output) must be identical for the same seed.
"""
import os
import sys

import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kad():
    import torch
    assert torch.cuda.is_available(), "no GPU"
    import paper_1604_08553_amd as k
    k.lib()
    return k


@pytest.fixture(scope="module")
def ctx(kad):
    c = kad.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def _compare_paths(kad, ctx, orc, csr, seed, phase, first, count, allow_flags=False):
    G = kad.Graph(ctx, csr)
    _say("sample_paths", csr.name, "n", csr.n, "seed", seed, "phase", phase, "ids", first, count)
    A = kad.sample_paths(ctx, G, seed, phase, first, count)
    B = orc.sample_paths(csr, seed, phase, first, count, threads=16)
    ok = A["flags"] == 0
    if not allow_flags:
        assert ok.all(), np.unique(A["flags"])
    assert np.array_equal(A["s"], B.s) and np.array_equal(A["t"], B.t)
    assert np.array_equal(A["arcs"][ok], B.arcs[ok])
    for k in np.nonzero(ok)[0]:
        a = A["nodes"][A["path_off"][k]:A["path_off"][k + 1]]
        b = B.path(k)
        assert np.array_equal(a, b), (k, a, b)
    G.close()
    return A, B


def test_paths_er2000_65536(kad, ctx, orc):
    g = gg.workload("er2000")
    _compare_paths(kad, ctx, orc, g, 1, 1, 0, 65536)
    _compare_paths(kad, ctx, orc, g, 7, 0, 12345, 3001)


@pytest.mark.parametrize("name", ["gnp_u", "gnp_d", "path", "star", "cycle", "grid", "union",
                                  "K2", "empty2", "kbip"])
def test_paths_small_graphs(kad, ctx, orc, name):
    g = {"gnp_u": lambda: gg.gnp(60, 0.05, 3), "gnp_d": lambda: gg.gnp(60, 0.04, 4, True),
         "path": lambda: gg.path_graph(40), "star": lambda: gg.star_graph(30),
         "cycle": lambda: gg.cycle_graph(25, True), "grid": lambda: gg.grid(12, 17),
         "union": lambda: gg.disjoint_union(gg.path_graph(9), gg.cycle_graph(6, True),
                                            gg.star_graph(5)),
         "K2": lambda: gg.path_graph(2),
         "empty2": lambda: gg.csr_from_edges(2, [], [], False, name="empty2"),
         "kbip": lambda: gg.complete_bipartite(30, 45)}[name]()
    _compare_paths(kad, ctx, orc, g, 11, 1, 0, 4099)


def test_paths_many_meeting_edges(kad, ctx, orc):
    """K_{1500,1500}: a pair on one side meets through 1500 candidate edges (more than
    the LDS staging holds, so the sort runs in the slot's global buffer)."""
    g = gg.complete_bipartite(1500, 1500)
    _compare_paths(kad, ctx, orc, g, 5, 1, 0, 300)


def test_paths_directed_chung_lu(kad, ctx, orc):
    g = gg.chung_lu_directed(200_000, 2.5, 2.1, 10.0, 9)
    _compare_paths(kad, ctx, orc, g, 3, 1, 0, 4000)


def test_paths_chung_lu_1m_sampled_ids(kad, ctx, orc):
    """The bench workload at full size: ids drawn across the main phase's range."""
    g = gg.workload("cl1m")
    _compare_paths(kad, ctx, orc, g, 1, 1, 0, 3000)
    _compare_paths(kad, ctx, orc, g, 1, 1, 150_000, 1000)
    _compare_paths(kad, ctx, orc, g, 1, 0, 0, 1000)


def _hub_layers(seed=21):
    return gg.hub_layers(seed)


@pytest.mark.parametrize("block", [64, 128, 256])
def test_paths_hub_rows_searched(kad, ctx, orc, block):
    """Touch scans that search long rows for the other frontier's nodes (several
    passes of pairs per chunk, endpoints that are hubs) give the oracle's paths.  Two
    endpoints off the regular layer (mostly two feeders) meet through up to ~370K
    candidate edges, more than a slot's 65,536-entry buffer: those samples are sampled
    again by the wide-count kernel, which keeps every candidate edge in its arena and
    picks one by a weighted radix select -- the same edge as the oracle's canonical
    prefix sum."""
    g = _hub_layers()
    G = kad.Graph(ctx, g)
    G.set_launch(block, 0)
    _say("hub_layers", block)
    A = kad.sample_paths(ctx, G, 4, 1, 0, 3000)
    B = orc.sample_paths(g, 4, 1, 0, 3000, threads=16)
    assert (A["flags"] == 0).all(), np.unique(A["flags"])
    assert np.array_equal(A["s"], B.s) and np.array_equal(A["t"], B.t)
    assert np.array_equal(A["arcs"], B.arcs)
    assert np.array_equal(A["path_off"], B.path_off.astype(np.uint64))
    assert np.array_equal(A["nodes"], B.nodes)
    lens = np.diff(B.path_off.astype(np.int64))
    # the layered case occurred: paths s -> A hub -> B hub -> t between regular nodes
    both = (B.s < 40_000) & (B.t < 40_000)
    assert (lens[both] == 4).sum() > 100
    # and the large meetings did: pairs of two feeder nodes
    feeders = (B.s >= 40_000) & (B.s < 90_000) & (B.t >= 40_000) & (B.t < 90_000)
    assert feeders.sum() > 500
    G.close()


def test_run_hub_layers_large_meetings(kad, ctx, orc):
    """Whole runs where about half the samples meet through more candidate edges than a
    slot holds: the single run and the engine equal the oracle."""
    g = _hub_layers()
    G = kad.Graph(ctx, g)
    kw = dict(epsilon=0.02, delta=0.1, seed=6)
    _say("hub_layers kad_run")
    a = kad.run(ctx, G, **kw)
    b = orc.run(g, threads=16, **kw)
    assert a["tau"] == b["tau"] and a["stop_reason"] == b["stop_rule"]
    assert a["arcs_scanned"] == b["arcs"] and a["pilot_arcs_scanned"] == b["pilot_arcs"]
    assert np.array_equal(a["count"], b["count"])
    assert np.array_equal(a["lower"], b["lower"]) and np.array_equal(a["upper"], b["upper"])
    assert a["overflow_samples"] > a["tau"] // 10   # sampled again for their candidate edges
    _say("hub_layers run_batch")
    c = kad.run_batch(ctx, [G, G], [kw, dict(kw, seed=7)])
    assert c[0]["tau"] == b["tau"] and np.array_equal(c[0]["count"], b["count"])
    assert np.array_equal(c[0]["lower"], b["lower"]) and np.array_equal(c[0]["upper"], b["upper"])
    d = orc.run(g, threads=16, **dict(kw, seed=7))
    assert c[1]["tau"] == d["tau"] and np.array_equal(c[1]["count"], d["count"])
    G.close()


_SHAPE_GRAPHS = {}


def _shape_graph(name):
    if name not in _SHAPE_GRAPHS:
        _SHAPE_GRAPHS[name] = {
            "er2000": lambda: (gg.workload("er2000"), 4099),
            "kbip1500": lambda: (gg.complete_bipartite(1500, 1500), 200),
            "dcl": lambda: (gg.chung_lu_directed(200_000, 2.5, 2.1, 10.0, 9), 1500),
            "union": lambda: (gg.disjoint_union(gg.path_graph(90), gg.star_graph(300),
                                                gg.grid(20, 30)), 3000),
        }[name]()
    return _SHAPE_GRAPHS[name]


@pytest.mark.parametrize("block", [64, 128, 256])
@pytest.mark.parametrize("small", [128, 2048])
@pytest.mark.parametrize("name", ["er2000", "kbip1500", "dcl", "union"])
def test_paths_every_launch_shape(kad, ctx, orc, block, small, name):
    """Workgroup size and scan threshold are performance choices only: every shape
    gives the oracle's paths."""
    g, cnt = _shape_graph(name)
    G = kad.Graph(ctx, g)
    G.set_launch(block, small)
    assert G.launch() == (block, small)
    _say("shape", block, small, name)
    A = kad.sample_paths(ctx, G, 3, 1, 17, cnt)
    B = orc.sample_paths(g, 3, 1, 17, cnt, threads=16)
    assert (A["flags"] == 0).all()
    assert np.array_equal(A["s"], B.s) and np.array_equal(A["t"], B.t)
    assert np.array_equal(A["arcs"], B.arcs)
    assert np.array_equal(A["path_off"], B.path_off.astype(np.uint64))
    assert np.array_equal(A["nodes"], B.nodes)
    G.close()


def test_autotune_keeps_results(kad, ctx, orc):
    g = gg.workload("er2000")
    G = kad.Graph(ctx, g)
    before = kad.run(ctx, G, epsilon=0.01, delta=0.1, seed=1)
    t = G.autotune(16384)
    _say("autotune er2000", t)
    assert t["block"] in (64, 128, 256) and t["seconds"] > 0
    assert G.launch() == (t["block"], t["small_expansion"])
    after = kad.run(ctx, G, epsilon=0.01, delta=0.1, seed=1)
    assert after["tau"] == before["tau"] and np.array_equal(after["count"], before["count"])
    G.close()


def test_paths_grid_wide_counts(kad, ctx, orc):
    """On a 500x500 grid the path counts of distant pairs pass 2^128 (a node l levels
    out on a diagonal has C(l, l/2) shortest paths): those samples are sampled again
    with multi-limb counts and must match the oracle's arbitrary precision exactly."""
    g = gg.grid(500, 500)
    A, B = _compare_paths(kad, ctx, orc, g, 2, 1, 0, 160)
    d = np.diff(B.path_off.astype(np.int64)) - 1
    assert (d >= 300).sum() >= 20  # far beyond 128-bit counts


def test_paths_high_diameter_all_wide(kad, ctx, orc):
    """A damaged grid with vertex diameter above 256: every sample goes straight to the
    wide-count kernel (no 128-bit attempt first); parity is unchanged."""
    g = gg.damaged_grid(200, 200, 0.05, 7)
    _compare_paths(kad, ctx, orc, g, 6, 1, 0, 300)
    _compare_paths(kad, ctx, orc, g, 6, 0, 1000, 100)


def test_hit_counts_wide(kad, ctx, orc):
    g = gg.damaged_grid(150, 150, 0.05, 3)
    G = kad.Graph(ctx, g)
    a, arcs = kad.hit_counts(ctx, G, 4, 1, 0, 3000)
    S = orc.sample_paths(g, 4, 1, 0, 3000, threads=16)
    b = np.zeros(g.n, dtype=np.uint64)
    for k in range(3000):
        p = S.path(k)
        b[p[1:-1]] += 1
    assert np.array_equal(a, b)
    assert arcs == int(S.arcs.sum())
    G.close()


def test_hit_counts_match(kad, ctx, orc):
    # er2000: short paths (hits pre-aggregated 64 samples at a time); 30x30 grid: longer
    # paths (fewer samples per aggregation); 600-node path: paths too long to aggregate.
    # Calls of at most 2^17 interior hits take the one-atomic-per-hit kernel instead:
    # er2000 with 4,096 samples, and a star whose centre lies on nearly every path (one
    # counter under ~4,000 concurrent atomics)
    for g, cnt in [(gg.workload("er2000"), 50000), (gg.gnp(300, 0.02, 5, True), 20000),
                   (gg.grid(30, 30), 20000), (gg.path_graph(600), 3000),
                   (gg.workload("er2000"), 4096), (gg.star_graph(3000), 4000)]:
        _say("hit_counts", g.name, cnt)
        G = kad.Graph(ctx, g)
        a, arcs = kad.hit_counts(ctx, G, 4, 1, 100, cnt)
        S = orc.sample_paths(g, 4, 1, 100, cnt, threads=16)
        b = np.zeros(g.n, dtype=np.uint64)
        for k in range(cnt):
            p = S.path(k)
            b[p[1:-1]] += 1
        assert np.array_equal(a, b)
        assert arcs == int(S.arcs.sum())
        G.close()


def _compare_run(kad, ctx, orc, g, **kw):
    _say("run", g.name, kw)
    G = kad.Graph(ctx, g)
    a = kad.run(ctx, G, **kw)
    okw = dict(kw)
    okw.pop("kernel_batch", None)
    b = orc.run(g, threads=16, **okw)
    for key in ("tau", "omega", "alpha", "vd"):
        assert a[key] == b[key], (key, a[key], b[key])
    assert a["stop_reason"] == b["stop_rule"]
    assert a["arcs_scanned"] == b["arcs"]
    assert np.array_equal(a["count"], b["count"])
    assert np.array_equal(a["bc"], b["bc"])
    assert np.array_equal(a["lower"], b["lower"]) and np.array_equal(a["upper"], b["upper"])
    G.close()
    return a, b


def test_run_er2000_all_nodes(kad, ctx, orc):
    a, b = _compare_run(kad, ctx, orc, gg.workload("er2000"), epsilon=0.01, delta=0.1, seed=1)
    assert a["omega"] == 29979 and a["alpha"] == 299 and a["stop_reason"] == 1


def test_run_kernel_batch_does_not_change_result(kad, ctx, orc):
    g = gg.workload("er2000")
    G = kad.Graph(ctx, g)
    r1 = kad.run(ctx, G, 0.01, 0.1, seed=3, kernel_batch=1024)
    r2 = kad.run(ctx, G, 0.01, 0.1, seed=3, kernel_batch=65536)
    assert r1["tau"] == r2["tau"] and np.array_equal(r1["count"], r2["count"])


def test_run_directed_and_disconnected(kad, ctx, orc):
    g = gg.disjoint_union(gg.chung_lu_directed(3000, 2.5, 2.1, 6.0, 4), gg.cycle_graph(50, True))
    _compare_run(kad, ctx, orc, g, epsilon=0.02, delta=0.1, seed=9)


def test_run_topk(kad, ctx, orc):
    g = gg.chung_lu(1500, 2.3, 6.0, 42)
    a, b = _compare_run(kad, ctx, orc, g, epsilon=0.004, delta=0.1, mode="topk", k=5, seed=2)
    rlo, rhi = orc.rank_intervals(b["lower"], b["upper"])
    sel = np.nonzero(rlo <= 5)[0]
    cnt = b["count"]
    sel = sorted(sel.tolist(), key=lambda v: (-int(cnt[v]), v))
    assert a["topk_node"].tolist() == sel
    assert a["rank_lo"].tolist() == [int(rlo[v]) for v in sel]
    assert a["rank_hi"].tolist() == [int(rhi[v]) for v in sel]


def test_run_damaged_grid_wide(kad, ctx, orc):
    """A high-diameter graph where most samples need counts beyond 128 bits."""
    g = gg.damaged_grid(120, 120, 0.05, 5)
    a, b = _compare_run(kad, ctx, orc, g, epsilon=0.03, delta=0.1, seed=4)
    assert a["overflow_samples"] > 0


def test_run_complete_graph_g_only(kad, ctx, orc):
    a, b = _compare_run(kad, ctx, orc, gg.complete_graph(20), epsilon=0.01, delta=0.1, seed=3)
    assert a["count"].sum() == 0 and a["stop_reason"] == 1


def test_device_memory_graph_and_torch_stream(kad, ctx, orc):
    import torch
    g = gg.workload("er2000")
    row = torch.from_numpy(g.row.astype(np.int32)).cuda()
    col = torch.from_numpy(g.col.astype(np.int32)).cuda()
    G = kad.Graph(ctx, n=g.n, row=row, col=col, directed=False, mem="device")
    s = torch.cuda.Stream()
    A = kad.sample_paths(ctx, G, 1, 1, 0, 2000, stream=s)
    B = orc.sample_paths(g, 1, 1, 0, 2000, threads=16)
    assert np.array_equal(A["nodes"], B.nodes)
    G.close()


@pytest.mark.parametrize("schedule", ["rk", "hoeffding"])
def test_run_fixed_schedule(kad, ctx, orc, schedule):
    """Fixed schedules: exactly tau main-phase samples (ids 0..tau-1), counts equal the
    oracle's hits over the same samples, intervals bc +- eps."""
    g = gg.workload("er2000")
    G = kad.Graph(ctx, g)
    r = kad.run(ctx, G, epsilon=0.02, delta=0.1, seed=5, schedule=schedule)
    tau = kad.fixed_samples(schedule, 0.02, 0.1, 8, g.n)
    assert r["tau"] == tau and r["stop_reason"] == kad.STOP_FIXED and r["alpha"] == 0
    S = orc.sample_paths(g, 5, 1, 0, tau, threads=16)
    b = np.zeros(g.n, dtype=np.uint64)
    for k in range(tau):
        p = S.path(k)
        b[p[1:-1]] += 1
    assert np.array_equal(r["count"], b)
    assert r["arcs_scanned"] == int(S.arcs.sum())
    assert np.array_equal(r["bc"], b / float(tau))
    assert np.array_equal(r["lower"], r["bc"] - 0.02) and np.array_equal(r["upper"], r["bc"] + 0.02)
    G.close()


@pytest.mark.parametrize("name", ["er2000", "dcl", "grid", "kbip", "union"])
def test_paths_forward_search(kad, ctx, orc, name):
    """The forward search (a plain BFS from s until t's level) gives the oracle's paths and
    arcs; on the 500x500 grid its counts pass 128 bits and go to the wide-count kernel."""
    g, cnt = {"er2000": (gg.workload("er2000"), 4099),
              "dcl": (gg.chung_lu_directed(200_000, 2.5, 2.1, 10.0, 9), 1500),
              "grid": (gg.grid(120, 120), 200),
              "kbip": (gg.complete_bipartite(300, 400), 500),
              "union": (gg.disjoint_union(gg.path_graph(90), gg.star_graph(300),
                                          gg.grid(20, 30)), 3000)}[name]
    G = kad.Graph(ctx, g)
    G.set_search("forward")
    assert G.search() == "forward"
    _say("forward search", name)
    A = kad.sample_paths(ctx, G, 3, 1, 11, cnt)
    B = orc.sample_paths(g, 3, 1, 11, cnt, threads=16, search="forward")
    assert (A["flags"] == 0).all()
    assert np.array_equal(A["s"], B.s) and np.array_equal(A["t"], B.t)
    assert np.array_equal(A["arcs"], B.arcs)
    assert np.array_equal(A["path_off"], B.path_off.astype(np.uint64))
    assert np.array_equal(A["nodes"], B.nodes)
    G.close()


def test_run_forward_search_equals_oracle(kad, ctx, orc):
    """Algorithm 1 with the forward search, and the RK algorithm (fixed RK sample count with
    the forward search: the comparison system of section 6) on the same graph."""
    g = gg.chung_lu(20_000, 2.5, 8.0, 12)
    G = kad.Graph(ctx, g)
    G.set_search("forward")
    a = kad.run(ctx, G, epsilon=0.01, delta=0.1, seed=4)
    b = orc.run(g, 0.01, 0.1, seed=4, threads=16, search="forward")
    assert a["tau"] == b["tau"] and a["stop_reason"] == b["stop_rule"]
    assert a["arcs_scanned"] == b["arcs"] and a["pilot_arcs_scanned"] == b["pilot_arcs"]
    assert np.array_equal(a["count"], b["count"])
    assert np.array_equal(a["lower"], b["lower"]) and np.array_equal(a["upper"], b["upper"])
    r = kad.run(ctx, G, epsilon=0.02, delta=0.1, seed=4, schedule="rk")
    S = orc.sample_paths(g, 4, 1, 0, r["tau"], threads=16, search="forward")
    cnt = np.zeros(g.n, dtype=np.uint64)
    for k in range(r["tau"]):
        p = S.path(k)
        cnt[p[1:-1]] += 1
    assert np.array_equal(r["count"], cnt) and r["arcs_scanned"] == int(S.arcs.sum())
    # the balanced search scans far fewer arcs for the same kind of run
    G.set_search("balanced")
    c = kad.run(ctx, G, epsilon=0.02, delta=0.1, seed=4, schedule="rk")
    assert c["arcs_scanned"] * 3 < r["arcs_scanned"]
    G.close()
