"""Edge betweenness on the GPU against the CPU oracle, bit for bit.

A sampled path hits every one of its edges (section 1: the method adapts to edges): the
library rewrites each path as edge ids and reduces them with the node-hit kernels; the
oracle counts the edges of its own paths.  Edge hit counts, whole adaptive runs over the
edges (all edges and top-k), the edge-id map and the engine's refusal are checked.
"""
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


@pytest.mark.parametrize("name", ["er2000", "dcl", "grid", "path", "hub", "forward"])
def test_edge_hit_counts_match(kad, ctx, orc, name):
    g, cnt = {"er2000": (gg.workload("er2000"), 40000),
              "dcl": (gg.chung_lu_directed(100_000, 2.5, 2.1, 8.0, 3), 8000),
              "grid": (gg.grid(90, 90), 3000),          # counts past 128 bits
              "path": (gg.path_graph(300), 3000),       # paths too long to aggregate
              "hub": (gg.hub_layers(), 1500),           # more candidate edges than a slot
              "forward": (gg.chung_lu(20_000, 2.3, 8.0, 5), 4000)}[name]
    G = kad.Graph(ctx, g)
    search = "forward" if name == "forward" else "balanced"
    G.set_search(search)
    _say("edge_hit_counts", name, cnt)
    a, arcs = kad.edge_hit_counts(ctx, G, 4, 1, 50, cnt)
    b, barcs = orc.edge_hits(g, 4, 1, 50, cnt, threads=16, search=search)
    assert len(a) == len(b) == G.edge_count()
    assert np.array_equal(a, b)
    assert arcs == barcs
    assert np.array_equal(G.edge_ids(), orc.edge_ids(g))
    G.close()


def _same_run(a, b, what):
    assert a["tau"] == b["tau"], (what, a["tau"], b["tau"])
    assert a["omega"] == b["omega"] and a["alpha"] == b["alpha"], what
    assert a["stop_reason"] == b["stop_rule"], what
    assert a["arcs_scanned"] == b["arcs"], what
    assert np.array_equal(a["count"], b["count"]), what
    assert np.array_equal(a["bc"], b["bc"]), what
    assert np.array_equal(a["lower"], b["lower"]), what
    assert np.array_equal(a["upper"], b["upper"]), what


@pytest.mark.parametrize("name,kw", [
    ("er2000", dict(epsilon=0.01, seed=1)),
    ("er2000", dict(epsilon=0.01, seed=3, kernel_batch=2048)),
    ("dcl", dict(epsilon=0.01, seed=2)),
    ("cl", dict(epsilon=0.004, seed=2, mode="topk", k=8)),
])
def test_run_edges_equals_oracle(kad, ctx, orc, name, kw):
    g = {"er2000": lambda: gg.workload("er2000"),
         "dcl": lambda: gg.chung_lu_directed(20_000, 2.5, 2.1, 6.0, 7),
         "cl": lambda: gg.chung_lu(5000, 2.3, 6.0, 9)}[name]()
    G = kad.Graph(ctx, g)
    _say("edge run", name, kw)
    a = kad.run(ctx, G, delta=0.1, target="edges", **kw)
    okw = {k: v for k, v in kw.items() if k != "kernel_batch"}
    b = orc.run(g, delta=0.1, threads=16, target="edges", **okw)
    assert a["items"] == G.edge_count() and a["count"].size == a["items"]
    _same_run(a, b, f"{name} {kw}")
    if kw.get("mode") == "topk":
        rlo, rhi = orc.rank_intervals(b["lower"], b["upper"])
        sel = sorted(np.nonzero(rlo <= kw["k"])[0].tolist(), key=lambda e: (-int(b["count"][e]), e))
        assert a["topk_node"].tolist() == sel
        assert a["rank_lo"].tolist() == [int(rlo[e]) for e in sel]
    G.close()


def test_run_edges_fixed_schedule(kad, ctx, orc):
    """The RK schedule over edges: floor(log2(VD - 1)) + 1 in the sample count, hits of
    main-phase ids 0..tau-1 on the edges."""
    g = gg.workload("er2000")
    G = kad.Graph(ctx, g)
    r = kad.run(ctx, G, epsilon=0.02, delta=0.1, seed=5, schedule="rk", target="edges")
    assert r["tau"] == orc.omega_edges(0.02, 0.2, 8)
    cnt, arcs = orc.edge_hits(g, 5, 1, 0, r["tau"], threads=16)
    assert np.array_equal(r["count"], cnt) and r["arcs_scanned"] == arcs
    G.close()


def test_engine_refuses_edges(kad, ctx):
    g = gg.workload("er2000")
    G = kad.Graph(ctx, g)
    with pytest.raises(kad.KadError) as e:
        kad.run_batch(ctx, [G], [dict(epsilon=0.01, delta=0.1, target="edges")])
    assert e.value.status == -1
    G.close()
