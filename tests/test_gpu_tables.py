"""Sampler slots as hash tables (kad_ctx_set_table) give the results of one record per node.

The searches of section 4 keep a tag and a 128-bit path count for every node they reach.
With tables, a slot holds 2^k records whatever the graph; nodes collide on their home
records and probe on, and a sample whose nodes find no free record within the probe limit
is sampled again by the wide-count kernel (dense records).  Checked against the CPU oracle
and against the dense layout, bit for bit:

* sampled paths (every sample unflagged after the wide pass) with tables of 2^12 records
  (collisions) and of 2^6 (most samples of a 30K-node graph overflow and are resampled);
* whole kad_run calls: all nodes, top-k, edges, several batches, in every launch mode;
* the multi-query engine;
* the library's own choice: tables when one record per node would leave fewer than four
  slots per CU (a small memory budget here), dense otherwise.
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
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="module")
def graphs():
    return {
        "er2000": gg.workload("er2000"),
        "cl30k": gg.chung_lu(30_000, 2.3, 10.0, 31),
        "dcl30k": gg.chung_lu_directed(30_000, 2.5, 2.1, 8.0, 32),
        "hub": gg.hub_layers(),
    }


def _ctx(kad, bits):
    c = kad.Context(0)
    c.set_table(bits)
    return c


_KEYS = ("tau", "omega", "alpha", "vd", "interval", "stop_reason", "arcs_scanned",
         "pilot_arcs_scanned", "items")
_ARRAYS = ("count", "bc", "lower", "upper")


def _same(a, b, what):
    for k in _KEYS:
        assert a[k] == b[k], (what, k, a[k], b[k])
    for k in _ARRAYS:
        assert np.array_equal(a[k], b[k]), (what, k)
    if "topk_node" in a or "topk_node" in b:
        assert np.array_equal(a["topk_node"], b["topk_node"]), what


@pytest.mark.parametrize("bits", [12, 6])
@pytest.mark.parametrize("name,count", [("er2000", 6000), ("cl30k", 6000), ("dcl30k", 4000),
                                        ("hub", 1500)])
def test_paths_with_tables(kad, orc, graphs, bits, name, count):
    g = graphs[name]
    ctx = _ctx(kad, bits)
    G = kad.Graph(ctx, g)
    _say("sample_paths tables", bits, name, count)
    A = kad.sample_paths(ctx, G, 3, 1, 100, count)
    info = ctx.table_info()
    assert info["log2_records"] == bits and info["slots"] > 0 and info["wide_slots"] > 0
    B = orc.sample_paths(g, 3, 1, 100, count, threads=16)
    assert (A["flags"] == 0).all(), np.unique(A["flags"])
    assert np.array_equal(A["s"], B.s) and np.array_equal(A["t"], B.t)
    assert np.array_equal(A["arcs"], B.arcs)
    assert np.array_equal(A["path_off"], B.path_off)
    assert np.array_equal(A["nodes"], B.nodes)
    G.close()
    ctx.close()


_RUNS = [
    ("er2000", dict(epsilon=0.01, seed=1)),
    ("cl30k", dict(epsilon=0.01, seed=2, kernel_batch=4096, check_interval=1024)),
    ("dcl30k", dict(epsilon=0.01, seed=3, kernel_batch=2048)),
    ("cl30k", dict(epsilon=0.005, seed=4, kernel_batch=2048, mode="topk", k=10)),
    ("er2000", dict(epsilon=0.01, seed=6, kernel_batch=2048, target="edges")),
    ("hub", dict(epsilon=0.02, seed=7)),
]


@pytest.mark.parametrize("name,kw", _RUNS)
def test_runs_with_tables_equal_dense(kad, orc, graphs, name, kw):
    g = graphs[name]
    dense = _ctx(kad, 1)
    Gd = kad.Graph(dense, g)
    _say("dense run", name, kw)
    ref = kad.run(dense, Gd, delta=0.1, **kw)
    assert dense.table_info()["log2_records"] == 0
    Gd.close()
    dense.close()
    for bits in (12, 6):
        ctx = _ctx(kad, bits)
        G = kad.Graph(ctx, g)
        for mode in ("graph", "stream", "plain"):
            ctx.set_exec(mode)
            _say("tables", bits, mode, name, kw)
            _same(kad.run(ctx, G, delta=0.1, **kw), ref, f"tables {bits} {mode} {name} {kw}")
        G.close()
        ctx.close()
    if "mode" not in kw and "target" not in kw:
        okw = {k: v for k, v in kw.items() if k != "kernel_batch"}
        b = orc.run(g, delta=0.1, threads=16, **okw)
        assert ref["tau"] == b["tau"] and ref["stop_reason"] == b["stop_rule"]
        for k in _ARRAYS:
            assert np.array_equal(ref[k], b[k]), (name, k)


def test_engine_with_tables(kad, graphs):
    mix = [("er2000", dict(epsilon=0.01, seed=21)),
           ("cl30k", dict(epsilon=0.01, seed=22)),
           ("dcl30k", dict(epsilon=0.02, seed=23, mode="topk", k=5)),
           ("hub", dict(epsilon=0.03, seed=24))]
    params = [dict(delta=0.1, **kw) for _, kw in mix]
    res = {}
    for bits in (1, 12, 6):
        ctx = _ctx(kad, bits)
        Gs = [kad.Graph(ctx, graphs[name]) for name, _ in mix]
        _say("engine tables", bits)
        res[bits] = kad.run_batch(ctx, Gs, params)
        for G in Gs:
            G.close()
        ctx.close()
    for bits in (12, 6):
        for (name, kw), a, b in zip(mix, res[bits], res[1]):
            _same(a, b, f"engine tables {bits} {name} {kw}")


def test_library_choice(kad, orc):
    """A 70K-node graph: dense under the default budget; tables of 2^16 under a budget that
    would leave fewer than four dense slots per CU."""
    g = gg.chung_lu(70_000, 2.3, 8.0, 41)
    kw = dict(epsilon=0.01, delta=0.1, seed=5)
    big = kad.Context(0)
    G = kad.Graph(big, g)
    _say("library choice, default budget")
    a = kad.run(big, G, **kw)
    assert big.table_info()["log2_records"] == 0
    G.close()
    big.close()
    small = kad.Context(0, 3 << 30)
    G = kad.Graph(small, g)
    _say("library choice, 3 GiB budget")
    b = kad.run(small, G, **kw)
    info = small.table_info()
    assert info["log2_records"] == 16 and info["wide_slots"] > 0, info
    _same(b, a, "tables chosen by the library")
    G.close()
    small.close()
    o = orc.run(g, threads=16, **kw)
    assert a["tau"] == o["tau"] and np.array_equal(a["count"], o["count"])


def test_table_knob_rejects(kad):
    ctx = kad.Context(0)
    for bad in (2, 5, 25):
        with pytest.raises(kad.KadError) as e:
            ctx.set_table(bad)
        assert e.value.status == -1
    ctx.close()


@pytest.mark.parametrize("bits", [12, 6])
def test_forward_search_and_edges_with_tables(kad, orc, graphs, bits):
    """The plain BFS from s (the forward search) and edge hits with slot tables."""
    g = graphs["cl30k"]
    ctx = _ctx(kad, bits)
    G = kad.Graph(ctx, g)
    G.set_search("forward")
    _say("forward search, tables", bits)
    A = kad.sample_paths(ctx, G, 5, 1, 0, 1500)
    B = orc.sample_paths(g, 5, 1, 0, 1500, threads=16, search="forward")
    assert (A["flags"] == 0).all()
    assert np.array_equal(A["arcs"], B.arcs) and np.array_equal(A["nodes"], B.nodes)
    G.set_search("balanced")
    _say("edge hits, tables", bits)
    a, arcs = kad.edge_hit_counts(ctx, G, 4, 1, 50, 3000)
    b, barcs = orc.edge_hits(g, 4, 1, 50, 3000, threads=16)
    assert np.array_equal(a, b) and arcs == barcs
    G.close()
    ctx.close()
