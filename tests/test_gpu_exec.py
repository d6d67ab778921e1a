"""kad_run's launch modes give one result.

KAD_EXEC_GRAPH (the default: main-phase batches replay recorded hipGraphs that read the
batch from a device descriptor), KAD_EXEC_STREAM (the same launches call by call) and
KAD_EXEC_PLAIN (the plain single-graph path: one sample per workgroup, a check after every
interval) are compared bit for bit, and with the CPU oracle, on runs of one batch and of
many batches, all-nodes and top-k, nodes and edges, 128-bit and wide path counts.  The
recorded chains are replayed many times in a row, with runs of the other modes and other
graphs in between, and every replay is checked against the call-by-call result.
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
    c.set_exec("graph")
    c.close()


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


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


def _vs_oracle(a, b, what):
    assert a["tau"] == b["tau"] and a["stop_reason"] == b["stop_rule"], what
    assert a["arcs_scanned"] == b["arcs"], what
    for k in _ARRAYS:
        assert np.array_equal(a[k], b[k]), (what, k)


def _graphs():
    return {
        "er2000": gg.workload("er2000"),
        "cl30k": gg.chung_lu(30_000, 2.3, 10.0, 31),
        "dcl30k": gg.chung_lu_directed(30_000, 2.5, 2.1, 8.0, 32),
        "grid90": gg.grid(90, 90),        # counts past 128 bits: wide fixes
        "grid140": gg.grid(140, 140),     # diameter >= 256: every sample wide
    }


_CASES = [
    ("er2000", dict(epsilon=0.01, seed=1)),                               # one batch
    ("er2000", dict(epsilon=0.006, seed=5, kernel_batch=2048)),           # many batches
    ("cl30k", dict(epsilon=0.01, seed=2, kernel_batch=4096, check_interval=1024)),
    ("dcl30k", dict(epsilon=0.01, seed=3, kernel_batch=2048)),
    ("cl30k", dict(epsilon=0.005, seed=4, kernel_batch=2048, mode="topk", k=10)),
    ("er2000", dict(epsilon=0.01, seed=6, kernel_batch=2048, target="edges")),
    ("grid90", dict(epsilon=0.03, seed=7, kernel_batch=1024)),
    ("grid140", dict(epsilon=0.08, seed=8, kernel_batch=1024)),
]


@pytest.fixture(scope="module")
def graphs(kad, ctx):
    gs = _graphs()
    Gs = {k: kad.Graph(ctx, v) for k, v in gs.items()}
    yield gs, Gs
    for G in Gs.values():
        G.close()


@pytest.mark.parametrize("name,kw", _CASES)
def test_modes_give_one_result(kad, ctx, orc, graphs, name, kw):
    gs, Gs = graphs
    res = {}
    for mode in ("stream", "graph", "plain"):
        ctx.set_exec(mode)
        _say("exec", mode, name, kw)
        res[mode] = kad.run(ctx, Gs[name], delta=0.1, **kw)
    ctx.set_exec("graph")
    _same(res["graph"], res["stream"], f"graph/stream {name} {kw}")
    _same(res["plain"], res["stream"], f"plain/stream {name} {kw}")
    if name in ("er2000", "cl30k", "dcl30k") and "mode" not in kw and "target" not in kw:
        okw = {k: v for k, v in kw.items() if k != "kernel_batch"}
        _say("oracle", name, okw)
        b = orc.run(gs[name], delta=0.1, threads=16, **okw)
        _vs_oracle(res["graph"], b, f"graph/oracle {name} {kw}")


def test_replays_in_a_row_match_call_by_call(kad, ctx, graphs):
    """Several kad_run calls replay the same recorded chains; between them come runs of the
    other modes, other graphs (which record other chains) and host synchronisations.
    Every graph-mode result equals the call-by-call result of the same call."""
    import torch
    gs, Gs = graphs
    seq = [("er2000", dict(epsilon=0.006, seed=11, kernel_batch=2048)),
           ("er2000", dict(epsilon=0.006, seed=12, kernel_batch=2048)),
           ("cl30k", dict(epsilon=0.01, seed=13, kernel_batch=2048)),
           ("er2000", dict(epsilon=0.006, seed=11, kernel_batch=2048)),
           ("er2000", dict(epsilon=0.008, seed=14, kernel_batch=2048)),
           ("dcl30k", dict(epsilon=0.01, seed=15, kernel_batch=4096)),
           ("er2000", dict(epsilon=0.006, seed=12, kernel_batch=2048))]
    ref = {}
    ctx.set_exec("stream")
    for j, (name, kw) in enumerate(seq):
        ref[j] = kad.run(ctx, Gs[name], delta=0.1, **kw)
    info0 = ctx.exec_info()
    for j, (name, kw) in enumerate(seq):
        ctx.set_exec("graph")
        _say("replay", j, name, kw)
        a = kad.run(ctx, Gs[name], delta=0.1, **kw)
        _same(a, ref[j], f"replay {j} {name} {kw}")
        torch.cuda.synchronize()
        ctx.set_exec("stream")  # eager work between the replays
        e = kad.run(ctx, Gs["er2000"], delta=0.1, epsilon=0.02, seed=100 + j)
        assert e["tau"] > 0
    ctx.set_exec("graph")
    info1 = ctx.exec_info()
    assert info1["replays"] - info0["replays"] >= 2 * len(seq)
    # a repeated call replays what the previous identical call recorded
    r0 = ctx.exec_info()["records"]
    a = kad.run(ctx, Gs["er2000"], delta=0.1, **seq[-1][1])
    b = kad.run(ctx, Gs["er2000"], delta=0.1, **seq[-1][1])
    _same(a, b, "repeat")
    _same(a, ref[len(seq) - 1], "repeat vs call by call")
    assert ctx.exec_info()["records"] == r0  # nothing recorded again


def test_exec_mode_rejects_unknown(kad, ctx):
    with pytest.raises(kad.KadError) as e:
        kad._check(kad.lib().kad_ctx_set_exec(ctx.handle, 7))
    assert e.value.status == -1
    assert ctx.exec_info()["mode"] == "graph"


def test_engine_ticks_replayed_equal_call_by_call(kad, ctx, graphs):
    """The engine replays each tick's sampling chain (segment table, sampler, wide-count
    passes, host mirrors) with the tick's size, segment count and stride read from a
    descriptor; its results equal the call-by-call engine's and kad_run's, twice in a row."""
    gs, Gs = graphs
    mix = [("er2000", dict(epsilon=0.01, seed=21)),
           ("cl30k", dict(epsilon=0.01, seed=22)),
           ("dcl30k", dict(epsilon=0.02, seed=23, mode="topk", k=5)),
           ("grid90", dict(epsilon=0.05, seed=24)),
           ("grid140", dict(epsilon=0.1, seed=25)),
           ("er2000", dict(epsilon=0.006, seed=26, kernel_batch=2048))]
    graphs_ = [Gs[name] for name, _ in mix]
    params = [dict(delta=0.1, **kw) for _, kw in mix]
    ctx.set_exec("stream")
    _say("engine call by call")
    a = kad.run_batch(ctx, graphs_, params)
    ctx.set_exec("graph")
    r0 = ctx.exec_info()["replays"]
    for rep in range(2):
        _say("engine replayed", rep)
        b = kad.run_batch(ctx, graphs_, params)
        for (name, kw), x, y in zip(mix, a, b):
            _same(y, x, f"engine replay {rep} {name} {kw}")
    assert ctx.exec_info()["replays"] > r0
    ctx.set_exec("stream")
    for (name, kw), x in zip(mix[:2], a):
        _same(kad.run(ctx, Gs[name], delta=0.1, **kw), x, f"kad_run {name}")
    ctx.set_exec("graph")
