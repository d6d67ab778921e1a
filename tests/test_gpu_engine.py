"""The multi-query engine (kad_run_batch, kad_server_*) against the single run.

Every query of a batch or of the server must give exactly kad_run's result for its
graph and parameters (tau, stop reason, arcs, counts, intervals, top-k output):
the engine only changes which launches carry the samples.  One mix is also checked
against the CPU oracle directly.
"""
import sys
import time

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


def _same(a, b, what=""):
    for key in ("tau", "omega", "alpha", "interval", "vd", "stop_reason", "arcs_scanned",
                "pilot_arcs_scanned"):
        assert a[key] == b[key], (what, key, a[key], b[key])
    for key in ("count", "bc", "lower", "upper"):
        assert np.array_equal(a[key], b[key]), (what, key)
    if "topk_node" in b:
        for key in ("topk_node", "rank_lo", "rank_hi"):
            assert np.array_equal(a[key], b[key]), (what, key)


def _mix():
    return [
        (gg.workload("er2000"), dict(epsilon=0.01, delta=0.1, seed=1)),
        (gg.disjoint_union(gg.chung_lu_directed(3000, 2.5, 2.1, 6.0, 4), gg.cycle_graph(50, True)),
         dict(epsilon=0.02, delta=0.1, seed=9)),
        (gg.chung_lu(1500, 2.3, 6.0, 42), dict(epsilon=0.004, delta=0.1, mode="topk", k=5, seed=2)),
        (gg.complete_graph(20), dict(epsilon=0.01, delta=0.1, seed=3)),
        (gg.workload("er2000"), dict(epsilon=0.02, delta=0.05, seed=7, check_interval=2048)),
        (gg.gnp(400, 0.02, 5, True), dict(epsilon=0.015, delta=0.1, seed=11)),
        (gg.grid(30, 30), dict(epsilon=0.02, delta=0.1, seed=4)),
        (gg.damaged_grid(120, 120, 0.05, 5), dict(epsilon=0.03, delta=0.1, seed=4)),
        (gg.damaged_grid(150, 150, 0.05, 6), dict(epsilon=0.05, delta=0.1, seed=8)),
    ]


def test_batch_equals_single_runs(kad, ctx):
    mix = _mix()
    Gs = [kad.Graph(ctx, g) for g, _ in mix]
    _say("run_batch of", len(mix), "queries")
    got = kad.run_batch(ctx, Gs, [kw for _, kw in mix])
    for (g, kw), G, a in zip(mix, Gs, got):
        _say("single run", g.name, kw)
        b = kad.run(ctx, G, **kw)
        _same(a, b, g.name)
    for G in Gs:
        G.close()


def test_batch_matches_oracle(kad, ctx):
    import oracle
    oracle.build(force=False)
    mix = _mix()[:4] + _mix()[-1:]
    Gs = [kad.Graph(ctx, g) for g, _ in mix]
    got = kad.run_batch(ctx, Gs, [kw for _, kw in mix])
    for (g, kw), a in zip(mix, got):
        _say("oracle run", g.name, kw)
        b = oracle.run(g, threads=16, **kw)
        assert a["tau"] == b["tau"] and a["stop_reason"] == b["stop_rule"]
        assert a["arcs_scanned"] == b["arcs"]
        assert np.array_equal(a["count"], b["count"])
        assert np.array_equal(a["lower"], b["lower"]) and np.array_equal(a["upper"], b["upper"])
    for G in Gs:
        G.close()


def test_batch_small_launches_and_repeated_graph(kad, ctx):
    """kernel_batch at the check interval forces one interval per query per launch;
    the same graph queried with several seeds shares launches."""
    g = gg.workload("er2000")
    G = kad.Graph(ctx, g)
    kws = [dict(epsilon=0.01, delta=0.1, seed=s, kernel_batch=1024) for s in range(1, 9)]
    got = kad.run_batch(ctx, [G] * len(kws), kws)
    for kw, a in zip(kws, got):
        b = kad.run(ctx, G, **kw)
        _same(a, b, f"seed {kw['seed']}")
    G.close()


def test_batch_graph_family(kad, ctx):
    """Graphs of the many-small-graphs family (half directed, Chung-Lu, 1e3..1e5
    nodes): a 24-graph batch equals the 24 single runs."""
    ids = list(range(24))
    gs = [gg.batch_graph(i) for i in ids]
    Gs = [kad.Graph(ctx, g) for g in gs]
    kws = [dict(epsilon=0.01, delta=0.1, seed=1) for _ in ids]
    _say("family batch", [g.n for g in gs])
    got = kad.run_batch(ctx, Gs, kws)
    for i, G, kw, a in zip(ids, Gs, kws, got):
        b = kad.run(ctx, G, **kw)
        _same(a, b, f"family graph {i}")
    for G in Gs:
        G.close()


def test_server_results_equal_alone(kad, ctx):
    """Queries arrive while others run (continuous batching); each result equals the
    query run alone."""
    mix = _mix()
    Gs = [kad.Graph(ctx, g) for g, _ in mix]
    alone = [kad.run(ctx, G, **kw) for G, (_, kw) in zip(Gs, mix)]
    with kad.Server(ctx) as srv:
        tickets = []
        for j, (G, (_, kw)) in enumerate(zip(Gs, mix)):
            tickets.append(srv.submit(G, **kw))
            time.sleep(0.002 * j)
        # the context belongs to the server meanwhile
        with pytest.raises(kad.KadError) as e:
            kad.run(ctx, Gs[0], epsilon=0.01, delta=0.1)
        assert e.value.status == kad.EBUSY
        res = [srv.wait(t, timeout=120.0) for t in tickets]
        st = srv.stats()
        assert st["completed"] == len(mix) and st["launches"] >= 2
    for (g, _), a, b in zip(mix, res, alone):
        assert a is not None
        _same(a, b, g.name)
    # the context is free again
    r = kad.run(ctx, Gs[0], epsilon=0.01, delta=0.1, seed=1)
    _same(r, alone[0])
    for G in Gs:
        G.close()


def test_server_poll_and_reuse(kad, ctx):
    g = gg.workload("er2000")
    G = kad.Graph(ctx, g)
    b = kad.run(ctx, G, epsilon=0.01, delta=0.1, seed=5)
    with kad.Server(ctx) as srv:
        t = srv.submit(G, epsilon=0.01, delta=0.1, seed=5)
        a = None
        deadline = time.time() + 120
        while a is None and time.time() < deadline:
            a = srv.poll(t)
            time.sleep(0.001)
        _same(a, b)
        # a second wave on the same server
        ts = [srv.submit(G, epsilon=0.01, delta=0.1, seed=5) for _ in range(3)]
        for t2 in ts:
            _same(srv.wait(t2, timeout=120.0), b)
    G.close()


def test_server_cancel(kad, ctx):
    """A long query is canceled; a query submitted afterwards still runs normally."""
    heavy = kad.Graph(ctx, gg.damaged_grid(200, 200, 0.05, 7))
    light_g = gg.workload("er2000")
    light = kad.Graph(ctx, light_g)
    b = kad.run(ctx, light, epsilon=0.01, delta=0.1, seed=3)
    with kad.Server(ctx) as srv:
        t1 = srv.submit(heavy, epsilon=0.004, delta=0.1, seed=1)
        time.sleep(0.5)
        srv.cancel()
        with pytest.raises(kad.KadError) as e:
            srv.wait(t1, timeout=120.0)
        assert e.value.status == -8
        t2 = srv.submit(light, epsilon=0.01, delta=0.1, seed=3)
        _same(srv.wait(t2, timeout=120.0), b)
    heavy.close()
    light.close()


def test_server_cancel_during_compute_delta(kad, ctx):
    """Queries canceled at several moments, some while their computeDelta task (top-k on a
    300K-node graph) runs beside the engine thread: each one either completes with the
    result of its single run or reports KAD_ECANCELED, and the server keeps serving."""
    g = gg.chung_lu(300_000, 2.3, 8.0, 51)
    G = kad.Graph(ctx, g)
    light = kad.Graph(ctx, gg.workload("er2000"))
    kw = [dict(epsilon=0.02, delta=0.1, seed=60 + i, mode="topk", k=10) for i in range(6)]
    ref = [kad.run(ctx, G, **p) for p in kw]
    b = kad.run(ctx, light, epsilon=0.01, delta=0.1, seed=3)
    with kad.Server(ctx) as srv:
        for delay in (0.0, 0.002, 0.005, 0.01, 0.02, 0.05):
            _say("cancel after", delay)
            ts = [srv.submit(G, **p) for p in kw]
            time.sleep(delay)
            srv.cancel()
            for t, r in zip(ts, ref):
                try:
                    _same(srv.wait(t, timeout=120.0), r)
                except kad.KadError as e:
                    assert e.status == -8
        _same(srv.wait(srv.submit(light, epsilon=0.01, delta=0.1, seed=3), timeout=120.0), b)
    G.close()
    light.close()
