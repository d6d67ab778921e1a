"""GPU parity with the CPU oracle at the sizes the measurements report.

* the full-size bench call (undirected Chung-Lu, n = 1e6, epsilon 0.005, 65,536 samples per
  launch): tau, stop reason, arcs, counts and bounds bit-equal to the oracle's whole run;
* runs spanning many sampler launches (kernel_batch at or near the check interval), which
  take the per-interval and the batched reductions, the next batch sized from the last
  check, the shortened last interval and a stop at omega;
* the directed top-k workload (n = 4e6, 6e7 arcs): sampled paths of id prefixes at the start
  and near 2^20, and hit counts of 2^16 ids;
* 16 graphs of the many-small-graphs family through the multi-query engine.
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


def _same_run(a, b, what):
    for key in ("tau", "omega", "alpha", "vd"):
        assert a[key] == b[key], (what, key, a[key], b[key])
    assert a["interval"] == b["interval"], what
    assert a["stop_reason"] == b["stop_rule"], what
    assert a["arcs_scanned"] == b["arcs"], what
    assert a["pilot_arcs_scanned"] == b["pilot_arcs"], what
    assert np.array_equal(a["count"], b["count"]), what
    assert np.array_equal(a["bc"], b["bc"]), what
    assert np.array_equal(a["lower"], b["lower"]), what
    assert np.array_equal(a["upper"], b["upper"]), what


def test_run_cl1m_bench_call_equals_oracle(kad, ctx, orc):
    """The exact call bench.py times, against the oracle's whole run."""
    g = gg.workload("cl1m")
    G = kad.Graph(ctx, g)
    _say("cl1m kad_run")
    a = kad.run(ctx, G, epsilon=0.005, delta=0.1, seed=1, kernel_batch=65536)
    _say("cl1m oracle run", a["tau"], a["omega"])
    b = orc.run(g, 0.005, 0.1, seed=1, threads=16)
    _same_run(a, b, "cl1m")
    assert a["stop_reason"] == 1 and a["tau"] > a["interval"] * 16  # several batches
    G.close()


_MULTI = {
    "er2000": lambda: gg.workload("er2000"),
    "cl30k": lambda: gg.chung_lu(30_000, 2.3, 10.0, 31),
    "dcl30k": lambda: gg.chung_lu_directed(30_000, 2.5, 2.1, 8.0, 32),
    "star100": lambda: gg.star_graph(100),
}
_GRAPHS = {}


def _graph(name):
    if name not in _GRAPHS:
        _GRAPHS[name] = _MULTI[name]()
    return _GRAPHS[name]


@pytest.mark.parametrize("name,kw", [
    # one check interval per launch: every interval reduced on its own
    ("er2000", dict(epsilon=0.01, kernel_batch=1024)),
    # two or four intervals per launch: the batched reduction, next batch from the last check
    ("er2000", dict(epsilon=0.01, kernel_batch=2048)),
    ("er2000", dict(epsilon=0.006, kernel_batch=4096, seed=5)),
    ("cl30k", dict(epsilon=0.01, kernel_batch=1024)),
    ("cl30k", dict(epsilon=0.01, kernel_batch=4096, check_interval=1024)),
    ("dcl30k", dict(epsilon=0.01, kernel_batch=2048)),
    ("cl30k", dict(epsilon=0.005, kernel_batch=2048, mode="topk", k=10)),
    # omega reached after 20 (10) launches; the last interval is shortened to omega
    ("star100", dict(epsilon=0.01, kernel_batch=1024)),
    ("star100", dict(epsilon=0.01, kernel_batch=2048)),
])
def test_run_many_launches_equals_oracle(kad, ctx, orc, name, kw):
    g = _graph(name)
    kw = dict(kw)
    kw.setdefault("seed", 2)
    G = kad.Graph(ctx, g)
    _say("multi-launch run", name, kw)
    a = kad.run(ctx, G, delta=0.1, **kw)
    okw = dict(kw)
    okw.pop("kernel_batch")
    b = orc.run(g, delta=0.1, threads=16, **okw)
    _same_run(a, b, f"{name} {kw}")
    assert a["tau"] > kw["kernel_batch"], "the run spans several launches"
    if name == "star100":
        assert a["stop_reason"] == 0 and a["tau"] == a["omega"]
    if kw.get("mode") == "topk":
        rlo, rhi = orc.rank_intervals(b["lower"], b["upper"])
        sel = sorted(np.nonzero(rlo <= kw["k"])[0].tolist(), key=lambda v: (-int(b["count"][v]), v))
        assert a["topk_node"].tolist() == sel
        assert a["rank_lo"].tolist() == [int(rlo[v]) for v in sel]
        assert a["rank_hi"].tolist() == [int(rhi[v]) for v in sel]
    G.close()


@pytest.fixture(scope="module")
def dcl4m():
    _say("generating dcl4m")
    return gg.workload("dcl4m")


@pytest.mark.parametrize("first,count", [(0, 2000), ((1 << 20) - 1000, 1000)])
def test_paths_dcl4m_id_prefixes(kad, ctx, orc, dcl4m, first, count):
    g = dcl4m
    G = kad.Graph(ctx, g)
    _say("dcl4m sample_paths", first, count)
    A = kad.sample_paths(ctx, G, 1, 1, first, count)
    B = orc.sample_paths(g, 1, 1, first, count, threads=16)
    assert (A["flags"] == 0).all(), np.unique(A["flags"])
    assert np.array_equal(A["s"], B.s) and np.array_equal(A["t"], B.t)
    assert np.array_equal(A["arcs"], B.arcs)
    assert np.array_equal(A["path_off"], B.path_off.astype(np.uint64))
    assert np.array_equal(A["nodes"], B.nodes)
    G.close()


def test_hit_counts_dcl4m(kad, ctx, orc, dcl4m):
    g = dcl4m
    G = kad.Graph(ctx, g)
    count = 1 << 16
    _say("dcl4m hit_counts", count)
    a, arcs = kad.hit_counts(ctx, G, 1, 1, 0, count)
    S = orc.sample_paths(g, 1, 1, 0, count, threads=16)
    b = np.zeros(g.n, dtype=np.uint64)
    lens = np.diff(S.path_off.astype(np.int64))
    for k in np.nonzero(lens > 2)[0]:
        p = S.path(k)
        b[p[1:-1]] += 1
    assert np.array_equal(a, b)
    assert arcs == int(S.arcs.sum())
    G.close()


def _family_pick():
    """The 4 smallest and the 4 largest graphs of each direction in the 256-graph family."""
    specs = [(gg.batch_family_spec(i)["n"], i, gg.batch_family_spec(i)["directed"])
             for i in range(256)]
    out = []
    for d in (False, True):
        side = sorted((n, i) for n, i, dd in specs if dd == d)
        out += [i for _, i in side[:4]] + [i for _, i in side[-4:]]
    return sorted(out)


def test_family_batch_equals_oracle(kad, ctx, orc):
    ids = _family_pick()
    assert len(ids) == 16
    gs = [gg.batch_graph(i) for i in ids]
    Gs = [kad.Graph(ctx, g) for g in gs]
    kws = [dict(epsilon=0.01, delta=0.1, seed=1) for _ in ids]
    _say("family batch vs oracle", [g.n for g in gs])
    got = kad.run_batch(ctx, Gs, kws)
    for i, g, kw, a in zip(ids, gs, kws, got):
        b = orc.run(g, threads=16, **kw)
        _same_run(a, b, f"family graph {i} (n={g.n}, directed={g.directed})")
    for G in Gs:
        G.close()
