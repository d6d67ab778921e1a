"""Multi-limb path counts at the sizes the measurements report, and the two wide passes.

* 2000x2000 damaged grid (every sample needs counts far past 128 bits): sampled paths of
  main-phase ids at the start and deep in the id space, and their hit counts, equal the
  oracle's arbitrary-precision results bit for bit;
* the second wide pass: with first-pass arenas too small for most samples of a
  high-diameter grid, the samples they cannot hold are sampled again by the larger second
  pass and every result still equals the oracle's (no sample is left flagged), in
  kad_sample_paths, kad_hit_counts and whole kad_run calls;
* the wide-arena layout knob and the layout it reports.
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


def _compare_paths(kad, ctx, orc, G, csr, seed, phase, first, count):
    _say("sample_paths", csr.name, "ids", first, count)
    A = kad.sample_paths(ctx, G, seed, phase, first, count)
    B = orc.sample_paths(csr, seed, phase, first, count, threads=16)
    assert (A["flags"] == 0).all(), np.unique(A["flags"])
    assert np.array_equal(A["s"], B.s) and np.array_equal(A["t"], B.t)
    assert np.array_equal(A["arcs"], B.arcs)
    for k in range(count):
        a = A["nodes"][A["path_off"][k]:A["path_off"][k + 1]]
        assert np.array_equal(a, B.path(k)), k
    return A, B


def _hits(n, S, count):
    """Interior hits per node of the oracle's sampled paths."""
    b = np.zeros(n, dtype=np.uint64)
    for k in range(count):
        p = S.path(k)
        b[p[1:-1]] += 1
    return b


def test_grid2000_paths_and_hits(kad, orc):
    g = gg.workload("grid2000")
    ctx = kad.Context(0)
    G = kad.Graph(ctx, g)
    A, B = _compare_paths(kad, ctx, orc, G, g, 1, 1, 0, 40)
    _compare_paths(kad, ctx, orc, G, g, 1, 1, 1 << 20, 10)
    d = np.diff(B.path_off.astype(np.int64)) - 1
    assert d.max() >= 1500  # counts of thousands of bits
    _say("hit_counts grid2000")
    a, arcs = kad.hit_counts(ctx, G, 1, 1, 0, 40)
    assert np.array_equal(a, _hits(g.n, B, 40)) and arcs == int(B.arcs.sum())
    w = ctx.wide_info()
    assert w["slots"] > 64  # more wide workgroups than the earlier fixed cap
    G.close()
    ctx.close()


@pytest.fixture(scope="module")
def small_ctx(kad):
    """First-pass arenas of 2^14 limbs: most samples of a 200x200 grid outgrow them."""
    c = kad.Context(0)
    c.set_wide(64, 1 << 14)
    yield c
    c.close()


def test_second_pass_paths(kad, orc, small_ctx):
    g = gg.damaged_grid(200, 200, 0.05, 7)
    G = kad.Graph(small_ctx, g)
    _compare_paths(kad, small_ctx, orc, G, g, 6, 1, 0, 300)
    w = small_ctx.wide_info()
    assert w["limbs"] == 1 << 14 and w["slots"] == 64
    assert w["slots2"] >= 1 and w["slots2"] * w["limbs2"] <= w["slots"] * w["limbs"]
    G.close()


def test_second_pass_hits_and_run(kad, orc, small_ctx):
    g = gg.damaged_grid(150, 150, 0.05, 3)
    G = kad.Graph(small_ctx, g)
    a, arcs = kad.hit_counts(small_ctx, G, 4, 1, 0, 2000)
    S = orc.sample_paths(g, 4, 1, 0, 2000, threads=16)
    assert np.array_equal(a, _hits(g.n, S, 2000)) and arcs == int(S.arcs.sum())
    for mode in ("graph", "stream"):
        small_ctx.set_exec(mode)
        _say("run", mode)
        r = kad.run(small_ctx, G, epsilon=0.05, delta=0.1, seed=2, kernel_batch=1024)
        o = orc.run(g, 0.05, 0.1, seed=2, threads=16)
        assert r["tau"] == o["tau"] and r["stop_reason"] == o["stop_rule"]
        assert np.array_equal(r["count"], o["count"])
        assert np.array_equal(r["lower"], o["lower"]) and np.array_equal(r["upper"], o["upper"])
    small_ctx.set_exec("graph")
    G.close()


def test_wide_knob_rejects_tiny_arenas(kad, small_ctx):
    with pytest.raises(kad.KadError) as e:
        small_ctx.set_wide(8, 100)
    assert e.value.status == -1
