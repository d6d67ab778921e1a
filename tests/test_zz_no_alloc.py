"""The entry point that allocates nothing (kad_hit_counts_noalloc) against kad_hit_counts.

Two calls in a row through the C ABI, the second on a smaller input, each compared bit for
bit with the allocating entry point on the same samples; then the rejections: a graph whose
path counts may pass 128 bits.
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


def _noalloc(kad, ctx, G, n, seed, phase, first, count, side_stream=True):
    """The call only enqueues: on a side stream (then waited for), or on the null stream
    (stream=None; then the device is synchronised)."""
    import torch
    cnt = torch.zeros(n, dtype=torch.int64, device="cuda")
    arcs = torch.zeros(1, dtype=torch.int64, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()  # the zeros are written before another stream reads them
    if side_stream:
        s = torch.cuda.Stream()
        kad.hit_counts_noalloc(ctx, G, seed, phase, first, count, cnt, arcs, flags, stream=s)
        s.synchronize()
    else:
        kad.hit_counts_noalloc(ctx, G, seed, phase, first, count, cnt, arcs, flags, stream=None)
        torch.cuda.synchronize()
    return (cnt.cpu().numpy().view(np.uint64), int(arcs.cpu().numpy()[0]),
            int(flags.cpu().numpy()[0]))


def test_noalloc_equals_hit_counts_two_calls(kad):
    with kad.Context(0) as ctx:
        cases = [(gg.workload("er2000"), 4, 1, 100, 20000),      # first call
                 (gg.gnp(300, 0.02, 5, True), 9, 0, 7, 3000)]     # second call, smaller input
        graphs = [kad.Graph(ctx, g) for g, *_ in cases]
        got = []
        for j, ((g, seed, phase, first, count), G) in enumerate(zip(cases, graphs)):
            _say("noalloc", g.name, seed, phase, first, count)
            got.append(_noalloc(kad, ctx, G, g.n, seed, phase, first, count, side_stream=j == 0))
        for (g, seed, phase, first, count), G, (c, arcs, flags) in zip(cases, graphs, got):
            _say("hit_counts", g.name)
            ref, ref_arcs = kad.hit_counts(ctx, G, seed, phase, first, count)
            assert flags == 0
            assert np.array_equal(c, ref), g.name
            assert arcs == ref_arcs, g.name
        # a larger input again after the smaller one: the scratch is cleared as needed
        g, seed, phase, first, count = cases[0]
        c, arcs, flags = _noalloc(kad, ctx, graphs[0], g.n, seed + 1, phase, first, count // 4)
        ref, ref_arcs = kad.hit_counts(ctx, graphs[0], seed + 1, phase, first, count // 4)
        assert flags == 0 and np.array_equal(c, ref) and arcs == ref_arcs
        for G in graphs:
            G.close()


def test_noalloc_many_candidate_edges(kad):
    """Samples whose candidate edges outgrow the scratch's per-slot buffer (4,096 entries;
    pairs of feeder nodes of the hub gadget meet through ~300K) are sampled again in the
    scratch's wide-count slot; the counts still equal kad_hit_counts'."""
    with kad.Context(0) as ctx:
        g = gg.hub_layers()
        G = kad.Graph(ctx, g)
        c, arcs, flags = _noalloc(kad, ctx, G, g.n, 5, 1, 0, 600)
        ref, ref_arcs = kad.hit_counts(ctx, G, 5, 1, 0, 600)
        assert flags == 0 and np.array_equal(c, ref) and arcs == ref_arcs
        G.close()


def test_noalloc_rejects_wide_count_graphs(kad):
    with kad.Context(0) as ctx:
        g = gg.damaged_grid(200, 200, 0.05, 7)   # vertex diameter above 256: wide counts
        G = kad.Graph(ctx, g)
        with pytest.raises(kad.KadError) as e:
            _noalloc(kad, ctx, G, g.n, 1, 1, 0, 100)
        assert e.value.status == -1
        G.close()
