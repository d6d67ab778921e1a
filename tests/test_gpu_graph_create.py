"""Graph registration (kad_graph_create): canonical CSR graphs are accepted, the rest are
rejected with KAD_EINVAL on the host before any device work, and the message names the
first bad node.

The library checks the rows on its worker threads and builds the in-rows of a directed
graph (or the transpose that proves an undirected one symmetric) by a parallel counting
pass; given in-rows are compared with that transpose, so accepting correct in-rows and
rejecting altered ones checks the transpose itself.  Sizes span one to many worker chunks.
A row pointer above the arc count that falls back later is rejected without reading past
the heads."""
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


def _register(kad, ctx, n, row, col, directed, rrow=None, rcol=None):
    assert len(row) == n + 1  # the library reads n + 1 row pointers
    return kad.Graph(ctx, n=n, row=np.asarray(row, np.uint32), col=np.asarray(col, np.uint32),
                     directed=directed, rrow=None if rrow is None else np.asarray(rrow, np.uint32),
                     rcol=None if rcol is None else np.asarray(rcol, np.uint32))


def _rejects(kad, ctx, text, *args, **kw):
    with pytest.raises(kad.KadError) as e:
        _register(kad, ctx, *args, **kw)
    assert e.value.status == -1, str(e.value)
    assert text in str(e.value), str(e.value)


_ACCEPT = {
    "path9": lambda: gg.path_graph(9),
    "cl3k": lambda: gg.chung_lu(3000, 2.3, 6.0, 7),
    "cl200k": lambda: gg.chung_lu(200_000, 2.3, 8.0, 11),
    "dcl3k": lambda: gg.chung_lu_directed(3000, 2.5, 2.1, 5.0, 8),
    "dcl120k": lambda: gg.chung_lu_directed(120_000, 2.5, 2.1, 8.0, 12),
}


@pytest.mark.parametrize("name", list(_ACCEPT))
def test_accepts_canonical_graphs(kad, ctx, name):
    g = _ACCEPT[name]()
    _say("register", name, g.n)
    G = _register(kad, ctx, g.n, g.row, g.col, g.directed)
    G.close()
    if g.directed:  # the caller's in-rows, compared with the library's transpose
        G = _register(kad, ctx, g.n, g.row, g.col, True, g.rrow, g.rcol)
        G.close()


def test_rejects_bad_rows(kad, ctx):
    g = gg.chung_lu_directed(20_000, 2.5, 2.1, 6.0, 3)
    n, row, col = g.n, g.row.astype(np.int64), g.col.astype(np.int64)
    deg = np.diff(row)
    v = int(np.flatnonzero(deg >= 3)[len(np.flatnonzero(deg >= 3)) // 2])  # a node in the middle
    e = int(row[v])
    _say("bad rows at node", v)

    c = col.copy(); c[e + 1] = n + 5
    _rejects(kad, ctx, f"node {v} has out-of-range neighbour {n + 5}", n, row, c, True)
    c = col.copy(); c[e + 1], c[e + 2] = col[e + 2], col[e + 1]
    _rejects(kad, ctx, f"row {v} is not strictly ascending", n, row, c, True)
    c = col.copy(); c[e + 1] = c[e]
    _rejects(kad, ctx, f"row {v} is not strictly ascending", n, row, c, True)
    # a self-loop that keeps the row ascending: w's first head replaced by w itself
    first_head = np.where(deg > 0, col[np.minimum(row[:-1], len(col) - 1)], -1)
    w = int(np.flatnonzero(first_head > np.arange(n))[0])
    c = col.copy(); c[row[w]] = w
    _rejects(kad, ctx, f"self-loop at node {w}", n, row, c, True)
    # the first bad node is reported when there are several
    c = col.copy(); c[e + 1] = n + 5; c[-1] = n + 9
    _rejects(kad, ctx, f"node {v} has out-of-range neighbour", n, row, c, True)

    r = row.copy(); r[v + 1] = r[v] - 1
    _rejects(kad, ctx, f"row_ptr decreases at node {v}", n, r, col, True)
    r = row.copy(); r[v + 1] = len(col) + 100  # above the arcs, then back down
    _rejects(kad, ctx, f"row_ptr[{v + 1}] passes the arc count", n, r, col, True)
    r = row.copy(); r[-1] = len(col) - 1
    _rejects(kad, ctx, "row_ptr[0] must be 0", n, r, col, True)


def test_rejects_asymmetric_and_wrong_in_rows(kad, ctx):
    g = gg.chung_lu_directed(20_000, 2.5, 2.1, 6.0, 4)
    _say("asymmetric as undirected")
    _rejects(kad, ctx, "undirected graph is not symmetric", g.n, g.row, g.col, False)
    rc = g.rcol.astype(np.int64)
    x = int(np.flatnonzero(np.diff(g.rrow.astype(np.int64)) >= 2)[0])
    lo = int(g.rrow[x])
    rc[lo], rc[lo + 1] = rc[lo + 1], rc[lo]
    _say("in-rows altered at node", x)
    _rejects(kad, ctx, "in-rows are not the transpose of the out-rows", g.n, g.row, g.col, True,
             g.rrow, rc)
