"""CPU checks of the C-ABI library: it loads, exports every declared symbol, and its
host-side binary64 statistics agree with the oracle (no device calls)."""
import ctypes
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

import graphgen as gg

kad = pytest.importorskip("paper_1604_08553_amd")


@pytest.fixture(scope="module")
def klib():
    if not os.path.exists(kad.library_path()):
        pytest.fail("libkadabra.so is not built (python -m paper_1604_08553_amd.build)")
    return kad.lib()


def test_exports_every_declared_symbol(klib):
    syms = kad.declared_symbols()
    assert len(syms) >= 19
    handle = ctypes.CDLL(kad.library_path())
    for name in syms:
        assert hasattr(handle, name), name


def test_no_device_gives_clean_error(klib):
    # CPU container: creating a context must fail with a status, never abort
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        pytest.skip("a GPU is present")
    with pytest.raises(kad.KadError) as e:
        kad.Context(0)
    assert e.value.status == -3


def test_schedule_matches_oracle(klib, oracle_lib):
    for lam in (0.03, 0.01, 0.005, 0.002, 0.0002):
        for delta in (0.1, 0.05, 0.2):
            for vd in (1, 2, 3, 4, 5, 8, 11, 30, 1000, 5000):
                om = kad.omega(lam, delta, vd)
                assert om == oracle_lib.omega(lam, delta, vd)
                assert kad.alpha(om) == oracle_lib.alpha(om)
                assert kad.default_interval(om) == oracle_lib.default_interval(om)


def _graphs():
    out = [gg.path_graph(9), gg.star_graph(7), gg.cycle_graph(8, True), gg.grid(6, 9),
           gg.complete_bipartite(3, 4), gg.disjoint_union(gg.path_graph(5), gg.cycle_graph(4, True)),
           gg.workload("er2000"), gg.chung_lu(3000, 2.3, 6.0, 7),
           gg.chung_lu_directed(3000, 2.5, 2.1, 5.0, 8)]
    for seed in range(8):
        out.append(gg.gnp(40, 0.06, seed))
        out.append(gg.gnp(40, 0.05, seed, directed=True))
    return out


def _cycle_chains():
    """Directed graphs of several strongly connected components in chains, where the node
    of largest degree sits in a single-node component, in a small one between a larger
    upstream and a downstream one, or in a DAG, and random chains of cycles with a hub."""
    out = []
    # hub 0 points at every node of two cycles, A (1..5) and B (6..12), and A -> B
    src = [0] * 12 + list(range(1, 6)) + list(range(6, 13)) + [3]
    dst = list(range(1, 13)) + [2, 3, 4, 5, 1] + [7, 8, 9, 10, 11, 12, 6] + [9]
    out.append(gg.csr_from_edges(13, src, dst, True, "hub_into_cycles"))
    # cycle U (0..19) -> two-node hub {20, 21} with many arcs -> cycle D (22..29)
    src = list(range(20)) + list(range(20)) + [20, 21] + [20] * 8 + list(range(22, 30))
    dst = [(i + 1) % 20 for i in range(20)] + [20 + (i % 2) for i in range(20)] + [21, 20] \
        + list(range(22, 30)) + [22 + (i + 1) % 8 for i in range(8)]
    out.append(gg.csr_from_edges(30, src, dst, True, "cycle_hub_cycle"))
    rng = np.random.default_rng(5)
    n = 60
    u, v = rng.integers(0, n, 300), rng.integers(0, n, 300)
    out.append(gg.csr_from_edges(n, np.minimum(u, v), np.maximum(u, v), True, "dag60"))
    for seed in range(6):
        rng = np.random.default_rng(100 + seed)
        sizes = rng.integers(1, 9, 12)
        start = np.concatenate([[0], np.cumsum(sizes)])
        n = int(start[-1]) + 1
        hub = int(rng.integers(0, n))
        src, dst = [], []
        for b in range(len(sizes)):
            members = np.arange(start[b], start[b + 1])
            src += list(members)
            dst += list(np.roll(members, -1))
        for _ in range(40):  # arcs between blocks, lower block to higher
            a, b = sorted(rng.choice(len(sizes), 2, replace=False))
            src.append(int(rng.integers(start[a], start[a + 1])))
            dst.append(int(rng.integers(start[b], start[b + 1])))
        others = [x for x in range(n) if x != hub]
        for x in rng.choice(others, 25, replace=False):  # hub degree above every other
            if rng.random() < 0.5:
                src.append(hub); dst.append(int(x))
            else:
                src.append(int(x)); dst.append(hub)
        out.append(gg.csr_from_edges(n, src, dst, True, f"cycle_chain{seed}"))
    return out


def test_vertex_diameter_matches_oracle(klib, oracle_lib):
    for g in _graphs() + _cycle_chains():
        for limit in (1e9, 0.0):
            assert kad.vertex_diameter(g, limit) == oracle_lib.vertex_diameter(g, limit), (g.name, limit)
    # levels of thousands of nodes: the bound's BFS runs them on several threads
    for g in (gg.chung_lu(200_000, 2.3, 8.0, 11), gg.damaged_grid(300, 300, 0.05, 2),
              gg.chung_lu_directed(200_000, 2.5, 2.1, 8.0, 12)):
        assert kad.vertex_diameter(g, 0.0) == oracle_lib.vertex_diameter(g, 0.0), g.name


def test_f_g_bitwise_equal_to_oracle(klib, oracle_lib):
    rng = np.random.default_rng(1)
    for _ in range(5000):
        om = float(rng.integers(1000, 10**8))
        tau = float(rng.integers(1, int(om) + 1))
        L = float(np.exp(rng.uniform(-1, 5)))
        b = float(rng.integers(0, int(tau) + 1)) / tau
        assert kad.bound_f(b, L, om, tau) == oracle_lib.f(b, L, om, tau)
        assert kad.bound_g(b, L, om, tau) == oracle_lib.g(b, L, om, tau)


def _pilot(n, alpha, seed, zero_frac=0.3):
    rng = np.random.default_rng(seed)
    c = rng.poisson(rng.exponential(1.5, n)).astype(np.uint64)
    c[rng.random(n) < zero_frac] = 0
    return np.minimum(c, alpha).astype(np.uint64)


def test_compute_delta_matches_oracle(klib, oracle_lib):
    for seed, n in enumerate((10, 1000, 20000)):
        alpha, om = 299, 29979
        c0 = _pilot(n, alpha, seed)
        lam = np.full(n, 0.01)
        a = kad.compute_delta(c0, alpha, om, lam, lam, 0.1, 0.001)
        b = oracle_lib.compute_delta(c0, alpha, om, lam, lam, 0.1, 0.001)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
        ll, lu = oracle_lib.topk_lambdas(c0, 5, alpha, 0.002)
        a = kad.compute_delta(c0, alpha, om, ll, lu, 0.1, 0.001)
        b = oracle_lib.compute_delta(c0, alpha, om, ll, lu, 0.1, 0.001)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_compute_delta_matches_oracle_large(klib, oracle_lib):
    """At 300,000 nodes, where the uniform path builds its count histogram and writes the
    per-node values over ranges on the worker threads: bit for bit with the oracle, for
    uniform half-widths and for the top-k ones (the per-node path)."""
    n, alpha, om = 300_000, 2999, 299_790
    c0 = _pilot(n, alpha, 11)
    lam = np.full(n, 0.004)
    a = kad.compute_delta(c0, alpha, om, lam, lam, 0.1, 0.001)
    b = oracle_lib.compute_delta(c0, alpha, om, lam, lam, 0.1, 0.001)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    ll, lu = oracle_lib.topk_lambdas(c0, 20, alpha, 0.002)
    a = kad.compute_delta(c0, alpha, om, ll, lu, 0.1, 0.001)
    b = oracle_lib.compute_delta(c0, alpha, om, ll, lu, 0.1, 0.001)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_compute_delta_hist_matches_oracle(klib, oracle_lib):
    """The all-nodes run solves computeDelta from the histogram of the pilot counts; the
    L value of each node (through its count's group) and C equal the oracle's per-node
    computeDelta bit for bit."""
    for seed, n in enumerate((10, 1000, 20000, 50000)):
        alpha, om = 299 + 40 * seed, 29979 + 1000 * seed
        c0 = _pilot(n, alpha, 50 + seed)
        lam = 0.004 + 0.003 * seed
        hist = np.bincount(c0.astype(np.int64), minlength=alpha + 1).astype(np.uint64)
        gof, gll, glu, cv = kad.compute_delta_hist(hist, alpha, om, lam, lam, 0.1, 0.001)
        b = oracle_lib.compute_delta(c0, alpha, om, np.full(n, lam), np.full(n, lam), 0.1, 0.001)
        g = gof[c0.astype(np.int64)]
        assert np.array_equal(gll[g], b[0]) and np.array_equal(glu[g], b[1]) and cv == b[2]
        # one group per count present, in ascending order of the count
        present = np.nonzero(hist)[0]
        assert np.array_equal(gof[present], np.arange(present.size))


def test_topk_lambdas_match_oracle(klib, oracle_lib):
    for seed in range(6):
        n = 500
        c0 = _pilot(n, 300, seed, zero_frac=0.1)
        for k in (1, 3, 10, n):
            for lam in (0.0005, 0.002, 0.05):
                a = kad.topk_lambdas(c0, k, 300, lam)
                b = oracle_lib.topk_lambdas(c0, k, 300, lam)
                assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), (seed, k, lam)


def test_topk_lambdas_match_oracle_large(klib, oracle_lib):
    """At 200,000 nodes the library finds only the k+1 largest pilot counts (per range on
    the worker threads) and writes every other node's half-widths from its own count; the
    oracle orders all nodes.  Small pilot counts tie at the boundary of the k+1 largest."""
    n, alpha = 200_000, 300
    for seed in range(2):
        c0 = _pilot(n, alpha, 70 + seed, zero_frac=0.3)
        for k in (1, 10, 100, 30_000):  # the last takes the full order
            for lam in (0.0005, 0.002, 0.05):
                a = kad.topk_lambdas(c0, k, alpha, lam)
                b = oracle_lib.topk_lambdas(c0, k, alpha, lam)
                assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), (seed, k, lam)


def test_grouped_stop_check_equals_plain_oracle(klib, oracle_lib):
    """The library groups nodes by (L_l, L_u) and tests only each group's largest count;
    the oracle tests every node.  Sweep tau across the decision boundary."""
    rng = np.random.default_rng(3)
    n, alpha, om = 3000, 300, 40000
    decisions = 0
    for trial in range(6):
        c0 = _pilot(n, alpha, 100 + trial)
        lam = 0.01 if trial % 2 == 0 else 0.004
        for mode, k in (("all", 0), ("topk", 1), ("topk", 7)):
            if mode == "topk":
                ll, lu = oracle_lib.topk_lambdas(c0, k, alpha, lam)
            else:
                ll = lu = np.full(n, lam)
            Ll, Lu, _ = oracle_lib.compute_delta(c0, alpha, om, ll, lu, 0.1)
            p = (c0.astype(np.float64) + 0.5) / (alpha + 1)
            for tau in np.unique(np.geomspace(1000, om, 14).astype(np.int64)):
                cnt = rng.binomial(int(tau), np.minimum(p, 1.0)).astype(np.uint64)
                a = kad.have_to_stop(cnt, int(tau), om, lam, Ll, Lu, mode=mode, k=k)
                if mode == "topk":
                    b = oracle_lib.stop_topk(cnt, k, int(tau), om, lam, Ll, Lu)
                else:
                    b = oracle_lib.stop_all(cnt, int(tau), om, lam, Ll, Lu)
                assert a == b, (trial, mode, k, tau)
                decisions += a
    assert decisions > 0


def test_grouped_stop_check_equals_plain_oracle_large(klib, oracle_lib):
    """The same at 200,000 nodes, where the check's node loops run in ranges on the
    worker threads (candidates gathered in id order, group maxima merged, the first
    check's k+1 largest chosen per range), with k small and large (many tied counts at
    the boundary of the k+1 largest)."""
    rng = np.random.default_rng(4)
    n, alpha, om = 200_000, 2000, 300_000
    decisions = 0
    for trial in range(2):
        c0 = _pilot(n, alpha, 200 + trial)
        lam = 0.004 if trial == 0 else 0.002
        for mode, k in (("all", 0), ("topk", 5), ("topk", 60)):
            if mode == "topk":
                ll, lu = oracle_lib.topk_lambdas(c0, k, alpha, lam)
            else:
                ll = lu = np.full(n, lam)
            Ll, Lu, _ = oracle_lib.compute_delta(c0, alpha, om, ll, lu, 0.1)
            p = (c0.astype(np.float64) + 0.5) / (alpha + 1)
            for tau in np.unique(np.geomspace(5000, om, 6).astype(np.int64)):
                cnt = rng.binomial(int(tau), np.minimum(p, 1.0)).astype(np.uint64)
                a = kad.have_to_stop(cnt, int(tau), om, lam, Ll, Lu, mode=mode, k=k)
                if mode == "topk":
                    b = oracle_lib.stop_topk(cnt, k, int(tau), om, lam, Ll, Lu)
                else:
                    b = oracle_lib.stop_all(cnt, int(tau), om, lam, Ll, Lu)
                assert a == b, (trial, mode, k, tau)
                decisions += a
    assert decisions > 0
    # five heavy nodes far apart: the top-k rule stops on their separation while other
    # nodes are still unconverged, so the decision rests on which nodes form the top k
    om = 3_000_000
    separated = 0
    for seed in range(2):
        rng = np.random.default_rng(50 + seed)
        c0 = _pilot(n, alpha, 300 + seed)
        heavy = rng.choice(n, 5, replace=False)
        ph = np.array([0.30, 0.24, 0.18, 0.13, 0.09])
        c0[heavy] = (ph * alpha).astype(np.uint64)
        lam = 0.005
        ll, lu = oracle_lib.topk_lambdas(c0, 5, alpha, lam)
        Ll, Lu, _ = oracle_lib.compute_delta(c0, alpha, om, ll, lu, 0.1)
        p = (c0.astype(np.float64) + 0.5) / (alpha + 1)
        p[heavy] = ph
        for tau in np.unique(np.geomspace(2000, om, 12).astype(np.int64)):
            cnt = rng.binomial(int(tau), np.minimum(p, 1.0)).astype(np.uint64)
            a = kad.have_to_stop(cnt, int(tau), om, lam, Ll, Lu, mode="topk", k=5)
            assert a == oracle_lib.stop_topk(cnt, 5, int(tau), om, lam, Ll, Lu), (seed, tau)
            separated += a and not oracle_lib.stop_all(cnt, int(tau), om, lam, Ll, Lu)
    assert separated > 0


def test_fixed_schedule_sample_counts(klib):
    """RK: the printed RK iteration counts of the appendix tables (delta = 0.1) are
    c/eps^2 (floor(log2(VD-2)) + 1 + ln(1/delta)) for some vertex diameter; Hoeffding:
    the smallest k with 2n exp(-2 k eps^2) <= delta."""
    import math
    golden = os.path.join(os.path.dirname(__file__), "golden", "appF_iterations.txt")
    rows = [l.split() for l in open(golden) if l.strip() and not l.startswith("#")]
    assert len(rows) == 180
    for kind, lam, _kad, rk in rows:
        lam, rk = float(lam), int(rk)
        assert any(kad.fixed_samples("rk", lam, 0.1, 2 ** j + 2, 1000) == rk for j in range(0, 40)), rk
    for n, eps, delta in [(1000, 0.01, 0.1), (2 ** 20, 0.005, 0.05), (7, 0.3, 0.5)]:
        k = kad.fixed_samples("hoeffding", eps, delta, 10, n)
        assert 2 * n * math.exp(-2 * k * eps * eps) <= delta
        assert 2 * n * math.exp(-2 * (k - 1) * eps * eps) > delta
    assert kad.fixed_samples("adaptive", 0.01, 0.1, 8, 100) == 0


def _bounds(n, seed, zero_frac=0.05, wide_frac=0.02):
    """Intervals like a run's: counts with many ties, bounds around count/tau, some of zero
    width and some very wide."""
    rng = np.random.default_rng(seed)
    count = rng.geometric(0.05, n).astype(np.uint64) - 1
    tau = 5000.0
    b = count / tau
    w = rng.uniform(0.0, 0.004, n)
    w[rng.random(n) < zero_frac] = 0.0
    w[rng.random(n) < wide_frac] *= 50
    lo = b - w * rng.uniform(0.5, 1.5, n)
    hi = b + w * rng.uniform(0.5, 1.5, n)
    return count, lo, hi


def test_topk_select_matches_oracle_rank_intervals(klib, oracle_lib):
    """kad_topk_select (which sorts only the bounds near the top) against the definition:
    every node's rank interval from the oracle, the nodes with rank_lo <= k, by count
    descending then id."""
    for seed in range(8):
        for n in (1, 2, 50, 3000):
            count, lo, hi = _bounds(n, seed)
            rlo, rhi = oracle_lib.rank_intervals(lo, hi)
            for k in sorted({1, 2, 10, 100, n}):
                if k > n:
                    continue
                want = sorted(np.nonzero(rlo <= k)[0].tolist(), key=lambda v: (-int(count[v]), v))
                node, a_lo, a_hi = kad.topk_select(count, lo, hi, k)
                assert node.tolist() == want, (seed, n, k)
                assert a_lo.tolist() == [int(rlo[v]) for v in want], (seed, n, k)
                assert a_hi.tolist() == [int(rhi[v]) for v in want], (seed, n, k)


def test_topk_select_large_against_definition(klib):
    """At 300,000 nodes, where the selection, the rank searches and the sort of the upper
    bounds run on the worker threads: against the definition written with numpy sorts
    (rank_lo = 1 + #{w != v: lo(w) >= hi(v)}, rank_hi = #{w: hi(w) > lo(v)}), including
    bounds loose enough that every node is selected."""
    n = 300_000
    for seed, (loose, k) in enumerate(((False, 10), (False, 100), (True, 100))):
        count, lo, hi = _bounds(n, 40 + seed)
        if loose:  # every interval reaches the top k
            lo, hi = lo - 1.0, hi + 1.0
        lo_sorted, hi_sorted = np.sort(lo), np.sort(hi)
        rlo = 1 + (n - np.searchsorted(lo_sorted, hi, side="left")) - (lo >= hi)
        rhi = n - np.searchsorted(hi_sorted, lo, side="right")
        sel = np.nonzero(rlo <= k)[0]
        want = sel[np.lexsort((sel, -count[sel].astype(np.int64)))]
        node, a_lo, a_hi = kad.topk_select(count, lo, hi, k)
        assert np.array_equal(node, want), (seed, len(node), len(want))
        assert np.array_equal(a_lo, rlo[want]) and np.array_equal(a_hi, rhi[want]), seed
        if loose:
            assert len(node) == n


def test_topk_select_rejects_bad_k(klib):
    count, lo, hi = _bounds(10, 0)
    for k in (0, 11):
        with pytest.raises(kad.KadError):
            kad.topk_select(count, lo, hi, k)


def test_host_memory_exhaustion_is_a_status(klib):
    """A host allocation that fails inside the library comes back as KAD_ENOMEM: the call
    returns, the process lives on, and the same call succeeds once memory is there again.
    A child process caps its own address space just above what it uses, then asks for the
    vertex-diameter bound of a 3M-node directed cycle (vectors of 12 MB each)."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = textwrap.dedent(f"""
        import resource, sys
        import numpy as np
        sys.path.insert(0, {root!r})
        import paper_1604_08553_amd as kad
        kad.lib()
        n = 3_000_000

        class Cycle:
            pass
        g = Cycle()
        g.n, g.directed = n, True
        g.row = np.arange(n + 1, dtype=np.uint32)
        g.col = ((np.arange(n) + 1) % n).astype(np.uint32)
        g.rrow = g.row
        g.rcol = ((np.arange(n) + n - 1) % n).astype(np.uint32)
        want = kad.vertex_diameter(g, 0.0)

        def vm_bytes():
            for line in open("/proc/self/status"):
                if line.startswith("VmSize:"):
                    return int(line.split()[1]) * 1024
        soft, hard = resource.getrlimit(resource.RLIMIT_AS)
        resource.setrlimit(resource.RLIMIT_AS, (vm_bytes() + (4 << 20), hard))
        try:
            kad.vertex_diameter(g, 0.0)
            print("NO ERROR")
        except kad.KadError as e:
            print("STATUS", e.status, e)
        resource.setrlimit(resource.RLIMIT_AS, (soft, hard))
        print("AGAIN", kad.vertex_diameter(g, 0.0) == want, want)
    """)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "STATUS -2 out of memory" in r.stdout, r.stdout + r.stderr
    assert "AGAIN True" in r.stdout, r.stdout


def test_vertex_diameter_rejects_malformed_rows(klib):
    """The host bound checks its CSR as graph registration does (rows on worker threads,
    the first bad node reported) instead of reading out of bounds: heads out of range,
    self-loops, rows not ascending, row pointers that decrease or pass the arc count."""
    g = gg.chung_lu_directed(300_000, 2.5, 2.1, 5.0, 9)  # several worker ranges
    n, row, col = g.n, g.row.astype(np.int64), g.col.astype(np.int64)
    deg = np.diff(row)
    v = int(np.flatnonzero(deg >= 3)[len(np.flatnonzero(deg >= 3)) // 2])
    e = int(row[v])

    class G:
        directed = True

    def call(r, c, rr=g.rrow, rc=g.rcol):
        h = G()
        h.n, h.row, h.col, h.rrow, h.rcol = n, r, c, rr, rc
        return kad.vertex_diameter(h, 0.0)

    def rejects(text, *a):
        with pytest.raises(kad.KadError) as err:
            call(*a)
        assert err.value.status == -1 and text in str(err.value), str(err.value)

    assert call(row, col) == kad.vertex_diameter(g, 0.0)
    c = col.copy(); c[e + 1] = n + 5; c[-1] = n + 9  # two bad heads: the first is reported
    rejects(f"out-rows: node {v} has out-of-range neighbour {n + 5}", row, c)
    c = col.copy(); c[e + 1], c[e + 2] = col[e + 2], col[e + 1]
    rejects(f"out-rows: row {v} is not strictly ascending", row, c)
    first_head = np.where(deg > 0, col[np.minimum(row[:-1], len(col) - 1)], -1)
    w = int(np.flatnonzero(first_head > np.arange(n))[0])
    c = col.copy(); c[row[w]] = w
    rejects(f"out-rows: self-loop at node {w}", row, c)
    r = row.copy(); r[v + 1] = r[v] - 1
    rejects(f"out-rows: row_ptr decreases at node {v}", r, col)
    r = row.copy(); r[v + 1] = len(col) + 100  # above the arcs, then back down
    rejects(f"out-rows: row_ptr[{v + 1}] passes the arc count", r, col)
    rc = g.rcol.astype(np.int64); rc[5] = n
    rejects("in-rows: node", row, col, g.rrow, rc)
