"""Pins of the CPU oracle against things other than itself.

Each test ties one oracle function to an independent authority: numpy's Philox
implementation, Python integers, networkx shortest paths and betweenness,
closed-form betweenness of textbook graphs, the numbers printed in the paper's
appendix tables, the quadratic identities f and g are derived from, and
exact/statistical properties of the sampling distribution.
"""
import math
import os

import numpy as np
import pytest

import graphgen as gg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------- Philox


def _numpy_block(seed, ctr):
    """Philox4x64-10 block at counter ``ctr`` from numpy's implementation.

    numpy advances its 256-bit counter before producing a block, so the block at
    counter c is numpy's first output after seeding the counter with c - 1.
    """
    c = sum(int(w) << (64 * j) for j, w in enumerate(ctr)) - 1
    c %= 1 << 256
    words = np.array([(c >> (64 * j)) & (2**64 - 1) for j in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64), counter=words)
    return [int(x) for x in bg.random_raw(4)]


def test_philox_matches_numpy(oracle_lib):
    rng = np.random.default_rng(5)
    cases = [([1, 0, 0, 0], 1), ([0, 0, 0, 0], 0), ([2**64 - 1, 7, 3, 1], 2**64 - 1)]
    for _ in range(40):
        ctr = [int(x) for x in rng.integers(0, 2**64, size=4, dtype=np.uint64)]
        cases.append((ctr, int(rng.integers(0, 2**64, dtype=np.uint64))))
    for ctr, seed in cases:
        assert oracle_lib.philox(ctr, [seed, 0]) == _numpy_block(seed, ctr), (ctr, seed)


def _ref_uniform_below(bound, seed, i, phase, purpose, step):
    if bound == 1:
        return 0
    W = (bound - 1).bit_length()
    q = (W + 63) // 64
    sword = (phase << 56) | (purpose << 48) | step
    for attempt in range(64):
        words = []
        for blk in range((q + 3) // 4):
            words += _numpy_block(seed, [i, sword, attempt, blk])
        x = sum(words[j] << (64 * j) for j in range(q)) & ((1 << W) - 1)
        if x < bound:
            return x
    raise AssertionError("unreachable")


def test_uniform_below_words_and_masking(oracle_lib):
    rng = np.random.default_rng(11)
    bounds = [1, 2, 3, 5, 1000, 2**63, 2**64 - 1, 2**64, 2**64 + 1, 2**128 - 1, 2**128,
              2**128 + 12345, 3**200, 2**255, 2**256 + 1]
    for bits in (7, 70, 130, 257, 600, 1500, 4096):
        for _ in range(3):
            bounds.append(int.from_bytes(rng.bytes((bits + 7) // 8), "little") % (1 << bits) + 1)
    for j, b in enumerate(bounds):
        for (i, phase, purpose, step) in [(0, 0, 0, 0), (j, 1, 2, 0), (2**40 + j, 1, 3, 17)]:
            got = oracle_lib.uniform_below(b, 77, i, phase, purpose, step)
            assert 0 <= got < b
            assert got == _ref_uniform_below(b, 77, i, phase, purpose, step), (b, i)


def test_uniform_below_is_uniform(oracle_lib):
    from scipy.stats import chisquare
    bound = 6
    draws = [oracle_lib.uniform_below(bound, 3, i, 1, 2, 0) for i in range(30000)]
    obs = np.bincount(draws, minlength=bound)
    assert chisquare(obs).pvalue > 1e-4


# ----------------------------------------------------------------------------- path counts and paths


def _nx(g):
    import networkx as nx
    G = nx.DiGraph() if g.directed else nx.Graph()
    G.add_nodes_from(range(g.n))
    s, d = g.edges()
    G.add_edges_from(zip(s.tolist(), d.tolist()))
    return G


def _small_graphs():
    out = []
    for seed in range(6):
        out.append(gg.gnp(11, 0.28, seed, directed=False))
        out.append(gg.gnp(10, 0.22, seed, directed=True))
    out += [gg.grid(3, 4), gg.complete_bipartite(2, 3), gg.cycle_graph(7, True),
            gg.disjoint_union(gg.path_graph(4), gg.star_graph(4))]
    return out


def test_sigma_st_matches_networkx(oracle_lib):
    import networkx as nx
    for g in _small_graphs():
        G = _nx(g)
        for s in range(g.n):
            for t in range(g.n):
                if s == t:
                    continue
                d, sig = oracle_lib.sigma_st(g, s, t)
                if nx.has_path(G, s, t):
                    assert d == nx.shortest_path_length(G, s, t)
                    assert sig == len(list(nx.all_shortest_paths(G, s, t)))
                else:
                    assert d == -1


def test_sigma_grid_binomial_beyond_128_bits(oracle_lib):
    g = gg.grid(80, 80)
    for (r, c) in [(79, 79), (40, 79), (79, 3), (70, 75)]:
        d, sig = oracle_lib.sigma_st(g, 0, r * 80 + c)
        assert d == r + c
        assert sig == math.comb(r + c, r)
    assert math.comb(158, 79).bit_length() > 128


def test_sampled_paths_are_shortest_paths(oracle_lib):
    import networkx as nx
    for g in _small_graphs():
        G = _nx(g)
        S = oracle_lib.sample_paths(g, 9, 1, 0, 400)
        for k in range(400):
            s, t = int(S.s[k]), int(S.t[k])
            assert s != t and 0 <= s < g.n and 0 <= t < g.n
            p = [int(x) for x in S.path(k)]
            if not nx.has_path(G, s, t):
                assert p == [] and S.sigma_bits[k] == 0
                continue
            assert p[0] == s and p[-1] == t
            assert len(p) - 1 == nx.shortest_path_length(G, s, t)
            for a, b in zip(p, p[1:]):
                assert G.has_edge(a, b)
            nsp = len(list(nx.all_shortest_paths(G, s, t)))
            assert int(S.sigma_bits[k]) == nsp.bit_length()


def test_pair_is_uniform_over_ordered_pairs(oracle_lib):
    from scipy.stats import chisquare
    g = gg.cycle_graph(5, True)
    S = oracle_lib.sample_paths(g, 4, 0, 0, 40000)
    cells = S.s.astype(np.int64) * 5 + S.t
    obs = np.bincount(cells, minlength=25)
    diag = [i * 5 + i for i in range(5)]
    assert obs[diag].sum() == 0
    assert chisquare(np.delete(obs, diag)).pvalue > 1e-4


@pytest.mark.parametrize("which", ["grid", "undirected", "directed"])
def test_paths_uniform_given_pair(oracle_lib, which):
    """Chi-square of sampled (s, t, path) triples against 1/(n(n-1) sigma_st)."""
    import networkx as nx
    from scipy.stats import chisquare
    g = {"grid": gg.grid(3, 4), "undirected": gg.gnp(9, 0.35, 3),
         "directed": gg.gnp(8, 0.35, 2, directed=True)}[which]
    G = _nx(g)
    N = 150000
    S = oracle_lib.sample_paths(g, 21, 1, 0, N, threads=4)
    index, expect = {}, []
    n = g.n
    for s in range(n):
        for t in range(n):
            if s == t or not nx.has_path(G, s, t):
                continue
            paths = list(nx.all_shortest_paths(G, s, t))
            for p in paths:
                index[tuple(p)] = len(expect)
                expect.append(N / (n * (n - 1)) / len(paths))
    obs = np.zeros(len(expect))
    for k in range(N):
        p = tuple(int(x) for x in S.path(k))
        if p:
            obs[index[p]] += 1
    expect = np.array(expect)
    # the disconnected pairs take the remaining mass
    assert abs(obs.sum() - expect.sum()) < 6 * math.sqrt(N)
    stat = ((obs - expect) ** 2 / expect).sum()
    from scipy.stats import chi2
    assert chi2.sf(stat, len(expect)) > 1e-5, (which, stat, len(expect))


# ----------------------------------------------------------------------------- betweenness


def test_brandes_matches_networkx(oracle_lib):
    import networkx as nx
    for g in _small_graphs() + [gg.gnp(40, 0.1, 1), gg.gnp(30, 0.08, 2, directed=True)]:
        bc = oracle_lib.brandes(g)
        ref = nx.betweenness_centrality(_nx(g), normalized=False)
        scale = (1.0 if g.directed else 2.0) / (g.n * (g.n - 1))
        for v in range(g.n):
            assert abs(bc[v] - ref[v] * scale) < 1e-12


def test_brandes_closed_forms(oracle_lib):
    n = 9
    bc = oracle_lib.brandes(gg.path_graph(n))
    for i in range(n):
        assert abs(bc[i] - 2 * i * (n - 1 - i) / (n * (n - 1))) < 1e-14
    bc = oracle_lib.brandes(gg.star_graph(n))
    assert abs(bc[0] - (n - 2) / n) < 1e-14 and np.all(bc[1:] == 0)
    bc = oracle_lib.brandes(gg.cycle_graph(n, True))
    assert np.allclose(bc, (n - 2) / (2 * n), atol=1e-14)
    assert np.all(oracle_lib.brandes(gg.complete_graph(6)) == 0)
    a, b = 3, 5
    bc = oracle_lib.brandes(gg.complete_bipartite(a, b))
    N = a + b
    assert np.allclose(bc[:a], b * (b - 1) / a / (N * (N - 1)), atol=1e-14)
    assert np.allclose(bc[a:], a * (a - 1) / b / (N * (N - 1)), atol=1e-14)


def test_expected_hits_equal_betweenness(oracle_lib):
    """E[X_i(v)] = bc(v): the hit frequency over many samples converges to Brandes."""
    for g in [gg.gnp(30, 0.12, 7), gg.gnp(25, 0.12, 8, directed=True),
              gg.disjoint_union(gg.path_graph(6), gg.cycle_graph(5, False))]:
        N = 120000
        S = oracle_lib.sample_paths(g, 5, 1, 0, N, threads=4)
        cnt = np.zeros(g.n)
        for k in range(N):
            p = S.path(k)
            cnt[p[1:-1]] += 1
        bt = cnt / N
        bc = oracle_lib.brandes(g)
        sd = np.sqrt(np.maximum(bc * (1 - bc), 1e-12) / N)
        assert np.all(np.abs(bt - bc) <= 5 * sd + 1e-9), np.max(np.abs(bt - bc) / sd)


# ----------------------------------------------------------------------------- vertex diameter


def test_vertex_diameter_exact_and_bound(oracle_lib):
    import networkx as nx
    graphs = _small_graphs() + [gg.gnp(60, 0.05, 3), gg.gnp(50, 0.04, 4, directed=True),
                                gg.path_graph(12), gg.grid(5, 7)]
    for g in graphs:
        G = _nx(g)
        lengths = dict(nx.all_pairs_shortest_path_length(G))
        exact = 1 + max(d for src in lengths.values() for d in src.values())
        vd, ex = oracle_lib.vertex_diameter(g)
        assert ex and vd == exact
        vb, exb = oracle_lib.vertex_diameter(g, exact_limit=0.0)
        assert not exb and vb >= exact
    # the bound is tight on a path's ends: r = node 1 (largest degree, lowest id)
    vb, _ = oracle_lib.vertex_diameter(gg.path_graph(10), exact_limit=0.0)
    assert vb == 2 * 8 + 1


def test_vertex_diameter_er2000_lcc(oracle_lib):
    vd, ex = oracle_lib.vertex_diameter(gg.workload("er2000"))
    assert ex and vd == 8


# ----------------------------------------------------------------------------- sample budget


def _appf_rows():
    rows = []
    for line in open(os.path.join(GOLDEN, "appF_iterations.txt")):
        if line.startswith("#") or not line.strip():
            continue
        kind, lam, kad, rk = line.split()
        rows.append((kind, float(lam), int(kad), int(rk)))
    return rows


def test_omega_formula_pinned_by_rk_column(oracle_lib):
    """RK's fixed sample size is c/lambda^2 (floor(log2(VD-2)) + 1 + ln(1/delta)); with
    delta' = delta/2 this is exactly the KADABRA cap omega.  Every printed RK count must
    be omega(lambda, 2*0.1, VD) for some VD: this pins c = 0.5, the natural log and the
    rounding up."""
    rows = _appf_rows()
    assert len(rows) == 180
    below = 0
    for kind, lam, kad, rk in rows:
        js = [j for j in range(1, 40) if oracle_lib.omega(lam, 0.2, 2 ** (j - 1) + 2) == rk]
        assert js, (kind, lam, rk)
        if kad <= oracle_lib.omega(lam, 0.1, 2 ** (js[0] - 1) + 2):
            below += 1
    assert below >= 178


def test_omega_alpha_interval_config1(oracle_lib):
    om = oracle_lib.omega(0.01, 0.1, 8)
    assert om == 29979
    assert oracle_lib.alpha(om) == 299
    assert oracle_lib.default_interval(om) == 1024
    assert oracle_lib.default_interval(2_000_000) == 65536
    assert oracle_lib.default_interval(200_000) == 8192
    assert oracle_lib.omega(0.01, 0.1, 3) == math.ceil(0.5 / 0.01 ** 2 * (1 + math.log(20)))


# ----------------------------------------------------------------------------- f and g


def test_f_g_satisfy_their_quadratics(oracle_lib):
    """g is the root of tau*g = L/3 + sqrt(L^2/9 + 2 omega (b+g) L) and f of
    tau*f = L/3 + sqrt(L^2/9 + 2 omega (b-f) L) (when tau*f >= L/3): the equations the
    appendix derives them from (McDiarmid's bound solved for the deviation)."""
    rng = np.random.default_rng(2)
    worst_g = worst_f = 0.0
    for _ in range(20000):
        om = float(rng.integers(1000, 10**7))
        tau = float(rng.integers(1, int(om) + 1))
        L = float(np.exp(rng.uniform(np.log(0.5), np.log(60))))
        b = float(10 ** rng.uniform(-9, -0.3))
        g = oracle_lib.g(b, L, om, tau)
        rhs = L / 3 + math.sqrt(L * L / 9 + 2 * om * (b + g) * L)
        worst_g = max(worst_g, abs(tau * g - rhs) / rhs)
        f = oracle_lib.f(b, L, om, tau)
        if tau * f >= L / 3 and b - f > 0:
            rhs = L / 3 + math.sqrt(L * L / 9 + 2 * om * (b - f) * L)
            worst_f = max(worst_f, abs(tau * f - rhs) / rhs)
    assert worst_g < 1e-12
    assert worst_f < 1e-9


def test_f_g_special_values(oracle_lib):
    L, om, tau = 7.3, 5000.0, 1200.0
    assert oracle_lib.f(0.0, L, om, tau) == 0.0
    assert abs(oracle_lib.g(0.0, L, om, tau) - 2 * L / tau * (1 / 3 + om / tau)) < 1e-15
    # monotone in the estimate
    xs = [oracle_lib.f(b, L, om, tau) for b in np.linspace(0, 0.5, 200)]
    assert all(x < y for x, y in zip(xs, xs[1:]))


# ----------------------------------------------------------------------------- computeDelta


def test_compute_delta_budget_and_balance(oracle_lib):
    rng = np.random.default_rng(4)
    n, alpha, om, delta, lam = 5000, 300, 29979, 0.1, 0.01
    count0 = rng.poisson(rng.exponential(2.0, n)).astype(np.uint64)
    count0[:1000] = 0
    Ll, Lu, C = oracle_lib.compute_delta(count0, alpha, om, np.full(n, lam), np.full(n, lam),
                                         delta, 0.001)
    dl, du = np.exp(-Ll), np.exp(-Lu)
    add = 0.001 * delta / (2 * n)
    assert abs((dl + du).sum() - delta / 2) < 1e-9
    assert np.all(dl >= add * (1 - 1e-12))
    # all terms equalised: c(v) * log(1/(delta(v) - add)) = C where c(v) > 0
    c = 2 * (count0 / alpha) * om / lam ** 2
    m = (c > 0) & (dl - add > 1e-2 * dl)          # well-conditioned subtraction only
    assert m.sum() > 100
    assert np.allclose(c[m] * -np.log(dl[m] - add), C, rtol=1e-9)


# ----------------------------------------------------------------------------- rank intervals


def test_rank_rule_reproduces_paper_tables(oracle_lib):
    tables, cur = [], None
    for line in open(os.path.join(GOLDEN, "appG_topk_tables.txt")):
        if line.startswith("#") or not line.strip():
            continue
        if line.startswith("table"):
            cur = []
            tables.append(cur)
            continue
        lo, hi, a, b, c = line.split()
        cur.append((int(lo), int(hi), float(a), float(b), float(c)))
    assert len(tables) == 17 and sum(len(t) for t in tables) == 232
    for t in tables:
        lower = np.array([r[2] for r in t])
        upper = np.array([r[4] for r in t])
        rlo, rhi = oracle_lib.rank_intervals(lower, upper)
        assert list(rlo) == [r[0] for r in t]
        assert list(rhi) == [r[1] for r in t]


# ----------------------------------------------------------------------------- whole runs


def test_run_complete_graph_stops_on_g_only(oracle_lib):
    g = gg.complete_graph(20)
    r = oracle_lib.run(g, 0.01, 0.1, seed=3)       # omega ~ 2e4 > interval 1024
    assert r["count"].sum() == 0 and r["stop_rule"] == 1
    assert r["tau"] < r["omega"] and r["tau"] % r["interval"] == 0


def test_run_invariants_er2000(oracle_lib):
    g = oracle_lib.Graph(gg.workload("er2000"))
    r1 = oracle_lib.run(g, 0.01, 0.1, seed=1, threads=1)
    r4 = oracle_lib.run(g, 0.01, 0.1, seed=1, threads=4)
    for key in ("count", "count0", "tau", "L_l", "L_u", "lower", "upper"):
        assert np.array_equal(np.asarray(r1[key]), np.asarray(r4[key])), key
    assert r1["omega"] == 29979 and r1["alpha"] == 299 and r1["vd"] == 8
    assert r1["tau"] <= r1["omega"] and (r1["tau"] % 1024 == 0 or r1["tau"] == r1["omega"])
    S = oracle_lib.sample_paths(g, 1, 1, 0, int(r1["tau"]), threads=4)
    cnt = np.zeros(g.n, dtype=np.uint64)
    for k in range(int(r1["tau"])):
        p = S.path(k)
        cnt[p[1:-1]] += 1
    assert np.array_equal(cnt, r1["count"])
    assert int(r1["count"].sum()) == int(sum(max(int(S.path_off[k + 1] - S.path_off[k]) - 2, 0)
                                             for k in range(int(r1["tau"]))))
    assert int(S.arcs.sum()) == r1["arcs"]


@pytest.mark.slow
def test_epsilon_guarantee_er2000(oracle_lib):
    """Theorem 1: with probability 1-delta every estimate is within its interval and
    (here all-nodes) within lambda of the exact betweenness."""
    g = oracle_lib.Graph(gg.workload("er2000"))
    bc = oracle_lib.brandes(g)
    bad_eps = bad_cov = 0
    runs = 200
    for seed in range(1, runs + 1):
        r = oracle_lib.run(g, 0.01, 0.1, seed=seed, threads=8)
        if np.max(np.abs(r["bc"] - bc)) > 0.01:
            bad_eps += 1
        if not np.all((r["lower"] <= bc) & (bc <= r["upper"])):
            bad_cov += 1
    # the theorem allows a fraction delta of failing runs; the bounds are loose, so in
    # practice none fails
    assert bad_eps <= 0.1 * runs and bad_cov <= 0.1 * runs
    assert bad_eps <= 2 and bad_cov <= 2


def test_topk_run_finds_true_top(oracle_lib):
    g = oracle_lib.Graph(gg.chung_lu(1500, 2.3, 6.0, 42))
    bc = oracle_lib.brandes(g)
    k = 5
    r = oracle_lib.run(g, 0.004, 0.1, mode="topk", k=k, seed=2, threads=8)
    rlo, rhi = oracle_lib.rank_intervals(r["lower"], r["upper"])
    reported = set(np.nonzero(rlo <= k)[0].tolist())
    true_top = set(np.argsort(-bc, kind="stable")[:k].tolist())
    assert true_top <= reported
    true_rank = np.empty(g.n, dtype=np.int64)
    true_rank[np.argsort(-bc, kind="stable")] = np.arange(1, g.n + 1)
    for v in reported:
        assert rlo[v] <= true_rank[v] <= rhi[v]


# ----------------------------------------------------------------------------- arcs scanned and the side rule
#
# Section 4: the side whose frontier has the smaller degree sum is expanded (out-degrees
# on the s side, in-degrees on the t side of a directed graph; ties expand s), a level is
# always processed whole, and every arc of an expanded level counts as one visited edge.
# On the small gadgets below the arcs of a pair follow from that rule by hand; each
# derivation is written next to its expected value.


def _pair_samples(oracle_lib, g, want, seed=3, count=40000):
    """Sample ids whose (s, t) is one of the pairs in ``want``; every pair must occur."""
    S = oracle_lib.sample_paths(g, seed, 1, 0, count, threads=4)
    seen = {}
    for k in range(count):
        key = (int(S.s[k]), int(S.t[k]))
        if key in want:
            seen.setdefault(key, []).append(k)
    assert set(seen) == set(want), sorted(set(want) - set(seen))
    return S, seen


def _gadget_directed_tie(k=6, r=3):
    """s=0 -> m=2 and s -> p_1..p_k (no out-arcs); m -> t=1; q_1..q_k -> t; every r_j -> every
    q_i.  out(s) = k+1 = in(t): a tie."""
    m, p0, q0, r0 = 2, 3, 3 + k, 3 + 2 * k
    n = r0 + r
    src = [0, m] + [0] * k + list(range(q0, q0 + k))
    dst = [m, 1] + list(range(p0, p0 + k)) + [1] * k
    for j in range(r):
        for i in range(k):
            src.append(r0 + j)
            dst.append(q0 + i)
    return gg.csr_from_edges(n, src, dst, True, name="tie_gadget"), dict(k=k, r=r, m=m, p0=p0,
                                                                            q0=q0, r0=r0)


def test_arcs_side_rule_directed_gadget(oracle_lib):
    g, P = _gadget_directed_tie()
    k, r, m, q0, r0, p0 = P["k"], P["r"], P["m"], P["q0"], P["r0"], P["p0"]
    want = {
        # D_S = out(s) = k+1 <= D_T = in(t) = k+1: expand s (k+1 arcs); its next level {m, p_*}
        # has out-degree sum 1 < k+1: expand it (1 arc, m -> t touches).  k+2 arcs.  Expanding
        # t first ("<") would cost in(t) = k+1, then the s level k+1 again: 2k+2.
        (0, 1): (k + 2, [0, m, 1]),
        # out(1) = 0 <= in(0) = 0: the s side is expanded and gains no node: disconnected.
        (1, 0): (0, []),
        # (m, t): out(m) = 1 <= 7: one arc, m -> t touches.
        (m, 1): (1, [m, 1]),
        # (p, t): out(p) = 0: the s side closes at once.
        (p0, 1): (0, []),
        # (s, q): in(q) = r < out(s) = k+1: expand q's in-row (r arcs) -> {r_*}, whose in-degree
        # sum is 0 < k+1: expanded again with no arcs and no node: disconnected after r arcs.
        (0, q0): (r, []),
    }
    # (r_j, t): out(r_j) = k <= in(t) = k+1: k arcs to the q's, whose out-degree sum k <= k+1:
    # expanded, k arcs, each q_i -> t touches.  2k arcs; the path is r_j, one q_i, t.
    for j in range(r):
        want[(r0 + j, 1)] = (2 * k, None)
    S, seen = _pair_samples(oracle_lib, g, want)
    for pair, ids in seen.items():
        arcs, path = want[pair]
        for i in ids:
            assert int(S.arcs[i]) == arcs, (pair, int(S.arcs[i]), arcs)
            got = [int(x) for x in S.path(i)]
            if path is not None:
                assert got == path, (pair, got)
            else:
                assert len(got) == 3 and q0 <= got[1] < q0 + k, (pair, got)


def test_arcs_whole_level_undirected_gadget(oracle_lib):
    """0-1, 0-2, 1-3, 2-{4..8}, 3-{9..12}: degrees 0:2, 1:2, 2:6, 3:5, leaves 1."""
    src = [0, 0, 1] + [2] * 5 + [3] * 4
    dst = [1, 2, 3] + list(range(4, 9)) + list(range(9, 13))
    g = gg.csr_from_edges(13, src, dst, False, name="level_gadget")
    want = {
        # (0, 3): 2 <= 5: expand 0 (2 arcs) -> {1, 2}, sum 8 > 5: expand 3 -- its whole row of 5
        # arcs, although the first (3 -> 1) already touches.  7 arcs (3 if the level were cut
        # at the first touching arc).
        (0, 3): (7, [0, 1, 3]),
        # (3, 0): 5 > 2: expand 0's row (2 arcs) -> {1, 2}, sum 8 > 5: expand 3 (5 arcs).  7.
        (3, 0): (7, [3, 1, 0]),
        # (4, 9): 1 <= 1: expand 4 (1 arc) -> {2}, sum 6 > 1: expand 9 (1) -> {3}, 5 < 6: expand
        # 3 (5 arcs) -> {1, 10, 11, 12}, sum 5 < 6: expand (5 arcs) -> {0}, 2 < 6: expand 0
        # (2 arcs; 0 -> 2 touches).  1+1+5+5+2 = 14 arcs, path 4, 2, 0, 1, 3, 9.
        (4, 9): (14, [4, 2, 0, 1, 3, 9]),
        # (1, 2): 2 <= 6: expand 1 (2 arcs) -> {0, 3}, sum 7 > 6: expand 2 (6 arcs; 2 -> 0
        # touches).  8 arcs.
        (1, 2): (8, [1, 0, 2]),
    }
    S, seen = _pair_samples(oracle_lib, g, want)
    for pair, ids in seen.items():
        arcs, path = want[pair]
        for i in ids:
            assert int(S.arcs[i]) == arcs, (pair, int(S.arcs[i]), arcs)
            assert [int(x) for x in S.path(i)] == path, (pair, S.path(i))


def test_arcs_star_and_path_closed_forms(oracle_lib):
    # star, centre 0: leaf-leaf 1 <= 1 expands the s leaf (1 arc) -> {0}, n-1 > 1: the t
    # leaf's arc touches (1): 2 arcs; a pair with the centre: the leaf's one arc: 1 arc
    n = 9
    g = gg.star_graph(n)
    S = oracle_lib.sample_paths(g, 2, 1, 0, 3000)
    for i in range(3000):
        s, t = int(S.s[i]), int(S.t[i])
        assert int(S.arcs[i]) == (1 if 0 in (s, t) else 2), (s, t)
    # path P_n, a pair at distance L >= 2 of nodes L away from both ends: the frontiers
    # have degree sums 2 at level 0 and 4 later, always tied, so the sides alternate s, t,
    # s, t, ...: 2 + 2 + 4 (L - 2) arcs; L = 1: one expansion of 2 arcs
    n = 40
    g = gg.path_graph(n)
    S = oracle_lib.sample_paths(g, 8, 1, 0, 20000, threads=4)
    checked = 0
    for i in range(20000):
        s, t = int(S.s[i]), int(S.t[i])
        L = abs(s - t)
        if min(s, t) >= L and max(s, t) <= n - 1 - L:
            assert int(S.arcs[i]) == (2 if L == 1 else 4 * L - 4), (s, t)
            checked += 1
    assert checked > 2000


# ----------------------------------------------------------------------------- tau on K_n
#
# On a complete graph every pair is adjacent, so no path has an interior node: the pilot
# and main counts are all zero.  computeDelta then gives c_L = c_U = 0, exp(-C/0) = 0 and
# delta_L = delta_U = eps * delta / (2n) for every node, i.e. L = ln(2n / (eps * delta)).
# f(0) = 0 exactly, and g(0) = (2L/tau)(1/3 + omega/tau): the run stops at the first
# multiple of the check interval B where that is <= lambda (VD = 2, so
# omega = ceil(c/lambda^2 (1 + ln(2/delta)))), or at omega.


def _kn_tau(n, lam, delta=0.1, eps=0.001, c=0.5):
    om = math.ceil(c / lam ** 2 * (1 + math.log(2 / delta)))
    b = 1
    while b * 2 <= om // 16:
        b *= 2
    B = min(max(b, 1024), 65536)
    L = math.log(2.0 * n / (eps * delta))
    tau = B
    while tau < om:
        if 2 * L / tau * (1 / 3 + om / tau) <= lam:
            return tau, om, 1
        tau += B
    return om, om, 0


@pytest.mark.parametrize("n,lam", [(20, 0.01), (30, 0.02), (12, 0.005), (50, 0.015), (8, 0.03),
                                   (10, 0.05)])
def test_run_complete_graph_tau_closed_form(oracle_lib, n, lam):
    tau, om, rule = _kn_tau(n, lam)
    r = oracle_lib.run(gg.complete_graph(n), lam, 0.1, seed=3)
    assert r["vd"] == 2 and r["omega"] == om
    assert int(r["count"].sum()) == 0 and int(r["count0"].sum()) == 0
    assert r["tau"] == tau and r["stop_rule"] == rule
    L = math.log(2.0 * n / (0.001 * 0.1))
    assert np.allclose(r["L_l"], L, rtol=1e-12) and np.allclose(r["L_u"], L, rtol=1e-12)
    if rule:
        assert np.all(r["lower"] == 0.0)   # f(0) = 0
        g0 = 2 * L / tau * (1 / 3 + om / tau)
        assert np.allclose(r["upper"], g0, rtol=1e-12)
    else:                                  # omega reached: [b - lambda, b + lambda]
        assert np.all(r["lower"] == -lam) and np.all(r["upper"] == lam)
    assert (10, 0.05) != (n, lam) or (rule == 0 and tau == om)   # omega < B: stops at omega


# ----------------------------------------------------------------------------- Algorithm 3
#
# Hand cases of the top-k stopping condition (appendix, Algorithm 3) with n = 6.  Positions
# v_1..v_6 are given in decreasing order of the estimate; node ids are scrambled.  A node
# is "narrow" (L = 1e-3: f, g about 2e-4 <= lambda = 0.01) or "wide" (L = 20 or 12:
# f, g about 0.02 > lambda).  Each case first checks that its intervals are laid out as
# described, then the decision written from the algorithm.

_A3_OM, _A3_TAU, _A3_LAM = 1_000_000, 100_000, 0.01
_A3_IDS = [4, 0, 5, 2, 1, 3]   # node id of position v_1..v_6
_N, _W = 1e-3, 20.0


def _alg3(oracle_lib, spec, k):
    """spec: (count, L) of v_1..v_6.  Returns (decision, lower[pos], upper[pos], wide[pos])."""
    n = len(spec)
    cnt = np.zeros(n, dtype=np.uint64)
    L = np.zeros(n)
    for pos, (c, l) in enumerate(spec):
        cnt[_A3_IDS[pos]] = c
        L[_A3_IDS[pos]] = l
    lo, hi, wide = [], [], []
    for c, l in spec:
        b = c / _A3_TAU
        f = oracle_lib.f(b, l, _A3_OM, _A3_TAU)
        g = oracle_lib.g(b, l, _A3_OM, _A3_TAU)
        lo.append(b - f)
        hi.append(b + g)
        wide.append(f > _A3_LAM or g > _A3_LAM)
    return oracle_lib.stop_topk(cnt, k, _A3_TAU, _A3_OM, _A3_LAM, L, L), lo, hi, wide


def test_alg3_all_narrow_stops_even_when_overlapping(oracle_lib):
    tail = [(10000, _N), (5000, _N), (1000, _N)]
    d, lo, hi, wide = _alg3(oracle_lib, [(20000, _N), (15000, _N), (12000, _N)] + tail, 2)
    assert not any(wide) and d
    # f, g <= lambda at every node: no separation test is made, so overlaps do not matter
    d, lo, hi, wide = _alg3(oracle_lib, [(20000, _N), (19990, _N), (19980, _N)] + tail, 2)
    assert lo[0] < hi[1] and lo[1] < hi[2] and not any(wide)
    assert d


def test_alg3_previous_neighbour(oracle_lib):
    # v_2 wide, its interval reaches above b(v_1) - f(v_1) (the i-1 test fails) but stays
    # above v_3's (the i+1 test passes): no stop
    spec = [(17600, _N), (15000, _W), (12000, _N), (10000, _N), (5000, _N), (1000, _N)]
    d, lo, hi, wide = _alg3(oracle_lib, spec, 2)
    assert wide == [False, True, False, False, False, False]
    assert lo[0] < hi[1] and lo[1] >= hi[2]
    assert not d
    # the same with v_1 far above: stop
    spec[0] = (20000, _N)
    d, lo, hi, wide = _alg3(oracle_lib, spec, 2)
    assert lo[0] >= hi[1] and lo[1] >= hi[2] and d


def test_alg3_next_neighbour(oracle_lib):
    # v_1 wide (there is no v_0, whose test never fails) overlapping v_2 below: no stop
    spec = [(20000, _W), (17500, _N), (12000, _N), (10000, _N), (5000, _N), (1000, _N)]
    d, lo, hi, wide = _alg3(oracle_lib, spec, 2)
    assert wide[0] and not any(wide[1:]) and lo[0] < hi[1]
    assert not d
    spec[1] = (15000, _N)
    d, lo, hi, wide = _alg3(oracle_lib, spec, 2)
    assert lo[0] >= hi[1] and d


def test_alg3_nodes_below_k_against_v_k(oracle_lib):
    # top two narrow and separated; v_4 (i > k) wide and reaching above b(v_k) - f(v_k): no stop
    spec = [(20000, _N), (15000, _N), (14000, _N), (13500, _W), (5000, _N), (1000, _N)]
    d, lo, hi, wide = _alg3(oracle_lib, spec, 2)
    assert wide == [False, False, False, True, False, False]
    assert lo[0] >= hi[1] and hi[3] > lo[1]
    assert not d
    # v_4's upper end between b(v_3) - f(v_3) and b(v_2) - f(v_2): the test is against v_k
    # (= v_2), so it passes (against v_{k+1} it would not): stop
    spec = [(20000, _N), (15000, _N), (14800, _N), (13000, 12.0), (5000, _N), (1000, _N)]
    d, lo, hi, wide = _alg3(oracle_lib, spec, 2)
    assert wide == [False, False, False, True, False, False]
    assert lo[2] < hi[3] <= lo[1]
    assert d


def test_alg3_last_position_has_no_successor(oracle_lib):
    # k = n: v_6 wide (L = 40); separated from v_5 it does not block the stop (there is no v_7)
    spec = [(20000, _N), (15000, _N), (12000, _N), (10000, _N), (5000, _N), (1000, 40.0)]
    d, lo, hi, wide = _alg3(oracle_lib, spec, 6)
    assert wide[5] and lo[4] >= hi[5] and d
    spec[5] = (4000, _W)
    d, lo, hi, wide = _alg3(oracle_lib, spec, 6)
    assert wide[5] and lo[4] < hi[5] and not d


# ----------------------------------------------------------------------------- top-k half-widths
#
# Section 5: pilot estimates b0 sorted decreasingly give v_1..v_n; for i <= k,
# lambda_U(v_i) = (b0(v_{i-1}) - b0(v_i))/2 (1 for v_1) and lambda_L(v_i) =
# (b0(v_i) - b0(v_{i+1}))/2 (1 when there is no v_{i+1}); a gap b0(v_i) - b0(v_{i+1}) < 2
# lambda for i <= k sets all four values of v_i and v_{i+1} to lambda; for i > k,
# lambda_L = 1 and lambda_U = b0(v_k) - lambda_L(v_k) - b0(v_i); every value is clamped to
# [lambda, 1].  Expected arrays below are worked by hand (per position v_1..v_6).


def _topk_case(oracle_lib, counts_by_pos, k, alpha, lam, ids):
    n = len(counts_by_pos)
    c0 = np.zeros(n, dtype=np.uint64)
    for pos, c in enumerate(counts_by_pos):
        c0[ids[pos]] = c
    ll, lu = oracle_lib.topk_lambdas(c0, k, alpha, lam)
    return [float(ll[ids[p]]) for p in range(n)], [float(lu[ids[p]]) for p in range(n)]


def test_topk_lambdas_hand_worked(oracle_lib):
    ids = [3, 0, 5, 1, 4, 2]
    # b0 = 0.80, 0.60, 0.59, 0.58, 0.30, 0.00; lambda = 0.05, k = 2.  Gap v_1-v_2 = 0.20
    # (no tie); gap v_2-v_3 = 0.01 < 0.10: v_2 and v_3 get (0.05, 0.05).  v_1: lambda_L =
    # 0.10, lambda_U = 1.  b0(v_k) - lambda_L(v_k) = 0.60 - 0.05 = 0.55, so v_4: 0.55 - 0.58 =
    # -0.03, clamped to 0.05; v_5: 0.25; v_6: 0.55; all of them lambda_L = 1.
    ll, lu = _topk_case(oracle_lib, [80, 60, 59, 58, 30, 0], 2, 100, 0.05, ids)
    assert np.allclose(ll, [0.10, 0.05, 0.05, 1.0, 1.0, 1.0], atol=1e-12, rtol=0)
    assert np.allclose(lu, [1.0, 0.05, 0.05, 0.05, 0.25, 0.55], atol=1e-12, rtol=0)
    # b0 = 0.80, 0.72, 0.50, 0.20, 0.10, 0.05; lambda = 0.05, k = 2.  Gap v_1-v_2 = 0.08 lies
    # between lambda and 2 lambda: a tie, v_1 and v_2 get (0.05, 0.05); gap v_2-v_3 = 0.22.
    # 0.72 - 0.05 = 0.67: v_3..v_6 get lambda_U = 0.17, 0.47, 0.57, 0.62.
    ll, lu = _topk_case(oracle_lib, [80, 72, 50, 20, 10, 5], 2, 100, 0.05, ids)
    assert np.allclose(ll, [0.05, 0.05, 1.0, 1.0, 1.0, 1.0], atol=1e-12, rtol=0)
    assert np.allclose(lu, [0.05, 0.05, 0.17, 0.47, 0.57, 0.62], atol=1e-12, rtol=0)
    # k = n = 3, b0 = 0.5, 0.3, 0.1 (alpha 10), lambda 0.05: no tie; v_3 has no successor
    ll, lu = _topk_case(oracle_lib, [5, 3, 1], 3, 10, 0.05, [2, 0, 1])
    assert np.allclose(ll, [0.1, 0.1, 1.0], atol=1e-12, rtol=0)
    assert np.allclose(lu, [1.0, 0.1, 0.1], atol=1e-12, rtol=0)
    # equal pilot counts are ordered by id: nodes 1 and 4 both at 0.6 (gap 0 < 2 lambda:
    # tied), node 1 is v_2 (k = 2) and node 4 is v_3
    c0 = np.array([90, 60, 10, 0, 60], dtype=np.uint64)
    ll, lu = oracle_lib.topk_lambdas(c0, 2, 100, 0.05)
    assert np.allclose([ll[0], lu[0]], [0.15, 1.0], atol=1e-12, rtol=0)
    assert np.allclose([ll[1], lu[1], ll[4], lu[4]], [0.05] * 4, atol=1e-12, rtol=0)
    # b0(v_k) - lambda_L(v_k) = 0.55: node 2 (0.10) gets 0.45, node 3 (0.00) 0.55
    assert np.allclose([ll[2], lu[2], ll[3], lu[3]], [1.0, 0.45, 1.0, 0.55], atol=1e-12, rtol=0)


# ----------------------------------------------------------------------------- forward search
#
# The search of the samplers section 6 compares against: a BFS from s only, level by level,
# until the level that reaches t is finished.  Its arcs follow from the levels of s alone.


def test_forward_search_closed_forms(oracle_lib):
    # star, centre 0: leaf -> leaf expands the leaf (1 arc) and the centre's whole row
    # (n-1 arcs): n; centre -> leaf: n-1; leaf -> centre: 1
    n = 9
    S = oracle_lib.sample_paths(gg.star_graph(n), 2, 1, 0, 3000, search="forward")
    for i in range(3000):
        s, t = int(S.s[i]), int(S.t[i])
        want = 1 if t == 0 else (n - 1 if s == 0 else n)
        assert int(S.arcs[i]) == want, (s, t)
    # path P_n: levels 0..d-1 of s are expanded, 2 arcs for s and 4 for each later level
    # when s is at least d from both ends: 4d - 2
    n = 40
    S = oracle_lib.sample_paths(gg.path_graph(n), 8, 1, 0, 20000, threads=4, search="forward")
    checked = 0
    for i in range(20000):
        s, t = int(S.s[i]), int(S.t[i])
        d = abs(s - t)
        if min(s, n - 1 - s) >= d:
            assert int(S.arcs[i]) == 4 * d - 2, (s, t)
            checked += 1
    assert checked > 1000
    # the directed tie gadget: (s, q) -- the balanced search stops after q's r in-arcs; the
    # forward search expands s (k+1 arcs), {m, p_*} (1 arc, m -> t), {t} (no arcs): k+2,
    # disconnected
    g, P = _gadget_directed_tie()
    k, q0 = P["k"], P["q0"]
    S, seen = _pair_samples(oracle_lib, g, {(0, q0): None, (0, 1): None})
    F = oracle_lib.sample_paths(g, 3, 1, 0, 40000, threads=4, search="forward")
    for i in seen[(0, q0)]:
        assert int(S.arcs[i]) == P["r"] and int(F.arcs[i]) == k + 2 and len(F.path(i)) == 0
    for i in seen[(0, 1)]:
        assert int(F.arcs[i]) == k + 2 and [int(x) for x in F.path(i)] == [0, P["m"], 1]


@pytest.mark.parametrize("which", ["grid", "undirected", "directed"])
def test_forward_search_paths_uniform(oracle_lib, which):
    """Chi-square of sampled (s, t, path) triples against 1/(n(n-1) sigma_st), forward search."""
    import networkx as nx
    from scipy.stats import chi2
    g = {"grid": gg.grid(3, 4), "undirected": gg.gnp(9, 0.35, 3),
         "directed": gg.gnp(8, 0.35, 2, directed=True)}[which]
    G = _nx(g)
    N = 150000
    S = oracle_lib.sample_paths(g, 23, 1, 0, N, threads=4, search="forward")
    index, expect = {}, []
    n = g.n
    for s in range(n):
        for t in range(n):
            if s == t or not nx.has_path(G, s, t):
                continue
            paths = list(nx.all_shortest_paths(G, s, t))
            for p in paths:
                index[tuple(p)] = len(expect)
                expect.append(N / (n * (n - 1)) / len(paths))
    obs = np.zeros(len(expect))
    for k in range(N):
        p = tuple(int(x) for x in S.path(k))
        if p:
            obs[index[p]] += 1
    expect = np.array(expect)
    assert abs(obs.sum() - expect.sum()) < 6 * math.sqrt(N)
    stat = ((obs - expect) ** 2 / expect).sum()
    assert chi2.sf(stat, len(expect)) > 1e-5, (which, stat, len(expect))


def test_forward_search_same_pairs_scans_more(oracle_lib):
    """Same sample ids give the same pairs and paths of the same length (both searches
    return shortest paths); on a power-law graph the forward search scans several times
    the arcs of the balanced one (section 6, Theorem 2)."""
    g = gg.chung_lu(3000, 2.3, 6.0, 7)
    B = oracle_lib.sample_paths(g, 5, 1, 0, 3000, threads=4)
    F = oracle_lib.sample_paths(g, 5, 1, 0, 3000, threads=4, search="forward")
    assert np.array_equal(B.s, F.s) and np.array_equal(B.t, F.t)
    assert np.array_equal(np.diff(B.path_off.astype(np.int64)), np.diff(F.path_off.astype(np.int64)))
    assert F.arcs.mean() > 3 * B.arcs.mean()


# ----------------------------------------------------------------------------- edge betweenness
#
# Section 1: the method adapts to the centrality of edges.  bc(e) = 1/(n(n-1)) * sum over
# ordered pairs s != t of sigma_st(e)/sigma_st; a sampled path hits every edge on it.


def test_edge_brandes_matches_networkx(oracle_lib):
    import networkx as nx
    for g in _small_graphs() + [gg.gnp(40, 0.1, 1), gg.gnp(30, 0.08, 2, directed=True)]:
        ebc = oracle_lib.edge_brandes(g)
        eid = oracle_lib.edge_ids(g)
        ref = nx.edge_betweenness_centrality(_nx(g), normalized=False)
        scale = (1.0 if g.directed else 2.0) / (g.n * (g.n - 1))
        src, dst = g.edges()
        for pos in range(g.arcs):
            u, v = int(src[pos]), int(dst[pos])
            key = (u, v) if (g.directed or (u, v) in ref) else (v, u)
            assert abs(ebc[eid[pos]] - ref[key] * scale) < 1e-12, (g.name, u, v)


def test_edge_brandes_closed_forms(oracle_lib):
    n = 9
    ebc = oracle_lib.edge_brandes(gg.path_graph(n))    # edge {i, i+1} has id i
    for i in range(n - 1):
        assert abs(ebc[i] - 2 * (i + 1) * (n - 1 - i) / (n * (n - 1))) < 1e-14
    assert np.allclose(oracle_lib.edge_brandes(gg.star_graph(n)), 2.0 / n, atol=1e-14)
    # directed cycle: arc i -> i+1 lies on the one path of every pair whose forward distance
    # passes it: sum over distances d of d pairs, i.e. n(n-1)/2 pairs
    assert np.allclose(oracle_lib.edge_brandes(gg.cycle_graph(n, True)), 0.5, atol=1e-14)
    # K_n: an edge carries only its own two ordered pairs
    assert np.allclose(oracle_lib.edge_brandes(gg.complete_graph(7)), 2.0 / (7 * 6), atol=1e-14)


def test_edge_ids_structure(oracle_lib):
    g = gg.gnp(50, 0.1, 4)
    eid = oracle_lib.edge_ids(g)
    src, dst = g.edges()
    m = oracle_lib.edge_count(g)
    assert m == g.arcs // 2 and np.array_equal(np.bincount(eid, minlength=m), np.full(m, 2))
    canon = {}
    for pos in range(g.arcs):
        canon.setdefault((min(src[pos], dst[pos]), max(src[pos], dst[pos])), set()).add(int(eid[pos]))
    assert all(len(ids) == 1 for ids in canon.values())
    # ids follow the order of the u < v arcs in CSR order
    order = [int(eid[p]) for p in range(g.arcs) if src[p] < dst[p]]
    assert order == list(range(m))
    d = gg.gnp(30, 0.1, 5, True)
    assert np.array_equal(oracle_lib.edge_ids(d), np.arange(d.arcs))


def test_expected_edge_hits_equal_edge_betweenness(oracle_lib):
    for g in [gg.gnp(30, 0.12, 7), gg.gnp(25, 0.12, 8, directed=True), gg.grid(5, 6)]:
        N = 120000
        cnt, _ = oracle_lib.edge_hits(g, 5, 1, 0, N, threads=4)
        bt = cnt / N
        bc = oracle_lib.edge_brandes(g)
        sd = np.sqrt(np.maximum(bc * (1 - bc), 1e-12) / N)
        assert np.all(np.abs(bt - bc) <= 5 * sd + 1e-9), np.max(np.abs(bt - bc) / sd)


def test_edge_hits_are_path_edges(oracle_lib):
    g = oracle_lib.Graph(gg.workload("er2000"))
    S = oracle_lib.sample_paths(g, 3, 1, 0, 5000, threads=4)
    cnt, arcs = oracle_lib.edge_hits(g, 3, 1, 0, 5000, threads=4)
    eid = oracle_lib.edge_ids(g)
    ref = np.zeros(oracle_lib.edge_count(g), dtype=np.uint64)
    row, col = g.row.astype(np.int64), g.col
    for k in range(5000):
        p = [int(x) for x in S.path(k)]
        for a, b in zip(p, p[1:]):
            pos = row[a] + int(np.searchsorted(col[row[a]:row[a + 1]], b))
            ref[eid[pos]] += 1
    assert np.array_equal(cnt, ref) and arcs == int(S.arcs.sum())
    assert int(cnt.sum()) == int(sum(max(len(S.path(k)) - 1, 0) for k in range(5000)))


def test_omega_edges_is_omega_with_one_more_node(oracle_lib):
    """floor(log2(VD - 1)) + 1 for edges is the nodes' floor(log2(VD' - 2)) + 1 at VD' = VD + 1."""
    for lam in (0.03, 0.01, 0.002):
        for vd in (2, 3, 4, 5, 8, 9, 17, 1000):
            assert oracle_lib.omega_edges(lam, 0.1, vd) == oracle_lib.omega(lam, 0.1, vd + 1)


def test_run_edges_invariants(oracle_lib):
    g = oracle_lib.Graph(gg.workload("er2000"))
    r1 = oracle_lib.run(g, 0.01, 0.1, seed=2, threads=1, target="edges")
    r4 = oracle_lib.run(g, 0.01, 0.1, seed=2, threads=4, target="edges")
    for key in ("count", "count0", "tau", "lower", "upper"):
        assert np.array_equal(np.asarray(r1[key]), np.asarray(r4[key])), key
    assert r1["omega"] == oracle_lib.omega_edges(0.01, 0.1, 8) and r1["vd"] == 8
    assert len(r1["count"]) == oracle_lib.edge_count(g)
    cnt, arcs = oracle_lib.edge_hits(g, 2, 1, 0, int(r1["tau"]), threads=4)
    assert np.array_equal(cnt, r1["count"]) and arcs == r1["arcs"]


@pytest.mark.slow
def test_epsilon_guarantee_edges(oracle_lib):
    """Theorem 1 over edges: every edge estimate within lambda in (nearly) every run."""
    g = oracle_lib.Graph(gg.workload("er2000"))
    bc = oracle_lib.edge_brandes(g)
    runs, bad_eps, bad_cov = 50, 0, 0
    for seed in range(1, runs + 1):
        r = oracle_lib.run(g, 0.01, 0.1, seed=seed, threads=8, target="edges")
        if np.max(np.abs(r["bc"] - bc)) > 0.01:
            bad_eps += 1
        if not np.all((r["lower"] <= bc) & (bc <= r["upper"])):
            bad_cov += 1
    assert bad_eps <= 0.1 * runs and bad_cov <= 0.1 * runs
