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
    runs = 24
    for seed in range(1, runs + 1):
        r = oracle_lib.run(g, 0.01, 0.1, seed=seed, threads=8)
        if np.max(np.abs(r["bc"] - bc)) > 0.01:
            bad_eps += 1
        if not np.all((r["lower"] <= bc) & (bc <= r["upper"])):
            bad_cov += 1
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
