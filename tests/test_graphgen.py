"""The random-graph models of the paper's appendix (inputs only): each generator's edges
follow its model's law.  Small graphs, many seeds, chi-square of edge counts per pair."""
import math

import numpy as np
import pytest

import graphgen as gg


def _pair_counts(gen, n, seeds):
    cnt = np.zeros((n, n))
    for s in seeds:
        g = gen(s)
        src, dst = g.edges()
        cnt[src, dst] += 1
    return cnt


def _weights(n, beta, mean):
    c = np.array([math.pow((i + 1) / n, -1.0 / (beta - 1.0)) for i in range(n)])
    return c * (mean * n / math.fsum(c.tolist()))


@pytest.mark.parametrize("model", ["nr", "grg"])
def test_irg_edge_probabilities(model):
    from scipy.stats import chi2
    n, beta, mean, runs = 12, 2.5, 3.0, 3000
    w = _weights(n, beta, mean)
    M = w.sum()
    x = np.outer(w, w) / M
    p = 1.0 - np.exp(-x) if model == "nr" else x / (1.0 + x)
    cnt = _pair_counts(lambda s: gg.random_model(model, n, beta, mean, s), n, range(runs))
    iu = np.triu_indices(n, 1)
    obs, exp = cnt[iu], p[iu] * runs
    assert np.allclose(cnt, cnt.T)           # undirected
    assert np.all(np.diag(cnt) == 0)         # no self-loops
    stat = (((obs - exp) ** 2) / (exp * (1 - p[iu]))).sum()
    assert chi2.sf(stat, iu[0].size) > 1e-4, stat


def test_configuration_model_degrees():
    """Node v gets round(w_v) half-edges (one more on one node if the total is odd); erasing
    self-loops and repeated edges only removes some.  With a finite second moment (beta 3.5)
    almost none are lost; with hubs (beta 2.5) a few percent."""
    for beta, lost in ((3.5, 0.01), (2.5, 0.06)):
        n, mean = 2000, 6.0
        g = gg.configuration_model(n, beta, mean, 3)
        want = np.maximum(1, np.rint(_weights(n, beta, mean))).astype(np.int64)
        deg = g.out_degree()
        assert np.all(deg <= want + 1)
        assert deg.sum() >= (1 - lost) * want.sum(), (beta, deg.sum(), want.sum())
        assert g.rrow is g.row


def test_chung_lu_edge_probabilities():
    from scipy.stats import chi2
    n, runs = 12, 3000
    cnt = _pair_counts(lambda s: gg.chung_lu(n, 2.5, 3.0, s), n, range(runs))
    g = gg.chung_lu(n, 2.5, 3.0, 0)
    iu = np.triu_indices(n, 1)
    assert np.allclose(cnt, cnt.T) and np.all(np.diag(cnt) == 0)
    # min(1, w_u w_v / W) with the generator's tuned scale
    ww = np.array([math.pow((i + 1) / n, -1.0 / 1.5) for i in range(n)]) * g.meta["xmin"]
    p = np.minimum(1.0, np.outer(ww, ww) / ww.sum())
    obs, exp = cnt[iu], p[iu] * runs
    keep = (p[iu] > 0) & (p[iu] < 1)
    stat = (((obs - exp)[keep] ** 2) / (exp * (1 - p[iu]))[keep]).sum()
    assert chi2.sf(stat, keep.sum()) > 1e-4, stat
    assert np.all(obs[p[iu] >= 1] == runs)
