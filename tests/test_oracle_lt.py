"""Pins of the oracle's LT-model sampler and SIEA_LT (reading R17; Sec. 5.3 and
the LT experiment of Sec. 6).

* Exact law: on a small graph, every combination of the nodes' in-edge
  choices (each node keeps one in-edge with probability w, or none) is
  enumerated, the reachable set from S computed, and the sampled law of
  |cascade| - |S| must fit it (chi-square).
* The threshold form of the LT model (each node draws a threshold uniform in
  [0, 1] and becomes active once the weights of its active in-neighbours
  reach it, in rounds from S) simulated here with numpy: the oracle's
  live-edge samples must have the same law (two-sample chi-square) on a
  larger graph, the equivalence of the two forms being that of Kempe et al.
* SIEA_LT meets (eps, delta) against the enumerated I(S); IS = OI + |S|.
* In-weights summing above 1 are rejected.
"""
import itertools

import numpy as np
import pytest
from scipy import stats

import oracle as O
from oi_inputs import chung_lu_graph, graph_from_edges, wc_probs
from test_oracle_sampler import _chi2_pvalue

SEED = 0x17044794


def _small_graph():
    src = [0, 0, 1, 1, 2, 2, 3, 4, 5, 5, 6, 7]
    dst = [1, 2, 2, 3, 3, 4, 5, 5, 6, 7, 7, 6]
    w = [0.6, 0.3, 0.5, 0.45, 0.35, 1.0, 0.7, 0.3, 0.4, 0.2, 0.55, 0.45]
    return graph_from_edges(8, src, dst, np.array(w, np.float32))


def _exact_lt_law(g, S):
    """Law of |reach(S)| - |S| over all in-edge choices (live-edge form)."""
    es, ed = g.edges()
    p = g.p.astype(np.float64)
    options = []
    for v in range(g.n):
        ins = np.flatnonzero(ed == v)
        opts = [(-1, 1.0 - p[ins].sum())] + [(int(e), p[e]) for e in ins]
        options.append([o for o in opts if o[1] > 0])
    law = np.zeros(g.n + 1)
    for combo in itertools.product(*options):
        pr = np.prod([c[1] for c in combo])
        live = [c[0] for c in combo if c[0] >= 0]
        adj = {}
        for e in live:
            adj.setdefault(int(es[e]), []).append(int(ed[e]))
        seen = set(S)
        stack = list(S)
        while stack:
            u = stack.pop()
            for v in adj.get(u, []):
                if v not in seen:
                    seen.add(v)
                    stack.append(v)
        law[len(seen) - len(S)] += pr
    return law


def _threshold_lt(g, S, N, rng):
    """N cascades of the threshold form, vectorized over samples: in each
    round an inactive node activates once the weights of its active
    in-neighbours reach its threshold."""
    es, ed = g.edges()
    W = np.zeros((g.n, g.n), np.float64)
    W[es, ed] = g.p.astype(np.float64)
    act = np.zeros((N, g.n), bool)
    act[:, S] = True
    theta = rng.random((N, g.n))
    while True:
        new = (~act) & (act.astype(np.float64) @ W >= theta)
        if not new.any():
            break
        act |= new
    return act.sum(1) - len(S)


@pytest.mark.parametrize("S", [[0], [1, 4], [2]])
def test_lt_law_matches_enumeration(S):
    g = _small_graph()
    law = _exact_lt_law(g, S)
    N = 200_000
    r = O.lt_fixed(g, S, qid=2, seed=SEED, stream=0, first=0, count=N, want_e=True)
    y = r["y"].astype(np.int64)
    counts = np.bincount(y, minlength=law.size)
    assert _chi2_pvalue(counts[:law.size], law) > 1e-4
    mean = (law * np.arange(law.size)).sum()
    assert abs(y.mean() - mean) < 5 * y.std() / np.sqrt(N)
    assert r["is_"] == len(S) + r["oi"]


def test_lt_matches_the_threshold_form():
    g = chung_lu_graph(400, 2400, 2.1, 5)
    g = g.with_p((0.9 * wc_probs(g)).astype(np.float32))
    S = [int(np.argmax(g.outdeg()))]
    N = 40_000
    a = O.lt_fixed(g, S, qid=0, seed=SEED, stream=0, first=0, count=N)["y"].astype(np.int64)
    b = _threshold_lt(g, S, N, np.random.default_rng(3))
    edges = np.unique(np.quantile(np.concatenate([a, b]), np.linspace(0, 1, 31)))
    ca, _ = np.histogram(a, bins=edges)
    cb, _ = np.histogram(b, bins=edges)
    keep = (ca + cb) > 0
    assert stats.chi2_contingency(np.vstack([ca[keep], cb[keep]]))[1] > 1e-4
    assert abs(a.mean() - b.mean()) < 5 * np.hypot(a.std(), b.std()) / np.sqrt(N)


def test_siea_lt_coverage():
    g = _small_graph()
    eps, delta = 0.1, 0.1
    fails = total = 0
    for S in ([0], [1, 4], [2]):
        law = _exact_lt_law(g, S)
        i_s = len(S) + (law * np.arange(law.size)).sum()
        for qid in range(8):
            r = O.estimate_lt(g, S, eps, delta, qid, SEED)
            assert r["is_"] == r["oi"] + len(S)
            fails += abs(r["is_"] - i_s) > eps * i_s
            total += 1
    assert fails <= max(2, int(0.1 * total))


def test_lt_rejects_in_weights_above_one():
    g = graph_from_edges(3, [0, 1], [2, 2], np.array([0.7, 0.6], np.float32))
    with pytest.raises(O.OracleError):
        O.lt_fixed(g, [0], 0, SEED, 0, 0, 10)
