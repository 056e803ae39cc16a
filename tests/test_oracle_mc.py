"""Pins of the oracle's classic IC Monte-Carlo sampler M^(S) (Sec. 2.3; the
MC_10K / MC_100K estimators of Sec. 6.1).

Pinned against: the enumerated law of |r_g(S) \\ S| over all live-edge
graphs (zero included), E[M] = I(S), the Poisson-binomial law of a star's
leaves, breadth-first reachability when every probability is 0 or 1, and
Lemma var (Sec. 5.2) with both variances taken from samples of the two
samplers.
"""
import numpy as np
import pytest

import oracle as O
from oi_inputs import chung_lu_graph, make_config, star_graph, tiny16_graph
from test_oracle_sampler import _chi2_pvalue

SEED = 0x17044794


@pytest.mark.parametrize("S", [[0], [3, 7], [2, 5, 9], [12]])
def test_mc_law_matches_enumeration(S):
    g = tiny16_graph()
    ex = O.exact(g, S)
    N = 200_000
    r = O.mc_fixed(g, S, qid=4, seed=SEED, stream=0, first=0, count=N)
    y = r["y"].astype(np.int64)
    assert y.min() >= 0 and y.max() <= g.n - len(S)
    counts = np.bincount(y, minlength=g.n + 1)
    assert _chi2_pvalue(counts, ex["dist"]) > 1e-4
    # E[M] = I(S) = |S| + Ext(S)
    assert abs(r["is_"] - (len(S) + ex["ext"])) < 5 * y.std() / np.sqrt(N)
    assert r["oi"] == r["sum_y"] / N and r["is_"] == len(S) + r["oi"]


def test_mc_star_is_poisson_binomial():
    """From the centre of a star, M - 1 is the number of live leaf edges: the
    Poisson-binomial law of the leaves' probabilities."""
    probs = np.array([0.1, 0.3, 0.5, 0.8, 0.05], np.float32)
    g = star_graph(probs)
    law = np.array([1.0])
    for p in probs.astype(np.float64):
        law = np.convolve(law, [1.0 - p, p])
    N = 200_000
    r = O.mc_fixed(g, [0], qid=0, seed=SEED, stream=1, first=0, count=N, want_e=True)
    counts = np.bincount(r["y"].astype(np.int64), minlength=law.size)
    assert _chi2_pvalue(counts, law) > 1e-4
    # E: the centre's out-degree; leaves have none
    assert np.all(r["e"] == probs.size)


def test_mc_deterministic_probabilities_are_reachability():
    """With every p in {0, 1} each sample is the set reachable from S over the
    p = 1 edges (breadth-first search written here)."""
    g = chung_lu_graph(3000, 12000, 2.1, 11)
    rng = np.random.default_rng(1)
    p = (rng.random(g.m) < 0.35).astype(np.float32)
    h = g.with_p(p)
    for S in ([0], [5, 17, 400], list(range(30))):
        seen = np.zeros(h.n, bool)
        seen[S] = True
        q = list(S)
        while q:
            u = q.pop()
            for e in range(h.row_ptr[u], h.row_ptr[u + 1]):
                v = h.col[e]
                if p[e] == 1.0 and not seen[v]:
                    seen[v] = True
                    q.append(v)
        want = int(seen.sum()) - len(S)
        r = O.mc_fixed(h, S, qid=1, seed=SEED, stream=0, first=0, count=64)
        assert np.all(r["y"] == want)


def test_lemma_var_with_both_samplers():
    """Var[Z] = beta_0 Var[M] - (1 - beta_0) Ext^2 (Lemma var, Sec. 5.2), with
    Var[Z] from IICP samples and Var[M] from classic Monte-Carlo samples, and
    the IICP variance never above the Monte-Carlo one."""
    g = tiny16_graph()
    for S in ([2, 5], [0], [9]):
        ex = O.exact(g, S)
        N = 400_000
        r = O.sample_fixed(g, S, qid=8, seed=SEED, stream=0, first=0, count=N)
        mc = O.mc_fixed(g, S, qid=9, seed=SEED, stream=0, first=0, count=N)
        b0 = r["beta0"]
        z = b0 * r["y"].astype(float) + len(S)
        m = mc["y"].astype(float) + len(S)
        want = b0 * m.var() - (1.0 - b0) * ex["ext"] ** 2
        zc, mcn = z - z.mean(), m - m.mean()
        se_z = np.sqrt(max((zc ** 4).mean() - z.var() ** 2, 1e-30) / N)
        se_m = b0 * np.sqrt(max((mcn ** 4).mean() - m.var() ** 2, 1e-30) / N)
        assert abs(z.var() - want) < 5 * np.hypot(se_z, se_m), S
        assert z.var() <= m.var()


def test_mc_thread_count_and_offsets():
    g, sets, _ = make_config("er2k")
    a = O.mc_fixed(g, sets[0], 0, SEED, 0, 0, 20_000, want_e=True, nthreads=1)
    b = O.mc_fixed(g, sets[0], 0, SEED, 0, 0, 20_000, want_e=True, nthreads=3)
    np.testing.assert_array_equal(a["y"], b["y"])
    np.testing.assert_array_equal(a["e"], b["e"])
    c = O.mc_fixed(g, sets[0], 0, SEED, 0, 12_345, 100, nthreads=1)
    np.testing.assert_array_equal(c["y"], a["y"][12_345:12_445])
