"""Pins of the oracle's Stage-1 table and IICP sampler (Sec. 3.1, Alg. 1).

Pinned against: exact enumeration (beta_0 = Pr[nontrivial cascade]; the law
of Y is the law of |r_g(S)\\S| conditioned on being >= 1; Lemma 2's
Ext = beta_0 E[Y]), a brute-force enumeration of the Stage-1 coins
(Pr[A_i]), closed forms for degenerate graphs, and Lemma var (Sec. 5.2).
"""
import itertools

import numpy as np
import pytest
from scipy import stats

import oracle as O
from oi_inputs import (graph_from_edges, make_config, path_graph, star_graph, tiny16_graph)

SEED = 0x17044794


def _chi2_pvalue(counts, probs):
    counts = np.asarray(counts, float)
    exp = np.asarray(probs, float) * counts.sum()
    # merge the tail into bins with expectation >= 5
    oc, ec, acc_o, acc_e = [], [], 0.0, 0.0
    for o, e in zip(counts, exp):
        acc_o += o
        acc_e += e
        if acc_e >= 5:
            oc.append(acc_o)
            ec.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0 or acc_o > 0:
        oc[-1] += acc_o
        ec[-1] += acc_e
    ec = np.array(ec)
    ec *= np.sum(oc) / ec.sum()
    return stats.chisquare(oc, ec).pvalue


def test_beta0_matches_enumeration():
    g = tiny16_graph()
    for S in ([0], [1], [3, 7], [2, 5, 9], [12]):
        t = O.stage1(g, S)
        ex = O.exact(g, S)
        assert t["beta0"] == pytest.approx(1.0 - ex["dist"][0], rel=1e-12, abs=1e-15)
        # partition identity of Eq. pal: sum_i Pr[A_i] + prod_j (1 - P_j) = 1
        assert t["beta0"] + np.prod(1.0 - t["P"]) == pytest.approx(1.0, abs=1e-15)
        assert np.all(np.diff(t["v"]) > 0)  # ascending node ids, no repeats
        assert not np.isin(t["v"], S).any()


def test_stage1_table_hand_cases():
    # S = {0, 1}; 0->2 (0.5), 0->3 (1.0), 1->2 (0.25), 1->0 (S-internal), 0->1 (S-internal), 1->4 (0.0)
    g = graph_from_edges(5, [0, 0, 0, 1, 1, 1], [1, 2, 3, 0, 2, 4],
                         [0.9, 0.5, 1.0, 0.7, 0.25, 0.0])
    t = O.stage1(g, [1, 0, 1])          # duplicate seed is removed
    assert t["k"] == 2
    assert list(t["v"]) == [2, 3, 4]
    assert t["P"][0] == 1.0 - (1.0 - 0.5) * (1.0 - 0.25)
    assert t["P"][1] == 1.0 and t["P"][2] == 0.0
    assert list(t["thr"]) == [int(t["P"][0] * 2**32), 2**32, 0]
    # Pr[A_1] = P_1; Pr[A_2] = (1-P_1)*1; after a P=1 entry the CDF is flat
    assert t["cdf"][1] == t["P"][0]
    assert t["cdf"][2] == 1.0 and t["cdf"][3] == 1.0 and t["beta0"] == 1.0
    # a seed set without out-neighbours outside S has beta_0 = 0
    t0 = O.stage1(g, [3])
    assert t0["l"] == 0 and t0["beta0"] == 0.0


def test_first_activation_law_brute_force():
    """Pr[A_i] from enumerating the S-edge coins directly, against the table
    and against sampled selection frequencies."""
    src = [0, 0, 0, 1, 1, 2, 2]
    dst = [3, 4, 5, 3, 6, 4, 7]
    probs = np.array([0.3, 0.2, 0.6, 0.4, 0.1, 0.5, 0.35], np.float32)
    g = graph_from_edges(8, src, dst, probs)
    S = [0, 1, 2]
    t = O.stage1(g, S)
    order = list(t["v"])
    es, ed = g.edges()
    pe = g.p.astype(np.float64)
    pa = np.zeros(len(order))
    for mask in itertools.product([0, 1], repeat=g.m):
        pr = np.prod([pe[e] if mask[e] else 1 - pe[e] for e in range(g.m)])
        live = {int(ed[e]) for e in range(g.m) if mask[e]}
        for i, v in enumerate(order):
            if v in live:
                pa[i] += pr
                break
    np.testing.assert_allclose(np.diff(t["cdf"]), pa, rtol=1e-13)
    sel = O.selection(g, S, 3, SEED, 0, 0, 200_000)
    counts = np.bincount(sel, minlength=len(order))
    assert _chi2_pvalue(counts, pa / pa.sum()) > 1e-4


@pytest.mark.parametrize("S", [[0], [3, 7], [2, 5, 9], [12]])
def test_iicp_law_matches_enumeration(S):
    """The law of Y is that of |r_g(S)\\S| given >= 1 (proof of Lemma 2);
    Lemma 2's Ext = beta_0 E[Y]; and 1 <= Y <= n - |S|."""
    g = tiny16_graph()
    ex = O.exact(g, S)
    N = 200_000
    r = O.sample_fixed(g, S, qid=11, seed=SEED, stream=0, first=0, count=N)
    y = r["y"].astype(np.int64)
    assert y.min() >= 1 and y.max() <= g.n - len(S)
    law = ex["dist"][1:] / (1.0 - ex["dist"][0])
    counts = np.bincount(y, minlength=g.n + 1)[1:]
    assert _chi2_pvalue(counts, law) > 1e-4
    se = r["beta0"] * y.std() / np.sqrt(N)
    assert abs(r["beta0"] * y.mean() - ex["ext"]) < 5 * se


def test_lemma_var_identity():
    """Var[Z] = beta_0 Var[M] - (1 - beta_0) Ext^2 (Lemma var, Sec. 5.2), with
    Var[Z] from sampled IICP outputs and Var[M] from the exact law of M."""
    g = tiny16_graph()
    S = [2, 5]
    ex = O.exact(g, S)
    N = 400_000
    r = O.sample_fixed(g, S, qid=5, seed=SEED, stream=1, first=0, count=N)
    b0 = r["beta0"]
    z = b0 * r["y"].astype(float) + len(S)
    y = np.arange(ex["dist"].size)
    var_m = (ex["dist"] * y * y).sum() - ex["ext"] ** 2
    want = b0 * var_m - (1.0 - b0) * ex["ext"] ** 2
    # standard error of a sample variance ~ sqrt((m4 - s^4)/N)
    zc = z - z.mean()
    se = np.sqrt(max((zc ** 4).mean() - z.var() ** 2, 1e-30) / N)
    assert abs(z.var() - want) < 5 * se


def test_no_stage2_edges_closed_form():
    """All probabilities outside S's edges zero: the cascade stops after
    Stage 1, and Ext = sum_j P_{S,v_j} (independent first-round activations)."""
    g = tiny16_graph()
    S = [0, 1]
    es, _ = g.edges()
    p = g.p.copy()
    p[~np.isin(es, S)] = 0.0
    h = g.with_p(p)
    t = O.stage1(h, S)
    ex = O.exact(h, S)
    assert ex["ext"] == pytest.approx(t["P"].sum(), rel=1e-13)
    N = 200_000
    r = O.sample_fixed(h, S, qid=1, seed=SEED, stream=0, first=0, count=N)
    y = r["y"].astype(float)
    assert abs(r["beta0"] * y.mean() - t["P"].sum()) < 5 * r["beta0"] * y.std() / np.sqrt(N)


def test_certain_first_round_is_plain_ic():
    """An S-edge with p = 1 makes beta_0 = 1: IICP then draws plain IC
    cascades, so E[Y] = Ext exactly and the law of Y is that of M - |S|."""
    g = tiny16_graph()
    S = [int(np.argmax(g.outdeg()))]
    p = g.p.copy()
    p[g.row_ptr[S[0]]] = 1.0
    h = g.with_p(p)
    ex = O.exact(h, S)
    assert ex["dist"][0] == 0.0
    N = 200_000
    r = O.sample_fixed(h, S, qid=2, seed=SEED, stream=0, first=0, count=N)
    assert r["beta0"] == 1.0
    counts = np.bincount(r["y"].astype(np.int64), minlength=h.n + 1)[1:]
    assert _chi2_pvalue(counts, ex["dist"][1:]) > 1e-4


def test_edges_examined_on_star_and_path():
    """E counts Stage-1 entries after the selected one plus the out-degree of
    every activated node: on a star (leaves have no out-edges) E = l-1-i; on
    a path from node 0, E = Y minus one if the last node is reached."""
    probs = np.array([0.3, 0.5, 0.2, 0.7, 0.4], np.float32)
    g = star_graph(probs)
    N = 5000
    r = O.sample_fixed(g, [0], 0, SEED, 0, 0, N, want_e=True)
    sel = O.selection(g, [0], 0, SEED, 0, 0, N)
    np.testing.assert_array_equal(r["e"], (probs.size - 1 - sel).astype(np.uint64))
    h = path_graph(np.array([0.9, 0.8, 0.7, 0.6], np.float32))
    r = O.sample_fixed(h, [0], 0, SEED, 0, 0, N, want_e=True)
    y = r["y"].astype(np.int64)
    np.testing.assert_array_equal(r["e"].astype(np.int64), y - (y == 4))


def test_thread_count_and_offsets_do_not_change_samples():
    g, sets, _ = make_config("er2k")
    a = O.sample_fixed(g, sets[0], 0, SEED, 0, 0, 20_000, want_e=True, nthreads=1)
    b = O.sample_fixed(g, sets[0], 0, SEED, 0, 0, 20_000, want_e=True, nthreads=3)
    np.testing.assert_array_equal(a["y"], b["y"])
    np.testing.assert_array_equal(a["e"], b["e"])
    assert a["sum_y"] == b["sum_y"] and a["sum_e"] == b["sum_e"]
    c = O.sample_fixed(g, sets[0], 0, SEED, 0, 12_345, 100, nthreads=1)
    np.testing.assert_array_equal(c["y"], a["y"][12_345:12_445])
    # 1 <= Y <= n - |S| (Lemma 2)
    assert a["y"].min() >= 1 and a["y"].max() <= g.n - 1
    # a different query id or stream gives different draws
    d = O.sample_fixed(g, sets[0], 1, SEED, 0, 0, 2000, nthreads=1)
    e = O.sample_fixed(g, sets[0], 0, SEED, 1, 0, 2000, nthreads=1)
    assert not np.array_equal(d["y"], a["y"][:2000]) and not np.array_equal(e["y"], a["y"][:2000])
