"""Pins of the oracle's exact enumeration and random-number generator.

The enumeration is the plain definition Ext(S) = sum_g |r_g(S) \\ S| Pr[g]
(Sec. 2); these tests tie it to values the paper prints (Fig. 1 and the
non-monotonicity paragraph of Sec. 2.2), to closed forms on stars, paths
and out-trees, to finite differences, and to the submodularity of Lemma 1.
"""
import itertools
import os

import numpy as np
import pytest

import oracle as O
from oi_inputs import (fig1_graph, graph_from_edges, out_tree_graph, path_graph, star_graph,
                       tiny16_graph)


def test_philox_known_answers(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = O.philox(r[0:4], r[4:6])
        assert [int(x) for x in out] == r[6:10]


def test_fig1_printed_values(golden_dir):
    names = {"u": 0, "v": 1, "w": 2, "x": 3}
    g = fig1_graph(0.1)
    with open(os.path.join(golden_dir, "fig1_values.txt")) as f:
        rows = [line.split() for line in f if line.strip() and not line.startswith("#")]
    assert len(rows) == 5
    for s, inf, ext in rows:
        S = [names[c] for c in s.split(",")]
        r = O.exact(g, S)
        # p is stored as fp32 0.1; the printed values have two decimals
        assert r["ext"] == pytest.approx(float(ext), abs=5e-8)
        if inf != "-":
            assert r["ext"] + len(S) == pytest.approx(float(inf), abs=5e-8)
    # the printed closed forms for u and v: p + 2p^2 and 2p
    p = float(np.float32(0.1))
    assert O.exact(g, [0])["ext"] == pytest.approx(p + 2 * p * p, rel=1e-15)
    assert O.exact(g, [1])["ext"] == pytest.approx(2 * p, rel=1e-15)


def test_star_closed_form():
    probs = np.array([0.1, 0.25, 0.5, 0.75, 1.0, 0.0], np.float32)
    g = star_graph(probs)
    r = O.exact(g, [0], want_grad=True)
    assert r["ext"] == pytest.approx(float(probs.astype(np.float64).sum()), rel=1e-14)
    np.testing.assert_allclose(r["grad"], np.ones(probs.size), rtol=1e-13)
    # a leaf as seed: nothing reachable
    assert O.exact(g, [3])["ext"] == 0.0


def test_path_closed_form():
    probs = np.array([0.9, 0.5, 0.3, 0.7, 0.2], np.float32)
    pp = probs.astype(np.float64)
    g = path_graph(probs)
    r = O.exact(g, [0], want_grad=True)
    want = sum(np.prod(pp[: k + 1]) for k in range(pp.size))
    assert r["ext"] == pytest.approx(want, rel=1e-14)
    for j in range(pp.size):
        gj = sum(np.prod(np.delete(pp[: k + 1], j)) for k in range(j, pp.size))
        assert r["grad"][j] == pytest.approx(gj, rel=1e-13)
    # seed in the middle: only the tail counts
    assert O.exact(g, [2])["ext"] == pytest.approx(pp[2] + pp[2] * pp[3] + pp[2] * pp[3] * pp[4], rel=1e-14)


def test_out_tree_closed_form():
    parent = [0, 0, 1, 1, 2, 4, 4, 0]
    probs = np.array([0.3, 0.6, 0.5, 0.2, 0.9, 0.4, 0.7, 0.1], np.float32)
    g = out_tree_graph(parent, probs)
    pp = probs.astype(np.float64)
    # OI(root) = sum over non-root nodes of the product of edge probabilities on the root path
    reach = np.zeros(len(parent) + 1)
    reach[0] = 1.0
    for i, par in enumerate(parent, start=1):
        reach[i] = reach[par] * pp[i - 1]
    assert O.exact(g, [0])["ext"] == pytest.approx(reach[1:].sum(), rel=1e-14)
    # seed set {0, 2}: node 2's subtree is counted from 2 directly, node 2 itself excluded
    r2 = np.zeros(len(parent) + 1)
    r2[0] = r2[2] = 1.0
    for i, par in enumerate(parent, start=1):
        if i != 2:
            r2[i] = r2[par] * pp[i - 1]
    want = r2.sum() - 2.0
    assert O.exact(g, [0, 2])["ext"] == pytest.approx(want, rel=1e-14)


def test_brute_force_python_small():
    """Independent pure-Python enumeration on a 5-node, 7-edge graph with a
    cycle and an edge into S."""
    src = [0, 0, 1, 2, 3, 3, 4]
    dst = [1, 2, 3, 3, 4, 0, 1]
    probs = np.array([0.3, 0.6, 0.5, 0.45, 0.8, 0.35, 0.25], np.float32)
    g = graph_from_edges(5, src, dst, probs)
    s_sorted, d_sorted = g.edges()
    pe = g.p.astype(np.float64)
    for S in ([0], [1], [0, 3], [2, 4]):
        tot = 0.0
        for mask in itertools.product([0, 1], repeat=g.m):
            pr = np.prod([pe[e] if mask[e] else 1 - pe[e] for e in range(g.m)])
            reach = set(S)
            changed = True
            while changed:
                changed = False
                for e in range(g.m):
                    if mask[e] and s_sorted[e] in reach and d_sorted[e] not in reach:
                        reach.add(int(d_sorted[e]))
                        changed = True
            tot += pr * (len(reach) - len(S))
        assert O.exact(g, S)["ext"] == pytest.approx(tot, rel=1e-13)


def test_gradient_is_exact_difference():
    """Ext is multilinear in each p_e, so dExt/dp_e = Ext|_{p_e=1} - Ext|_{p_e=0}."""
    g = tiny16_graph(seed=7, n=10, m=16)
    S = [int(np.argmax(g.outdeg()))]
    r = O.exact(g, S, want_grad=True)
    for e in range(g.m):
        p1 = g.p.copy()
        p1[e] = 1.0
        p0 = g.p.copy()
        p0[e] = 0.0
        diff = O.exact(g.with_p(p1), S)["ext"] - O.exact(g.with_p(p0), S)["ext"]
        assert r["grad"][e] == pytest.approx(diff, rel=1e-10, abs=1e-13)


def test_submodular_and_non_monotone():
    """Lemma 1 (submodularity of Ext) on a random 10-node graph; non-monotonicity
    as in Sec. 2.2."""
    g = tiny16_graph(seed=11, n=10, m=18)
    rng = np.random.default_rng(5)
    for _ in range(40):
        T = sorted(rng.choice(10, size=4, replace=False).tolist())
        S = T[:2]
        x = int(rng.choice([v for v in range(10) if v not in T]))
        f = lambda A: O.exact(g, A)["ext"]  # noqa: E731
        assert f(S + [x]) - f(S) >= f(T + [x]) - f(T) - 1e-12
    # non-monotone on Fig. 1: adding w lowers Ext, adding v raises it
    h = fig1_graph(0.1)
    assert O.exact(h, [0, 2])["ext"] < O.exact(h, [0])["ext"] < O.exact(h, [0, 1])["ext"]


def test_exact_distribution_sums_to_one():
    g = tiny16_graph()
    for S in ([0], [3, 7]):
        r = O.exact(g, S)
        assert r["dist"].sum() == pytest.approx(1.0, abs=1e-12)
        y = np.arange(r["dist"].size)
        assert (r["dist"] * y).sum() == pytest.approx(r["ext"], rel=1e-12)
