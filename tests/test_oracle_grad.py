"""Pins of the oracle's fp64 score-function gradient of the fixed-count
estimate beta_0 * mean(Y) of Ext(S).

The paper gives no gradient; the estimator is checked against the exact
derivative of the enumerated Ext (Ext is multilinear in each p_e, so
dExt/dp_e = Ext|_{p_e=1} - Ext|_{p_e=0}) within 4 standard errors per edge,
and against closed forms on a star (dOI/dp_i = 1) and a path.
"""
import numpy as np
import pytest

import oracle as O
from oi_inputs import graph_from_edges, path_graph, star_graph, tiny16_graph

SEED = 0x17044794


def _grad_and_se(g, S, N, qid=0):
    r = O.backward(g, S, qid, SEED, 0, N, want_sq=True)
    b0 = r["beta0"]
    mean = b0 * r["acc"] / N
    m2 = b0 * b0 * r["acc2"] / N
    se = np.sqrt(np.maximum(m2 - mean * mean, 0.0) / N)
    return mean, se


@pytest.mark.parametrize("S", [[0], [3, 7], [2, 5, 9]])
def test_gradient_matches_enumeration(S):
    g = tiny16_graph()
    exact = O.exact(g, S, want_grad=True)["grad"]
    est, se = _grad_and_se(g, S, 300_000, qid=len(S))
    es, ed = g.edges()
    # edges into S, and edges the cascade can never reveal (exact gradient 0 up
    # to the enumeration's cancellation error), get no score at all
    zero = np.isin(ed, S) | (np.abs(exact) < 1e-12)
    np.testing.assert_array_equal(est[zero], 0.0)
    z = np.abs(est - exact)[~zero] / np.maximum(se[~zero], 1e-300)
    assert z.max() < 4.0, (z.max(), np.argmax(z))


def test_gradient_star_is_one():
    probs = np.array([0.1, 0.3, 0.5, 0.8], np.float32)
    g = star_graph(probs)
    est, se = _grad_and_se(g, [0], 200_000)
    assert np.all(np.abs(est - 1.0) < 4 * se + 1e-12)


def test_gradient_path_closed_form():
    probs = np.array([0.6, 0.5, 0.8], np.float32)
    pp = probs.astype(np.float64)
    g = path_graph(probs)
    est, se = _grad_and_se(g, [0], 300_000)
    want = np.array([sum(np.prod(np.delete(pp[: k + 1], j)) for k in range(j, 3)) for j in range(3)])
    assert np.all(np.abs(est - want) < 4 * se)


def test_gradient_near_certain_and_impossible_edges():
    """Probabilities close to 1 and 0, and two seeds sharing an out-neighbour.
    (The likelihood-ratio identity needs 0 < p_e < 1: at p_e = 0 or 1 one
    outcome of the coin has probability zero and its branch is invisible to
    the score, so the estimate there is not the derivative.)"""
    src = [0, 0, 1, 1, 2, 3, 3, 4]
    dst = [2, 3, 2, 4, 5, 5, 1, 0]
    probs = np.array([0.97, 0.4, 0.3, 0.03, 0.6, 0.5, 0.7, 0.2], np.float32)
    g = graph_from_edges(6, src, dst, probs)
    S = [0, 1]
    exact = O.exact(g, S, want_grad=True)["grad"]
    est, se = _grad_and_se(g, S, 300_000)
    ok = np.abs(est - exact) < 4 * se + 1e-12
    assert ok.all(), (est, exact, se)
