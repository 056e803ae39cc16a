"""GPU parity of Stage-1 skip sampling (long Stage-1 tables; the
specification in include/oi.h, oi_set_stage1_skip) with the oracle: per-sample
Y and E bit for bit, the backward per edge, and an RSA estimate, with the
threshold lowered and the density test off so that tables of a few hundred
dense entries use it; and the density test's decision at the default
settings, taken alike on both sides (the configured workloads' long tables
are dense and keep their plain coins; they are covered by the 4M-node
tests)."""
import numpy as np
import pytest

import oracle as O
from oi_inputs import chung_lu_graph, star_graph, uniform_seed_set, wc_probs
from oi_inputs.configs import RUN_SEED

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1704_04794_amd as P
    return P


@pytest.fixture
def skip65():
    O.set_stage1_skip(65)
    O.set_stage1_skip_cost(0)
    yield 65
    O.set_stage1_skip(4096)
    O.set_stage1_skip_cost(8)


def _graph(P, g, min_l):
    G = P.Graph.from_inputs(g)
    P.oi_set_stage1_skip(G.h, min_l)
    P.oi_set_stage1_skip_cost(G.h, 0)
    return G


def _compare(G, g, S, N, qid, stream=0, first=0, label=""):
    print(f"[gpu] skip {label} |S|={len(S)} N={N} qid={qid}", flush=True)
    y, e, r = G.sample_fixed(S, N, first=first, stream=stream, query_id=qid, want_e=True)
    o = O.sample_fixed(g, S, qid, RUN_SEED, stream, first, N, want_e=True)
    yg = y.cpu().numpy().view(np.uint32)
    bad = np.flatnonzero(yg != o["y"])
    assert bad.size == 0, (label, bad[:5], yg[bad[:5]], o["y"][bad[:5]])
    assert np.array_equal(e.cpu().numpy().view(np.uint64), o["e"]), label
    assert r["sum_y"] == o["sum_y"] and r["oi"] == o["oi"], label
    return r, yg


def _star():
    rng = np.random.default_rng(4)
    p = rng.uniform(0.0, 0.2, 700)
    heavy = rng.random(700) < 0.08
    p[heavy] = rng.uniform(0.5, 0.99, heavy.sum())
    p[rng.random(700) < 0.05] = 0.0
    p[rng.random(700) < 0.01] = 1.0
    return star_graph(p.astype(np.float32))


def test_skip_star_bit_exact(P, skip65):
    g = _star()
    G = _graph(P, g, skip65)
    r, _ = _compare(G, g, [0], 50_000, qid=3, label="star 700")
    assert r["l"] == 700
    _compare(G, g, [0], 20_000, qid=4, stream=1, first=123_456_789, label="star 700 stream 1")
    # the default threshold keeps these tables on their plain coins, on both sides
    P.oi_set_stage1_skip(G.h, 4096)
    O.set_stage1_skip(4096)
    _compare(G, g, [0], 20_000, qid=3, label="star 700 plain")
    G.close()


def test_skip_chung_lu_forward_backward_and_rsa(P, skip65):
    import torch
    c = chung_lu_graph(20000, 200000, 2.1, 7)
    c = c.with_p(wc_probs(c))
    G = _graph(P, c, skip65)
    for k, sd in ((60, 9), (200, 10)):
        S = uniform_seed_set(c, k, sd)
        _compare(G, c, S, 20_000, qid=k, label=f"cl20k wc k={k}")
    S = uniform_seed_set(c, 60, 9)
    # backward: every edge against the fp64 oracle on the same keys
    N = 20_000
    grad = torch.empty(c.m, dtype=torch.float32, device="cuda")
    G.backward(S, N, grad, query_id=5)
    got = grad.cpu().numpy().astype(np.float64)
    o = O.backward(c, S, 5, RUN_SEED, 0, N)
    ref = o["beta0"] * o["acc"] / N
    tol = 1e-6 * np.abs(ref) + 1e-7 * np.abs(ref).max()
    bad = np.flatnonzero(np.abs(got - ref) > tol)
    assert bad.size == 0, (bad[:5], got[bad[:5]], ref[bad[:5]])
    # an RSA estimate drawing skip-sampled samples on both streams
    a = G.estimate(S, 0.2, 0.05, query_id=6)
    b = O.estimate(c, S, 0.2, 0.05, 0, 6, RUN_SEED)
    for f in ("T1", "h1", "nsigma", "D", "T", "hT"):
        assert a[f] == b["rsa"][f], (f, a[f], b["rsa"][f])
    assert a["oi"] == b["oi"]
    G.close()


def test_skip_noalloc_matches(P, skip65):
    import torch
    g = _star()
    G = _graph(P, g, skip65)
    N = 30_000
    y1 = torch.empty(N, dtype=torch.int32, device="cuda")
    r1 = P.oi_sample_fixed_noalloc(G.h, 7, [0], 0, 0, N, RUN_SEED, y1, None)
    y2, _, r2 = G.sample_fixed([0], N, query_id=7)
    assert torch.equal(y1, y2) and r1["sum_y"] == r2["sum_y"]
    G.close()


@pytest.mark.parametrize("p", [0.027, 0.0275, "mixed"])
def test_density_test_agrees_with_the_oracle(P, p):
    """Stars of 4096 leaves with every P_j = p, at the default settings
    (tables from 4096 entries, cost 8): the density test skip-samples the
    first (8 W = 8 (16 + 4096 p) = 1013 <= 1024) and not the second (1029),
    and skip-samples a star of 2048 heavy (0.9) and 2048 light (0.02)
    leaves, whose heavy entries do not count; both sides take the same
    decision, so the samples agree bit for bit."""
    if p == "mixed":
        q = np.full(4096, 0.02, np.float32)
        q[::2] = 0.9
    else:
        q = np.full(4096, p, np.float32)
    g = star_graph(q)
    G = P.Graph.from_inputs(g)
    try:
        r, _ = _compare(G, g, [0], 1 << 14, qid=11, label=f"density test p={p}")
        assert r["l"] == 4096
    finally:
        G.close()


def test_density_cost_validation(P):
    """oi_set_stage1_skip_cost takes a finite, non-negative ratio."""
    g = star_graph(np.full(8, 0.1, np.float32))
    G = P.Graph.from_inputs(g)
    try:
        for bad in (-1.0, float("nan"), float("inf")):
            with pytest.raises(P.OiError) as ei:
                P.oi_set_stage1_skip_cost(G.h, bad)
            assert ei.value.status == P._binding.OI_EINVAL
        P.oi_set_stage1_skip_cost(G.h, 0.0)
        P.oi_set_stage1_skip_cost(G.h, 8.0)
    finally:
        G.close()
