"""GPU parity of the IICP sampler (Alg. 1) and its Stage-1 table against the
CPU oracle, through the C ABI.  Per-sample Y and examined-edge counts E are
integers and must match bit for bit; Stage-1 tables must match exactly.

Inputs come from oi_inputs (seeded); expected values only from oracle/.
"""
import numpy as np
import pytest

import oracle as O
from oi_inputs import (chung_lu_graph, er_graph, fig1_graph, graph_from_edges, make_config, path_graph,
                       seed_node_outdeg_ge1, star_graph, tiny16_graph, top_outdeg_seed_set, trivalency_probs,
                       uniform_seed_set, wc_probs)
from oi_inputs.configs import RUN_SEED

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_1704_04794_amd as P
    return P


def _gpu_graph(P, g):
    return P.Graph.from_inputs(g)


def _compare(P, g, S, N, first=0, stream=0, qid=0, G=None, variant=None, label=""):
    print(f"[gpu] {label} n={g.n} m={g.m} |S|={len(np.atleast_1d(S))} N={N} first={first} stream={stream} "
          f"variant={variant}", flush=True)
    own = G is None
    G = G or _gpu_graph(P, g)
    if variant is not None:
        G.tune(variant=variant)
    y, e, r = G.sample_fixed(S, N, first=first, stream=stream, query_id=qid, want_e=True)
    o = O.sample_fixed(g, S, qid, RUN_SEED, stream, first, N, want_e=True)
    if o["beta0"] == 0.0:
        assert r["beta0"] == 0.0 and r["sum_y"] == 0
        return r
    yg = y.cpu().numpy().view(np.uint32)
    eg = e.cpu().numpy().view(np.uint64)
    bad = np.flatnonzero(yg != o["y"])
    assert bad.size == 0, (label, bad[:10], yg[bad[:10]], o["y"][bad[:10]])
    np.testing.assert_array_equal(eg, o["e"])
    assert r["sum_y"] == o["sum_y"] and r["edges_examined"] == o["sum_e"]
    assert r["beta0"] == o["beta0"]
    if own:
        G.close()
    return r


def test_stage1_tables_bit_exact(P):
    cases = [(fig1_graph(), [[0], [1], [2], [0, 1]]),
             (tiny16_graph(), [[i] for i in range(16)] + [[0, 1, 2], [3, 7, 11], [5, 5, 9]])]
    g = chung_lu_graph(20000, 200000, 2.1, 7)
    g = g.with_p(trivalency_probs(g, 5))
    cases.append((g, [seed_node_outdeg_ge1(g, 3), uniform_seed_set(g, 50, 4), top_outdeg_seed_set(g, 300, 5)]))
    h = graph_from_edges(5, [0, 0, 0, 1, 1, 1], [1, 2, 3, 0, 2, 4], [0.9, 0.5, 1.0, 0.7, 0.25, 0.0])
    cases.append((h, [[0, 1], [1], [3]]))
    for g, sets in cases:
        G = _gpu_graph(P, g)
        for S in sets:
            a = G.stage1(S)
            b = O.stage1(g, S)
            assert a["l"] == b["l"] and a["beta0"] == b["beta0"]
            np.testing.assert_array_equal(a["v"], b["v"])
            np.testing.assert_array_equal(a["P"], b["P"])
            np.testing.assert_array_equal(a["cdf"], b["cdf"])
            np.testing.assert_array_equal(a["thr"], b["thr"])
        G.close()


def test_small_graphs_bit_exact(P):
    g = fig1_graph(0.3)
    for S in ([0], [1], [2], [0, 1]):
        _compare(P, g, S, 20000, label="fig1")
    _compare(P, star_graph(np.array([0.1, 0.3, 0.5, 0.8, 1.0, 0.0], np.float32)), [0], 20000, label="star")
    _compare(P, path_graph(np.array([0.9, 0.8, 0.7, 0.6, 1.0], np.float32)), [0], 20000, label="path")
    g = tiny16_graph()
    G = _gpu_graph(P, g)
    for v in range(16):
        _compare(P, g, [v], 20000, qid=v, G=G, label=f"tiny16 {v}")
    for S in ([0, 1, 2], [3, 7, 11], [2, 5, 9, 12]):
        _compare(P, g, S, 20000, qid=7, G=G, label="tiny16 multi")
    G.close()


def test_er2k_workload_bit_exact(P):
    """The ER n=2000 m=20000 weighted-cascade workload: 100,000 samples, query 0."""
    g, sets, extra = make_config("er2k")
    r = _compare(P, g, sets[0], extra["samples"], label="er2k")
    o = O.sample_fixed(g, sets[0], 0, RUN_SEED, 0, 0, extra["samples"], want_y=False)
    assert r["oi"] == o["oi"] > 0.0 and r["is_"] == o["is_"] == r["oi"] + 1


@pytest.mark.parametrize("variant,tiny", [(0, 1), (1, 1), (2, 1), (3, 1), (4, 1), (5, 1), (0, 0), (1, 0)])
def test_variants_bit_exact(P, variant, tiny):
    g = chung_lu_graph(20000, 200000, 2.1, 7)
    gw = g.with_p(wc_probs(g))
    G = _gpu_graph(P, gw)
    # the small kernel samples what it is handed (no direct hand-over), so
    # that every variant does some of the work
    G.tune(tiny=tiny, small_direct=2)
    G.timing(True)
    S1 = seed_node_outdeg_ge1(gw, 3)
    _compare(P, gw, S1, 30000, G=G, variant=variant, label=f"cl20k wc |S|=1 tiny={tiny}")
    _compare(P, gw, uniform_seed_set(gw, 20, 9), 20000, qid=3, G=G, variant=variant, label="cl20k wc |S|=20")
    t = G.timing()
    # every kernel of the pipeline finished some of the samples
    assert t["handed_large"] > 0 and t["large_y"] > 0 and t["small_y"] > 0
    if tiny:
        assert t["handed_small"] > 0 and t["tiny_y"] > 0
    else:
        assert t["tiny_y"] == 0
    G.close()
    gt = g.with_p(trivalency_probs(g, 5))
    G = _gpu_graph(P, gt)
    G.tune(tiny=tiny, small_direct=2)
    _compare(P, gt, S1, 50000, stream=1, first=123_457, G=G, variant=variant, label="cl20k tri X'")
    G.close()


def test_large_seed_sets_and_hubs(P):
    g = chung_lu_graph(20000, 200000, 2.1, 7)
    gt = g.with_p(trivalency_probs(g, 5))
    G = _gpu_graph(P, gt)
    _compare(P, gt, top_outdeg_seed_set(gt, 500, 5), 5000, qid=11, G=G, label="tri top-500")
    _compare(P, gt, uniform_seed_set(gt, 1000, 6), 5000, qid=12, G=G, label="tri uniform-1000")
    G.close()
    gw = g.with_p(wc_probs(g))
    _compare(P, gw, top_outdeg_seed_set(gw, 200, 8), 3000, qid=13, label="wc top-200")
    # a hub with 6000 out-edges reached in Stage 1: rows split over many passes
    k = 6000
    src = np.concatenate([[1], np.zeros(k, np.int64), np.arange(2, 40)])
    dst = np.concatenate([[0], np.arange(2, k + 2), np.arange(3, 41)])
    for p_hub in (0.01, 0.3):
        p = np.concatenate([[0.9], np.full(k, p_hub), np.full(38, 0.5)]).astype(np.float32)
        h = graph_from_edges(k + 2, src, dst, p)
        _compare(P, h, [1], 4000, label=f"hub p={p_hub}")


def test_cl1m_workload_sampled(P):
    """The 1M-node Chung-Lu trivalency workload at full size: a 2^22-sample
    launch on the GPU; 3,000 sample ids recomputed one by one by the oracle;
    every sample checked against 1 <= Y <= n - |S| (Lemma 2)."""
    g, sets, extra = make_config("cl1m")
    S = sets[0]
    G = _gpu_graph(P, g)
    N = 1 << 22
    print(f"[gpu] cl1m sampled N={N}", flush=True)
    y, e, r = G.sample_fixed(S, N, want_e=True)
    yg = y.cpu().numpy().view(np.uint32)
    eg = e.cpu().numpy().view(np.uint64)
    assert yg.min() >= 1 and yg.max() <= g.n - 1
    assert int(yg.sum(dtype=np.uint64)) == r["sum_y"] and int(eg.sum(dtype=np.uint64)) == r["edges_examined"]
    rng = np.random.default_rng(2)
    ids = np.sort(rng.choice(N, size=3000, replace=False))
    for i in ids:
        o = O.sample_fixed(g, S, 0, RUN_SEED, 0, int(i), 1, want_e=True, nthreads=1)
        assert yg[i] == o["y"][0] and eg[i] == o["e"][0], int(i)
    # and one contiguous block in full
    o = O.sample_fixed(g, S, 0, RUN_SEED, 0, 1_000_000, 50_000, want_e=True)
    np.testing.assert_array_equal(yg[1_000_000:1_050_000], o["y"])
    G.close()


def test_degenerate_inputs(P):
    g = tiny16_graph()
    G = _gpu_graph(P, g)
    leaf = int(np.flatnonzero(g.outdeg() == 0)[0])
    y, e, r = G.sample_fixed([leaf], 100)
    assert r["beta0"] == 0.0 and r["sum_y"] == 0
    y, e, r = G.sample_fixed([0], 0)
    assert r["sum_y"] == 0
    with pytest.raises(P.OiError):
        G.sample_fixed([16], 10)
    with pytest.raises(P.OiError):
        G.sample_fixed([], 10)
    # all nodes in S: nothing outside S to activate
    y, e, r = G.sample_fixed(list(range(16)), 10)
    assert r["beta0"] == 0.0
    G.close()
    # an empty graph and a graph without edges out of S
    h = graph_from_edges(3, [], [], [])
    H = _gpu_graph(P, h)
    assert H.sample_fixed([0], 10)[2]["beta0"] == 0.0
    H.close()


def test_few_handed_samples_go_straight_to_the_large_kernel(P):
    """A 40-leaf star at p = 0.2 from the centre: only the rare samples with
    more than 16 activated leaves leave the tiny kernel, few enough that the
    small kernel forwards them to the large kernel unprocessed.  Y and E stay
    bit-exact, and so does the backward's use of the same path."""
    import torch
    g = star_graph(np.full(40, 0.2, np.float32))
    G = _gpu_graph(P, g)
    G.timing(True)
    _compare(P, g, [0], 20000, G=G, label="star40 few hand-overs")
    t = G.timing()
    assert 0 < t["handed_small"] <= 512 and t["small_y"] == 0 and t["large_y"] > 0, t
    grad = torch.empty(g.m, dtype=torch.float32, device="cuda")
    G.backward([0], 20000, grad)
    o = O.backward(g, [0], 0, RUN_SEED, 0, 20000)
    ref = o["beta0"] * o["acc"] / 20000
    got = grad.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref)
    G.close()


def test_soft_cap_departures_bit_exact(P):
    """The large kernel's adaptive soft cap.  On this graph its mark is an
    eighth of the pool's queues (2,500 activations) and 52 of the first
    20,000 samples of this seed set pass it: after the first launch has
    counted them, the next launch sends such samples to the full-queue pass
    once they pass the mark.  Per-sample Y and E stay bit-exact with the
    oracle, and so do an RSA estimate and the backward run after it."""
    import torch
    g = chung_lu_graph(20000, 200000, 2.1, 7)
    gw = g.with_p(wc_probs(g))
    S = uniform_seed_set(gw, 5, 2)
    G = _gpu_graph(P, gw)
    G.timing(True)
    _compare(P, gw, S, 20000, G=G, label="cl20k wc soft cap, first launch")
    t = G.timing()
    assert t["left_soft"] == 0, t
    G.timing(True)
    _compare(P, gw, S, 20000, G=G, label="cl20k wc soft cap, second launch")
    t = G.timing()
    assert 0 < t["left_soft"] <= t["handed_full"], t
    a = G.estimate(S, 0.2, 1e-2, mode=0, query_id=0)
    b = O.estimate(gw, S, 0.2, 1e-2, 0, 0, RUN_SEED)
    assert a["oi"] == b["oi"] and a["T"] == b["rsa"]["T"] and a["D"] == b["rsa"]["D"]
    N = 20000
    grad = torch.empty(gw.m, dtype=torch.float32, device="cuda")
    G.backward(S, N, grad)
    o = O.backward(gw, S, 0, RUN_SEED, 0, N)
    ref = o["beta0"] * o["acc"] / N
    got = grad.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref)
    G.close()


@pytest.mark.parametrize("small_direct,qcap", [(1, 24), (2, 24), (0, 1 << 20)])
def test_routing_and_capped_queues_bit_exact(P, small_direct, qcap):
    """Routing settings do not change results: hand-overs forced through or
    around the small kernel, and large-kernel queues capped far below the
    cascades so most large samples take the second pass with n-entry queues.
    The backward under the same settings matches the oracle."""
    import torch
    g = chung_lu_graph(20000, 200000, 2.1, 7)
    gw = g.with_p(wc_probs(g))
    G = _gpu_graph(P, gw)
    G.tune(small_direct=small_direct, large_qcap=qcap)
    G.timing(True)
    S = uniform_seed_set(gw, 5, 2)
    _compare(P, gw, S, 20000, G=G, label=f"cl20k wc routing {small_direct} qcap {qcap}")
    t = G.timing()
    assert t["large_y"] > 0
    if small_direct == 1:
        assert t["small_y"] == 0
    N = 20000
    grad = torch.empty(gw.m, dtype=torch.float32, device="cuda")
    G.backward(S, N, grad)
    o = O.backward(gw, S, 0, RUN_SEED, 0, N)
    ref = o["beta0"] * o["acc"] / N
    got = grad.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref)
    G.close()


def test_single_entry_tables_bit_exact(P):
    """Seed sets whose Stage-1 table has one entry v_0 (the one-sample-per-lane
    kernel tests each sample's out-edges of v_0 in a first pass and runs the
    cascade only for samples with a live one): v_0's row inside one edge
    group, across two, four and seven groups, longer than sixteen groups,
    empty, with edges back into S, with p = 1 edges, and with several seeds.
    Every table runs under each first-level mode (the host's choice, none,
    and each pass instantiation forced), so that pending samples also start
    from the live out-edges their pass drew, including a v_0 with 20 certain
    out-edges, which overflows the per-lane list at once.  Y and E bit-exact
    against the oracle, and the estimate's sums equal."""
    rng = np.random.default_rng(11)
    n = 300
    edges = []  # (src, dst, p)
    pick = lambda: float(rng.choice([0.05, 0.2, 0.5, 1.0], p=[0.5, 0.3, 0.15, 0.05]))
    # seeds 0, 1 and 2 point only at node 3 (v_0 for S = {0}, {0, 1}, {0, 1, 2})
    for s_ in (0, 1, 2):
        edges.append((s_, 3, pick()))
    # node 3: edges back into {0, 1, 2} and out to 10 nodes (edge ids 3..15)
    for t in (0, 1, 2, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19):
        edges.append((3, t, pick()))
    # single-entry seeds a -> b, where b has d out-edges of probability q:
    # 6 mixed (misaligned), 20 mixed, none, 25 at 0.02 (seven groups, mostly
    # dead), 70 at 0.01 (more than sixteen groups), 20 certain
    for a, b, d, q in ((4, 5, 6, None), (6, 7, 20, None), (8, 9, 0, None), (20, 21, 25, 0.02), (22, 23, 70, 0.01),
                       (24, 25, 20, 1.0)):
        edges.append((a, b, pick()))
        for t in rng.choice(np.arange(30, n), size=d, replace=False):
            edges.append((b, int(t), pick() if q is None else q))
    # a random sparse remainder so that cascades continue
    for u in range(30, n):
        for t in rng.choice(n, size=3, replace=False):
            if t != u:
                edges.append((u, int(t), pick()))
    src = np.array([e[0] for e in edges])
    dst = np.array([e[1] for e in edges])
    p = np.array([e[2] for e in edges], np.float32)
    _, keep = np.unique(src * n + dst, return_index=True)
    keep = np.sort(keep)
    g = graph_from_edges(n, src[keep], dst[keep], p[keep])
    G = _gpu_graph(P, g)
    for mode in (-1, 0, 1, 2):
        P.oi_set_first_level(G.h, mode)
        for qid, S in enumerate(([0], [0, 1], [0, 1, 2], [4], [6], [8], [20], [22], [24], [3])):
            tab = O.stage1(g, S)
            r = _compare(P, g, S, 40_000, qid=qid, G=G, label=f"single-entry mode {mode} S={S} l={tab['l']}")
            _compare(P, g, S, 30_000, qid=qid, stream=1, first=987_654_321, G=G,
                     label=f"single-entry mode {mode} S={S} X'")
            if S != [3]:
                assert tab["l"] == 1 and r["l"] == 1
    P.oi_set_first_level(G.h, -1)
    a = G.estimate([0, 1], 0.1, 0.05, query_id=9)
    b = O.estimate(g, [0, 1], 0.1, 0.05, 0, 9, RUN_SEED)
    for f in ("T1", "h1", "nsigma", "D", "T", "hT"):
        assert a[f] == b["rsa"][f], (f, a[f], b["rsa"][f])
    assert a["oi"] == b["oi"]
    G.close()


def test_multi_entry_first_level_bit_exact(P):
    """Seed sets with Stage-1 tables of 2..16 entries whose samples mostly end
    at their first activated node (low probabilities), so that the tiny
    kernel runs its first-level passes over them: the selection, the later
    entries' coins and the selected node's out-edge coins are taken in the
    pass, everything else in the cascade.  Entries whose rows span more than
    sixteen groups, edges back into S, p = 1 edges, a 17-entry table (beyond
    the passes) and several seeds.  Y and E bit-exact against the oracle."""
    rng = np.random.default_rng(23)
    n = 2000
    edges = {}
    low = lambda: float(rng.choice([0.002, 0.01, 0.05, 1.0], p=[0.5, 0.35, 0.149, 0.001]))
    # seed u in 0..9 has k_u out-neighbours among 20..59 (table entries)
    sizes = [2, 3, 4, 5, 7, 8, 11, 16, 17, 6]
    for u, k in enumerate(sizes):
        for t in rng.choice(np.arange(20, 60), size=k, replace=False):
            edges[(u, int(t))] = float(rng.choice([0.003, 0.01, 0.05]))
    # rows of the entries: mostly short, a few longer than sixteen groups,
    # some edges back to the seeds
    for v in range(20, 60):
        d = 80 if v % 13 == 0 else int(rng.integers(0, 8))
        for t in rng.choice(np.arange(60, n), size=d, replace=False):
            edges[(v, int(t))] = low()
        if v % 5 == 0:
            edges[(v, int(v % 10))] = 0.5
    for u in range(60, n):
        for t in rng.choice(n, size=4, replace=False):
            if t != u:
                edges[(u, int(t))] = low()
    src = np.array([a for a, _ in edges])
    dst = np.array([b for _, b in edges])
    p = np.array(list(edges.values()), np.float32)
    g = graph_from_edges(n, src, dst, p)
    G = _gpu_graph(P, g)
    sets = [[u] for u in range(10)] + [[0, 1], [2, 3, 4]]
    # the host's choice, then the general instantiation forced on every table
    for mode in (-1, 2):
        P.oi_set_first_level(G.h, mode)
        for qid, S in enumerate(sets):
            tab = O.stage1(g, S)
            _compare(P, g, S, 40_000, qid=qid, G=G, label=f"multi-entry mode {mode} S={S} l={tab['l']}")
            _compare(P, g, S, 20_000, qid=qid, stream=1, first=555_555_555, G=G,
                     label=f"multi-entry mode {mode} S={S} X'")
    P.oi_set_first_level(G.h, -1)
    # every set in one batched estimate (one launch per round over all of
    # them), replayed by the oracle set by set
    qids = np.arange(40, 40 + len(sets), dtype=np.uint32)
    batch = G.estimate_batch([np.array(S, np.int32) for S in sets], 0.2, 0.1, query_ids=qids)
    for S, q, a in zip(sets, qids, batch):
        b = O.estimate(g, S, 0.2, 0.1, 0, int(q), RUN_SEED)
        for f in ("T1", "h1", "nsigma", "D", "T", "hT"):
            assert a[f] == b["rsa"][f], (S, f, a[f], b["rsa"][f])
        assert a["oi"] == b["oi"], S
    G.close()


def test_first_level_mode_validation(P):
    """oi_set_first_level takes -1, 0, 1 or 2."""
    g = fig1_graph()
    G = _gpu_graph(P, g)
    try:
        for bad in (-2, 3):
            with pytest.raises(P.OiError) as ei:
                P.oi_set_first_level(G.h, bad)
            assert ei.value.status == P._binding.OI_EINVAL
        for ok in (-1, 0, 1, 2):
            P.oi_set_first_level(G.h, ok)
    finally:
        G.close()
