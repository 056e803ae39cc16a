"""GPU parity of the stopping-rule controller (GSRA, Alg. 2; RSA, Alg. 3) and
of SOIEA / SIEA (Algs. 4, 5): every RSA quantity (T1, h1, N_sigma, D, T, hT)
and the returned fp64 estimates must equal the oracle's, and batched
estimation must equal one-at-a-time estimation per seed set."""
import numpy as np
import pytest

import oracle as O
from oi_inputs import (chung_lu_graph, make_config, seed_node_outdeg_ge1, tiny16_graph, trivalency_probs,
                       uniform_seed_set, wc_probs)
from oi_inputs.configs import RUN_SEED

pytestmark = pytest.mark.gpu

FIELDS = ("T1", "h1", "nsigma", "D", "T", "hT", "gsra_only", "early")


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1704_04794_amd as P
    return P


def _check(P, G, g, S, eps, delta, mode, qid, label):
    print(f"[gpu] rsa {label} |S|={len(S)} eps={eps} delta={delta} mode={mode} qid={qid}", flush=True)
    a = G.estimate(S, eps, delta, mode=mode, query_id=qid)
    b = O.estimate(g, S, eps, delta, mode, qid, RUN_SEED)
    for f in FIELDS:
        assert a[f] == b["rsa"][f], (label, f, a[f], b["rsa"][f])
    assert a["mu"] == b["rsa"]["mu"] and a["mu1"] == b["rsa"]["mu1"]
    assert a["oi"] == b["oi"] and a["is_"] == b["is_"] and a["beta0"] == b["beta0"]
    assert a["k"] == b["k"]
    return a


def test_rsa_er2k(P):
    g, sets, _ = make_config("er2k")
    G = P.Graph.from_inputs(g)
    for eps, delta, mode in [(0.1, 0.01, 0), (0.1, 0.01, 1), (0.3, 0.05, 0), (0.3, 0.05, 1), (0.05, 1e-3, 0),
                             (0.2, 0.1, 1)]:
        _check(P, G, g, sets[0], eps, delta, mode, 0, "er2k")
    G.close()


def test_rsa_tiny16_all_modes(P):
    g = tiny16_graph()
    G = P.Graph.from_inputs(g)
    for S in ([0], [3, 7], [2, 5, 9], [12], [int(np.flatnonzero(g.outdeg() == 0)[0])]):
        for mode in (0, 1):
            a = _check(P, G, g, S, 0.1, 0.05, mode, 3, "tiny16")
            assert a["is_"] == a["oi"] + a["k"] if mode == 0 else a["oi"] == a["is_"] - a["k"]
    G.close()


def test_rsa_small_rounds_same_answer(P):
    """Many small rounds (crossings inside rounds, step 3 within drawn
    samples, X' split over rounds) give the same result."""
    g, sets, _ = make_config("er2k")
    G = P.Graph.from_inputs(g)
    G.tune(round_max=8192)
    for eps, delta, mode in [(0.1, 0.01, 0), (0.05, 1e-3, 1)]:
        _check(P, G, g, sets[0], eps, delta, mode, 0, "er2k rounds=8192")
    G.close()


def test_queued_rounds_same_answer(P):
    """Rounds queued before the previous one is read back (steps 2 and 3),
    also as one captured graph per round, give exactly the results of rounds
    read back one at a time, also when a sample outgrows the large kernel's
    queues and its round is run again with the full-size pass."""
    g = chung_lu_graph(20000, 200000, 2.1, 7)
    gw = g.with_p(wc_probs(g))
    rng = np.random.default_rng(11)
    sets = [uniform_seed_set(gw, int(k), int(s)) for k, s in zip(rng.integers(1, 30, 5), rng.integers(0, 1 << 30, 5))]
    keys = FIELDS + ("oi", "is_", "mu", "mu1", "samples_x", "samples_xp", "rounds", "sum_y", "edges_examined")
    for qcap in (-1, 24):
        res = {}
        # the third run starts every sample in the small kernel; the fourth
        # launches every round as one captured graph
        for key, pipe, tiny in ((0, 0, 1), (1, 1, 1), (2, 1, 0), (3, 2, 1)):
            print(f"[gpu] queued rounds pipeline={pipe} tiny={tiny} large_qcap={qcap}", flush=True)
            G = P.Graph.from_inputs(gw)
            G.tune(round_max=16384, large_qcap=qcap, pipeline=pipe, tiny=tiny)
            res[key] = (G.estimate_batch(sets, 0.2, 1e-2, mode=0, query_ids=np.arange(5, dtype=np.uint32)),
                        [G.estimate(sets[0], 0.1, 1e-2, mode=1, query_id=9)])
            if pipe == 2:  # with event timing on, rounds are issued one operation at a time
                G.timing(True)
                again = G.estimate(sets[0], 0.1, 1e-2, mode=1, query_id=9)
                tm = G.timing()
                G.timing(False)
                assert again["oi"] == res[key][1][0]["oi"] and again["T"] == res[key][1][0]["T"]
                assert tm["launches"] > 4 and tm["tiny_ms"] > 0 and tm["samples"] > 0
            G.close()
        for other in (1, 2, 3):
            for a_list, b_list in zip(res[0], res[other]):
                for a, b in zip(a_list, b_list):
                    for f in keys:
                        assert a[f] == b[f], (qcap, other, f, a[f], b[f])
        assert res[1][1][0]["rounds"] > 4
    one = res[1][1][0]
    b = O.estimate(gw, sets[0], 0.1, 1e-2, 1, 9, RUN_SEED)
    assert one["oi"] == b["oi"] and one["T"] == b["rsa"]["T"] and one["D"] == b["rsa"]["D"]


def test_rsa_chung_lu(P):
    g = chung_lu_graph(20000, 200000, 2.1, 7)
    gt = g.with_p(trivalency_probs(g, 5))
    G = P.Graph.from_inputs(gt)
    S = seed_node_outdeg_ge1(gt, 3)
    _check(P, G, gt, S, 0.2, 1e-3, 0, 0, "cl20k tri")
    _check(P, G, gt, uniform_seed_set(gt, 30, 4), 0.2, 1e-3, 1, 1, "cl20k tri |S|=30")
    G.close()
    gw = g.with_p(wc_probs(g))
    G = P.Graph.from_inputs(gw)
    _check(P, G, gw, S, 0.2, 1e-2, 0, 2, "cl20k wc")
    G.close()


def test_batched_equals_single(P):
    g = chung_lu_graph(20000, 200000, 2.1, 7)
    gw = g.with_p(wc_probs(g))
    G = P.Graph.from_inputs(gw)
    rng = np.random.default_rng(8)
    sets = [uniform_seed_set(gw, int(k), int(s)) for k, s in zip(rng.integers(1, 40, 12), rng.integers(0, 1 << 30, 12))]
    sets.append(np.array([int(np.flatnonzero(gw.outdeg() == 0)[0])], np.int32))  # beta_0 = 0
    qids = np.arange(100, 100 + len(sets), dtype=np.uint32)
    for mode in (0, 1):
        batch = G.estimate_batch(sets, 0.2, 1e-2, mode=mode, query_ids=qids)
        for q, S in enumerate(sets):
            one = G.estimate(S, 0.2, 1e-2, mode=mode, query_id=int(qids[q]))
            for f in FIELDS + ("oi", "is_", "mu", "samples_x", "samples_xp"):
                assert batch[q][f] == one[f], (q, f)
        # and the oracle agrees on a few of them
        for q in (0, 5, len(sets) - 1):
            b = O.estimate(gw, sets[q], 0.2, 1e-2, mode, int(qids[q]), RUN_SEED)
            assert batch[q]["oi"] == b["oi"] and batch[q]["T"] == b["rsa"]["T"]
    G.close()


def test_rsa_rejects_bad_parameters(P):
    g = tiny16_graph()
    G = P.Graph.from_inputs(g)
    for mode in (-1, 3):
        with pytest.raises(P.OiError):
            G.tune(pipeline=mode)
    for eps, delta in [(0.0, 0.1), (1.0, 0.1), (0.1, 0.5), (0.1, 0.0), (float("nan"), 0.1)]:
        with pytest.raises(P.OiError):
            G.estimate([0], eps, delta)
    with pytest.raises(P.OiError):
        G.estimate([0], 0.1, 0.1, mode=3)
    G.close()


def test_autotune_keeps_results(P):
    """The autotuner times every schedule on a pilot and applies the fastest;
    batched estimates before and after it are identical."""
    import numpy as np
    g = chung_lu_graph(20000, 200000, 2.1, 7)
    gw = g.with_p(wc_probs(g))
    sets = [uniform_seed_set(gw, k, 30 + k) for k in (1, 5, 40)]
    G = P.Graph.from_inputs(gw)
    before = G.estimate_batch(sets, 0.2, 0.01)
    r = G.autotune(sets, pilot=8192)
    nv = P.oi_num_variants()
    assert r["candidates"] == 2 * 2 * nv and r["seed_sets"] == 3
    assert 0 <= r["variant"] < nv and r["tiny"] in (0, 1) and r["small_direct"] in (0, 1)
    assert 0 < r["best_ms"] <= r["default_ms"]
    after = G.estimate_batch(sets, 0.2, 0.01)
    for a, b in zip(before, after):
        assert a["oi"] == b["oi"] and a["T"] == b["T"] and a["samples_x"] == b["samples_x"]
    G.close()


def test_cl1m_full_estimate_replayed_by_the_oracle(P):
    """The 1M-node single-query workload at full size, in the configuration
    the bench times (eps = 0.05, delta = 1e-6, SOIEA): the oracle draws the
    same two streams itself (as many samples as the GPU's stopping indices
    need) and replays RSA on them; every stopping index, sum and estimate
    must agree.  The GPU's counts only size the oracle's arrays: a wrong
    count leaves the oracle without the samples it needs or with a
    different answer."""
    g, sets, extra = make_config("cl1m")
    S = sets[0]
    G = P.Graph.from_inputs(g)
    print("[gpu] rsa cl1m full size", flush=True)
    a = G.estimate(S, extra["eps"], extra["delta"], mode=0, query_id=0)
    G.close()
    nx = max(a["T1"], a["T"]) + 4096
    nxp = 2 * a["nsigma"]
    print(f"[gpu] oracle draws {nx} + {nxp} samples", flush=True)
    nt = O.nthreads_default()
    x = O.sample_fixed(g, S, 0, RUN_SEED, 0, 0, nx, nthreads=nt)
    xp = O.sample_fixed(g, S, 0, RUN_SEED, 1, 0, nxp, nthreads=nt)
    b0 = x["beta0"]
    r = O.rsa_arrays(x["y"], xp["y"], extra["eps"], extra["delta"], 1.0, float(g.n - len(S)))
    del x, xp
    for f in FIELDS:
        assert a[f] == r[f], (f, a[f], r[f])
    assert a["mu"] == r["mu"] and a["oi"] == b0 * r["mu"]
