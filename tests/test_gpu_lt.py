"""GPU parity of the LT-model sampler (oi_sample_lt) and of SIEA_LT
(OI_MODE_SIEA_LT) with the oracle (reading R17): per-sample cascade sizes and
examined edges bit for bit, RSA estimates equal, batched equal to one at a
time, invalid LT weights rejected, and new probabilities taking effect."""
import numpy as np
import pytest

import oracle as O
from oi_inputs import chung_lu_graph, graph_from_edges, make_config, uniform_seed_set, wc_probs
from oi_inputs.configs import RUN_SEED

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1704_04794_amd as P
    return P


def _compare(G, g, S, N, qid=0, stream=0, first=0, label=""):
    print(f"[gpu] lt {label} |S|={len(S)} N={N} qid={qid}", flush=True)
    y, e, r = G.sample_lt(S, N, first=first, stream=stream, query_id=qid, want_e=True)
    o = O.lt_fixed(g, S, qid, RUN_SEED, stream, first, N, want_e=True)
    yg = y.cpu().numpy().view(np.uint32)
    bad = np.flatnonzero(yg != o["y"])
    assert bad.size == 0, (label, bad[:5], yg[bad[:5]], o["y"][bad[:5]])
    assert np.array_equal(e.cpu().numpy().view(np.uint64), o["e"]), label
    assert r["sum_y"] == o["sum_y"] and r["is_"] == o["is_"] and r["oi"] == o["oi"], label
    return r


def _small_graph():
    src = [0, 0, 1, 1, 2, 2, 3, 4, 5, 5, 6, 7]
    dst = [1, 2, 2, 3, 3, 4, 5, 5, 6, 7, 7, 6]
    w = [0.6, 0.3, 0.5, 0.45, 0.35, 1.0, 0.7, 0.3, 0.4, 0.2, 0.55, 0.45]
    return graph_from_edges(8, src, dst, np.array(w, np.float32))


def test_lt_samples_bit_exact(P):
    g = _small_graph()
    G = P.Graph.from_inputs(g)
    for S in ([0], [1, 4], [2], list(range(8))):
        _compare(G, g, S, 50_000, qid=len(S), label="small")
    G.close()
    g, sets, _ = make_config("er2k")
    G = P.Graph.from_inputs(g)
    _compare(G, g, sets[0], 100_000, label="er2k")
    _compare(G, g, [3, 99, 1500], 30_000, qid=2, stream=1, first=77_777, label="er2k multi")
    G.close()
    c = chung_lu_graph(20000, 200000, 2.1, 7)
    c = c.with_p(wc_probs(c))
    G = P.Graph.from_inputs(c)
    for k, sd in ((1, 2), (5, 3), (60, 4)):
        _compare(G, c, uniform_seed_set(c, k, sd), 20_000, qid=k, label=f"cl20k wc k={k}")
    G.close()


def test_siea_lt_estimates(P):
    g, sets, _ = make_config("er2k")
    G = P.Graph.from_inputs(g)
    picks = [sets[0], np.array([17], np.int32), np.array([5, 600, 1200], np.int32)]
    batch = G.estimate_batch(picks, 0.1, 0.01, mode=P.OI_MODE_SIEA_LT)
    for q, S in enumerate(picks):
        a = G.estimate(S, 0.1, 0.01, mode=P.OI_MODE_SIEA_LT, query_id=q)
        b = O.estimate_lt(g, S, 0.1, 0.01, q, RUN_SEED)
        for f in ("T1", "h1", "nsigma", "D", "T", "hT"):
            assert a[f] == b["rsa"][f] == batch[q][f], (q, f, a[f], b["rsa"][f], batch[q][f])
        assert a["is_"] == b["is_"] == batch[q]["is_"] and a["oi"] == a["is_"] - a["k"]
    G.close()


def test_lt_weights_validated_and_updated(P):
    import torch
    bad = graph_from_edges(3, [0, 1], [2, 2], np.array([0.7, 0.6], np.float32))
    G = P.Graph.from_inputs(bad)
    y = torch.empty(8, dtype=torch.int32, device="cuda")
    with pytest.raises(P.OiError) as ei:
        P.oi_sample_lt(G.h, 0, [0], 0, 0, 8, RUN_SEED, y)
    assert ei.value.status == P._binding.OI_EINVAL
    # lower weights: valid, and the intervals follow the new probabilities
    ok = bad.with_p(np.array([0.4, 0.6], np.float32))
    G.set_probs(ok.p)
    _compare(G, ok, [0], 20_000, label="updated weights")
    G.close()
