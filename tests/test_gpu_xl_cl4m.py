"""Full-size parity on the 4M-node weighted-cascade batched workload
(Chung-Lu n = 4e6, m ~ 7e7, 4,096 seed sets of 1..1000 nodes): per-sample Y
and E of a uniform and a top-1% seed set, sampled across launches of the
sizes a batched estimate uses, bit-exact against the oracle computed one
sample at a time; complete RSA estimates of both sets at eps = 0.1 (the
workload's) and 0.05, replayed by the oracle's controller on the GPU's two
streams, with 200 random sample ids of each stream recomputed by the oracle;
and batched estimates of several sets equal to the same sets estimated one
at a time."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
from oi_inputs import make_config
from oi_inputs.configs import RUN_SEED

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    import torch
    assert torch.cuda.is_available()
    import paper_1704_04794_amd as P
    g, sets, extra = make_config("cl4m")
    print(f"[gpu] cl4m n={g.n} m={g.m}", flush=True)
    G = P.Graph.from_inputs(g)
    yield P, g, sets, extra, G
    G.close()


@pytest.mark.parametrize("which", ["uniform", "top"])
def test_sampled_outputs_bit_exact(big, which):
    import torch
    P, g, sets, extra, G = big
    qi = 0 if which == "uniform" else len(sets) // 2
    S = sets[qi]
    N = 1 << 16
    print(f"[gpu] cl4m {which} set {qi} |S|={len(S)} N={N}", flush=True)
    y, e, r = G.sample_fixed(S, N, query_id=qi, want_e=True)
    idx = np.unique(np.random.default_rng(qi).integers(0, N, 6))
    sel = torch.from_numpy(idx).cuda()
    yg = y[sel].cpu().numpy().view(np.uint32)
    eg = e[sel].cpu().numpy().view(np.uint64)
    for j, k in enumerate(idx):
        o = O.sample_fixed(g, S, qi, RUN_SEED, 0, int(k), 1, want_e=True, nthreads=1)
        assert int(o["y"][0]) == int(yg[j]) and int(o["e"][0]) == int(eg[j]), (qi, int(k))
    assert r["sum_y"] == int(y.to(dtype=torch.int64).sum().item())


def test_batched_equals_single(big):
    P, g, sets, extra, G = big
    pick = [0, 1, 2, 3]
    sub = [sets[i] for i in pick]
    q = np.array(pick, np.uint32)
    print(f"[gpu] cl4m batched vs single, sets {pick}", flush=True)
    batch = G.estimate_batch(sub, 0.25, extra["delta"], query_ids=q)
    for S, qi, b in zip(sub, pick, batch):
        a = G.estimate(S, 0.25, extra["delta"], query_id=qi)
        for f in ("oi", "is_", "T", "T1", "hT", "h1", "samples_x"):
            assert a[f] == b[f], (qi, f, a[f], b[f])


def _oracle_ids(g, S, qi, stream, ids):
    """Y of the given sample ids from the oracle, one sample per call, on the
    host's cores."""
    def one(k):
        return int(O.sample_fixed(g, S, qi, RUN_SEED, stream, int(k), 1, nthreads=1)["y"][0])
    with ThreadPoolExecutor(max_workers=min(16, O.nthreads_default())) as ex:
        return np.array(list(ex.map(one, ids)), np.int64)


RSA_FIELDS = ("T1", "h1", "nsigma", "D", "T", "hT")


@pytest.mark.parametrize("which", ["uniform", "top"])
def test_rsa_estimates_replayed_by_the_oracle(big, which):
    """RSA (Alg. 3, SOIEA) at eps = 0.1 and 0.05, delta = 1e-3: the oracle's
    controller replays each estimate on the GPU's streams X and X' (dumped
    with oi_sample_fixed, as many samples as the stopping indices need) and
    must reach every stopping index, sum and estimate; 200 random ids of each
    stream (over the longer eps = 0.05 streams) are recomputed by the
    oracle."""
    import torch
    P, g, sets, extra, G = big
    qi = 1 if which == "uniform" else len(sets) // 2 + 1
    S = sets[qi]
    delta = extra["delta"]
    streams = {}
    for eps in (0.1, 0.05):
        print(f"[gpu] cl4m {which} set {qi} |S|={len(S)} RSA eps={eps}", flush=True)
        r = G.estimate(S, eps, delta, query_id=qi)
        assert not r["gsra_only"] and r["T"] > 0
        nx, nxp = max(r["T1"], r["T"]), 2 * r["nsigma"]
        x, _, _ = G.sample_fixed(S, nx, stream=0, query_id=qi)
        xp, _, _ = G.sample_fixed(S, nxp, stream=1, query_id=qi)
        x = x.cpu().numpy().view(np.uint32)
        xp = xp.cpu().numpy().view(np.uint32)
        rep = O.rsa_arrays(x, xp, eps, delta, 1.0, float(g.n - r["k"]))
        for f in RSA_FIELDS:
            assert r[f] == rep[f], (which, eps, f, r[f], rep[f])
        assert r["mu"] == rep["mu"] and r["oi"] == r["beta0"] * rep["mu"] and r["is_"] == r["oi"] + r["k"]
        streams[eps] = (x, xp)
    x, xp = streams[0.05]
    rng = np.random.default_rng(100 + qi)
    ix = np.unique(rng.integers(0, x.size, 200))
    ixp = np.unique(rng.integers(0, xp.size, 200))
    print(f"[gpu] cl4m {which}: oracle recomputes {ix.size} + {ixp.size} sample ids", flush=True)
    assert np.array_equal(_oracle_ids(g, S, qi, 0, ix), x[ix].astype(np.int64))
    assert np.array_equal(_oracle_ids(g, S, qi, 1, ixp), xp[ixp].astype(np.int64))
