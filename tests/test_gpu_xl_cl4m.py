"""Full-size parity on the 4M-node weighted-cascade batched workload
(Chung-Lu n = 4e6, m ~ 7e7, 4,096 seed sets of 1..1000 nodes): per-sample Y
and E of a uniform and a top-1% seed set, sampled across launches of the
sizes a batched estimate uses, bit-exact against the oracle computed one
sample at a time; and batched estimates of several sets equal to the same
sets estimated one at a time."""
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
