"""Full-size parity on the billion-edge weighted-cascade workload (Chung-Lu,
n = 1e8, m ~ 1.5e9): per-sample Y and E, sampled across launches of the
sizes the bench times, bit-exact against the oracle computed one sample at
a time, for one seed set of each size (1, 10, 100); the backward over all
edges for the |S| = 100 set from 1,024 samples, every edge against the fp64
oracle on the same keys; and a SIEA estimate of the |S| = 1 set at the
workload's eps = 0.05, delta = 1e-6, its stopping decisions replayed by the
oracle's controller from the GPU's integer sums (its streams, ~1e11 samples,
are too long to copy out) with 200 random ids of each stream recomputed by
the oracle."""
import time

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
    t0 = time.perf_counter()

    def progress(done, total):
        if done % 16 == 0 or done == total:
            print(f"[gpu] cl100m generated {done}/{total} blocks ({time.perf_counter() - t0:.0f}s)", flush=True)

    g, sets, extra = make_config("cl100m", progress=progress)
    print(f"[gpu] cl100m n={g.n} m={g.m} built in {time.perf_counter() - t0:.0f}s", flush=True)
    G = P.Graph.from_inputs(g)
    yield g, sets, G
    G.close()


@pytest.mark.parametrize("qi,N", [(0, 1 << 26), (1, 1 << 20), (2, 1 << 15)])
def test_sampled_outputs_bit_exact(big, qi, N):
    import torch
    g, sets, G = big
    S = sets[qi]
    print(f"[gpu] cl100m |S|={len(S)} query {qi} N={N}", flush=True)
    y, e, r = G.sample_fixed(S, N, query_id=qi, want_e=True)
    rng = np.random.default_rng(qi)
    idx = np.unique(np.concatenate([np.linspace(0, N - 1, 12).astype(np.int64), rng.integers(0, N, 12)]))
    sel = torch.from_numpy(idx).cuda()
    yg = y[sel].cpu().numpy().view(np.uint32)
    eg = e[sel].cpu().numpy().view(np.uint64)
    for j, k in enumerate(idx):
        o = O.sample_fixed(g, S, qi, RUN_SEED, 0, int(k), 1, want_e=True, nthreads=1)
        assert int(o["y"][0]) == int(yg[j]) and int(o["e"][0]) == int(eg[j]), (qi, int(k))
    # the launch's integer sums agree with its own outputs
    assert r["sum_y"] == int(y.to(dtype=torch.int64).sum().item())
    assert r["edges_examined"] == int(e.sum().item())


def test_backward_over_all_edges(big):
    import torch
    g, sets, G = big
    S = sets[2]
    N = 1024
    print(f"[gpu] cl100m backward |S|={len(S)} N={N} over {g.m} edges", flush=True)
    grad = torch.empty(g.m, dtype=torch.float32, device="cuda")
    G.backward(S, N, grad, query_id=2)
    got = grad.cpu().numpy()
    del grad
    o = O.backward(g, S, 2, RUN_SEED, 0, N, nthreads=1)
    ref = o["acc"]
    ref *= o["beta0"] / N
    assert np.count_nonzero(got) > 0
    # every edge, in slices (each entry differs from the fp64 oracle only by
    # the fp32 rounding of the output and the oracle's summation order)
    C = 1 << 27
    top = max(float(np.abs(ref[i:i + C]).max()) for i in range(0, ref.size, C))
    sq_d = sq_r = 0.0
    for i in range(0, ref.size, C):
        b = ref[i:i + C]
        d = got[i:i + C].astype(np.float64) - b
        bad = np.flatnonzero(np.abs(d) > 1e-6 * np.abs(b) + 1e-7 * top)
        assert bad.size == 0, (i + bad[:8], got[i + bad[:8]], b[bad[:8]])
        sq_d += float(d @ d)
        sq_r += float(b @ b)
    assert np.sqrt(sq_d) <= 1e-4 * np.sqrt(sq_r)


def test_siea_estimate_decisions_replayed(big):
    """SIEA (Alg. 5) of the |S| = 1 set at eps = 0.05, delta = 1e-6.  The
    oracle's controller, given the GPU's sums, must reach the same decisions:
    step 1 stops at T1 (the sum of Z reaches the threshold at T1 and not at
    T1 - 1, with Y_T1 recomputed by the oracle), N_sigma from (h1, T1), T
    from D, and the estimate from hT; 200 random ids of each stream are
    recomputed by the oracle."""
    import torch
    g, sets, G = big
    S = sets[0]
    eps, delta = 0.05, 1e-6
    print(f"[gpu] cl100m SIEA |S|=1 eps={eps} delta={delta}", flush=True)
    t = time.perf_counter()
    r = G.estimate(S, eps, delta, mode=1, query_id=0)
    print(f"[gpu] cl100m SIEA: {time.perf_counter() - t:.1f}s, T1={r['T1']} nsigma={r['nsigma']} T={r['T']}",
          flush=True)
    k, b0 = r["k"], r["beta0"]
    a, b = k + b0, k + b0 * (g.n - k)
    plan = O.rsa_plan(eps, delta, a, b, [r["h1"]], [r["T1"]], [r["D"]], scale=b0, offset=float(k))
    assert r["nsigma"] == int(plan["nsigma"][0]) and r["T"] == int(plan["T"][0])
    yT1 = int(O.sample_fixed(g, S, 0, RUN_SEED, 0, r["T1"] - 1, 1, nthreads=1)["y"][0])
    assert b0 * r["h1"] + k * r["T1"] >= plan["ups1"] > b0 * (r["h1"] - yT1) + k * (r["T1"] - 1)
    mu = (b0 * r["hT"] + k * r["T"]) / r["T"]
    assert r["mu"] == mu and r["is_"] == mu and r["oi"] == r["is_"] - k
    rng = np.random.default_rng(5)
    for stream, hi in ((0, max(r["T1"], r["T"])), (1, 2 * r["nsigma"])):
        ids = np.unique(rng.integers(0, hi, 200))
        got = []
        for i in ids:
            y, _, _ = G.sample_fixed(S, 1, first=int(i), stream=stream, query_id=0)
            got.append(int(y.item()))
        want = [int(O.sample_fixed(g, S, 0, RUN_SEED, stream, int(i), 1, nthreads=1)["y"][0]) for i in ids]
        assert got == want, stream
