"""oi_sample_fixed_noalloc (the entry point for callers that cannot allocate)
against oi_sample_fixed, through the C ABI: per-sample Y and E and the sums
bit for bit, on two calls in a row (the second smaller, with another seed
set), on workloads that reach each sampling tier, including the pass for
samples that outgrow the main pool's queues."""
import ctypes as C

import numpy as np
import pytest

from oi_inputs import chung_lu_graph, graph_from_edges, make_config, uniform_seed_set, wc_probs
from oi_inputs.configs import RUN_SEED

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1704_04794_amd as P
    return P


def _run(P, G, S, qid, first, count, noalloc):
    import torch
    y = torch.full((count,), -1, dtype=torch.int32, device="cuda")
    e = torch.full((count,), -1, dtype=torch.int64, device="cuda")
    fn = P.oi_sample_fixed_noalloc if noalloc else P.oi_sample_fixed
    r = fn(G.h, qid, S, 0, first, count, RUN_SEED, y, e)
    torch.cuda.synchronize()
    return y.cpu().numpy(), e.cpu().numpy(), r


def _same(a, b, label):
    ya, ea, ra = a
    yb, eb, rb = b
    assert np.array_equal(ya, yb), label
    assert np.array_equal(ea, eb), label
    for f in ("sum_y", "edges_examined", "beta0", "k", "l", "oi", "is_", "mu", "T", "hT", "samples_x"):
        assert ra[f] == rb[f], (label, f, ra[f], rb[f])


def _star(n_leaves):
    src = np.zeros(n_leaves, np.int64)
    dst = np.arange(1, n_leaves + 1, dtype=np.int64)
    return graph_from_edges(n_leaves + 1, src, dst, np.ones(n_leaves, np.float32))


def test_noalloc_matches_oi_sample_fixed(P):
    import torch
    cases = []
    g, sets, _ = make_config("er2k")
    cases.append(("er2k", g, [sets[0], [5, 17]], [100_000, 30_000]))
    c = chung_lu_graph(20000, 200000, 2.1, 7)
    c = c.with_p(wc_probs(c))
    cases.append(("cl20k wc", c, [uniform_seed_set(c, 5, 2), uniform_seed_set(c, 1, 3)], [20_000, 7_000]))
    # every sample activates all 99,999 leaves: past the main pool's 2^16-entry queues
    cases.append(("star 1e5 p=1", _star(99_999), [[0], [0]], [24, 5]))
    for label, g, ss, counts in cases:
        G = P.Graph.from_inputs(g)
        for call, (S, N) in enumerate(zip(ss, counts)):
            print(f"[gpu] noalloc {label} call {call} |S|={len(S)} N={N}", flush=True)
            qid = 3 + call
            a = _run(P, G, S, qid, 11, N, True)
            b = _run(P, G, S, qid, 11, N, False)
            _same(a, b, f"{label} call {call}")
            assert a[2]["rounds"] >= 1 and (a[0] >= 1).all()
        G.close()


def test_noalloc_allocates_no_device_memory(P):
    import torch
    g, sets, _ = make_config("er2k")
    G = P.Graph.from_inputs(g)
    S = sets[0]
    _run(P, G, S, 0, 0, 50_000, True)  # first use: code objects and the scratch array are in place after it
    y = torch.empty(50_000, dtype=torch.int32, device="cuda")
    import gc
    gc.collect()  # graphs of earlier tests free their memory now, not inside the window
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for first in (0, 50_000, 7):
        P.oi_sample_fixed_noalloc(G.h, 0, S, 0, first, 50_000, RUN_SEED, y, None)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    # an allocation would lower the free memory; nothing else in this
    # process allocates inside the window
    assert free1 >= free0, (free0, free1)
    G.close()


def test_noalloc_limits(P):
    import torch
    y = torch.empty(16, dtype=torch.int32, device="cuda")
    g, sets, _ = make_config("er2k")
    G = P.Graph.from_inputs(g)
    with pytest.raises(P.OiError) as ei:  # y_out is required
        P.oi_sample_fixed_noalloc(G.h, 0, sets[0], 0, 0, 16, RUN_SEED, None, None)
    assert ei.value.status == P._binding.OI_EINVAL
    G.close()
    n = (1 << 22) + 1  # one node more than the scratch array is sized for
    big = P.Graph(n, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    with pytest.raises(P.OiError) as ei:
        P.oi_sample_fixed_noalloc(big.h, 0, [0], 0, 0, 16, RUN_SEED, y, None)
    assert ei.value.status == P._binding.OI_ERANGE
    big.close()
