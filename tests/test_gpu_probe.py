"""The random-gather probe reads exactly the rows it claims: on a circulant
graph where every node has out-degree d, `count` nodes give count * d edges."""
import numpy as np
import pytest

from oi_inputs import graph_from_edges

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,d,count", [(1000, 3, 1 << 16), (5000, 7, 100_003), (64, 1, 1)])
def test_gather_probe_counts_rows(n, d, count):
    import paper_1704_04794_amd as P
    src = np.repeat(np.arange(n), d)
    dst = (src + np.tile(np.arange(1, d + 1), n)) % n
    g = graph_from_edges(n, src, dst, np.full(n * d, 0.25, np.float32))
    G = P.Graph.from_inputs(g)
    print(f"[gpu] gather probe n={n} d={d} count={count}", flush=True)
    r = G.gather_probe(count, seed=7)
    assert r["edges"] == count * d
    assert r["useful_bytes"] == 16 * count + 8 * count * d
    assert r["ms"] > 0
    G.close()


@pytest.mark.parametrize("samples,gps,seed,qid", [(1000, 3, 0x17044794, 0), (4099, 1, 5, 77)])
def test_coin_probe_counts_the_edge_coins(samples, gps, seed, qid):
    """The coin probe draws the samplers' edge coins: its count of words
    below the four fixed thresholds equals the oracle's Philox count."""
    import oracle as O
    import paper_1704_04794_amd as P
    thr = np.array([0x19999999, 0x028F5C28, 0x00418937, 0x80000000], np.uint64)
    want = 0
    for s in range(samples):
        for g in range(gps):
            w = np.asarray(O.philox([g, 0, s & 0xFFFFFFFF, (s >> 32) & 0x07FFFFFF], [qid, seed]), np.uint64)
            want += int((w < thr).sum())
    G = P.Graph.from_inputs(graph_from_edges(4, [0, 1], [1, 2], np.full(2, 0.5, np.float32)))
    print(f"[gpu] coin probe samples={samples} gps={gps}", flush=True)
    r = G.coin_probe(samples, gps, seed=seed, query_id=qid)
    assert r["live"] == want and r["words"] == 4 * samples * gps and r["ms"] > 0
    with pytest.raises(P.OiError):
        G.coin_probe(0, 4)
    G.close()
