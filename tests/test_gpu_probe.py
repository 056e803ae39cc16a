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
