"""The seeded input generators: parallel block generation gives the same
graph as sequential generation, and the graphs have the recipe's shape."""
import numpy as np

from oi_inputs import chung_lu_graph


def test_chung_lu_parallel_blocks_match_sequential():
    a = chung_lu_graph(200_000, 2_000_000, 2.1, 11, block=1 << 15)
    b = chung_lu_graph(200_000, 2_000_000, 2.1, 11, block=1 << 15, workers=3)
    np.testing.assert_array_equal(a.row_ptr, b.row_ptr)
    np.testing.assert_array_equal(a.col, b.col)
    # CSR well formed: sorted unique targets per row, no self-loops
    assert a.row_ptr[0] == 0 and a.row_ptr[-1] == a.m
    src = np.repeat(np.arange(a.n), np.diff(a.row_ptr))
    assert not np.any(src == a.col)
    key = src.astype(np.int64) * a.n + a.col
    assert np.all(np.diff(key) > 0)
    assert 0.8 * 2_000_000 < a.m < 1.05 * 2_000_000
