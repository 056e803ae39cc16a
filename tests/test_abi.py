"""The HIP library builds, loads and exports every symbol include/oi.h declares;
host-side validation rejects malformed input before touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oi.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(oi_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("oi_graph_create", "oi_graph_destroy", "oi_sample_fixed", "oi_estimate", "oi_estimate_batch",
                 "oi_backward", "oi_stage1_table", "oi_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1704_04794_amd import _binding
    lib = C.CDLL(_binding.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_library_is_not_the_oracle():
    """The product library must not link or embed the oracle."""
    from paper_1704_04794_amd import _binding
    data = open(_binding.LIB_PATH, "rb").read()
    assert b"oo_rsa" not in data and b"oo_sample_fixed" not in data and b"liboi_oracle" not in data


def test_malformed_graphs_are_rejected_on_the_host():
    import paper_1704_04794_amd as P
    rp = np.array([0, 1, 2, 2], np.int64)
    col = np.array([1, 2], np.int32)
    p = np.array([0.5, 0.5], np.float32)
    bad = [
        (3, rp, np.array([1, 3], np.int32), p),          # target out of range
        (3, rp, col, np.array([0.5, 1.5], np.float32)),  # probability above 1
        (3, rp, col, np.array([0.5, np.nan], np.float32)),
        (3, np.array([0, 2, 1, 2], np.int64), col, p),   # decreasing row_ptr
        (3, np.array([1, 1, 2, 2], np.int64), col, p),   # row_ptr[0] != 0
        (0, np.array([0], np.int64), col[:0], p[:0]),    # n = 0
    ]
    with pytest.raises(P.OiError) as ei:                 # more edges than 32-bit edge ids allow
        P.oi_graph_create(3, 1 << 32, rp, col, p)
    assert ei.value.status == P._binding.OI_EINVAL
    for n, r, c, q in bad:
        with pytest.raises(P.OiError) as ei:
            P.oi_graph_create(n, c.size, r, c, q)
        assert ei.value.status == P._binding.OI_EINVAL


def test_variants_are_described():
    import paper_1704_04794_amd as P
    nv = P.oi_num_variants()
    assert nv >= 1
    for v in range(nv):
        info = P.oi_variant_info(v)
        # the LDS set of a slot keeps its load factor at most 1/2
        cmax = info["ring_cap"] // info["slots_per_wave"] - 1
        assert 2 * cmax <= info["hash_cap"]
    with pytest.raises(P.OiError):
        P.oi_variant_info(nv)


def test_null_handles_are_rejected():
    """Entry points given no graph fail with OI_EINVAL instead of touching a GPU."""
    import paper_1704_04794_amd as P
    for call in (lambda: P.oi_gather_probe(None, 1024),
                 lambda: P.oi_coin_probe(None, 1024, 4),
                 lambda: P.oi_timing_get(None),
                 lambda: P.oi_set_tuning(None, 0),
                 lambda: P.oi_set_routing(None, 0),
                 lambda: P.oi_set_pipeline(None, 1),
                 lambda: P.oi_autotune(None, np.array([0, 1], np.int64), np.array([0], np.int32),
                                       np.array([0], np.uint32), 4096, 1)):
        with pytest.raises(P.OiError) as ei:
            call()
        assert ei.value.status == P._binding.OI_EINVAL
