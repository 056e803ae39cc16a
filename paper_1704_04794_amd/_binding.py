"""ctypes binding of include/oi.h.

Argument marshalling only: every function forwards to the C entry point of
the same name in liboi_hip.so; all computation happens in the library's HIP
kernels.  Arrays may be numpy arrays (host memory) or torch tensors; device
buffers must be CUDA (HIP) tensors of the graph's GPU.  If the library has
not been built this module raises at import time: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboi_hip.so")

OI_OK, OI_EINVAL, OI_ERANGE, OI_ENOMEM, OI_EHIP, OI_ESTATE = 0, -1, -2, -3, -4, -5
OI_MODE_SOIEA, OI_MODE_SIEA, OI_MODE_SIEA_LT = 0, 1, 2
OI_PARAM_P, OI_PARAM_THETA = 0, 1


class oi_result(C.Structure):
    _fields_ = [
        ("oi", C.c_double), ("is_", C.c_double), ("beta0", C.c_double), ("mu", C.c_double),
        ("mu1", C.c_double),
        ("T1", C.c_uint64), ("h1", C.c_uint64), ("nsigma", C.c_uint64), ("D_lo", C.c_uint64),
        ("D_hi", C.c_uint64), ("T", C.c_uint64), ("hT", C.c_uint64),
        ("samples_x", C.c_uint64), ("samples_xp", C.c_uint64), ("sum_y", C.c_uint64),
        ("edges_examined", C.c_uint64), ("k", C.c_int64), ("l", C.c_int64),
        ("gsra_only", C.c_int32), ("early", C.c_int32), ("status", C.c_int32), ("rounds", C.c_int32),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["D"] = (int(self.D_hi) << 64) | int(self.D_lo)
        return d


class oi_autotune_result(C.Structure):
    _fields_ = [("variant", C.c_int32), ("tiny", C.c_int32), ("small_direct", C.c_int32),
                ("candidates", C.c_int32), ("seed_sets", C.c_int32), ("pad", C.c_int32),
                ("best_ms", C.c_double), ("default_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class oi_timing(C.Structure):
    _fields_ = [
        ("tiny_ms", C.c_double), ("small_ms", C.c_double), ("large_ms", C.c_double),
        ("launches", C.c_uint64), ("samples", C.c_uint64), ("handed_small", C.c_uint64),
        ("handed_large", C.c_uint64), ("tiny_y", C.c_uint64), ("tiny_edges", C.c_uint64),
        ("small_y", C.c_uint64), ("small_edges", C.c_uint64), ("large_y", C.c_uint64),
        ("large_edges", C.c_uint64), ("handed_full", C.c_uint64), ("left_soft", C.c_uint64),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class OiError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} failed ({status}): {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1704_04794_amd.build`")
    # torch first: its HIP runtime is then the one the library binds to, so a
    # process has a single runtime, and device pointers and streams pass
    # between torch and the library unchanged
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    i64, u64, u32, i32, dbl, vp, ci = C.c_int64, C.c_uint64, C.c_uint32, C.c_int32, C.c_double, C.c_void_p, C.c_int
    P = C.POINTER
    sig = {
        "oi_graph_create": [i64, i64, vp, vp, vp, ci, vp, P(vp)],
        "oi_graph_set_probs": [vp, vp, ci],
        "oi_set_stream": [vp, vp],
        "oi_graph_set_theta": [vp, vp, ci],
        "oi_graph_get_probs": [vp, vp],
        "oi_stage1_table": [vp, vp, i64, i64, P(i64), P(dbl), vp, vp, vp, vp],
        "oi_sample_fixed": [vp, u32, vp, i64, ci, u64, u64, u32, vp, vp, P(oi_result)],
        "oi_sample_fixed_noalloc": [vp, u32, vp, i64, ci, u64, u64, u32, vp, vp, P(oi_result)],
        "oi_sample_mc": [vp, u32, vp, i64, ci, u64, u64, u32, vp, vp, P(oi_result)],
        "oi_sample_lt": [vp, u32, vp, i64, ci, u64, u64, u32, vp, vp, P(oi_result)],
        "oi_estimate": [vp, u32, vp, i64, dbl, dbl, ci, u32, P(oi_result)],
        "oi_estimate_batch": [vp, i32, vp, vp, vp, dbl, dbl, ci, u32, vp],
        "oi_backward": [vp, u32, vp, i64, u64, u64, u32, vp, ci, dbl, vp],
        "oi_timing_enable": [vp, ci],
        "oi_timing_get": [vp, P(oi_timing)],
        "oi_set_tuning": [vp, ci, ci, ci, ci, i64],
        "oi_variant_info": [ci, P(ci), P(ci), P(ci), P(ci)],
        "oi_gather_probe": [vp, u64, u32, P(u64), P(u64), P(dbl)],
        "oi_coin_probe": [vp, u64, u32, u32, u32, P(u64), P(dbl)],
        "oi_set_routing": [vp, ci, i64],
        "oi_set_pipeline": [vp, ci],
        "oi_set_stage1_skip": [vp, i64],
        "oi_set_stage1_skip_cost": [vp, C.c_double],
        "oi_set_first_level": [vp, C.c_int],
        "oi_autotune": [vp, i32, vp, vp, vp, u64, u32, P(oi_autotune_result)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ci
    L.oi_graph_destroy.argtypes = [vp]
    L.oi_graph_destroy.restype = None
    L.oi_num_variants.argtypes = []
    L.oi_num_variants.restype = ci
    L.oi_last_error.argtypes = []
    L.oi_last_error.restype = C.c_char_p
    return L


_lib = _load()


def lib():
    return _lib


def oi_last_error() -> str:
    return _lib.oi_last_error().decode(errors="replace")


def _check(fn, st):
    if st != OI_OK:
        raise OiError(fn, st, oi_last_error())


def _ptr(x):
    """Raw address of a numpy array or torch tensor (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return int(x.data_ptr())


def _host(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _stream_handle(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except Exception:  # pragma: no cover
            pass
        return None
    return getattr(stream, "cuda_stream", stream)


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def oi_graph_create(n, m, row_ptr, col, p, device_ptrs=0, hip_stream=None):
    h = C.c_void_p()
    _check("oi_graph_create", _lib.oi_graph_create(int(n), int(m), _ptr(row_ptr), _ptr(col), _ptr(p),
                                                    int(device_ptrs), _stream_handle(hip_stream), C.byref(h)))
    return h


def oi_graph_set_probs(g, p, device_ptr=0):
    _check("oi_graph_set_probs", _lib.oi_graph_set_probs(g, _ptr(p), int(device_ptr)))


def oi_graph_set_theta(g, theta, device_ptr=0):
    _check("oi_graph_set_theta", _lib.oi_graph_set_theta(g, _ptr(theta), int(device_ptr)))


def oi_graph_get_probs(g, m):
    out = np.zeros(int(m), np.float32)
    _check("oi_graph_get_probs", _lib.oi_graph_get_probs(g, _ptr(out)))
    return out


def oi_set_stream(g, hip_stream):
    _check("oi_set_stream", _lib.oi_set_stream(g, _stream_handle(hip_stream)))


def oi_graph_destroy(g):
    _lib.oi_graph_destroy(g)


def oi_stage1_table(g, seeds, cap=1 << 24):
    s = _host(seeds, np.int32)
    l = C.c_int64()
    b0 = C.c_double()
    _check("oi_stage1_table", _lib.oi_stage1_table(g, _ptr(s), s.size, 0, C.byref(l), C.byref(b0),
                                                    None, None, None, None))
    L = l.value
    v = np.zeros(L, np.int32)
    P = np.zeros(L, np.float64)
    cdf = np.zeros(L + 1, np.float64)
    thr = np.zeros(L, np.uint64)
    if L <= cap:
        _check("oi_stage1_table", _lib.oi_stage1_table(g, _ptr(s), s.size, L, C.byref(l), C.byref(b0),
                                                        _ptr(v), _ptr(P), _ptr(cdf), _ptr(thr)))
    return dict(l=L, beta0=b0.value, v=v, P=P, cdf=cdf, thr=thr)


def oi_sample_fixed(g, query_id, seeds, stream, first, count, run_seed, y_out=None, e_out=None):
    s = _host(seeds, np.int32)
    r = oi_result()
    _check("oi_sample_fixed", _lib.oi_sample_fixed(g, int(query_id), _ptr(s), s.size, int(stream), int(first),
                                                    int(count), int(run_seed), _ptr(y_out), _ptr(e_out),
                                                    C.byref(r)))
    return r.as_dict()


def oi_sample_mc(g, query_id, seeds, stream, first, count, run_seed, y_out=None, e_out=None):
    s = _host(seeds, np.int32)
    r = oi_result()
    _check("oi_sample_mc", _lib.oi_sample_mc(g, int(query_id), _ptr(s), s.size, int(stream), int(first),
                                              int(count), int(run_seed), _ptr(y_out), _ptr(e_out), C.byref(r)))
    return r.as_dict()


def oi_sample_lt(g, query_id, seeds, stream, first, count, run_seed, y_out=None, e_out=None):
    s = _host(seeds, np.int32)
    r = oi_result()
    _check("oi_sample_lt", _lib.oi_sample_lt(g, int(query_id), _ptr(s), s.size, int(stream), int(first),
                                              int(count), int(run_seed), _ptr(y_out), _ptr(e_out), C.byref(r)))
    return r.as_dict()


def oi_sample_fixed_noalloc(g, query_id, seeds, stream, first, count, run_seed, y_out, e_out=None):
    s = _host(seeds, np.int32)
    r = oi_result()
    _check("oi_sample_fixed_noalloc", _lib.oi_sample_fixed_noalloc(g, int(query_id), _ptr(s), s.size, int(stream),
                                                                    int(first), int(count), int(run_seed),
                                                                    _ptr(y_out), _ptr(e_out), C.byref(r)))
    return r.as_dict()


def oi_estimate(g, query_id, seeds, eps, delta, mode, run_seed):
    s = _host(seeds, np.int32)
    r = oi_result()
    _check("oi_estimate", _lib.oi_estimate(g, int(query_id), _ptr(s), s.size, float(eps), float(delta),
                                            int(mode), int(run_seed), C.byref(r)))
    return r.as_dict()


def oi_estimate_batch(g, seed_off, seeds, query_ids, eps, delta, mode, run_seed):
    off = _host(seed_off, np.int64)
    s = _host(seeds, np.int32)
    q = _host(query_ids, np.uint32)
    nq = off.size - 1
    out = (oi_result * nq)()
    _check("oi_estimate_batch", _lib.oi_estimate_batch(g, nq, _ptr(off), _ptr(s), _ptr(q), float(eps),
                                                        float(delta), int(mode), int(run_seed), out))
    return [out[i].as_dict() for i in range(nq)]


def oi_backward(g, query_id, seeds, first, count, run_seed, y_in, param, grad_scale, grad_out):
    s = _host(seeds, np.int32)
    _check("oi_backward", _lib.oi_backward(g, int(query_id), _ptr(s), s.size, int(first), int(count),
                                            int(run_seed), _ptr(y_in), int(param), float(grad_scale),
                                            _ptr(grad_out)))


def oi_timing_enable(g, enable=True):
    _check("oi_timing_enable", _lib.oi_timing_enable(g, int(bool(enable))))


def oi_timing_get(g):
    t = oi_timing()
    _check("oi_timing_get", _lib.oi_timing_get(g, C.byref(t)))
    return t.as_dict()


def oi_set_tuning(g, variant=-1, chunk=-1, tiny=-1, tiny_chunk=-1, round_max=-1):
    _check("oi_set_tuning", _lib.oi_set_tuning(g, int(variant), int(chunk), int(tiny), int(tiny_chunk),
                                                int(round_max)))


def oi_set_routing(g, small_direct=-1, large_qcap=-1):
    _check("oi_set_routing", _lib.oi_set_routing(g, int(small_direct), int(large_qcap)))


def oi_set_stage1_skip(g, min_l):
    """Stage-1 tables of at least max(min_l, 65) entries that pass the density
    test use skip sampling."""
    _check("oi_set_stage1_skip", _lib.oi_set_stage1_skip(g, int(min_l)))


def oi_set_stage1_skip_cost(g, cost):
    """Draw-cost ratio of skip sampling's density test (default 8; 0: none)."""
    _check("oi_set_stage1_skip_cost", _lib.oi_set_stage1_skip_cost(g, float(cost)))


def oi_set_first_level(g, mode):
    """Tiny kernel's first-level passes: -1 automatic, 0 none, 1 / 2 that instantiation always."""
    _check("oi_set_first_level", _lib.oi_set_first_level(g, int(mode)))


def oi_set_pipeline(g, mode):
    """0: read every RSA round back; 1: queue rounds whose plan is fixed; 2: as 1, one graph per round."""
    _check("oi_set_pipeline", _lib.oi_set_pipeline(g, int(mode)))


def oi_autotune(g, seed_off, seeds, query_ids, pilot, run_seed):
    off = _host(seed_off, np.int64)
    s = _host(seeds, np.int32)
    q = _host(query_ids, np.uint32)
    r = oi_autotune_result()
    _check("oi_autotune", _lib.oi_autotune(g, int(off.size - 1), _ptr(off), _ptr(s), _ptr(q), int(pilot),
                                           int(run_seed) & 0xFFFFFFFF, C.byref(r)))
    return r.as_dict()


def oi_num_variants():
    return int(_lib.oi_num_variants())


def oi_variant_info(v):
    a, b, c, d = C.c_int(), C.c_int(), C.c_int(), C.c_int()
    _check("oi_variant_info", _lib.oi_variant_info(int(v), C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
    return dict(slots_per_wave=a.value, hash_cap=b.value, ring_cap=c.value, rounds_per_pass=d.value)


def oi_gather_probe(g, count, seed=0):
    """Random-gather bandwidth probe: dict(useful_bytes, edges, ms, gbps)."""
    b, e, t = C.c_uint64(), C.c_uint64(), C.c_double()
    _check("oi_gather_probe", _lib.oi_gather_probe(g, int(count), int(seed) & 0xFFFFFFFF, C.byref(b), C.byref(e),
                                                   C.byref(t)))
    return dict(useful_bytes=b.value, edges=e.value, ms=t.value,
                gbps=b.value / (t.value * 1e-3) / 1e9 if t.value > 0 else 0.0)


def oi_coin_probe(g, samples, groups_per_sample, seed=0, qid=0):
    """Coin-generation rate probe: dict(live, words, ms, words_per_s)."""
    live, t = C.c_uint64(), C.c_double()
    _check("oi_coin_probe", _lib.oi_coin_probe(g, int(samples), int(groups_per_sample), int(seed) & 0xFFFFFFFF,
                                               int(qid) & 0xFFFFFFFF, C.byref(live), C.byref(t)))
    words = 4 * int(samples) * int(groups_per_sample)
    return dict(live=live.value, words=words, ms=t.value,
                words_per_s=words / (t.value * 1e-3) if t.value > 0 else 0.0)
