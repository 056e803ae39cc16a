"""MI355X (gfx950) outward-influence estimation: IICP sampling driven by RSA.

The computation lives in liboi_hip.so (HIP kernels + C ABI, include/oi.h);
this package is its binding.  `Graph` owns a library graph handle; the
module-level `oi_*` functions are the C entry points one to one.
"""
from __future__ import annotations

import numpy as np

from ._binding import (  # noqa: F401
    LIB_PATH, OI_MODE_SIEA, OI_MODE_SIEA_LT, OI_MODE_SOIEA, OI_PARAM_P, OI_PARAM_THETA, OiError, oi_autotune, oi_backward,
    oi_coin_probe, oi_gather_probe,
    oi_estimate, oi_estimate_batch, oi_graph_create, oi_graph_destroy, oi_graph_get_probs, oi_graph_set_probs,
    oi_graph_set_theta, oi_last_error,
    oi_num_variants, oi_sample_fixed, oi_set_first_level, oi_sample_fixed_noalloc, oi_sample_lt, oi_sample_mc, oi_set_pipeline, oi_set_routing, oi_set_stage1_skip, oi_set_stage1_skip_cost, oi_set_stream, oi_set_tuning, oi_stage1_table,
    oi_timing_enable, oi_timing_get, oi_variant_info)

RUN_SEED = 0x17044794


def _is_device_tensor(x) -> bool:
    return hasattr(x, "is_cuda") and bool(x.is_cuda)


class Graph:
    """A CSR graph with fp32 IC edge probabilities resident on the GPU.

    row_ptr int64[n+1], col int32[m], p float32[m]: numpy arrays (host) or
    torch CUDA tensors (device)."""

    def __init__(self, n, row_ptr, col, p, stream=None):
        dev = _is_device_tensor(row_ptr)
        if dev:
            row_ptr, col, p = row_ptr.contiguous(), col.contiguous(), p.contiguous()
        else:
            row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
            col = np.ascontiguousarray(col, dtype=np.int32)
            p = np.ascontiguousarray(p, dtype=np.float32)
        self.n = int(n)
        self.m = int(col.shape[0])
        self.h = oi_graph_create(self.n, self.m, row_ptr, col, p, 1 if dev else 0, stream)
        # bumped by every change of the edge probabilities (set_probs,
        # set_theta), so that holders of earlier results can tell
        self.version = 0

    @classmethod
    def from_inputs(cls, g, stream=None):
        """From an object with n, row_ptr, col, p (e.g. oi_inputs.Graph)."""
        return cls(g.n, g.row_ptr, g.col, g.p, stream)

    def close(self):
        if getattr(self, "h", None) is not None:
            oi_graph_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def set_probs(self, p):
        dev = _is_device_tensor(p)
        self.version += 1
        oi_graph_set_probs(self.h, p.contiguous() if dev else np.ascontiguousarray(p, np.float32),
                           1 if dev else 0)

    def set_theta(self, theta):
        """p = sigmoid(theta), computed by the library on the GPU."""
        dev = _is_device_tensor(theta)
        self.version += 1
        oi_graph_set_theta(self.h, theta.contiguous() if dev else np.ascontiguousarray(theta, np.float32),
                           1 if dev else 0)

    def probs(self):
        return oi_graph_get_probs(self.h, self.m)

    def stage1(self, seeds):
        return oi_stage1_table(self.h, seeds)

    def sample_fixed(self, seeds, count, first=0, stream=0, query_id=0, run_seed=RUN_SEED, want_e=False,
                     device="cuda"):
        """Y (and optionally E) of `count` samples as torch tensors on the GPU."""
        import torch
        y = torch.empty(count, dtype=torch.int32, device=device)
        e = torch.empty(count, dtype=torch.int64, device=device) if want_e else None
        r = oi_sample_fixed(self.h, query_id, seeds, stream, first, count, run_seed, y, e)
        return y, e, r

    def sample_mc(self, seeds, count, first=0, stream=0, query_id=0, run_seed=RUN_SEED, want_e=False,
                  device="cuda"):
        """Classic IC Monte-Carlo samples M - |S| (and optionally E) of `count`
        cascades as torch tensors on the GPU, with the MC_N estimates."""
        import torch
        y = torch.empty(count, dtype=torch.int32, device=device)
        e = torch.empty(count, dtype=torch.int64, device=device) if want_e else None
        r = oi_sample_mc(self.h, query_id, seeds, stream, first, count, run_seed, y, e)
        return y, e, r

    def sample_lt(self, seeds, count, first=0, stream=0, query_id=0, run_seed=RUN_SEED, want_e=False,
                  device="cuda"):
        """LT-model cascades (edge probabilities as LT weights): Y = |cascade|
        - |S| (and optionally E) of `count` samples as torch tensors, with the
        fixed-count estimates."""
        import torch
        y = torch.empty(count, dtype=torch.int32, device=device)
        e = torch.empty(count, dtype=torch.int64, device=device) if want_e else None
        r = oi_sample_lt(self.h, query_id, seeds, stream, first, count, run_seed, y, e)
        return y, e, r

    def estimate(self, seeds, eps, delta, mode=OI_MODE_SOIEA, query_id=0, run_seed=RUN_SEED):
        return oi_estimate(self.h, query_id, seeds, eps, delta, mode, run_seed)

    def estimate_batch(self, seed_sets, eps, delta, mode=OI_MODE_SOIEA, query_ids=None, run_seed=RUN_SEED):
        off = np.zeros(len(seed_sets) + 1, np.int64)
        off[1:] = np.cumsum([len(s) for s in seed_sets])
        seeds = np.concatenate([np.asarray(s, np.int32) for s in seed_sets]) if seed_sets else np.zeros(0, np.int32)
        q = np.arange(len(seed_sets), dtype=np.uint32) if query_ids is None else np.asarray(query_ids, np.uint32)
        return oi_estimate_batch(self.h, off, seeds, q, eps, delta, mode, run_seed)

    def backward(self, seeds, count, grad_out, y_in=None, first=0, param=OI_PARAM_P, grad_scale=1.0,
                 query_id=0, run_seed=RUN_SEED):
        oi_backward(self.h, query_id, seeds, first, count, run_seed, y_in, param, grad_scale, grad_out)
        return grad_out

    def gather_probe(self, count, seed=0):
        """Random-read bandwidth of this graph's CSR under the samplers' access
        pattern (no coins or visited sets): dict(useful_bytes, edges, ms, gbps)."""
        return oi_gather_probe(self.h, count, seed)

    def coin_probe(self, samples, groups_per_sample, seed=0, query_id=0):
        """Rate at which the GPU draws and tests the samplers' edge coins alone
        (no loads, queues or visited sets): dict(live, words, ms, words_per_s)."""
        return oi_coin_probe(self.h, samples, groups_per_sample, seed, query_id)

    def autotune(self, seed_sets, pilot=1 << 16, query_ids=None, run_seed=RUN_SEED):
        """Time the sampler's schedules on a pilot of up to four of the seed
        sets and keep the fastest (results never depend on the choice)."""
        off = np.zeros(len(seed_sets) + 1, np.int64)
        off[1:] = np.cumsum([len(s) for s in seed_sets])
        seeds = np.concatenate([np.asarray(s, np.int32) for s in seed_sets]) if seed_sets else np.zeros(0, np.int32)
        q = np.arange(len(seed_sets), dtype=np.uint32) if query_ids is None else np.asarray(query_ids, np.uint32)
        return oi_autotune(self.h, off, seeds, q, pilot, run_seed)

    def timing(self, enable=None):
        """Kernel timing with HIP events: timing(True) turns it on and resets
        the counters, timing(False) turns it off; returns the counters."""
        if enable is not None:
            oi_timing_enable(self.h, enable)
        return oi_timing_get(self.h)

    def tune(self, variant=-1, chunk=-1, tiny=-1, tiny_chunk=-1, round_max=-1, small_direct=-1, large_qcap=-1,
             pipeline=None):
        """Sampler knobs (oi_set_tuning, oi_set_routing, oi_set_pipeline); -1
        (or None) keeps a setting.  large_qcap > 0 fixes the large kernel's
        queue size, 0 restores the default adaptive soft cap.  Results never
        depend on any of them."""
        oi_set_tuning(self.h, variant, chunk, tiny, tiny_chunk, round_max)
        if small_direct >= 0 or large_qcap >= 0:
            oi_set_routing(self.h, small_direct, large_qcap)
        if pipeline is not None:
            oi_set_pipeline(self.h, pipeline)
