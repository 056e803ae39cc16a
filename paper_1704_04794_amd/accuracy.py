"""The accuracy experiment of Sec. 6 (Tables 3-5): relative errors of SOIEA,
SIEA and classic Monte-Carlo estimates against a "ground truth" estimated
with a very small error.

For each seed set the ground truth is an SOIEA estimate at eps = 0.005,
delta = 1/n (Sec. 6.1, ground-truth computation) drawn with its own Philox
run seed, so that it shares no sample with the estimates it judges.  The
estimators under test are SOIEA and SIEA at the paper's default eps = 0.1,
delta = 1/n (Algs. 4 and 5, all seed sets in one batched call each) and
MC_N, the mean cascade size of N classic Monte-Carlo cascades (Sec. 2.3;
N = 10,000 and 100,000 as MC_10K and MC_100K).  The relative error of an
estimate of Ext(S) is |est / truth - 1| * 100%, and likewise for I(S)
(Sec. 6.1, metrics).  Every estimate comes from the library's kernels; this
module only schedules the calls and forms the error statistics.
"""
from __future__ import annotations

import time

import numpy as np

from . import OI_MODE_SIEA, OI_MODE_SOIEA, RUN_SEED

TRUTH_SEED = 0x5EED7A1E  # Philox run seed of the ground-truth estimates


def _rel_err(est, truth):
    est = np.asarray(est, np.float64)
    truth = np.asarray(truth, np.float64)
    return np.abs(est / truth - 1.0) * 100.0


def accuracy(G, seed_sets, eps=0.1, delta=None, truth_eps=0.005, truth_delta=None, mc_samples=(10_000, 100_000),
             run_seed=RUN_SEED, truth_seed=TRUTH_SEED, query_ids=None, truth_chunk=None, progress=None):
    """Run the experiment on graph G (a paper_1704_04794_amd.Graph) for the
    given seed sets (every set needs an out-neighbour outside itself, so that
    its outward influence is positive).  Returns a dict with, per estimator
    ("soiea", "siea", "mc_<N>"), the per-set estimates of OI and IS, the
    average and maximum relative errors (%) of both, and the wall time of the
    estimator's calls; plus the ground truth and its time.  The ground truth
    is estimated in batched calls of `truth_chunk` sets (default: all at
    once), calling progress(done, total) after each."""
    import torch
    n = G.n
    delta = 1.0 / n if delta is None else delta
    truth_delta = delta if truth_delta is None else truth_delta
    q = np.arange(len(seed_sets), dtype=np.uint32) if query_ids is None else np.asarray(query_ids, np.uint32)
    k = np.array([len(np.unique(s)) for s in seed_sets], np.float64)
    out = {"sets": len(seed_sets), "eps": eps, "delta": delta, "truth_eps": truth_eps, "truth_delta": truth_delta}

    t = time.perf_counter()
    tr = []
    step = truth_chunk or len(seed_sets)
    for lo in range(0, len(seed_sets), step):
        tr += G.estimate_batch(seed_sets[lo:lo + step], truth_eps, truth_delta, mode=OI_MODE_SOIEA,
                               query_ids=q[lo:lo + step], run_seed=truth_seed)
        if progress:
            progress(len(tr), len(seed_sets))
    out["truth"] = {"seconds": time.perf_counter() - t,
                    "oi": [r["oi"] for r in tr], "is": [r["is_"] for r in tr],
                    "samples": int(sum(r["samples_x"] + r["samples_xp"] for r in tr))}
    t_oi = np.array(out["truth"]["oi"])
    t_is = np.array(out["truth"]["is"])
    if np.any(t_oi <= 0):
        raise ValueError("a seed set has no outward influence: relative errors are undefined")

    def summarize(name, oi, is_, seconds, extra=None):
        e_oi, e_is = _rel_err(oi, t_oi), _rel_err(is_, t_is)
        out[name] = {"seconds": seconds, "oi": list(map(float, oi)), "is": list(map(float, is_)),
                     "avg_rel_err_oi": float(e_oi.mean()), "max_rel_err_oi": float(e_oi.max()),
                     "avg_rel_err_is": float(e_is.mean()), "max_rel_err_is": float(e_is.max()), **(extra or {})}

    for name, mode in (("soiea", OI_MODE_SOIEA), ("siea", OI_MODE_SIEA)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = G.estimate_batch(seed_sets, eps, delta, mode=mode, query_ids=q, run_seed=run_seed)
        dt = time.perf_counter() - t
        summarize(name, [r["oi"] for r in res], [r["is_"] for r in res], dt,
                  {"samples": int(sum(r["samples_x"] + r["samples_xp"] for r in res))})
    for N in mc_samples:
        oi, is_ = [], []
        torch.cuda.synchronize()
        t = time.perf_counter()
        for S, qi in zip(seed_sets, q):
            _, _, r = G.sample_mc(S, N, query_id=int(qi), run_seed=run_seed)
            oi.append(r["oi"])
            is_.append(r["is_"])
        dt = time.perf_counter() - t
        summarize(f"mc_{N}", oi, is_, dt, {"samples": N * len(seed_sets)})
    out["k"] = list(map(float, k))
    return out
