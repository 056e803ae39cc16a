"""Throughput of the IICP + RSA hot path on one MI355X.

One step is one complete (eps, delta)-estimate of the outward influence of
the seed set of the 1M-node Chung-Lu workload (n = 1,000,000, expected
m = 1e7, degree exponent 2.1, trivalency edge probabilities, |S| = 1, SOIEA
with eps = 0.05, delta = 1/n), i.e. every IICP sample the three RSA steps
draw, on inputs already resident in HBM.

Prints one JSON line: `value` = IICP samples per second over the timed
steps; GTEPS and seed-set estimates/s are reported beside it, with the
roofline of the sampling kernel that took the most time (bytes it must read
per activated node and per examined edge, over its HIP-event time on the
library's stream) and the CPU oracle's rate on a bounded sample of the same
query.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --workload cl4m [--queries Q] [--eps E] [--no-autotune]
        seed-set estimates/s, batched vs one at a time, on the 4M-node
        weighted-cascade graph, with the large-cascade kernel's roofline
    python bench.py --workload accuracy [--queries Q]
        relative errors of SOIEA, SIEA, MC_10K and MC_100K against a ground
        truth (Sec. 6.1) on NetHEP- and NetPHY-sized synthetic graphs
    python bench.py --workload cl100m [--c5-sets K] [--c5-only]
        the 1e8-node / 1.5e9-edge graph: fixed-count throughput for
        |S| = 1, 10, 100, a SIEA estimate, the queue-cap comparison and the
        backward over all edges; with --c5-sets, SOIEA estimates at the
        workload's eps = 0.05, delta = 1e-6 for K sets of each size
    python bench.py --workload skip-density
        Stage-1 skip sampling against one coin per entry on a 1,000-seed
        table of the 1M-node graph under edge models from dense to sparse,
        and which of the two the default density test picks
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "IICP samples/s + GTEPS; seed-set estimates/s batched vs single at ε=0.05"
HBM_PEAK_GBS = 8000.0
BYTES_PER_NODE = 16  # row_ptr[u], row_ptr[u+1] (int64) per activated node
BYTES_PER_EDGE = 8   # col (int32) + coin threshold (uint32) per examined edge
# Algorithmic vector ALU work, in 32-bit lane operations of this ISA: one
# Philox4x32-10 draw is 10 rounds of two 32x32->64 products (one multiply-add
# with a 64-bit result each) and two three-input exclusive ors (the key
# schedule is the same for every lane: scalar work), 40 operations for four
# coin words.  A coin (Alg. 1: one per Stage-1 entry after the selected one
# and per out-edge of an activated node) is a quarter draw and a compare; the
# selection of a sample's first entry, needed only when the Stage-1 table
# has more than one entry, is one draw.
PHILOX_OPS = 10 * (2 + 2)
OPS_PER_COIN = PHILOX_OPS / 4 + 1
OPS_PER_SELECTION = PHILOX_OPS
# MI355X vector ALU peak for 32-bit integer operations: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz (one wave64 instruction per CU per clock; the 157.3 TFLOP/s
# fp32 figure counts an FMA as two and packed pairs as two)
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


# Counter figures for tiny_kernel on the default workload (rocprofv3 --pmc
# passes over `bench.py --minimal --warmup 1 --steps 2`): HBM bytes per launch
# = FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (the scales a 1 GiB device copy gives
# those counters), the L2 hit rate, VALU busy (percent of the active cycles
# the vector ALUs issued), and VALU instructions per examined edge
# (SQ_INSTS_VALU x 64 lanes over the launch's examined edges); means over the
# launches of one estimate.  Reported only while the sampler's source up to
# the small-sample kernel (its code, comments aside) and the device header
# hash to what was measured, and an estimate takes as many launches.
COUNTERS = {"sources_sha1": "ba0ddfb5a59f6bde3027e7a023683cfd7f59f36f", "kernel": "tiny_kernel",
            "launches_per_estimate": 7, "bytes_per_launch": 2.0 * 17628.289 * 1024 + 1.0 * 5286963.970 * 1024,
            "l2_hit_rate": 0.794, "valu_busy": 0.515, "valu_lane_ops_per_edge": 62.7}
KERNEL_SOURCES = ("paper_1704_04794_amd/csrc/iicp_kernels.hip", "paper_1704_04794_amd/csrc/oi_device.hpp")
TINY_REGION_END = "template <int K, int HCAP, int RCAP, int R, bool BWD>\n__global__ void __launch_bounds__(256) small_kernel"


def kernel_sources_sha1():
    """SHA-1 of the tiny sampler's sources (the kernel file up to the
    small-sample kernel, and the device header) with comments and blank space
    removed, so that only a change of its code voids the counter figures."""
    import hashlib
    import re
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            text = fh.read()
        if f.endswith(".hip"):
            end = text.find(TINY_REGION_END)
            text = text[:end] if end >= 0 else text
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_counters(kernel, launches_per_estimate):
    if (COUNTERS["sources_sha1"] is None or kernel_sources_sha1() != COUNTERS["sources_sha1"]
            or kernel != COUNTERS["kernel"] or launches_per_estimate != COUNTERS["launches_per_estimate"]):
        return None
    return COUNTERS


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info():
    """CPU model, logical CPUs and RAM of the host the oracle runs on."""
    model, ram = None, None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    ram = round(int(line.split()[1]) / 2**20, 1)
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_logical_cpus": os.cpu_count(), "ram_gib": ram}


def cpu_baseline(g, S, seconds):
    import oracle as O
    from oi_inputs.configs import RUN_SEED
    nt = O.nthreads_default()
    n0 = 2_000_000
    t = time.perf_counter()
    O.sample_fixed(g, S, 0, RUN_SEED, 0, 0, n0, want_y=False, nthreads=nt)
    rate0 = n0 / max(time.perf_counter() - t, 1e-6)
    N = int(min(max(rate0 * seconds, n0), 2e10))
    log(f"cpu baseline: {N} samples on {nt} threads (calibrated {rate0:.3g}/s)")
    t = time.perf_counter()
    r = O.sample_fixed(g, S, 0, RUN_SEED, 0, 0, N, want_y=False, nthreads=nt)
    dt = time.perf_counter() - t
    # the same oracle on one thread, over a slice of about 4 s
    n1 = max(n0 // 4, int(N / nt * 4.0 / max(dt, 1e-6)))
    t = time.perf_counter()
    O.sample_fixed(g, S, 0, RUN_SEED, 0, 0, n1, want_y=False, nthreads=1)
    dt1 = time.perf_counter() - t
    return {"value": N / dt, "unit": "samples/s", "cores": nt, "kind": "oracle", **host_info(),
            "sample": f"IICP samples 0..{N - 1} of stream X of the same query (fixed count, oracle in C, "
                      f"{nt} threads), {dt:.1f} s; GTEPS {r['sum_e'] / dt / 1e9:.4f}; one thread: "
                      f"{n1} samples in {dt1:.1f} s",
            "one_thread_value": n1 / dt1}


def gather_roofline(G, count=1 << 26, reps=3):
    """Best of `reps` runs of the library's random-gather probe on the same
    graph: the samplers' row_ptr + edge-group reads without coins or visited
    sets, i.e. the random-read bandwidth the sampling kernels are bound by."""
    best = None
    for r in range(reps):
        x = G.gather_probe(count, seed=r)
        if best is None or x["gbps"] > best["gbps"]:
            best = x
    return best


def backward_ratio(P, N=1_000_000, reps=5):
    """Time of oi_backward over N samples (reusing the forward's Y) over the
    time of oi_sample_fixed over the same N, on the 1M-node sigmoid(theta)
    workload with |S| = 50."""
    import torch

    from oi_inputs import make_config
    g, sets, extra = make_config("cl1m_sig")
    S = sets[0]
    G = P.Graph.from_inputs(g)
    grad = torch.empty(g.m, dtype=torch.float32, device="cuda")
    y, _, _ = G.sample_fixed(S, N)
    G.backward(S, N, grad, y_in=y)
    torch.cuda.synchronize()
    tf = tb = float("inf")
    for _ in range(reps):
        t = time.perf_counter()
        y, _, r = G.sample_fixed(S, N)
        torch.cuda.synchronize()
        tf = min(tf, time.perf_counter() - t)
        t = time.perf_counter()
        G.backward(S, N, grad, y_in=y)
        torch.cuda.synchronize()
        tb = min(tb, time.perf_counter() - t)
    G.close()
    return {"workload": "cl1m_sig: Chung-Lu n=1e6 m~1e7 gamma=2.1, p=sigmoid(theta), theta~N(-3,1), |S|=50",
            "samples": N, "forward_ms": tf * 1e3, "backward_ms": tb * 1e3, "ratio": tb / tf,
            "note": "wall time per call incl. host work, best of %d; backward reuses the forward's Y" % reps}


def billion_edge(P, args):
    """The 1e8-node / 1.5e9-edge weighted-cascade workload: build and upload
    time, the random-gather probe, fixed-count IICP throughput for one seed
    set of each size (1, 10, 100), one backward dOI/dp over all edges for the
    |S| = 100 set, and the CPU oracle on the |S| = 1 set."""
    import torch

    from oi_inputs import make_config
    t0 = time.perf_counter()

    def progress(done, total):
        if done % 16 == 0 or done == total:
            log(f"generated {done}/{total} blocks of sources ({time.perf_counter() - t0:.0f}s)")

    g, sets, extra = make_config("cl100m", progress=progress)
    build_s = time.perf_counter() - t0
    log(f"cl100m n={g.n} m={g.m} built in {build_s:.1f}s")
    t = time.perf_counter()
    G = P.Graph.from_inputs(g)
    torch.cuda.synchronize()
    upload_s = time.perf_counter() - t
    probe = gather_roofline(G)
    out = {"metric": "IICP samples/s and GTEPS per seed-set size; backward over all edges",
           "workload": f"cl100m: Chung-Lu n=1e8 m={g.m} gamma=2.1 WC p, seed sets of the 256-set list "
                       "(|S| = 1, 10, 100: sets 0, 1, 2)",
           "build_s": build_s, "upload_s": upload_s, "gather_probe_gbps": probe["gbps"], "fixed": []}
    if args.c5_sets > 0:
        out["estimates"] = c5_estimates(P, G, g, sets, extra, args.c5_sets)
    if args.c5_only:
        G.close()
        return out
    for qi, N in ((0, 1 << 26), (1, 1 << 20), (2, 1 << 15)):
        S = sets[qi]
        # a warm-up of the same size: the large kernel's queue cap adapts to
        # what the previous launch saw
        G.sample_fixed(S, N, query_id=qi)
        G.timing(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        y, _, r = G.sample_fixed(S, N, query_id=qi)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        tm = G.timing()
        row = {"k": int(len(S)), "query": qi, "samples": N, "seconds": dt, "samples_per_s": N / dt,
               "gteps": r["edges_examined"] / dt / 1e9, "sum_y": r["sum_y"], "y_mean": r["sum_y"] / N,
               "beta0": r["beta0"],
               "kernel_ms": {k: tm[f"{k}_ms"] for k in ("tiny", "small", "large")}}
        out["fixed"].append(row)
        log(f"fixed |S|={len(S)}: {row}")
    # one SIEA estimate of the |S| = 1 set at the paper's default accuracy
    # (eps = 0.1, delta = 1/n), for comparison with its runtimes on graphs of
    # this size
    S = sets[0]
    t = time.perf_counter()
    r = G.estimate(S, 0.1, 1.0 / g.n, mode=P.OI_MODE_SIEA, query_id=0)
    dt = time.perf_counter() - t
    out["siea_estimate"] = {"k": int(len(S)), "eps": 0.1, "delta": 1.0 / g.n, "seconds": dt, "is": r["is_"],
                            "oi": r["oi"], "samples": r["samples_x"] + r["samples_xp"], "rounds": r["rounds"],
                            "samples_per_s": (r["samples_x"] + r["samples_xp"]) / dt}
    log(f"SIEA estimate: {out['siea_estimate']}")
    # the same two runs with the large kernel's queue cap fixed at 2^20 (no
    # adaptation): the rare giant cascades then keep one 256-thread block
    # busy long after the rest of a launch has finished (results identical)
    G.tune(large_qcap=1 << 20)
    S = sets[0]
    G.sample_fixed(S, 1 << 26, query_id=0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, _, rq = G.sample_fixed(S, 1 << 26, query_id=0)
    torch.cuda.synchronize()
    tq = time.perf_counter() - t
    t = time.perf_counter()
    rs = G.estimate(S, 0.1, 1.0 / g.n, mode=P.OI_MODE_SIEA, query_id=0)
    dt = time.perf_counter() - t
    out["fixed_queue_cap_2e20"] = {"fixed_k1_seconds": tq, "fixed_k1_samples_per_s": (1 << 26) / tq,
                                   "siea_seconds": dt,
                                   "siea_samples_per_s": (rs["samples_x"] + rs["samples_xp"]) / dt,
                                   "identical": rq["sum_y"] == out["fixed"][0]["sum_y"] and rs["is_"] == r["is_"]
                                   and rs["T"] == r["T"]}
    log(f"queue cap fixed at 2^20: {out['fixed_queue_cap_2e20']}")
    G.tune(large_qcap=0)
    S = sets[2]
    N = 1 << 14
    grad = torch.empty(g.m, dtype=torch.float32, device="cuda")
    y, _, _ = G.sample_fixed(S, N, query_id=2)
    G.backward(S, N, grad, y_in=y, query_id=2)
    torch.cuda.synchronize()
    t = time.perf_counter()
    y, _, _ = G.sample_fixed(S, N, query_id=2)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t
    t = time.perf_counter()
    G.backward(S, N, grad, y_in=y, query_id=2)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    out["backward"] = {"k": int(len(S)), "samples": N, "edges": g.m, "forward_ms": tf * 1e3,
                       "backward_ms": tb * 1e3, "ratio": tb / tf,
                       "nonzero_grad_edges": int((grad != 0).sum().item())}
    log(f"backward: {out['backward']}")
    del grad
    G.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, sets[0], args.cpu_seconds)
    return out


def c5_estimates(P, G, g, sets, extra, per_size):
    """SOIEA estimates at the billion-edge workload's own accuracy (eps =
    0.05, delta = 1e-6) for the first `per_size` seed sets of each size (1,
    10, 100) in its seed-set list, one at a time, with each estimate's wall
    time, sample count and rounds."""
    eps, delta = extra["eps"], extra["delta"]
    rows = []
    for k in sorted(set(int(len(S)) for S in sets)):
        picks = [qi for qi, S in enumerate(sets) if len(S) == k][:per_size]
        for qi in picks:
            t = time.perf_counter()
            r = G.estimate(sets[qi], eps, delta, mode=P.OI_MODE_SOIEA, query_id=qi)
            dt = time.perf_counter() - t
            n_s = r["samples_x"] + r["samples_xp"]
            row = {"k": k, "query": qi, "eps": eps, "delta": delta, "seconds": dt, "oi": r["oi"], "is": r["is_"],
                   "beta0": r["beta0"], "samples": n_s, "rounds": r["rounds"], "T1": r["T1"], "T": r["T"],
                   "samples_per_s": n_s / dt, "gteps": r["edges_examined"] / dt / 1e9}
            rows.append(row)
            log(f"estimate |S|={k} set {qi}: {dt:.2f}s OI={r['oi']:.6g} samples={n_s} rounds={r['rounds']}")
    return rows


def batched_vs_single(P, args, per_stratum=False):
    """Seed-set estimates/s on the 4M-node weighted-cascade workload: a seeded
    stratified subset of its 4,096 seed sets (equal numbers from the uniform
    and the top-1% halves), estimated in one batched call and one at a time
    (with per_stratum, each half in a batched call of its own, so that the
    two kinds of seed set are timed apart)."""
    import numpy as np

    from oi_inputs import make_config
    t = time.perf_counter()
    g, sets, extra = make_config("cl4m")
    log(f"cl4m graph n={g.n} m={g.m} built in {time.perf_counter() - t:.1f}s")
    half = len(sets) // 2
    k = max(1, (args.queries or 32) // 2)
    rng = np.random.default_rng(7)
    pick = np.concatenate([rng.choice(half, size=k, replace=False),
                           half + rng.choice(len(sets) - half, size=k, replace=False)])
    sub = [sets[i] for i in pick]
    qids = pick.astype(np.uint32)
    eps = args.eps if args.eps > 0 else extra["eps"]
    delta = extra["delta"]
    G = P.Graph.from_inputs(g)
    G.estimate(sub[0], 0.5, delta, query_id=int(qids[0]))  # warm up kernels and workspaces
    tune = None
    if not args.no_autotune:
        t = time.perf_counter()
        tune = G.autotune(sub, pilot=4096, query_ids=qids)
        log(f"autotune ({time.perf_counter() - t:.1f}s): {tune}")
    probe = gather_roofline(G)
    import torch
    torch.cuda.synchronize()
    # both passes with HIP-event kernel timing on (same cost for both)
    G.timing(True)
    strata = {}
    if per_stratum:
        batch, tb = [], 0.0
        for name, lo in (("uniform", 0), ("top1pct", k)):
            t = time.perf_counter()
            batch += G.estimate_batch(sub[lo:lo + k], eps, delta, query_ids=qids[lo:lo + k])
            dt = time.perf_counter() - t
            tb += dt
            strata[name] = {"sets": k, "batched_s": dt, "batched_estimates_per_s": k / dt}
            log(f"batched {name}: {k} sets in {dt:.2f}s")
    else:
        t = time.perf_counter()
        batch = G.estimate_batch(sub, eps, delta, query_ids=qids)
        tb = time.perf_counter() - t
    tm = G.timing()
    log(f"batched: {len(sub)} sets in {tb:.2f}s")
    G.timing(True)
    single, ts = [], 0.0
    for j, (S, q) in enumerate(zip(sub, qids)):
        t = time.perf_counter()
        single.append(G.estimate(S, eps, delta, query_id=int(q)))
        dt = time.perf_counter() - t
        ts += dt
        if per_stratum:
            st = strata["uniform" if j < k else "top1pct"]
            st["single_s"] = st.get("single_s", 0.0) + dt
    for st in strata.values():
        st["single_estimates_per_s"] = st["sets"] / st["single_s"]
        st["speedup"] = st["single_s"] / st["batched_s"]
    G.timing(False)
    log(f"one at a time: {len(sub)} sets in {ts:.2f}s")
    # the large-cascade kernel of the batched pass against the random-read
    # roofline: algorithmic bytes of the samples it finished over its time
    kbytes = BYTES_PER_NODE * tm["large_y"] + BYTES_PER_EDGE * tm["large_edges"]
    kgbps = kbytes / (tm["large_ms"] * 1e-3) / 1e9 if tm["large_ms"] > 0 else 0.0
    large = {"kernel": "large_kernel", "ms": tm["large_ms"], "launches": tm["launches"],
             "activated": tm["large_y"], "edges": tm["large_edges"],
             "gteps": tm["large_edges"] / (tm["large_ms"] * 1e-3) / 1e9 if tm["large_ms"] > 0 else 0.0,
             "achieved_gbps": kgbps, "frac_of_hbm_peak": kgbps / HBM_PEAK_GBS,
             "gather_probe_gbps": probe["gbps"], "frac_of_measured_gather": kgbps / probe["gbps"],
             "share_of_batched_time": tm["large_ms"] * 1e-3 / tb}
    same = all(a["oi"] == b["oi"] and a["T"] == b["T"] for a, b in zip(batch, single))
    samples = sum(r["samples_x"] + r["samples_xp"] for r in batch)
    G.close()
    return {"metric": "seed-set estimates/s, batched vs one at a time", "workload":
            f"cl4m: Chung-Lu n=4e6 m~7e7 gamma=2.1 WC p, {len(sub)} of the 4,096 seed sets "
            f"({k} uniform + {k} top-1% out-degree, |S| in [1,1000]), SOIEA eps={eps} delta={delta}",
            "batched_estimates_per_s": len(sub) / tb, "single_estimates_per_s": len(sub) / ts,
            "speedup": ts / tb, "identical_results": same, "samples": samples,
            "batched_samples_per_s": samples / tb, "large_kernel": large, "autotune": tune,
            **({"strata": strata} if per_stratum else {})}


def batched_vs_single_small(P, args):
    """Seed-set estimates/s, batched vs one at a time, where one query alone
    leaves the GPU idle: the 2k-node ER weighted-cascade graph, Q seeded
    single-node seed sets, SOIEA at eps = 0.05, delta = 1e-3.  Each estimate
    needs only a few million short samples, so one at a time it is bound by
    the per-round launch and read-back; batched, every round serves all
    unfinished queries."""
    import numpy as np
    import torch

    from oi_inputs import make_config, uniform_seed_set
    g, _, _ = make_config("er2k")
    q = args.queries or 256
    sub = [uniform_seed_set(g, 1, 1000 + i) for i in range(q)]
    qids = np.arange(q, dtype=np.uint32)
    eps = args.eps if args.eps > 0 else 0.05
    delta = 1e-3
    G = P.Graph.from_inputs(g)
    G.estimate(sub[0], 0.5, delta, query_id=0)  # warm up kernels and workspaces
    G.estimate_batch(sub[:4], 0.5, delta, query_ids=qids[:4])
    torch.cuda.synchronize()
    t = time.perf_counter()
    batch = G.estimate_batch(sub, eps, delta, query_ids=qids)
    tb = time.perf_counter() - t
    log(f"batched: {q} sets in {tb:.3f}s")
    t = time.perf_counter()
    single = [G.estimate(S, eps, delta, query_id=int(i)) for S, i in zip(sub, qids)]
    ts = time.perf_counter() - t
    log(f"one at a time: {q} sets in {ts:.3f}s")
    same = all(a["oi"] == b["oi"] and a["T"] == b["T"] for a, b in zip(batch, single))
    samples = sum(r["samples_x"] + r["samples_xp"] for r in batch)
    G.close()
    return {"metric": "seed-set estimates/s, batched vs one at a time", "workload":
            f"er2k: Erdos-Renyi n=2000 m=20000 WC p, {q} seeded single-node seed sets, SOIEA eps={eps} "
            f"delta={delta}",
            "batched_estimates_per_s": q / tb, "single_estimates_per_s": q / ts, "speedup": ts / tb,
            "identical_results": same, "samples": samples, "batched_samples_per_s": samples / tb,
            "rounds_per_estimate": sum(r["rounds"] for r in single) / q}


def stage1_skip_gain(P, g, S, models, N, qid=99, repeats=1):
    """Stage-1 skip sampling against one coin per table entry, on the long
    Stage-1 table of one seed set under several edge models: fixed-count
    IICP time (best of `repeats` after a warm run) with skip sampling forced
    (density test off), with plain coins (skip sampling off), and at the
    default settings, whose choice is named by which of the two it
    reproduces (same law, different samples).  The table's light mass per
    256-entry segment and the walks' and coins' draw counts come from the
    library's own table."""
    import numpy as np
    import torch

    from oi_inputs import Graph as InputGraph
    rows = []
    for label, p in models:
        gg = g if p is None else InputGraph(g.n, g.row_ptr, g.col, p)
        G = P.Graph.from_inputs(gg)
        t = P.oi_stage1_table(G.h, S)
        Pj = t["P"]
        light = (Pj > 0.0) & (Pj < 0.5)
        nseg = (t["l"] + 255) // 256
        row = {"model": label, "samples": N, "l": t["l"], "light_mass_per_segment": float(Pj[light].sum()) / nseg,
               "walk_draws": nseg + float(Pj[light].sum()), "coin_blocks": t["l"] / 4}
        for name, min_l, cost in (("plain", 1 << 62, 8.0), ("skip", 4096, 0.0), ("default", 4096, 8.0)):
            P.oi_set_stage1_skip(G.h, min_l)
            P.oi_set_stage1_skip_cost(G.h, cost)
            G.sample_fixed(S, N, query_id=qid)  # warm
            torch.cuda.synchronize()
            best, r = None, None
            for _ in range(repeats):
                t0 = time.perf_counter()
                _, _, r = G.sample_fixed(S, N, query_id=qid)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
            row[name] = {"seconds": best, "samples_per_s": N / best, "mean_y": r["sum_y"] / N, "sum_y": r["sum_y"]}
        row["skip_vs_plain"] = row["plain"]["seconds"] / row["skip"]["seconds"]
        d = row["default"]["sum_y"]
        row["default_takes"] = ("skip" if d == row["skip"]["sum_y"] else
                                "plain" if d == row["plain"]["sum_y"] else "unknown")
        G.close()
        log(f"stage-1 skip sampling, {label}: {row}")
        rows.append(row)
    return rows


def skip_models(g, consts):
    """The workload's own trivalency p, then constant p for each of `consts`."""
    import numpy as np
    return [("trivalency", None)] + [(f"p = {c}", np.full(g.m, c, np.float32)) for c in consts]


def seed_spread(P, G, g, eps, delta, count):
    """One complete estimate for each of `count` seeded single-node seed sets
    (uniform over nodes with out-degree >= 1; the first is the headline's):
    the throughput spread over seed sets, with each set's Stage-1 size l."""
    from oi_inputs import seed_node_outdeg_ge1
    from oi_inputs.configs import CONFIGS
    rows = []
    seeds = [100 + CONFIGS["cl1m"]["number"]] + [1000 + i for i in range(count - 1)]
    for qi, sd in enumerate(seeds):
        S = seed_node_outdeg_ge1(g, sd)
        G.estimate(S, 0.5, delta, query_id=qi)  # warm: table and workspaces
        t = time.perf_counter()
        r = G.estimate(S, eps, delta, query_id=qi)
        dt = time.perf_counter() - t
        n = r["samples_x"] + r["samples_xp"]
        rows.append({"seed_node": int(S[0]), "l": r["l"], "samples": n, "seconds": dt, "samples_per_s": n / dt,
                     "gteps": r["edges_examined"] / dt / 1e9, "mean_y": r["sum_y"] / max(n, 1), "oi": r["oi"]})
        log(f"spread {qi}: {rows[-1]}")
    v = np.array([x["samples_per_s"] for x in rows])
    return {"sets": rows, "samples_per_s_min": float(v.min()), "samples_per_s_median": float(np.median(v)),
            "samples_per_s_max": float(v.max())}


def accuracy_experiment(P, args):
    """Sec. 6.1's accuracy comparison on stand-ins for NetHEP and NetPHY
    (Chung-Lu graphs of their sizes) under the weighted-cascade and constant
    edge models: average and maximum relative errors of SOIEA / SIEA at
    eps = 0.1, delta = 1/n and of MC_10K / MC_100K against a ground truth
    estimated at eps = 0.005, delta = 1/n, over `--queries` (default 1,000)
    random single-node seed sets with out-degree >= 1, with each estimator's
    GPU time."""
    from oi_inputs.configs import ACCURACY_GRAPHS, ACCURACY_MODELS, accuracy_workload
    from paper_1704_04794_amd.accuracy import accuracy
    rows = []
    graphs = args.accuracy_graphs.split(",") if args.accuracy_graphs else list(ACCURACY_GRAPHS)
    models = args.accuracy_models.split(",") if args.accuracy_models else list(ACCURACY_MODELS)
    for name in graphs:
        for model in models:
            g, sets = accuracy_workload(name, model, args.queries or 1000)
            G = P.Graph.from_inputs(g)
            G.estimate_batch(sets[:4], 0.5, 0.1)  # warm up kernels and workspaces
            t0 = time.perf_counter()
            r = accuracy(G, sets, truth_chunk=50,
                         progress=lambda d, n: log(f"{name} {model}: ground truth {d}/{n} "
                                                   f"({time.perf_counter() - t0:.0f}s)"))
            G.close()
            row = {"graph": name, "model": model, "n": g.n, "m": g.m, "sets": len(sets),
                   "truth_seconds": r["truth"]["seconds"], "truth_samples": r["truth"]["samples"]}
            for est in ("soiea", "siea", "mc_10000", "mc_100000"):
                x = r[est]
                row[est] = {f: round(x[f], 4) for f in ("avg_rel_err_oi", "max_rel_err_oi", "avg_rel_err_is",
                                                         "max_rel_err_is", "seconds")}
            rows.append(row)
            log(f"accuracy {name} {model}: {row}")
    return {"metric": "average / maximum relative error (%) of OI and IS estimates against a ground truth "
                      "(eps = 0.005, delta = 1/n), as in the accuracy comparison of Sec. 6.1",
            "data": "synthetic stand-ins (Chung-Lu, gamma 2.1) of NetHEP and NetPHY sizes", "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-backward", action="store_true", help="skip the backward/forward ratio")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--variant", type=int, default=-1)
    ap.add_argument("--pipeline", type=int, choices=(0, 1, 2), default=None,
                    help="RSA rounds: 0 read back one at a time, 1 queued (default), 2 queued, one graph each")
    ap.add_argument("--workload", choices=("cl1m", "cl4m", "cl100m", "er2k", "accuracy", "skip-density"),
                    default="cl1m",
                    help="cl1m: the single-query throughput line (default); cl4m: batched vs one-at-a-time; "
                         "cl100m: the billion-edge graph; er2k: batched vs one-at-a-time where one query "
                         "leaves the GPU idle; skip-density: Stage-1 skip sampling against plain coins over "
                         "table densities")
    ap.add_argument("--queries", type=int, default=None,
                    help="cl4m: seed sets in the subset (default 32); er2k: seed sets (default 256)")
    ap.add_argument("--no-autotune", action="store_true", help="cl4m: keep the default sampler schedule")
    ap.add_argument("--eps", type=float, default=-1.0, help="cl4m: eps (default: the workload's 0.1)")
    ap.add_argument("--minimal", action="store_true",
                    help="cl1m: only the timed estimates (for profiler runs): no spread, gather probe, backward, "
                         "CPU baseline or batched block")
    ap.add_argument("--no-batched", action="store_true",
                    help="cl1m: skip the batched-vs-single block (er2k and the 4M-node subset)")
    ap.add_argument("--batched-per-stratum", type=int, default=16,
                    help="cl1m: seed sets per stratum (uniform, top-1%%) of the 4M-node subset")
    ap.add_argument("--c5-sets", type=int, default=0,
                    help="cl100m: SOIEA estimates at eps=0.05, delta=1e-6 for this many sets of each size")
    ap.add_argument("--c5-only", action="store_true", help="cl100m: only the build, probe and those estimates")
    ap.add_argument("--spread", type=int, default=8, help="cl1m: seed sets of the headline's spread")
    ap.add_argument("--accuracy-graphs", default="", help="accuracy: comma-separated graphs (default: all)")
    ap.add_argument("--accuracy-models", default="", help="accuracy: comma-separated edge models (default: all)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device-to-device with torch (a plain copy kernel of known size, "
                         "to scale hardware byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (each GPU would run its own "
              "samples and only per-round integer sums would be exchanged); run with --gpus 1.",
              file=sys.stderr, flush=True)
        sys.exit(2)

    import torch

    import paper_1704_04794_amd as P
    from oi_inputs import make_config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copied 1 GiB device-to-device for counter calibration")
    if args.workload == "cl4m":
        print(json.dumps(batched_vs_single(P, args)), flush=True)
        return
    if args.workload == "er2k":
        print(json.dumps(batched_vs_single_small(P, args)), flush=True)
        return
    if args.workload == "cl100m":
        print(json.dumps(billion_edge(P, args)), flush=True)
        return
    if args.workload == "accuracy":
        print(json.dumps(accuracy_experiment(P, args)), flush=True)
        return
    if args.workload == "skip-density":
        from oi_inputs import top_outdeg_seed_set
        g, _, _ = make_config("cl1m")
        out = {"workload": "cl1m graph, 1,000 seeds from the top-1% out-degree nodes, under its trivalency p "
                           "and constant p from 0.03 down to 0.001; 2^20 fixed-count samples, best of 3",
               "rows": stage1_skip_gain(P, g, top_outdeg_seed_set(g, 1000, 7),
                                        skip_models(g, (0.03, 0.01, 0.003, 0.001)), 1 << 20, repeats=3)}
        print(json.dumps(out), flush=True)
        return
    t = time.perf_counter()
    g, sets, extra = make_config("cl1m")
    S = sets[0]
    log(f"graph n={g.n} m={g.m} seed={S.tolist()} built in {time.perf_counter() - t:.1f}s")
    G = P.Graph.from_inputs(g)
    if args.variant >= 0:
        G.tune(variant=args.variant)
    if args.pipeline is not None:
        G.tune(pipeline=args.pipeline)
    eps, delta = extra["eps"], extra["delta"]
    for w in range(args.warmup):
        t = time.perf_counter()
        r = G.estimate(S, eps, delta, mode=P.OI_MODE_SOIEA)
        log(f"warmup {w}: {time.perf_counter() - t:.2f}s OI={r['oi']:.6g} samples={r['samples_x'] + r['samples_xp']}")
    G.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot_samples = tot_edges = 0
    res = None
    for k in range(args.steps):
        res = G.estimate(S, eps, delta, mode=P.OI_MODE_SOIEA)
        tot_samples += res["samples_x"] + res["samples_xp"]
        tot_edges += res["edges_examined"]
        log(f"step {k}: OI={res['oi']:.6g} IS={res['is_']:.6g} T={res['T']} rounds={res['rounds']}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tm = G.timing()
    G.timing(False)
    # roofline of the kernel that took the most time: its algorithmic ALU
    # operations (a coin per examined edge, a selection draw per sample) over
    # its event-timed duration, against the vector ALU peak; the bytes it
    # must read over the same time are reported beside it
    kern = max(("tiny", "small", "large"), key=lambda k: tm[f"{k}_ms"])
    launches = max(tm["launches"], 1)
    lpe = tm["launches"] / args.steps
    avg_ms = tm[f"{kern}_ms"] / launches
    kbytes = BYTES_PER_NODE * tm[f"{kern}_y"] + BYTES_PER_EDGE * tm[f"{kern}_edges"]
    sel = tm["samples"] if (kern == "tiny" and res and res["l"] > 1) else 0
    kops = OPS_PER_COIN * tm[f"{kern}_edges"] + OPS_PER_SELECTION * sel
    sec = avg_ms * 1e-3
    achieved = (kops / launches) / sec / 1e12 if avg_ms > 0 else 0.0
    alg_gbps = (kbytes / launches) / sec / 1e9 if avg_ms > 0 else 0.0
    cnt = measured_counters(f"{kern}_kernel", lpe)
    coin = G.coin_probe(1 << 22, 64)
    coins_per_s = tm[f"{kern}_edges"] / (tm[f"{kern}_ms"] * 1e-3) if tm[f"{kern}_ms"] > 0 else 0.0
    roofline = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                "frac": achieved / ALU_PEAK_TOPS, "traffic": cnt["bytes_per_launch"] if cnt else None,
                "kernel": f"{kern}_kernel", "avg_launch_ms": avg_ms, "launches": tm["launches"],
                "ops_per_launch": kops / launches, "ops_per_coin": OPS_PER_COIN,
                "valu_busy": cnt["valu_busy"] if cnt else None,
                "valu_lane_ops_per_edge": cnt["valu_lane_ops_per_edge"] if cnt else None,
                "l2_hit_rate": cnt["l2_hit_rate"] if cnt else None,
                "hbm_gbps": cnt["bytes_per_launch"] / sec / 1e9 if cnt and avg_ms > 0 else None,
                "algorithmic_bytes_per_launch": kbytes / launches, "algorithmic_gbps": alg_gbps,
                "coin_ceiling_words_per_s": coin["words_per_s"],
                "frac_of_coin_ceiling": coins_per_s / coin["words_per_s"] if coin["words_per_s"] > 0 else None}
    out = {
        "metric": METRIC,
        "value": tot_samples / dt,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "cl1m: Chung-Lu n=1e6 m~1e7 gamma=2.1 trivalency p, |S|=1, SOIEA eps=0.05 "
                               "delta=1e-6 (one full RSA estimate per step)",
                   "n": g.n, "m": g.m, "seed_set": S.tolist(), "eps": eps, "delta": delta},
        "gteps": tot_edges / dt / 1e9,
        "estimates_per_s": args.steps / dt,
        "samples_per_step": tot_samples / args.steps,
        "oi": res["oi"] if res else None,
        "roofline": roofline,
        "sampler": {k: tm[k] for k in ("tiny_ms", "small_ms", "large_ms", "samples", "handed_small",
                                       "handed_large", "tiny_y", "small_y", "large_y")},
    }
    if args.minimal:
        G.close()
        print(json.dumps(out), flush=True)
        return
    out["spread"] = seed_spread(P, G, g, eps, delta, args.spread)
    from oi_inputs import top_outdeg_seed_set
    out["stage1_skip"] = {
        "workload": "cl1m graph, 1,000 seeds from the top-1% out-degree nodes: its own trivalency p (a dense "
                    "table) and constant p = 0.003 (a sparse one)",
        "rows": stage1_skip_gain(P, g, top_outdeg_seed_set(g, 1000, 7), skip_models(g, (0.003,)), 1 << 18)}
    gr = gather_roofline(G)
    out["roofline"]["measured_gather_gbps"] = gr["gbps"]
    out["roofline"]["frac_of_measured_gather"] = alg_gbps / gr["gbps"] if gr["gbps"] > 0 else None
    out["roofline"]["gather_probe"] = {"nodes": 1 << 26, "edges": gr["edges"], "ms": gr["ms"]}
    G.close()
    if not args.no_backward:
        out["backward"] = backward_ratio(P)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, S, args.cpu_seconds)
    if not args.no_batched:
        # the metric's second half: seed-set estimates/s batched vs one at a
        # time at eps = 0.05, where single queries leave the GPU idle (er2k)
        # and on the 4M-node workload's stratified subset
        a = argparse.Namespace(**vars(args))
        a.queries, a.eps = 256, 0.05
        small = batched_vs_single_small(P, a)
        a.queries, a.eps = 2 * args.batched_per_stratum, 0.05
        big = batched_vs_single(P, a, per_stratum=True)
        big.pop("autotune", None)
        out["batched"] = {"er2k": small, "cl4m": big}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
