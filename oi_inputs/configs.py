"""The five measured workloads, as seeded recipes.

  er2k      ER n=2,000 m=20,000, weighted cascade, |S|=1 (out-degree >= 1),
            100,000 fixed-count samples, query id 0; plus the 16-node/24-edge
            enumeration graph.
  cl1m      Chung-Lu n=1e6, m~1e7, exponent 2.1, trivalency p, |S|=1,
            estimate to eps=0.05, delta=1/n.
  cl4m      Chung-Lu n=4e6, m~7e7, exponent 2.1, weighted cascade, 4,096 seed
            sets |S| in [1,1000] (half uniform, half top-1% out-degree),
            eps=0.1, delta=1e-3.
  cl1m_sig  Chung-Lu n=1e6, m~1e7, p = sigmoid(theta), theta ~ N(-3,1),
            |S|=50, 1e6 fixed-count samples, forward + backward.
  cl100m    Chung-Lu n=1e8, m~1.5e9, weighted cascade, 256 seed sets with
            |S| in {1,10,100}, eps=0.05, delta=1e-6.

Seeds: graph seed = workload number (1..5; the 16-node graph uses 16),
probability seed = 200 + number, seed-set seed = 100 + number, theta seed 40.
The Philox run seed used by tests and the bench is RUN_SEED.
"""
from __future__ import annotations

import os

import numpy as np

from . import graphs as G

RUN_SEED = 0x17044794

CONFIGS = {
    "er2k": dict(number=1, n=2000, m=20000, model="wc", samples=100_000),
    "cl1m": dict(number=2, n=1_000_000, m=10_000_000, gamma=2.1, model="trivalency",
                 eps=0.05, delta=1e-6),
    "cl4m": dict(number=3, n=4_000_000, m=70_000_000, gamma=2.1, model="wc",
                 eps=0.1, delta=1e-3, queries=4096, kmin=1, kmax=1000),
    "cl1m_sig": dict(number=4, n=1_000_000, m=10_000_000, gamma=2.1, model="sigmoid",
                     k=50, samples=1_000_000),
    "cl100m": dict(number=5, n=100_000_000, m=1_500_000_000, gamma=2.1, model="wc",
                   eps=0.05, delta=1e-6, queries=256, sizes=(1, 10, 100)),
}


def _probs(g, model, number):
    if model == "wc":
        return G.wc_probs(g), None
    if model == "trivalency":
        return G.trivalency_probs(g, 200 + number), None
    if model == "sigmoid":
        theta, p = G.sigmoid_theta_probs(g, 40)
        return p, theta
    raise ValueError(model)


def make_config(name: str, n: int | None = None, m: int | None = None, progress=None):
    """Build (graph, seed_sets, extra) for a workload.  `n`/`m` override the
    size (for scaled-down parity cases with the same recipe).

    seed_sets is a list of int32 arrays.  extra holds theta where relevant and
    the eps/delta/sample counts of the workload.  `progress(done, total)` is
    passed to the graph generator (called once per block of sources)."""
    c = dict(CONFIGS[name])
    num = c["number"]
    nn = c["n"] if n is None else n
    mm = c["m"] if m is None else m
    extra = dict(c)
    if name == "er2k":
        g = G.er_graph(nn, mm, num)
    else:
        # blocks generated in parallel for large graphs (same output)
        workers = min(16, os.cpu_count() or 1) if nn >= (1 << 22) else 1
        g = G.chung_lu_graph(nn, mm, c["gamma"], num, workers=workers, progress=progress)
    p, theta = _probs(g, c["model"], num)
    g = g.with_p(p)
    extra["theta"] = theta
    if name in ("er2k", "cl1m"):
        sets = [G.seed_node_outdeg_ge1(g, 100 + num)]
    elif name == "cl1m_sig":
        sets = [G.uniform_seed_set(g, c["k"], 100 + num)]
    elif name == "cl4m":
        off, seeds = G.batched_seed_sets(g, c["queries"], c["kmin"], c["kmax"], 100 + num)
        sets = [seeds[off[i]:off[i + 1]] for i in range(c["queries"])]
    elif name == "cl100m":
        rng = np.random.Generator(np.random.PCG64(100 + num))
        sizes = np.array(c["sizes"])[np.arange(c["queries"]) % len(c["sizes"])]
        sets = [np.sort(rng.choice(g.n, size=int(k), replace=False)).astype(np.int32)
                for k in sizes]
    else:
        raise ValueError(name)
    return g, sets, extra


# Stand-ins for the two smallest networks of the accuracy experiment (Sec. 6,
# Table 2: NetHEP about 15K nodes / 59K edges, NetPHY about 37K / 181K):
# Chung-Lu graphs of those sizes, under the weighted-cascade model and the
# constant models p = 0.1, 0.01, 0.001 of Sec. 6.1.
ACCURACY_GRAPHS = {"hep15k": dict(n=15_000, m=59_000, seed=31), "phy37k": dict(n=37_000, m=181_000, seed=32)}
ACCURACY_MODELS = ("wc", "p0.1", "p0.01", "p0.001")


def accuracy_workload(name: str, model: str, sets: int = 1000):
    """(graph, seed sets) of the accuracy experiment: `sets` distinct single
    nodes with out-degree >= 1 (seed 300 + the graph's seed)."""
    c = ACCURACY_GRAPHS[name]
    g = G.chung_lu_graph(c["n"], c["m"], 2.1, c["seed"])
    if model == "wc":
        p = G.wc_probs(g)
    elif model.startswith("p"):
        p = G.constant_probs(g, float(model[1:]))
    else:
        raise ValueError(model)
    g = g.with_p(p)
    nodes = G.outdeg_ge1_nodes(g, sets, 300 + c["seed"])
    return g, [np.array([v], np.int32) for v in nodes]
