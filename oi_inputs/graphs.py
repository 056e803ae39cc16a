"""Deterministic graph, probability and seed-set generators.

Every generator takes an explicit integer seed and uses numpy's PCG64, so the
same call gives the same arrays on every machine that runs this numpy build.

Graph representation (the layout both implementations read):
  row_ptr : int64[n+1]  CSR offsets, row u holds the out-edges of u
  col     : int32[m]    edge targets, sorted ascending inside each row
  p       : float32[m]  IC activation probability w(u, v) of each edge
Edge ids are CSR positions 0..m-1.  No generator emits self-loops or parallel
edges.

The paper's workloads (Sec. 6: SNAP / Twitter / Friendster networks and GTgraph
synthetics, weighted-cascade and constant edge models) are not available here;
these generators produce stand-ins of the same kind: power-law (Chung-Lu)
directed graphs, weighted-cascade p = 1/indeg(v), trivalency-style constant
probabilities, and the small graphs used for exact enumeration.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray  # int32[m]
    p: np.ndarray  # float32[m]
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def outdeg(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def indeg(self) -> np.ndarray:
        return np.bincount(self.col, minlength=self.n).astype(np.int64)

    def with_p(self, p: np.ndarray) -> "Graph":
        assert p.shape == self.col.shape and p.dtype == np.float32
        return Graph(self.n, self.row_ptr, self.col, p, dict(self.meta))

    def edges(self):
        """(src, dst) arrays in edge-id order."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.outdeg())
        return src, self.col.astype(np.int64)


def graph_from_edges(n: int, src, dst, p=None) -> Graph:
    """Build a CSR graph from an edge list; edges are sorted by (src, dst).

    Raises on self-loops or duplicate edges.  `p` follows the input order and
    is permuted along with the edges.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if src.size and (src.min() < 0 or src.max() >= n or dst.min() < 0 or dst.max() >= n):
        raise ValueError("edge endpoint out of range")
    if np.any(src == dst):
        raise ValueError("self-loop")
    key = src * n + dst
    order = np.argsort(key, kind="stable")
    key = key[order]
    if key.size and np.any(key[1:] == key[:-1]):
        raise ValueError("duplicate edge")
    s = src[order]
    d = dst[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, s + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int64)
    if p is None:
        pp = np.zeros(s.size, dtype=np.float32)
    else:
        pp = np.asarray(p, dtype=np.float32)[order]
    return Graph(int(n), row_ptr, d.astype(np.int32), pp)


# ---------------------------------------------------------------------------
# topologies
# ---------------------------------------------------------------------------

def er_graph(n: int, m: int, seed: int) -> Graph:
    """Uniform directed G(n, m): m distinct ordered pairs, no self-loops."""
    if m > n * (n - 1):
        raise ValueError("too many edges")
    rng = np.random.Generator(np.random.PCG64(seed))
    keys = np.empty(0, dtype=np.int64)
    while keys.size < m:
        need = m - keys.size
        draw = rng.integers(0, n * n, size=int(need * 1.2) + 16, dtype=np.int64)
        draw = draw[(draw // n) != (draw % n)]
        # keep first occurrences, in draw order, of keys not seen before
        allk = np.concatenate([keys, draw])
        _, first = np.unique(allk, return_index=True)
        first.sort()
        keys = allk[first][:m]
    keys = np.sort(keys)
    g = graph_from_edges(n, keys // n, keys % n)
    g.meta.update(kind="er", n=n, m=m, seed=seed)
    return g


def chung_lu_weights(n: int, m_target: float, gamma: float) -> np.ndarray:
    """Power-law expected degrees w_i ~ i^(-1/(gamma-1)), summing to about
    m_target, capped at sqrt(m_target) (the cap keeps the largest expected
    degree a small fraction of n)."""
    i = np.arange(1, n + 1, dtype=np.float64)
    w = i ** (-1.0 / (gamma - 1.0))
    cap = np.sqrt(m_target)
    for _ in range(100):
        w *= m_target / w.sum()
        over = w > cap
        if not over.any():
            break
        w[over] = cap
    np.minimum(w, cap, out=w)
    return w


# Per-process state of the block generator (set before worker processes are
# forked, so the large arrays are shared copy-on-write rather than pickled).
_CL_STATE: dict = {}


def _chung_lu_block(b0: int):
    n, block, seed = _CL_STATE["n"], _CL_STATE["block"], _CL_STATE["seed"]
    w_out, cdf = _CL_STATE["w_out"], _CL_STATE["cdf"]
    b1 = min(n, b0 + block)
    rng = np.random.Generator(np.random.PCG64([seed, b0 // block]))
    d = rng.poisson(w_out[b0:b1])
    tot = int(d.sum())
    u = rng.random(tot)
    # the same searchsorted, evaluated in sorted order of u (cache friendly)
    order = np.argsort(u)
    tgt = np.empty(tot, dtype=np.int64)
    tgt[order] = np.searchsorted(cdf, u[order], side="right")
    del order
    np.minimum(tgt, n - 1, out=tgt)
    src = np.repeat(np.arange(b0, b1, dtype=np.int64), d)
    keep = tgt != src
    key = np.unique(src[keep] * n + tgt[keep])
    s = key // n
    return (key % n).astype(np.int32), np.bincount(s - b0, minlength=b1 - b0)


def chung_lu_graph(n: int, m_target: float, gamma: float, seed: int,
                   block: int = 1 << 20, workers: int = 1, progress=None) -> Graph:
    """Directed Chung-Lu graph.

    Out- and in-weights use the same capped power-law sequence, each assigned
    to nodes through its own seeded random permutation (so in- and out-degree
    are independent).  Source u draws d_u ~ Poisson(w_out[u]) targets i.i.d.
    from the in-weight distribution; self-loops and duplicates are dropped.
    Sources are generated in blocks of `block` nodes, each block with its own
    PCG64 stream keyed by (seed, block index), so memory stays bounded and
    `workers` processes can generate blocks in parallel with the same result.
    `progress(done, total)` is called after each block if given.
    """
    top = np.random.Generator(np.random.PCG64(seed))
    w = chung_lu_weights(n, m_target, gamma)
    w_out = w[top.permutation(n)]
    w_in = w[top.permutation(n)]
    del w
    cdf = np.cumsum(w_in)
    del w_in
    cdf /= cdf[-1]
    _CL_STATE.update(n=n, block=block, seed=seed, w_out=w_out, cdf=cdf)
    starts = list(range(0, n, block))
    try:
        parts = []
        if workers > 1 and len(starts) > 1:
            import multiprocessing as mp
            with mp.get_context("fork").Pool(min(workers, len(starts))) as pool:
                for part in pool.imap(_chung_lu_block, starts, chunksize=1):
                    parts.append(part)
                    if progress:
                        progress(len(parts), len(starts))
        else:
            for b0 in starts:
                parts.append(_chung_lu_block(b0))
                if progress:
                    progress(len(parts), len(starts))
    finally:
        _CL_STATE.clear()
    degs = np.concatenate([d for _, d in parts]) if parts else np.zeros(0, dtype=np.int64)
    col = np.concatenate([c for c, _ in parts]) if parts else np.zeros(0, dtype=np.int32)
    del parts
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(degs, out=row_ptr[1:])
    g = Graph(int(n), row_ptr, col, np.zeros(col.size, dtype=np.float32))
    g.meta.update(kind="chung_lu", n=n, m_target=m_target, m=int(col.size),
                  gamma=gamma, seed=seed)
    return g


def tiny16_graph(seed: int = 16, n: int = 16, m: int = 24) -> Graph:
    """16 nodes, 24 distinct non-loop edges, p ~ U[0.05, 0.5] in fp32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pairs = [(a, b) for a in range(n) for b in range(n) if a != b]
    pick = rng.choice(len(pairs), size=m, replace=False)
    src = np.array([pairs[i][0] for i in pick])
    dst = np.array([pairs[i][1] for i in pick])
    p = rng.uniform(0.05, 0.5, size=m).astype(np.float32)
    g = graph_from_edges(n, src, dst, p)
    g.meta.update(kind="tiny16", seed=seed)
    return g


def fig1_graph(p: float = 0.1) -> Graph:
    """A 4-node graph consistent with the worked example of Fig. 1: nodes
    u=0, v=1, w=2, x=3 and edges u->v, v->w, v->x, all with probability p.
    (The figure itself is not in the paper text; this topology reproduces all
    of the printed influence values.)"""
    return graph_from_edges(4, [0, 1, 1], [1, 2, 3], [p, p, p])


def star_graph(probs) -> Graph:
    """Centre 0 with out-edges 0 -> i (i = 1..k) of the given probabilities."""
    probs = np.asarray(probs, dtype=np.float32)
    k = probs.size
    return graph_from_edges(k + 1, np.zeros(k, dtype=np.int64), np.arange(1, k + 1), probs)


def path_graph(probs) -> Graph:
    """Directed path 0 -> 1 -> ... -> k with edge i -> i+1 of probability probs[i]."""
    probs = np.asarray(probs, dtype=np.float32)
    k = probs.size
    return graph_from_edges(k + 1, np.arange(k), np.arange(1, k + 1), probs)


def out_tree_graph(parent, probs) -> Graph:
    """Out-tree: node i (i >= 1) has parent parent[i-1] < i, edge parent -> i."""
    parent = np.asarray(parent, dtype=np.int64)
    k = parent.size
    return graph_from_edges(k + 1, parent, np.arange(1, k + 1), probs)


# ---------------------------------------------------------------------------
# edge models (Sec. 6 settings: weighted cascade and constant probabilities)
# ---------------------------------------------------------------------------

def wc_probs(g: Graph) -> np.ndarray:
    """Weighted cascade: p(u, v) = 1 / indeg(v), as fp32 division."""
    indeg = g.indeg().astype(np.float32)
    return (np.float32(1.0) / indeg[g.col]).astype(np.float32)


def trivalency_probs(g: Graph, seed: int) -> np.ndarray:
    """Each edge's p drawn uniformly from {0.1, 0.01, 0.001} (fp32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    vals = np.array([0.1, 0.01, 0.001], dtype=np.float32)
    return vals[rng.integers(0, 3, size=g.m)]


def sigmoid_theta_probs(g: Graph, seed: int, mu: float = -3.0, sd: float = 1.0):
    """theta ~ N(mu, sd) in fp32; p = sigmoid(theta) evaluated in fp64 from the
    fp32 theta, then rounded to fp32.  Returns (theta, p)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = rng.normal(mu, sd, size=g.m).astype(np.float32)
    t = theta.astype(np.float64)
    p = (1.0 / (1.0 + np.exp(-t))).astype(np.float32)
    return theta, p


def constant_probs(g: Graph, p: float) -> np.ndarray:
    """The constant edge model of Sec. 6: every edge has probability p."""
    return np.full(g.m, p, dtype=np.float32)


def uniform_probs(g: Graph, seed: int, lo: float, hi: float) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=g.m).astype(np.float32)


# ---------------------------------------------------------------------------
# seed sets
# ---------------------------------------------------------------------------

def seed_node_outdeg_ge1(g: Graph, seed: int) -> np.ndarray:
    """One node drawn uniformly among nodes with out-degree >= 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cand = np.flatnonzero(g.outdeg() >= 1)
    return np.array([cand[rng.integers(0, cand.size)]], dtype=np.int32)


def outdeg_ge1_nodes(g: Graph, count: int, seed: int) -> np.ndarray:
    """`count` distinct nodes drawn uniformly among nodes with out-degree >= 1
    (single-node seed sets whose outward influence is positive)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cand = np.flatnonzero(g.outdeg() >= 1)
    return np.sort(rng.choice(cand, size=min(count, cand.size), replace=False)).astype(np.int32)


def uniform_seed_set(g: Graph, k: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(g.n, size=k, replace=False)).astype(np.int32)


def top_outdeg_seed_set(g: Graph, k: int, seed: int, frac: float = 0.01) -> np.ndarray:
    """k nodes drawn without replacement from the top `frac` of nodes by
    out-degree (ties broken by node id)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    deg = g.outdeg()
    order = np.lexsort((np.arange(g.n), -deg))
    top = order[: max(1, int(round(frac * g.n)))]
    k = min(k, top.size)
    return np.sort(rng.choice(top, size=k, replace=False)).astype(np.int32)


def batched_seed_sets(g: Graph, count: int, kmin: int, kmax: int, seed: int,
                      top_frac: float = 0.01):
    """`count` seed sets with |S| uniform in [kmin, kmax]; the first half drawn
    uniformly over all nodes, the second half from the top `top_frac`
    out-degree nodes.  Returns (offsets int64[count+1], seeds int32[...])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(kmin, kmax + 1, size=count)
    deg = g.outdeg()
    order = np.lexsort((np.arange(g.n), -deg))
    top = order[: max(1, int(round(top_frac * g.n)))]
    sets = []
    for i, k in enumerate(sizes):
        pool_top = i >= count // 2
        if pool_top:
            kk = min(int(k), top.size)
            s = rng.choice(top, size=kk, replace=False)
        else:
            s = rng.choice(g.n, size=int(k), replace=False)
        sets.append(np.sort(s).astype(np.int32))
    off = np.zeros(count + 1, dtype=np.int64)
    off[1:] = np.cumsum([s.size for s in sets])
    return off, np.concatenate(sets) if sets else np.zeros(0, dtype=np.int32)
