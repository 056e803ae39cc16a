"""Pins of the oracle's Stage-1 skip sampling (Alg. 1, Stage 1 drawn as in
reading R16 for long tables: own coins for entries with P >= 1/2, one walk
per 256-entry segment for the others).  The law must be Stage 1's: after the
selection i, every later entry live independently with probability P_j.

* A star whose centre is S has no Stage-2 edges, so Y = 1 + the number of
  live entries after i.  Its exact law is the mixture over i (weights
  Pr[A_i] / beta_0, Eq. pai) of Poisson-binomial laws of the later P_j,
  computed here by a recursion over the table; the skip-sampled Y must fit
  it (chi-square), across heavy, light, zero and certain entries and
  several segments.
* On a weighted-cascade Chung-Lu graph (Stage 2 included) the law of Y
  under skip sampling equals the law under the plain coins (two-sample
  chi-square), as do the estimates and the examined-edge counts' definition.
* Tables below the threshold keep the plain coins bit for bit.
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O
from oi_inputs import chung_lu_graph, make_config, star_graph, uniform_seed_set, wc_probs
from test_oracle_sampler import _chi2_pvalue

SEED = 0x17044794


@pytest.fixture
def skip_from_65():
    O.set_stage1_skip(65)
    O.set_stage1_skip_cost(0)    # no density test: the tables here are dense
    yield
    O.set_stage1_skip(4096)
    O.set_stage1_skip_cost(8)


def _star_probs(l, rng):
    """Light entries in (0, 0.2), some heavy ones in [0.5, 0.99), some zero,
    a few certain (p = 1) and a few tiny (1e-3)."""
    p = rng.uniform(0.0, 0.2, l)
    heavy = rng.random(l) < 0.08
    p[heavy] = rng.uniform(0.5, 0.99, heavy.sum())
    p[rng.random(l) < 0.05] = 0.0
    p[rng.random(l) < 0.01] = 1.0
    p[rng.random(l) < 0.05] = 0.001
    return p.astype(np.float32)


def _star_law(P, cdf):
    """Exact law of Y on a star with Stage-1 table (P, cdf): Y = 1 + number of
    live entries after the selected one."""
    l = P.size
    beta0 = cdf[-1]
    law = np.zeros(l + 1)
    suffix = np.array([1.0])   # law of the number of live entries in (i, l)
    for i in range(l - 1, -1, -1):
        w = (cdf[i + 1] - cdf[i]) / beta0   # Pr[A_i] / beta_0
        if w > 0:
            law[1:1 + suffix.size] += w * suffix
        suffix = np.convolve(suffix, [1.0 - P[i], P[i]])
    return law


def test_skip_law_on_a_star_matches_the_exact_law(skip_from_65):
    rng = np.random.default_rng(4)
    probs = _star_probs(700, rng)
    g = star_graph(probs)
    t = O.stage1(g, [0])
    assert t["l"] == 700
    law = _star_law(t["P"], t["cdf"])
    assert law.sum() == pytest.approx(1.0, abs=1e-12)
    N = 300_000
    r = O.sample_fixed(g, [0], qid=3, seed=SEED, stream=0, first=0, count=N, want_e=True)
    y = r["y"].astype(np.int64)
    counts = np.bincount(y, minlength=law.size)
    assert _chi2_pvalue(counts[:law.size], law) > 1e-4
    mean = (law * np.arange(law.size)).sum()
    assert abs(y.mean() - mean) < 5 * y.std() / np.sqrt(N)
    # the examined-edge count keeps l - 1 - i (reading R15) on a star
    sel = O.selection(g, [0], 3, SEED, 0, 0, N)
    np.testing.assert_array_equal(r["e"], (700 - 1 - sel).astype(np.uint64))


def test_skip_and_plain_give_the_same_law_with_stage2(skip_from_65):
    """Chung-Lu graph with weighted-cascade p, seed set of 60 nodes (table of
    several hundred entries): skip sampling and plain coins draw different
    samples with the same law."""
    g = chung_lu_graph(20000, 200000, 2.1, 7)
    g = g.with_p(wc_probs(g))
    S = uniform_seed_set(g, 60, 9)
    t = O.stage1(g, S)
    assert t["l"] >= 300
    N = 120_000
    a = O.sample_fixed(g, S, qid=1, seed=SEED, stream=0, first=0, count=N)
    O.set_stage1_skip(1 << 40)
    b = O.sample_fixed(g, S, qid=2, seed=SEED, stream=0, first=0, count=N)
    O.set_stage1_skip(65)
    assert not np.array_equal(a["y"], b["y"])
    ya, yb = a["y"].astype(np.int64), b["y"].astype(np.int64)
    edges = np.unique(np.quantile(np.concatenate([ya, yb]), np.linspace(0, 1, 41)))
    ca, _ = np.histogram(ya, bins=edges)
    cb, _ = np.histogram(yb, bins=edges)
    keep = (ca + cb) > 0
    p = stats.chi2_contingency(np.vstack([ca[keep], cb[keep]]))[1]
    assert p > 1e-4
    se = np.hypot(ya.std(), yb.std()) / np.sqrt(N)
    assert abs(ya.mean() - yb.mean()) < 5 * se


def test_short_tables_keep_the_plain_coins():
    """Below the threshold (and always below 65 entries) nothing changes: the
    samples are those of reading R4."""
    g, sets, _ = make_config("er2k")
    S = sets[0]
    a = O.sample_fixed(g, S, 0, SEED, 0, 0, 5000, want_e=True)
    O.set_stage1_skip(1)     # floor of 65: the 1-entry..small tables stay plain
    try:
        b = O.sample_fixed(g, S, 0, SEED, 0, 0, 5000, want_e=True)
    finally:
        O.set_stage1_skip(4096)
    np.testing.assert_array_equal(a["y"], b["y"])
    np.testing.assert_array_equal(a["e"], b["e"])


def test_skip_backward_star_gradient_is_one(skip_from_65):
    """The score-function backward reads each sample's Stage-1 live set, so it
    stays unbiased under skip sampling: on a star, Ext = sum of the leaves'
    p, whose gradient with respect to each leaf's p is 1; every leaf's
    estimate is within 5 standard errors of 1."""
    rng = np.random.default_rng(8)
    probs = np.clip(rng.uniform(0.02, 0.45, 300), 0.02, 0.45).astype(np.float32)
    g = star_graph(probs)
    N = 200_000
    r = O.backward(g, [0], 0, SEED, 0, N, want_sq=True)
    b0 = r["beta0"]
    est = b0 * r["acc"] / N
    se = np.sqrt(np.maximum(b0 * b0 * r["acc2"] / N - est * est, 0.0) / N)
    assert np.all(np.abs(est - 1.0) < 5 * se + 1e-9)


def _walk_draws(P):
    """W of the density test in the order the specification fixes: the
    segment count, then the light entries' P_j in ascending j."""
    W = float((len(P) + 255) // 256)
    for x in P:
        x = float(x)
        if 0.0 < x < 0.5:
            W = W + x
    return W


def _star_probs_of(p):
    """Leaf probabilities: every leaf p, or (for p = "mixed") 2048 heavy
    leaves at 0.9 interleaved with 2048 light ones at 0.02."""
    if p == "mixed":
        q = np.full(4096, 0.02, np.float32)
        q[::2] = 0.9
        return q
    return np.full(4096, p, np.float32)


@pytest.mark.parametrize("p, skipped", [(0.002, True), (0.027, True), (0.0275, False), (0.2, False),
                                        ("mixed", True)])
def test_density_test_decides_by_the_expected_draws(p, skipped):
    """A star of 4096 leaves with every P_j = p: W = 16 + 4096 p walk draws
    against 1024 coin blocks, so with the default cost 8 the table is
    skip-sampled iff p <= 0.02734375.  Its samples are then those drawn with
    the density test off (cost 0), else those of the plain coins (skip
    sampling off); the two differ.  Heavy entries (P >= 1/2) keep their
    coins and do not count: half the leaves at 0.9 and half at 0.02 give
    W = 16 + 2048 * 0.02, skip-sampled (counting the heavy ones would not
    be)."""
    g = star_graph(_star_probs_of(p))
    t = O.stage1(g, [0])
    assert t["l"] == 4096
    W = _walk_draws(t["P"])
    closed = 16 + 2048 * 0.02 if p == "mixed" else 16 + 4096 * p
    assert abs(W - closed) < 1e-3 * W
    assert (W * 8.0 <= 4096 / 4.0) == skipped
    N = 4000
    d = O.sample_fixed(g, [0], 5, SEED, 0, 0, N, want_e=True)
    O.set_stage1_skip_cost(0)
    try:
        s = O.sample_fixed(g, [0], 5, SEED, 0, 0, N, want_e=True)
    finally:
        O.set_stage1_skip_cost(8)
    O.set_stage1_skip(1 << 40)
    try:
        c = O.sample_fixed(g, [0], 5, SEED, 0, 0, N, want_e=True)
    finally:
        O.set_stage1_skip(4096)
    assert not np.array_equal(s["y"], c["y"])
    np.testing.assert_array_equal(d["y"], (s if skipped else c)["y"])
    np.testing.assert_array_equal(d["e"], (s if skipped else c)["e"])
