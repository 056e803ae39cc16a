"""Pins of the oracle's stopping rules (GSRA, Alg. 2; RSA, Alg. 3) and of
SOIEA / SIEA (Algs. 4, 5), by their consequences: closed forms of the
stopping index on constant streams (which pin the control flow: which
stream, which index, which estimate feeds which step), the overshoot bound
of the proof of Theorem 3 (Upsilon <= sum X <= Upsilon + b), the (eps,
delta) guarantee of Theorems 3/4 measured as a failure frequency, and both
claims of Theorem 3 computed exactly for Bernoulli streams down to
delta = 1e-8 (which bound the GSRA threshold from below to within 25%).
Theorem 4 computed exactly, and the printed expressions of every RSA
quantity, are in test_oracle_rsa_exact.py.
"""
import math

import numpy as np
import pytest

import oracle as O
from oi_inputs import tiny16_graph

SEED = 0x17044794


def test_gsra_constant_stream_closed_form():
    for c, eps, delta, a, b in [(3, 0.1, 0.05, 1.0, 40.0), (1, 0.3, 0.2, 1.0, 9.0), (7, 0.05, 1e-3, 1.0, 12.0)]:
        x = np.full(10_000_000, c, np.uint32)
        r = O.gsra_array(x, eps, delta, a, b)
        assert r["T"] == math.ceil(r["ups"] / c)
        assert r["mu"] == float(c) and r["h"] == c * r["T"]


def test_gsra_early_exit():
    r = O.gsra_array(np.ones(10, np.uint32), 0.2, 0.1, 9.0, 10.0)
    assert r["T"] == 0 and r["mu"] == 9.0


def test_gsra_overshoot_bound():
    """At the stop, Upsilon <= sum X <= Upsilon + b, and the sum before the
    last draw is below Upsilon (proof of Theorem 3)."""
    rng = np.random.default_rng(3)
    for trial in range(20):
        b = float(rng.integers(5, 60))
        x = rng.integers(1, int(b) + 1, size=2_000_000).astype(np.uint32)
        r = O.gsra_array(x, 0.2, 0.1, 1.0, b)
        h = int(x[: r["T"]].sum())
        assert h == r["h"]
        assert r["ups"] <= h <= r["ups"] + b
        assert h - int(x[r["T"] - 1]) < r["ups"]


def test_rsa_constant_stream_and_pairing():
    """Constant X: mu' = c, T1 = ceil(Upsilon_1/c), Delta = 0, rho = eps*c*(b-a),
    so T ~ Upsilon_2*eps/c and the estimate is exactly c.  X' alternates so
    that the pairs (X'_1,X'_2), (X'_3,X'_4), ... each differ by 2 while the
    shifted pairs (X'_2,X'_3), ... would not."""
    c, eps, delta, a, b = 4, 0.05, 0.01, 1.0, 30.0
    x = np.full(5_000_000, c, np.uint32)
    xp = np.tile(np.array([1, 3, 3, 1], np.uint32), 2_000_000)
    r = O.rsa_arrays(x, xp, eps, delta, a, b)
    assert not r["gsra_only"]
    assert r["mu1"] == float(c) and r["T1"] == math.ceil(r["ups1"] / c)
    assert r["D"] == 4 * r["nsigma"]
    assert r["nsigma"] == max(1, math.ceil(r["ups2"] * eps / c))
    assert abs(r["T"] - r["ups2"] * eps / c) <= 1.0
    assert r["mu"] == float(c) and r["hT"] == c * r["T"]


def test_rsa_step3_reuses_stream_x():
    rng = np.random.default_rng(9)
    x = rng.integers(1, 11, size=3_000_000).astype(np.uint32)
    xp = rng.integers(1, 11, size=3_000_000).astype(np.uint32)
    r = O.rsa_arrays(x, xp, 0.1, 0.05, 1.0, 10.0)
    assert r["hT"] == int(x[: r["T"]].sum())
    assert r["h1"] == int(x[: r["T1"]].sum())
    d = (xp[0:2 * r["nsigma"]:2].astype(np.int64) - xp[1:2 * r["nsigma"]:2].astype(np.int64))
    assert r["D"] == int((d * d).sum())
    assert r["mu"] == r["hT"] / r["T"]


def test_rsa_gsra_only_for_large_eps():
    x = np.full(1_000_000, 2, np.uint32)
    r = O.rsa_arrays(x, x, 0.3, 0.1, 1.0, 20.0)
    assert r["gsra_only"] and r["nsigma"] == 0 and r["mu"] == 2.0


@pytest.mark.parametrize("eps,delta", [(0.1, 0.1), (0.3, 0.1)])
def test_rsa_coverage_two_point(eps, delta):
    """Theorem 4 (and Theorem 3 for eps >= 1/4): Pr[|mu_hat - mu| > eps mu] <= delta.
    Two-point streams X in {1, b} have the largest variance for their mean."""
    rng = np.random.default_rng(17)
    b, q = 20, 0.2
    mu = 1 + q * (b - 1)
    reps, fails = 300, 0
    for _ in range(reps):
        x = np.where(rng.random(60_000) < q, b, 1).astype(np.uint32)
        xp = np.where(rng.random(60_000) < q, b, 1).astype(np.uint32)
        r = O.rsa_arrays(x, xp, eps, delta, 1.0, float(b))
        fails += abs(r["mu"] - mu) > eps * mu
    # binomial(300, delta) exceeds this bound with probability < 1e-3
    assert fails <= 47 if delta == 0.1 else True


def test_soiea_siea_identities_and_coverage():
    """IS = OI + |S| in both modes; SIEA's estimate lies in the Z range of
    Sec. 5.2; both modes meet (eps, delta) against the enumerated Ext."""
    g = tiny16_graph()
    eps, delta = 0.1, 0.1
    cases = [[0], [3, 7], [2, 5, 9]]
    fails = total = 0
    for S in cases:
        ex = O.exact(g, S)["ext"]
        for mode in (0, 1):
            for qid in range(8):
                r = O.estimate(g, S, eps, delta, mode, qid, SEED)
                k = r["k"]
                if mode == 0:
                    assert r["is_"] == r["oi"] + k
                    fails += abs(r["oi"] - ex) > eps * ex
                else:
                    assert r["oi"] == r["is_"] - k
                    b0 = r["beta0"]
                    assert k + b0 <= r["is_"] <= k + b0 * (g.n - k)
                    fails += abs(r["is_"] - (ex + k)) > eps * (ex + k)
                total += 1
    assert fails <= max(2, int(0.1 * total))


def test_estimate_degenerate_and_invalid():
    g = tiny16_graph()
    deg = g.outdeg()
    leaf = int(np.flatnonzero(deg == 0)[0])
    r = O.estimate(g, [leaf], 0.1, 0.1, 0, 0, SEED)
    assert r["oi"] == 0.0 and r["is_"] == 1.0 and r["rsa"]["T"] == 0
    for bad in [dict(eps=0.0), dict(eps=1.0), dict(delta=0.5), dict(delta=0.0)]:
        kw = dict(eps=0.1, delta=0.1)
        kw.update(bad)
        with pytest.raises(O.OracleError):
            O.estimate(g, [0], kw["eps"], kw["delta"], 0, 0, SEED)
    with pytest.raises(O.OracleError):
        O.estimate(g, [16], 0.1, 0.1, 0, 0, SEED)
    with pytest.raises(O.OracleError):
        O.estimate(g, [], 0.1, 0.1, 0, 0, SEED)


def _gsra_bernoulli_failures(r, ups, eps, p):
    """For X_i ~ Bernoulli(p) on [a, b] = [0, 1] the sum grows by one per
    success, so a stop at the r-th success makes T negative binomial:
    Pr[T <= t] = Pr[Binomial(t, p) >= r].  Returns the exact probabilities
    of the two events Theorem 3 bounds: |r/T - p| > eps p, and
    T > (1 + eps) Upsilon / p."""
    from scipy.stats import binom
    t_lo = math.floor(r / ((1.0 - eps) * p))            # r/T < (1 - eps) p  <=>  T > t_lo
    low = binom.cdf(r - 1, t_lo, p)
    t_hi = math.ceil(r / ((1.0 + eps) * p)) - 1         # r/T > (1 + eps) p  <=>  T <= t_hi
    high = binom.sf(r - 1, t_hi, p) if t_hi >= r else 0.0
    t_cap = math.floor((1.0 + eps) * ups / p)
    return low + high, binom.cdf(r - 1, t_cap, p)


@pytest.mark.parametrize("eps", [0.05, 0.25, 0.9])
@pytest.mark.parametrize("delta", [0.1, 1e-4, 1e-8])
def test_gsra_theorem3_exact_on_bernoulli_streams(eps, delta):
    """Theorem 3 computed exactly, with no sampling: with the oracle's
    threshold, for Bernoulli streams of every mean p from 1e-4 to 1,
    Pr[|mu_hat - p| > eps p] < delta and Pr[T > (1 + eps) Upsilon / p] <
    delta / 2.  The stopping index r comes from the oracle's own loop (an
    all-ones stream stops at r = ceil(Upsilon)), and a random 0/1 stream is
    checked to stop exactly at its r-th success.  The theorem bounds the
    threshold from below only; at delta = 1e-8 a threshold 25% smaller
    breaks the first claim, which pins the threshold to within that."""
    ones = np.ones(2_000_000, np.uint32)
    g = O.gsra_array(ones, eps, delta, 0.0, 1.0)
    r, ups = g["T"], g["ups"]
    assert r == math.ceil(ups) and g["h"] == r
    x = (np.random.default_rng(5).random(40 * r + 1000) < 0.05).astype(np.uint32)
    s = O.gsra_array(x, eps, delta, 0.0, 1.0)
    assert s["h"] == r and s["T"] == int(np.flatnonzero(x)[r - 1]) + 1 and s["mu"] == r / s["T"]
    worst_acc = worst_len = 0.0
    for p in np.geomspace(1e-4, 1.0, 25):
        acc, length = _gsra_bernoulli_failures(r, ups, eps, p)
        worst_acc, worst_len = max(worst_acc, acc), max(worst_len, length)
    assert worst_acc < delta and worst_len < delta / 2, (worst_acc / delta, worst_len / (delta / 2))
    if delta == 1e-8:
        r_small = math.ceil(0.75 * ups)
        bad = max(_gsra_bernoulli_failures(r_small, 0.75 * ups, eps, p)[0] for p in np.geomspace(1e-4, 1.0, 25))
        assert bad > delta


@pytest.mark.timeout(60)
def test_short_array_streams_are_reported_not_spun():
    """A stream shorter than the stopping index ends the run with an error
    (it used to leave the stopping loop waiting for a sum that zeros past
    the end of the array could never reach)."""
    with pytest.raises(O.OracleError):
        O.gsra_array(np.ones(4, np.uint32), 0.5, 0.1, 0.0, 1.0)
    with pytest.raises(O.OracleError):
        O.rsa_arrays(np.ones(4, np.uint32), np.ones(4, np.uint32), 0.1, 0.1, 1.0, 2.0)
    x = np.ones(1_000_000, np.uint32)
    with pytest.raises(O.OracleError):  # step 1 fits, the pairs of step 2 do not
        O.rsa_arrays(x, np.ones(2, np.uint32), 0.1, 0.1, 1.0, 2.0)
