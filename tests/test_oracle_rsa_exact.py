"""Pins of the oracle's RSA controller (Alg. 3) and of SIEA's range of Z
(Sec. 5.2) beyond the sampled coverage tests.

* Theorem 4 (1), evaluated exactly with no sampling (tests/rsa_exact.py):
  for two-point streams (the law of largest variance on [a, b]) the
  oracle's RSA misses mu by more than eps*mu with probability at most delta,
  in SOIEA form (X = Y on {0, 1}) and in SIEA form (X = beta_0 Y + |S| on
  [|S| + beta_0, |S| + beta_0 (n - |S|)]).  The theorem bounds the sizes
  from below only, and loosely: the same computation with Upsilon_2 six to
  seven times too small is still within delta at delta = 1e-3; one
  written out with Upsilon_2 = 0.15 of its value breaks it.
* The values themselves: every threshold and size the oracle reports
  (Upsilon of step 1, Upsilon, Upsilon_2, N_sigma, rho, T, the estimate) is
  recomputed here from the printed expressions of Table 1, Alg. 2 and
  Alg. 3, on the oracle's own streams (replayed from oracle.sample_fixed),
  in both modes.  This is a transcription check: it pins the oracle's code
  to the printed formulas (and would catch a dropped factor), not the
  formulas to an independent source; the paper prints no worked value for
  these steps.
* SIEA's lower end a = |S| + beta_0: when Alg. 2's early exit applies
  (b - a < eps b), SIEA returns IS = a, which equals the smallest value Z
  can take (Y >= 1), with beta_0 taken from the enumeration.
"""
import math

import numpy as np
import pytest

import oracle as O
import rsa_exact as X
from oi_inputs import tiny16_graph

SEED = 0x17044794


@pytest.mark.parametrize("eps,delta,ps", [
    (0.1, 1e-3, (0.05, 0.25, 0.6, 0.95)),
    (0.2, 0.05, (0.05, 0.3, 0.8)),
])
def test_rsa_theorem4_exact_bernoulli(eps, delta, ps):
    """SOIEA form: X_i in {0, 1} on [a, b] = [0, 1]."""
    ups1, plan = X.oracle_plan(O, eps, delta, 0.0, 1.0, 1.0, 0.0)
    for p in ps:
        f, lost = X.rsa_failure(eps, p, 0, 1, 1.0, 0.0, ups1, plan)
        assert lost < 1e-9
        assert f <= delta, (p, f / delta)


@pytest.mark.parametrize("k,nk,beta0", [(3, 12, 0.3), (1, 40, 0.85)])
def test_rsa_theorem4_exact_siea_two_point(k, nk, beta0):
    """SIEA form: Y in {1, n - |S|}, X = beta_0 Y + |S| on the range
    [|S| + beta_0, |S| + beta_0 (n - |S|)] that the oracle's SIEA uses."""
    eps, delta = 0.1, 1e-3
    a, b = k + beta0, k + beta0 * nk
    ups1, plan = X.oracle_plan(O, eps, delta, a, b, beta0, float(k))
    for p in (0.05, 0.3, 0.7):
        f, lost = X.rsa_failure(eps, p, 1, nk, beta0, float(k), ups1, plan)
        assert lost < 1e-9
        assert f <= delta, (p, f / delta)


def test_rsa_exact_sensitivity_to_upsilon2():
    """What the exact guarantee can see: the oracle's plan and the written-out
    plan agree on every cell; a plan with Upsilon_2 at 0.15 of its value
    fails more often than delta allows, one at 0.3 does not (RSA's sample
    sizes carry that much slack at these parameters)."""
    eps, delta, p = 0.05, 1e-3, 0.25
    ups1, plan = X.oracle_plan(O, eps, delta, 0.0, 1.0, 1.0, 0.0)
    u1, pplan = X.paper_plan(eps, delta, 0.0, 1.0, 1.0, 0.0)
    assert u1 == pytest.approx(ups1, rel=1e-14)
    t, s, x, w, _ = X.step1_cells(ups1, 0, 1, p, 1.0, 0.0)
    h1 = s + x
    ns_o, _ = plan(h1, t, None)
    ns_p, _ = pplan(h1, t, None)
    assert np.array_equal(ns_o.astype(np.int64), ns_p)
    D = (np.arange(h1.size) % 997).astype(np.uint64)
    _, T_o = plan(h1, t, D)
    _, T_p = pplan(h1, t, D)
    assert np.array_equal(T_o.astype(np.int64), T_p)
    f_ok, _ = X.rsa_failure(eps, p, 0, 1, 1.0, 0.0, ups1, plan)
    u1, small = X.paper_plan(eps, delta, 0.0, 1.0, 1.0, 0.0, factor_ups2=0.15)
    f_bad, _ = X.rsa_failure(eps, p, 0, 1, 1.0, 0.0, u1, small)
    u1, mid = X.paper_plan(eps, delta, 0.0, 1.0, 1.0, 0.0, factor_ups2=0.3)
    f_mid, _ = X.rsa_failure(eps, p, 0, 1, 1.0, 0.0, u1, mid)
    assert f_ok < 1e-6 * delta
    assert f_bad > delta
    assert f_mid < delta


# ---------------------------------------------------------------------------
# the printed expressions, written out here from Table 1 and Algs. 2-5
# ---------------------------------------------------------------------------
def _c(e, d):  # Table 1: c(eps, delta) = (2 + 2/3 eps) ln(2/delta) / eps^2
    return (2.0 + 2.0 / 3.0 * e) * math.log(2.0 / d) / e ** 2


def _upsilon(e, d, a, b):  # Alg. 2, line 2
    ep = e * (1.0 - e * b / ((2.0 + 2.0 / 3.0 * e) * math.log(2.0 / d) * (b - a)))
    return (1.0 + e) * _c(ep, d) * (b - a)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("S", [[0], [3, 7], [2, 5, 9]])
def test_rsa_fields_match_the_printed_formulas(mode, S):
    """Every quantity the oracle's RSA reports, recomputed from the printed
    expressions on the oracle's own streams X and X' (Alg. 3 with the
    pairing (X'_{2i-1}, X'_{2i}) and step 3 reusing X_1..X_T; Alg. 4 / 5)."""
    g = tiny16_graph()
    eps, delta = 0.05, 0.01
    r = O.estimate(g, S, eps, delta, mode, 5, SEED)
    rs, k, b0, n = r["rsa"], r["k"], r["beta0"], g.n
    if mode == 0:
        a, b, scale, off = 1.0, float(n - k), 1.0, 0.0      # Lemma 2: 1 <= Y <= n - |S|
    else:
        a, b, scale, off = k + b0, k + b0 * (n - k), b0, float(k)  # Sec. 5.2, range of Z
    # step 1: GSRA(sqrt(eps), delta/3) on X
    se = math.sqrt(eps)
    assert rs["ups1"] == pytest.approx(_upsilon(se, delta / 3, a, b), rel=1e-13)
    T1 = rs["T1"]
    x = O.sample_fixed(g, S, 5, SEED, 0, 0, max(T1, rs["T"]))["y"].astype(np.int64)
    zsum = lambda h, T: scale * h + off * T
    h1 = int(x[:T1].sum())
    assert rs["h1"] == h1
    assert zsum(h1, T1) >= rs["ups1"] > zsum(h1 - x[T1 - 1], T1 - 1)   # the first crossing
    mu1 = zsum(h1, T1) / T1
    assert rs["mu1"] == pytest.approx(mu1, rel=1e-14)
    # step 2
    ups = _upsilon(eps, delta, a, b)
    ups2 = 2.0 * (1.0 + se) / (1.0 - se) * (1.0 + math.log(1.5) / math.log(2.0 / delta)) * ups
    assert rs["ups"] == pytest.approx(ups, rel=1e-13)
    assert rs["ups2"] == pytest.approx(ups2, rel=1e-13)
    nsig = max(1, math.ceil(ups2 * eps / mu1))
    assert rs["nsigma"] == nsig
    xp = O.sample_fixed(g, S, 5, SEED, 1, 0, 2 * nsig)["y"].astype(np.int64)
    D = int(((xp[0::2] - xp[1::2]) ** 2).sum())
    assert rs["D"] == D
    Delta = scale * scale * D / 2.0
    rho = max(Delta / nsig, eps * mu1 * (b - a))
    # step 3
    T = max(1, math.ceil(ups2 * rho / (mu1 ** 2 * (b - a))))
    assert rs["T"] == T
    hT = int(x[:T].sum())
    assert rs["hT"] == hT
    mu = zsum(hT, T) / T
    assert rs["mu"] == pytest.approx(mu, rel=1e-14)
    if mode == 0:
        assert r["oi"] == pytest.approx(b0 * mu, rel=1e-14)          # Alg. 4
    else:
        assert r["is_"] == pytest.approx(mu, rel=1e-14)              # Alg. 5


def test_siea_early_exit_returns_the_smallest_z():
    """With |S| = 13 of 16 nodes, SIEA's range has b - a = beta_0 (n - |S| - 1)
    < eps b, so Alg. 2 returns a without sampling: IS = |S| + beta_0, the
    smallest value Z = beta_0 Y + |S| takes (Y >= 1), beta_0 being the
    enumerated probability of a non-trivial cascade.  SOIEA on the same set
    (range [1, 3]) samples."""
    g = tiny16_graph()
    S = list(range(13))
    ex = O.exact(g, S)
    beta0 = 1.0 - ex["dist"][0]
    r = O.estimate(g, S, 0.3, 0.05, 1, 0, SEED)
    assert r["rsa"]["early"] == 1 and r["rsa"]["T"] == 0
    assert r["is_"] == pytest.approx(13 + beta0, rel=1e-14)
    assert r["oi"] == pytest.approx(beta0, rel=1e-13)
    r0 = O.estimate(g, S, 0.3, 0.05, 0, 0, SEED)
    assert r0["rsa"]["early"] == 0 and r0["rsa"]["T"] > 0
    # one seed: no early exit in either mode
    r1 = O.estimate(g, [0], 0.3, 0.05, 1, 0, SEED)
    assert r1["rsa"]["early"] == 0 and r1["rsa"]["T"] > 0
