"""Exact, sampling-free failure probabilities of RSA (Alg. 3) on two-point
streams, for the oracle's pins of Theorem 4 (1).

The stream is Y_i in {y0, y1} (y0 < y1, integers) with Pr[Y_i = y1] = p,
i.i.d., and the estimator sees X_i = scale * Y_i + offset, as SOIEA
(scale 1, offset 0) and SIEA (scale beta_0, offset |S|, Eq. z_s) do.  A
two-point law on [a, b] has the largest variance for its mean, the case the
Chernoff-like bounds behind Theorems 3 and 4 are written for.

Every decision of RSA depends on the streams only through integer sums, so
its law can be summed out exactly:

  step 1 (GSRA with sqrt(eps), delta/3): the running sum of X is
      nondecreasing, so step 1 stops at T1 = t with s_{t-1} = sigma successes
      among the first t - 1 draws and X_t = x iff the sum at (t - 1, sigma)
      is below the threshold and the sum at (t, sigma + x) is not; given
      that, the first t - 1 draws are exchangeable;
  step 2: N_sigma pairs of the independent stream X', each pair differing
      with probability 2p(1 - p), so the integer sum of squared
      differences is (y1 - y0)^2 * Binomial(N_sigma, 2p(1 - p));
  step 3: the estimate sums X_1..X_T: for T < t its successes are
      hypergeometric (sigma successes among t - 1 draws, T taken); for
      T >= t they are sigma + x + Binomial(T - t, p).

The thresholds, N_sigma and T come from `plan`, so the oracle's own
controller (oracle.rsa_plan) is what gets evaluated; a hand-written plan
with a deliberately changed constant shows which changes the theorem can
detect.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.stats import binom, hypergeom


def _first_true(pred, lo, hi):
    """Smallest integer s in [lo, hi] with pred(s) (pred monotone nondecreasing
    in s, vectorized over numpy arrays lo/hi); hi + 1 where none."""
    lo = lo.astype(np.int64).copy()
    hi = hi.astype(np.int64).copy() + 1
    while True:
        act = lo < hi
        if not act.any():
            return lo
        mid = (lo + hi) // 2
        ok = pred(mid)
        hi = np.where(act & ok, mid, hi)
        lo = np.where(act & ~ok, mid + 1, lo)


def step1_cells(ups1, y0, y1, p, scale, offset, tail=1e-19, chunk=1 << 16):
    """The law of step 1's stop: arrays (t, sigma, x, prob) over every cell
    with prob > tail, and the probability mass those cells leave out."""
    dy = y1 - y0

    def crossing(t):
        """Smallest number of successes among t draws at which the stopping
        loop's test (keep drawing while scale * h + offset * T < ups1) ends."""
        t = np.asarray(t, np.int64)
        return _first_true(lambda s: ~(scale * (t * y0 + dy * s).astype(np.float64)
                                        + offset * t.astype(np.float64) < ups1), np.zeros_like(t), t)

    # last t that step 1 reaches with probability above tail
    t_max = 1
    while binom.cdf(crossing([t_max])[0] - 1, t_max, p) > tail * 1e-3:
        t_max *= 2
    out_t, out_s, out_x, out_w = [], [], [], []
    for t0 in range(1, t_max + 1, chunk):
        t = np.arange(t0, min(t0 + chunk, t_max + 1), dtype=np.int64)
        c_t, c_tm1 = crossing(t), crossing(t - 1)
        for x in (0, 1):
            s_lo = np.maximum(c_t - x, 0)
            s_hi = np.minimum(c_tm1 - 1, t - 1)
            width = np.maximum(s_hi - s_lo + 1, 0)
            if width.sum() == 0:
                continue
            tt = np.repeat(t, width)
            ss = np.repeat(s_lo, width) + (np.arange(width.sum()) - np.repeat(np.cumsum(width) - width, width))
            w = binom.pmf(ss, tt - 1, p) * (p if x else 1.0 - p)
            keep = w > tail
            out_t.append(tt[keep]); out_s.append(ss[keep]); out_x.append(np.full(int(keep.sum()), x))
            out_w.append(w[keep])
    t = np.concatenate(out_t); s = np.concatenate(out_s); x = np.concatenate(out_x); w = np.concatenate(out_w)
    return t, s, x, w, max(0.0, 1.0 - float(w.sum()))


def rsa_failure(eps, p, y0, y1, scale, offset, ups1, plan, z=9.5):
    """Exact Pr[|mu_hat - mu| > eps * mu] of RSA (eps < 1/4) on the two-point
    stream, with step 1's threshold ups1 and plan(h1, T1, D) -> (nsigma, T)
    (vectorized).  Returns (failure probability, mass left out by the
    truncations)."""
    t, s, x, w, lost = step1_cells(ups1, y0, y1, p, scale, offset)
    dy = y1 - y0
    h1 = t * y0 + dy * (s + x)
    nsig, _ = plan(h1, t, None)
    nsig = nsig.astype(np.int64)
    q = 2.0 * p * (1.0 - p)
    # window of the pair-difference count K per cell
    mean = nsig * q
    sd = np.sqrt(np.maximum(nsig * q * (1.0 - q), 1e-300))
    k_lo = np.maximum(np.floor(mean - z * sd - 1), 0).astype(np.int64)
    k_hi = np.minimum(np.ceil(mean + z * sd + 1), nsig).astype(np.int64)
    width = k_hi - k_lo + 1
    cell = np.repeat(np.arange(t.size), width)
    K = np.repeat(k_lo, width) + (np.arange(width.sum()) - np.repeat(np.cumsum(width) - width, width))
    pk = binom.pmf(K, nsig[cell], q)
    lost += float(w.sum() - (w[cell] * pk).sum())
    D = K.astype(np.uint64) * np.uint64(dy * dy)
    _, T = plan(h1[cell], t[cell], D)
    T = T.astype(np.int64)
    mu = scale * (y0 + dy * p) + offset

    def est(S, TT):  # the oracle's estimate from its integer sums (R11)
        hT = TT * y0 + dy * S
        return (scale * hT.astype(np.float64) + offset * TT.astype(np.float64)) / TT.astype(np.float64)

    def first(pred, target):
        """Smallest S in [0, T] with pred(S) (monotone), T + 1 if none: start
        from where est(S) = target in real arithmetic, then step to the exact
        boundary of the fp64 predicate."""
        g = np.ceil(((target - offset) / scale - y0) * T / dy)
        S = np.clip(g, 0, T + 1).astype(np.int64)
        while True:  # step down while the predecessor also satisfies pred
            down = (S > 0) & pred(np.maximum(S - 1, 0))
            if not down.any():
                break
            S = np.where(down, S - 1, S)
        while True:  # step up while S does not satisfy pred
            up = (S <= T) & ~pred(np.minimum(S, T))
            if not up.any():
                break
            S = np.where(up, S + 1, S)
        return S

    s_ok_lo = first(lambda S: est(S, T) >= (1.0 - eps) * mu, (1.0 - eps) * mu)   # first S not failing low
    s_bad_hi = first(lambda S: est(S, T) > (1.0 + eps) * mu, (1.0 + eps) * mu)   # first S failing high
    tc, sc, xc = t[cell], s[cell], x[cell]
    fail = np.zeros(T.size)
    less = T < tc
    if less.any():
        M, n, N = tc[less] - 1, sc[less], T[less]
        fail[less] = hypergeom.cdf(s_ok_lo[less] - 1, M, n, N) + hypergeom.sf(s_bad_hi[less] - 1, M, n, N)
    same = T == tc
    if same.any():
        S = sc[same] + xc[same]
        fail[same] = ((S < s_ok_lo[same]) | (S >= s_bad_hi[same])).astype(np.float64)
    more = T > tc
    if more.any():
        base = sc[more] + xc[more]
        m = T[more] - tc[more]
        fail[more] = binom.cdf(s_ok_lo[more] - 1 - base, m, p) + binom.sf(s_bad_hi[more] - 1 - base, m, p)
    return float((w[cell] * pk * fail).sum()), lost


def paper_plan(eps, delta, a, b, scale, offset, factor_ups2=1.0, factor_ups1=1.0):
    """Steps 2 and 3 of Alg. 3 written out from the paper (Alg. 2's Upsilon
    with c(eps', delta) of Table 1; Upsilon_2, N_sigma, rho and T of Alg. 3),
    with optional factors on Upsilon_2 and on step 1's threshold: the
    perturbations whose effect on the guarantee the tests report.  Returns
    (ups1, plan)."""
    def ups(e, d):
        L = math.log(2.0 / d)
        ep = e * (1.0 - (e * b) / ((2.0 + (2.0 / 3.0) * e) * L * (b - a)))
        c = (2.0 + (2.0 / 3.0) * ep) * L / (ep * ep)
        return (1.0 + e) * c * (b - a)

    se = math.sqrt(eps)
    L = math.log(2.0 / delta)
    u2 = 2.0 * (1.0 + se) / (1.0 - se) * (1.0 + math.log(1.5) / L) * ups(eps, delta) * factor_ups2

    def plan(h1, T1, D):
        h1 = np.asarray(h1, np.float64)
        T1 = np.asarray(T1, np.float64)
        mu1 = (scale * h1 + offset * T1) / T1
        ns = np.maximum(np.ceil(u2 * eps / mu1), 1.0)
        if D is None:
            return ns.astype(np.int64), None
        Dd = np.asarray(D).astype(np.float64)
        rho = np.maximum(scale * scale * Dd / 2.0 / ns, eps * mu1 * (b - a))
        T = np.maximum(np.ceil(u2 * rho / (mu1 * mu1 * (b - a))), 1.0)
        return ns.astype(np.int64), T.astype(np.int64)

    return ups(se, delta / 3.0) * factor_ups1, plan


def oracle_plan(O, eps, delta, a, b, scale, offset):
    """(ups1, plan) of the oracle's controller."""
    info = O.rsa_plan(eps, delta, a, b, [1], [1], scale=scale, offset=offset)

    def plan(h1, T1, D):
        r = O.rsa_plan(eps, delta, a, b, h1, T1, D, scale=scale, offset=offset)
        return r["nsigma"], r["T"]

    return info["ups1"], plan
