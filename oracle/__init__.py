"""Python access to the CPU oracle (oracle/oi_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check in
__graft_entry__.py and by bench.py's cpu_baseline leg.  The HIP library never
imports, links or calls anything here, and nothing here imports the HIP
library.  Inputs come from `oi_inputs` (seeded generators).

Functions take a graph as (n, row_ptr int64, col int32, p float32) numpy
arrays, or any object with those attributes.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

_lib = None

OK, EINVAL, ERANGE, ENOMEM = 0, -1, -2, -3


class RsaResult(C.Structure):
    _fields_ = [
        ("mu", C.c_double), ("mu1", C.c_double), ("ups", C.c_double),
        ("ups1", C.c_double), ("ups2", C.c_double),
        ("T1", C.c_uint64), ("h1", C.c_uint64), ("nsigma", C.c_uint64),
        ("D_lo", C.c_uint64), ("D_hi", C.c_uint64), ("T", C.c_uint64), ("hT", C.c_uint64),
        ("drawn_x", C.c_uint64), ("drawn_xp", C.c_uint64),
        ("gsra_only", C.c_int32), ("early", C.c_int32),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["D"] = (int(self.D_hi) << 64) | int(self.D_lo)
        return d


def _P(t):
    return C.POINTER(t)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        i64, u64, u32, i32, dbl = C.c_int64, C.c_uint64, C.c_uint32, C.c_int32, C.c_double
        vp = C.c_void_p
        L.oo_philox.argtypes = [vp, vp, vp]
        L.oo_philox.restype = None
        L.oo_set_stage1_skip.argtypes = [i64]
        L.oo_set_stage1_skip.restype = None
        L.oo_set_stage1_skip_cost.argtypes = [C.c_double]
        L.oo_set_stage1_skip_cost.restype = None
        g = [i64, i64, vp, vp, vp]
        L.oo_sample_fixed.argtypes = g + [vp, i64, u32, u32, u32, u64, u64, vp, vp, vp, vp, C.c_int]
        L.oo_stage1.argtypes = g + [vp, i64, i64, _P(i64), _P(dbl), vp, vp, vp, vp, _P(i64)]
        L.oo_mc_fixed.argtypes = g + [vp, i64, u32, u32, u32, u64, u64, vp, vp, vp, _P(i64), C.c_int]
        L.oo_lt_fixed.argtypes = g + [vp, i64, u32, u32, u32, u64, u64, vp, vp, vp, _P(i64), C.c_int]
        L.oo_estimate_lt.argtypes = g + [vp, i64, dbl, dbl, u32, u32, _P(dbl), _P(dbl), _P(i64), _P(RsaResult)]
        L.oo_selection.argtypes = g + [vp, i64, u32, u32, u32, u64, u64, vp]
        L.oo_rsa_arrays.argtypes = [vp, u64, vp, u64, dbl, dbl, dbl, dbl, dbl, dbl, _P(RsaResult)]
        L.oo_gsra_array.argtypes = [vp, u64, dbl, dbl, dbl, dbl, dbl, dbl, _P(dbl), _P(u64), _P(u64), _P(dbl)]
        L.oo_rsa_plan.argtypes = [dbl, dbl, dbl, dbl, dbl, dbl, u64, vp, vp, vp, vp, vp, vp, vp]
        L.oo_estimate.argtypes = g + [vp, i64, dbl, dbl, C.c_int, u32, u32, _P(dbl), _P(dbl), _P(dbl),
                                      _P(i64), _P(RsaResult)]
        L.oo_exact.argtypes = g + [vp, i64, _P(dbl), vp, vp]
        L.oo_backward.argtypes = g + [vp, i64, u32, u32, u64, u64, vp, vp, _P(u64), _P(dbl), C.c_int]
        for f in ("oo_sample_fixed", "oo_mc_fixed", "oo_lt_fixed", "oo_estimate_lt", "oo_stage1", "oo_selection", "oo_rsa_arrays", "oo_gsra_array", "oo_rsa_plan",
                  "oo_estimate", "oo_exact", "oo_backward"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, fn, rc):
        super().__init__(f"oracle {fn} failed with status {rc}")
        self.rc = rc


def _chk(fn, rc):
    if rc != OK:
        raise OracleError(fn, rc)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _graph(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    p = np.ascontiguousarray(g.p, dtype=np.float32)
    return (int(g.n), int(col.shape[0]), rp, col, p)


def _gargs(gg):
    n, m, rp, col, p = gg
    return [n, m, _ptr(rp), _ptr(col), _ptr(p)]


def _seeds(seeds):
    return np.ascontiguousarray(np.atleast_1d(seeds), dtype=np.int32)


def nthreads_default() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


# ---------------------------------------------------------------------------

def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oo_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def set_stage1_skip(min_l: int):
    """Tables of at least max(min_l, 65) entries use Stage-1 skip sampling
    (the default min_l is 4096) when they pass its density test; a
    process-wide setting of the oracle."""
    lib().oo_set_stage1_skip(int(min_l))


def set_stage1_skip_cost(cost: float):
    """Draw-cost ratio of skip sampling's density test (default 8): a long
    table is skip-sampled iff W * cost <= l / 4, W = ceil(l / 256) + the sum
    of its light entries' P_j; 0 drops the test.  Process-wide."""
    lib().oo_set_stage1_skip_cost(float(cost))


def stage1(g, seeds, cap: int = 1 << 24):
    """Stage-1 table: dict(l, beta0, k, v, P, cdf, thr)."""
    gg = _graph(g)
    s = _seeds(seeds)
    l = C.c_int64()
    b0 = C.c_double()
    kk = C.c_int64()
    rc = lib().oo_stage1(*_gargs(gg), _ptr(s), s.size, 0, C.byref(l), C.byref(b0), None, None,
                         None, None, C.byref(kk))
    _chk("stage1", rc)
    L = l.value
    v = np.zeros(L, np.int32)
    P = np.zeros(L, np.float64)
    cdf = np.zeros(L + 1, np.float64)
    thr = np.zeros(L, np.uint64)
    if L <= cap:
        rc = lib().oo_stage1(*_gargs(gg), _ptr(s), s.size, L, C.byref(l), C.byref(b0), _ptr(v),
                             _ptr(P), _ptr(cdf), _ptr(thr), C.byref(kk))
        _chk("stage1", rc)
    return dict(l=L, beta0=b0.value, k=kk.value, v=v, P=P, cdf=cdf, thr=thr)


def sample_fixed(g, seeds, qid: int, seed: int, stream: int, first: int, count: int,
                 want_y: bool = True, want_e: bool = False, nthreads: int | None = None):
    """Per-sample Y (uint32) and E (uint64) of samples first..first+count-1.

    Returns dict(y, e, sum_y, sum_e, beta0, oi, is_) with the fixed-count
    estimate oi = beta_0 * mean(Y) (Lemma 2) and is_ = oi + |S|."""
    gg = _graph(g)
    s = _seeds(seeds)
    y = np.zeros(count, np.uint32) if want_y else None
    e = np.zeros(count, np.uint64) if want_e else None
    sums = np.zeros(2, np.uint64)
    b0 = np.zeros(1, np.float64)
    nt = nthreads_default() if nthreads is None else nthreads
    rc = lib().oo_sample_fixed(*_gargs(gg), _ptr(s), s.size, qid, seed, stream, first, count,
                               _ptr(y), _ptr(e), _ptr(sums), _ptr(b0), nt)
    _chk("sample_fixed", rc)
    # the fixed-count estimate of Lemma 2 (and the FPRAS of Sec. 3.2):
    # OI = beta_0 * mean(Y); IS = OI + |S| (Eq. def)
    k = int(np.unique(s).size)
    b = float(b0[0])
    oi = b * (int(sums[0]) / count) if (b > 0.0 and count > 0) else 0.0
    return dict(y=y, e=e, sum_y=int(sums[0]), sum_e=int(sums[1]), beta0=b, oi=oi, is_=oi + k)


def mc_fixed(g, seeds, qid: int, seed: int, stream: int, first: int, count: int,
             want_y: bool = True, want_e: bool = False, nthreads: int | None = None):
    """Classic IC Monte-Carlo samples (Sec. 2.3): per-sample M - |S| (uint32)
    and E (uint64) of samples first..first+count-1.

    Returns dict(y, e, sum_y, sum_e, k, is_, oi) with the MC_N estimate
    is_ = |S| + mean(M - |S|) of I(S) and oi = is_ - |S|."""
    gg = _graph(g)
    s = _seeds(seeds)
    y = np.zeros(count, np.uint32) if want_y else None
    e = np.zeros(count, np.uint64) if want_e else None
    sums = np.zeros(2, np.uint64)
    kk = C.c_int64()
    nt = nthreads_default() if nthreads is None else nthreads
    rc = lib().oo_mc_fixed(*_gargs(gg), _ptr(s), s.size, qid, seed, stream, first, count,
                           _ptr(y), _ptr(e), _ptr(sums), C.byref(kk), nt)
    _chk("mc_fixed", rc)
    k = kk.value
    oi = int(sums[0]) / count if count else 0.0
    return dict(y=y, e=e, sum_y=int(sums[0]), sum_e=int(sums[1]), k=k, oi=oi, is_=k + oi)


def lt_fixed(g, seeds, qid: int, seed: int, stream: int, first: int, count: int,
             want_y: bool = True, want_e: bool = False, nthreads: int | None = None):
    """LT-model cascades (reading R17): per-sample Y = |cascade| - |S| and E of
    samples first..first+count-1.  Returns dict(y, e, sum_y, sum_e, k, is_, oi)
    with the fixed-count estimates is_ = |S| + mean(Y), oi = mean(Y)."""
    gg = _graph(g)
    s = _seeds(seeds)
    y = np.zeros(count, np.uint32) if want_y else None
    e = np.zeros(count, np.uint64) if want_e else None
    sums = np.zeros(2, np.uint64)
    kk = C.c_int64()
    nt = nthreads_default() if nthreads is None else nthreads
    rc = lib().oo_lt_fixed(*_gargs(gg), _ptr(s), s.size, qid, seed, stream, first, count,
                           _ptr(y), _ptr(e), _ptr(sums), C.byref(kk), nt)
    _chk("lt_fixed", rc)
    k = kk.value
    oi = int(sums[0]) / count if count else 0.0
    return dict(y=y, e=e, sum_y=int(sums[0]), sum_e=int(sums[1]), k=k, oi=oi, is_=k + oi)


def estimate_lt(g, seeds, eps, delta, qid: int, seed: int):
    """SIEA_LT: RSA on LT cascade sizes.  Returns dict(oi, is_, k, rsa)."""
    gg = _graph(g)
    s = _seeds(seeds)
    oi, is_ = C.c_double(), C.c_double()
    kk = C.c_int64()
    r = RsaResult()
    rc = lib().oo_estimate_lt(*_gargs(gg), _ptr(s), s.size, eps, delta, qid, seed, C.byref(oi), C.byref(is_),
                              C.byref(kk), C.byref(r))
    _chk("estimate_lt", rc)
    return dict(oi=oi.value, is_=is_.value, k=kk.value, rsa=r.as_dict())


def selection(g, seeds, qid: int, seed: int, stream: int, first: int, count: int):
    gg = _graph(g)
    s = _seeds(seeds)
    out = np.zeros(count, np.int64)
    rc = lib().oo_selection(*_gargs(gg), _ptr(s), s.size, qid, seed, stream, first, count, _ptr(out))
    _chk("selection", rc)
    return out


def rsa_arrays(x, xp, eps, delta, a, b, scale=1.0, offset=0.0):
    x = np.ascontiguousarray(x, dtype=np.uint32)
    xp = np.ascontiguousarray(xp, dtype=np.uint32)
    r = RsaResult()
    rc = lib().oo_rsa_arrays(_ptr(x), x.size, _ptr(xp), xp.size, eps, delta, a, b, scale, offset,
                             C.byref(r))
    _chk("rsa_arrays", rc)
    return r.as_dict()


def gsra_array(x, eps, delta, a, b, scale=1.0, offset=0.0):
    x = np.ascontiguousarray(x, dtype=np.uint32)
    mu, T, h, ups = C.c_double(), C.c_uint64(), C.c_uint64(), C.c_double()
    rc = lib().oo_gsra_array(_ptr(x), x.size, eps, delta, a, b, scale, offset, C.byref(mu),
                             C.byref(T), C.byref(h), C.byref(ups))
    _chk("gsra_array", rc)
    return dict(mu=mu.value, T=T.value, h=h.value, ups=ups.value)


def rsa_plan(eps, delta, a, b, h1, T1, D=None, scale=1.0, offset=0.0):
    """RSA's step-2 and step-3 sizes (Alg. 3, eps < 1/4) as the oracle's
    controller computes them from the sums it observes: step 1 stopped after
    T1 samples whose Y sum to h1; D (optional) is step 2's integer sum of
    squared paired differences of Y' (below 2^128).  Arrays of equal length.
    Returns dict(nsigma, T (None without D), ups1 (step 1's threshold), ups,
    ups2)."""
    h1 = np.ascontiguousarray(np.atleast_1d(h1), dtype=np.uint64)
    T1 = np.ascontiguousarray(np.atleast_1d(T1), dtype=np.uint64)
    n = h1.size
    assert T1.size == n
    ns = np.zeros(n, np.uint64)
    T = None
    dlo = dhi = None
    if D is not None:
        Da = np.atleast_1d(D)
        if Da.dtype == object:  # Python integers, possibly of 65..128 bits
            dlo = np.array([int(d) & ((1 << 64) - 1) for d in Da], dtype=np.uint64)
            dhi = np.array([int(d) >> 64 for d in Da], dtype=np.uint64)
        else:
            dlo = np.ascontiguousarray(Da, dtype=np.uint64)
            dhi = np.zeros(n, np.uint64)
        assert dlo.size == n
        T = np.zeros(n, np.uint64)
    thr = np.zeros(3, np.float64)
    rc = lib().oo_rsa_plan(float(eps), float(delta), float(a), float(b), float(scale), float(offset), n,
                           _ptr(h1), _ptr(T1), _ptr(dlo), _ptr(dhi), _ptr(ns), _ptr(T), _ptr(thr))
    _chk("rsa_plan", rc)
    return dict(nsigma=ns, T=T, ups1=float(thr[0]), ups=float(thr[1]), ups2=float(thr[2]))


def estimate(g, seeds, eps, delta, mode: int, qid: int, seed: int):
    """SOIEA (mode 0) or SIEA (mode 1).  Returns dict(oi, is_, beta0, k, rsa)."""
    gg = _graph(g)
    s = _seeds(seeds)
    oi, is_, b0 = C.c_double(), C.c_double(), C.c_double()
    kk = C.c_int64()
    r = RsaResult()
    rc = lib().oo_estimate(*_gargs(gg), _ptr(s), s.size, eps, delta, mode, qid, seed,
                           C.byref(oi), C.byref(is_), C.byref(b0), C.byref(kk), C.byref(r))
    _chk("estimate", rc)
    return dict(oi=oi.value, is_=is_.value, beta0=b0.value, k=kk.value, rsa=r.as_dict())


def exact(g, seeds, want_grad: bool = False):
    """Exact Ext(S), the law of |r_g(S)\\S| and optionally dExt/dp by
    enumerating every live-edge graph.  Returns dict(ext, dist, grad)."""
    gg = _graph(g)
    s = _seeds(seeds)
    ext = C.c_double()
    dist = np.zeros(gg[0] + 1, np.float64)
    grad = np.zeros(gg[1], np.float64) if want_grad else None
    rc = lib().oo_exact(*_gargs(gg), _ptr(s), s.size, C.byref(ext), _ptr(dist), _ptr(grad))
    _chk("exact", rc)
    return dict(ext=ext.value, dist=dist, grad=grad)


def backward(g, seeds, qid: int, seed: int, first: int, count: int, want_sq: bool = False,
             nthreads: int | None = None):
    """Score-function sums over samples first..first+count-1 of stream X.

    Returns dict(acc, acc2, sum_y, beta0, count) with acc[e] = sum_s Y_s sc_s(e);
    the gradient of beta0*mean(Y) is beta0/count*acc."""
    gg = _graph(g)
    s = _seeds(seeds)
    acc = np.zeros(gg[1], np.float64)
    acc2 = np.zeros(gg[1], np.float64) if want_sq else None
    sy = C.c_uint64()
    b0 = C.c_double()
    nt = nthreads_default() if nthreads is None else nthreads
    rc = lib().oo_backward(*_gargs(gg), _ptr(s), s.size, qid, seed, first, count, _ptr(acc),
                           _ptr(acc2), C.byref(sy), C.byref(b0), nt)
    _chk("backward", rc)
    return dict(acc=acc, acc2=acc2, sum_y=sy.value, beta0=b0.value, count=count)


def grad_p(g, seeds, qid, seed, count, first=0, nthreads=None):
    """fp64 estimate of dOI/dp over `count` samples."""
    r = backward(g, seeds, qid, seed, first, count, nthreads=nthreads)
    return r["beta0"] / count * r["acc"]
