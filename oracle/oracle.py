"""ctypes wrapper of the FP64 CPU oracle (oracle/liboracle.so) on numpy arrays.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU baseline of the benchmark.  The product path never imports it.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional

import numpy as np

from . import build as _build

_lib = None

ORC_OK, ORC_ERR_ARG, ORC_ERR_NOT_PD, ORC_ERR_NONFINITE, ORC_ERR_DEGENERATE = 0, -1, -3, -4, -5
RW, MALA = 0, 1
RESIDUAL, MULTINOMIAL = 0, 1

_d = ct.POINTER(ct.c_double)
_i32 = ct.POINTER(ct.c_int32)
_i64 = ct.POINTER(ct.c_int64)
_u64 = ct.POINTER(ct.c_uint64)
_u32 = ct.POINTER(ct.c_uint32)
_i8 = ct.POINTER(ct.c_int8)


class Config(ct.Structure):
    _fields_ = [("J", ct.c_int32), ("N", ct.c_int32), ("kind", ct.c_int32),
                ("scheme", ct.c_int32), ("rne_rule", ct.c_int32), ("R_max", ct.c_int32),
                ("max_cycles", ct.c_int32), ("pad_", ct.c_int32),
                ("ess_frac", ct.c_double), ("K_mid", ct.c_double), ("K_final", ct.c_double),
                ("h_init", ct.c_double), ("h_step", ct.c_double), ("h_min", ct.c_double),
                ("h_max", ct.c_double), ("acc_target", ct.c_double), ("seed", ct.c_uint64)]


class Summary(ct.Structure):
    _fields_ = [("logml", ct.c_double), ("logml_nse", ct.c_double), ("meanlog", ct.c_double),
                ("meanlog_nse", ct.c_double), ("cycles", ct.c_int32), ("m_iters", ct.c_int32),
                ("hit_R_max", ct.c_int32), ("status", ct.c_int32)]


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ct.CDLL(path)
        L.orc_philox4x32_10.argtypes = [_u32, _u32, _u32]
        L.orc_u53.argtypes = [ct.c_uint64, ct.c_uint64, ct.c_int64, _u64]
        L.orc_uniforms.argtypes = [ct.c_uint64, ct.c_uint64, ct.c_int64, _d]
        L.orc_normals.argtypes = [ct.c_uint64, ct.c_uint64, ct.c_int64, ct.c_int32, _d]
        L.orc_loglik.argtypes = [_d, _i32, ct.c_int64, ct.c_int32, ct.c_int32, _d, ct.c_int64,
                                 ct.c_int64, ct.c_int64, _d]
        L.orc_loglik_grad.argtypes = L.orc_loglik.argtypes + [_d]
        L.orc_logprior.argtypes = [_d, ct.c_int64, ct.c_int32, _d, _d, _d, _d]
        L.orc_logprior.restype = None
        L.orc_init_prior.argtypes = [_d, _d, ct.c_int32, ct.c_int64, ct.c_uint64, ct.c_uint64, _d]
        L.orc_init_prior.restype = None
        L.orc_gprior_cov.argtypes = [_d, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_double, _d]
        L.orc_correct.argtypes = [_d, _i32, ct.c_int64, ct.c_int32, ct.c_int32, _d, _d,
                                  ct.c_int32, ct.c_int32, ct.c_int64, ct.c_double, _d, _i64, _d]
        L.orc_ess.argtypes = [_d, ct.c_int64]
        L.orc_ess.restype = ct.c_double
        L.orc_logml_update.argtypes = [_d, ct.c_int32, ct.c_int32, _d]
        L.orc_logml_total.argtypes = [_d, ct.c_int32, _d, _d, _d, _d]
        L.orc_logml_total.restype = None
        L.orc_resample_int.argtypes = [_u64, ct.c_int32, ct.c_int32, ct.c_int32, _u64, _i32]
        L.orc_resample.argtypes = [_d, ct.c_int32, ct.c_int32, ct.c_int32, _u64, _i32, _u64]
        L.orc_gather.argtypes = [_i32, ct.c_int64, ct.c_int32, _d, _d]
        L.orc_gather.restype = None
        L.orc_cov.argtypes = [_d, ct.c_int64, ct.c_int32, _d, _d]
        L.orc_cov.restype = None
        L.orc_cholesky.argtypes = [_d, ct.c_int32, _d]
        L.orc_mutate.argtypes = [_d, _i32, ct.c_int64, ct.c_int32, ct.c_int32, _d, _d, _d, _d, _d,
                                 ct.c_int32, ct.c_int32, ct.c_int64, ct.c_double, ct.c_int32,
                                 _d, _d, _d, _d, _i8, _d]
        L.orc_mutate_cov.argtypes = [_d, _i32, ct.c_int64, ct.c_int32, ct.c_int32, _d, _d, _d, _d,
                                     _d, ct.c_int32, ct.c_int32, ct.c_int64, _d, ct.c_int32,
                                     _d, _d, _d, _d, _i8]
        L.orc_moments.argtypes = [_d, ct.c_int32, ct.c_int32, ct.c_int32, _d, _d, _d, _d]
        L.orc_moments.restype = None
        L.orc_sps_run.argtypes = [_d, _i32, ct.c_int64, ct.c_int32, ct.c_int32, _d, _d,
                                  ct.POINTER(Config), _d, _d, _d, _d, _d, _d, _i64, _i32, _d, _d,
                                  _d, ct.c_int64, ct.POINTER(Summary)]
        L.orc_sps_run_fixed.argtypes = [_d, _i32, ct.c_int64, ct.c_int32, ct.c_int32, _d, _d,
                                        ct.POINTER(Config), ct.c_int32, _i64, _i32, _d, _d, _d,
                                        _d, _d, _d, _d, ct.POINTER(Summary)]
        L.orc_threads.argtypes = [ct.c_int]
        L.orc_threads.restype = ct.c_int
        _lib = L
    return _lib


def threads(n: int = 0) -> int:
    """Set the oracle's OpenMP thread count (n > 0); return the count in use."""
    return int(lib().orc_threads(int(n)))


def _p(a, typ):
    return None if a is None else a.ctypes.data_as(typ)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(status, what):
    if status != ORC_OK:
        raise OracleError(status, what)


# ---------------------------------------------------------------- randoms
def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c, _u32), _p(k, _u32), _p(o, _u32))
    return o


def u53(seed: int, stream: int, count: int) -> np.ndarray:
    o = np.zeros(count, dtype=np.uint64)
    lib().orc_u53(seed, stream, count, _p(o, _u64))
    return o


def uniforms(seed: int, stream: int, count: int) -> np.ndarray:
    o = np.zeros(count)
    lib().orc_uniforms(seed, stream, count, _p(o, _d))
    return o


def normals(seed: int, stream: int, P: int, d: int) -> np.ndarray:
    o = np.zeros((P, d))
    lib().orc_normals(seed, stream, P, d, _p(o, _d))
    return o


# ---------------------------------------------------------------- model
def loglik(X, y, C, theta, t0=0, t1=None, grad=False):
    X = _f64(X)
    y = np.ascontiguousarray(y, dtype=np.int32)
    theta = _f64(theta)
    T, k = X.shape
    t1 = T if t1 is None else t1
    P = theta.shape[0]
    ll = np.zeros(P)
    if grad:
        g = np.zeros_like(theta)
        _check(lib().orc_loglik_grad(_p(X, _d), _p(y, _i32), T, k, C, _p(theta, _d), P, t0, t1,
                                     _p(ll, _d), _p(g, _d)), "loglik_grad")
        return ll, g
    _check(lib().orc_loglik(_p(X, _d), _p(y, _i32), T, k, C, _p(theta, _d), P, t0, t1,
                            _p(ll, _d)), "loglik")
    return ll


def prior_factor(d, sd=1.0, cov=None):
    """Lower Cholesky factor L (d x d) of the prior covariance: diag(sd) for
    independent components, else the oracle's own Cholesky of cov."""
    if cov is None:
        return np.diag(_f64(np.broadcast_to(sd, (d,))).copy())
    return cholesky(cov)


def logprior(theta, mean, sd=1.0, cov=None):
    theta = _f64(theta)
    P, d = theta.shape
    mean = _f64(np.broadcast_to(mean, (d,)))
    L = prior_factor(d, sd, cov)
    lp = np.zeros(P)
    g = np.zeros_like(theta)
    lib().orc_logprior(_p(theta, _d), P, d, _p(mean, _d), _p(L, _d), _p(lp, _d), _p(g, _d))
    return lp, g


def init_prior(mean, sd, P, seed, stream, cov=None):
    mean = _f64(mean)
    d = mean.shape[0]
    L = prior_factor(d, sd, cov)
    th = np.zeros((P, d))
    lib().orc_init_prior(_p(mean, _d), _p(L, _d), d, P, seed, stream, _p(th, _d))
    return th


def gprior_cov(X, C, g):
    """Covariance of the free parameters under the normalised g-prior."""
    X = _f64(X)
    T, k = X.shape
    d = k * (C - 1)
    cov = np.zeros((d, d))
    _check(lib().orc_gprior_cov(_p(X, _d), T, k, C, float(g), _p(cov, _d)), "gprior_cov")
    return cov


# ---------------------------------------------------------------- C phase
def correct(X, y, C, theta, ll, J, N, s0, ess_frac=0.5):
    """Returns (log_w, ll_new, t_end, ess_end); ll is not modified."""
    X = _f64(X)
    y = np.ascontiguousarray(y, dtype=np.int32)
    theta = _f64(theta)
    ll = _f64(ll).copy()
    T, k = X.shape
    lw = np.zeros(J * N)
    t_end = ct.c_int64(0)
    ess = ct.c_double(0.0)
    _check(lib().orc_correct(_p(X, _d), _p(y, _i32), T, k, C, _p(theta, _d), _p(ll, _d), J, N,
                             s0, ess_frac, _p(lw, _d), ct.byref(t_end), ct.byref(ess)), "correct")
    return lw, ll, t_end.value, ess.value


def ess(log_w):
    lw = _f64(log_w)
    return lib().orc_ess(_p(lw, _d), lw.shape[0])


# ---------------------------------------------------------------- logML
def logml_update(log_w, J, N, logml_j):
    lw = _f64(log_w)
    lj = _f64(logml_j).copy()
    _check(lib().orc_logml_update(_p(lw, _d), J, N, _p(lj, _d)), "logml_update")
    return lj


def logml_total(logml_j):
    lj = _f64(logml_j)
    a, b, c, e = ct.c_double(), ct.c_double(), ct.c_double(), ct.c_double()
    lib().orc_logml_total(_p(lj, _d), lj.shape[0], ct.byref(a), ct.byref(b), ct.byref(c),
                          ct.byref(e))
    return a.value, b.value, c.value, e.value


# ---------------------------------------------------------------- S phase
def resample_int(W, J, N, scheme, u53_):
    W = np.ascontiguousarray(W, dtype=np.uint64)
    U = np.ascontiguousarray(u53_, dtype=np.uint64)
    anc = np.zeros(J * N, dtype=np.int32)
    _check(lib().orc_resample_int(_p(W, _u64), J, N, scheme, _p(U, _u64), _p(anc, _i32)),
           "resample_int")
    return anc


def resample(log_w, J, N, scheme, u53_):
    lw = _f64(log_w)
    U = np.ascontiguousarray(u53_, dtype=np.uint64)
    anc = np.zeros(J * N, dtype=np.int32)
    W = np.zeros(J * N, dtype=np.uint64)
    _check(lib().orc_resample(_p(lw, _d), J, N, scheme, _p(U, _u64), _p(anc, _i32), _p(W, _u64)),
           "resample")
    return anc, W


# ---------------------------------------------------------------- M phase
def cov(theta):
    theta = _f64(theta)
    P, d = theta.shape
    mean = np.zeros(d)
    V = np.zeros((d, d))
    lib().orc_cov(_p(theta, _d), P, d, _p(mean, _d), _p(V, _d))
    return mean, V


def cholesky(V):
    V = _f64(V)
    d = V.shape[0]
    L = np.zeros_like(V)
    _check(lib().orc_cholesky(_p(V, _d), d, _p(L, _d)), "cholesky")
    return L


def mutate_cov(X, y, C, prior_mean, prior_sd, theta, ll, grad, J, N, t, Sigma, kind, z, u,
               prior_cov=None):
    """One M step with proposal covariance Sigma (d x d).  Returns
    (theta, ll, grad, rate, log_alpha, accepted); inputs untouched."""
    X = _f64(X)
    y = np.ascontiguousarray(y, dtype=np.int32)
    T, k = X.shape
    theta = _f64(theta).copy()
    d = theta.shape[1]
    ll = _f64(ll).copy()
    grad = None if grad is None else _f64(grad).copy()
    pm = _f64(np.broadcast_to(prior_mean, (d,)))
    ps = prior_factor(d, prior_sd, prior_cov)
    S = _f64(Sigma)
    z = _f64(z)
    u = _f64(u)
    P = J * N
    rate = ct.c_double(0.0)
    la = np.zeros(P)
    acc = np.zeros(P, dtype=np.int8)
    _check(lib().orc_mutate_cov(_p(X, _d), _p(y, _i32), T, k, C, _p(pm, _d), _p(ps, _d),
                                _p(theta, _d), _p(ll, _d), _p(grad, _d), J, N, t, _p(S, _d), kind,
                                _p(z, _d), _p(u, _d), ct.byref(rate), _p(la, _d), _p(acc, _i8)),
           "mutate_cov")
    return theta, ll, grad, rate.value, la, acc.astype(bool)


def mutate(X, y, C, prior_mean, prior_sd, theta, ll, grad, J, N, t, h, kind, z, u, prior_cov=None):
    """One M step.  Returns (theta, ll, grad, rate, log_alpha, accepted); inputs untouched."""
    X = _f64(X)
    y = np.ascontiguousarray(y, dtype=np.int32)
    T, k = X.shape
    theta = _f64(theta).copy()
    d = theta.shape[1]
    ll = _f64(ll).copy()
    grad = None if grad is None else _f64(grad).copy()
    pm = _f64(np.broadcast_to(prior_mean, (d,)))
    ps = prior_factor(d, prior_sd, prior_cov)
    z = _f64(z)
    u = _f64(u)
    P = J * N
    rate = ct.c_double(0.0)
    la = np.zeros(P)
    acc = np.zeros(P, dtype=np.int8)
    _check(lib().orc_mutate(_p(X, _d), _p(y, _i32), T, k, C, _p(pm, _d), _p(ps, _d),
                            _p(theta, _d), _p(ll, _d), _p(grad, _d), J, N, t, h, kind,
                            _p(z, _d), _p(u, _d), ct.byref(rate), _p(la, _d), _p(acc, _i8), None),
           "mutate")
    return theta, ll, grad, rate.value, la, acc.astype(bool)


# ---------------------------------------------------------------- accuracy
def moments(g, J, N):
    g = _f64(g)
    if g.ndim == 1:
        g = g[:, None]
    m = g.shape[1]
    mean, sd, nse, rne = (np.zeros(m) for _ in range(4))
    lib().orc_moments(_p(g, _d), J, N, m, _p(mean, _d), _p(sd, _d), _p(nse, _d), _p(rne, _d))
    return mean, sd, nse, rne


def sps_run(X, y, C, prior_mean, prior_sd, J, N, seed, kind=RW, scheme=RESIDUAL, rne_rule=0,
            R_max=100, ess_frac=0.5, K_mid=0.35, K_final=0.9, h_init=0.5, h_step=0.01,
            h_min=0.1, h_max=1.0, acc_target=0.25, max_cycles=4096, record_sigma=0,
            prior_cov=None):
    """Full adaptive SPS (Algorithm 2).  Returns a dict of results; with
    record_sigma = n > 0 the proposal covariances of the first n M steps are
    returned too (the design of Algorithm 3's first pass)."""
    X = _f64(X)
    y = np.ascontiguousarray(y, dtype=np.int32)
    T, k = X.shape
    d = k * (C - 1)
    m = d + C - 1
    P = J * N
    pm = _f64(np.broadcast_to(prior_mean, (d,)))
    ps = prior_factor(d, prior_sd, prior_cov)
    cfg = Config(J=J, N=N, kind=kind, scheme=scheme, rne_rule=rne_rule, R_max=R_max,
                 max_cycles=max_cycles, pad_=0, ess_frac=ess_frac, K_mid=K_mid,
                 K_final=K_final, h_init=h_init, h_step=h_step, h_min=h_min, h_max=h_max,
                 acc_target=acc_target, seed=seed)
    theta = np.zeros((P, d))
    ll = np.zeros(P)
    mean, sd, nse, rne = (np.zeros(m) for _ in range(4))
    rt = np.zeros(max_cycles, dtype=np.int64)
    rR = np.zeros(max_cycles, dtype=np.int32)
    rh = np.zeros(max_cycles)
    ra = np.zeros(max_cycles)
    s = Summary()
    sig = np.zeros((record_sigma, d, d)) if record_sigma else None
    _check(lib().orc_sps_run(_p(X, _d), _p(y, _i32), T, k, C, _p(pm, _d), _p(ps, _d),
                             ct.byref(cfg), _p(theta, _d), _p(ll, _d), _p(mean, _d), _p(sd, _d),
                             _p(nse, _d), _p(rne, _d), _p(rt, _i64), _p(rR, _i32), _p(rh, _d),
                             _p(ra, _d), _p(sig, _d), record_sigma, ct.byref(s)), "sps_run")
    L = s.cycles
    out = dict(theta=theta, ll=ll, mean=mean, sd=sd, nse=nse, rne=rne,
               logml=s.logml, logml_nse=s.logml_nse, meanlog=s.meanlog,
               meanlog_nse=s.meanlog_nse, cycles=L, m_iters=s.m_iters,
               hit_R_max=s.hit_R_max, t=rt[:L].copy(), R=rR[:L].copy(), h=rh[:L].copy(),
               acc=ra[:L].copy())
    if record_sigma:
        if s.m_iters > record_sigma:
            raise ValueError(f"record_sigma={record_sigma} < {s.m_iters} M steps")
        out["sigma"] = sig[:s.m_iters].copy()
    return out


def sps_run_fixed(X, y, C, prior_mean, prior_sd, J, N, seed, t, R, sigma, kind=RW,
                  scheme=RESIDUAL, prior_cov=None):
    """Algorithm 1 with a fixed design (the second pass of Algorithm 3)."""
    X = _f64(X)
    y = np.ascontiguousarray(y, dtype=np.int32)
    T, k = X.shape
    d = k * (C - 1)
    m = d + C - 1
    P = J * N
    pm = _f64(np.broadcast_to(prior_mean, (d,)))
    ps = prior_factor(d, prior_sd, prior_cov)
    cfg = Config(J=J, N=N, kind=kind, scheme=scheme, seed=seed)
    tt = np.ascontiguousarray(t, dtype=np.int64)
    RR = np.ascontiguousarray(R, dtype=np.int32)
    S = _f64(sigma)
    theta = np.zeros((P, d))
    ll = np.zeros(P)
    mean, sd, nse, rne = (np.zeros(m) for _ in range(4))
    s = Summary()
    _check(lib().orc_sps_run_fixed(_p(X, _d), _p(y, _i32), T, k, C, _p(pm, _d), _p(ps, _d),
                                   ct.byref(cfg), len(tt), _p(tt, _i64), _p(RR, _i32), _p(S, _d),
                                   _p(theta, _d), _p(ll, _d), _p(mean, _d), _p(sd, _d),
                                   _p(nse, _d), _p(rne, _d), ct.byref(s)), "sps_run_fixed")
    return dict(theta=theta, ll=ll, mean=mean, sd=sd, nse=nse, rne=rne, logml=s.logml,
                logml_nse=s.logml_nse, cycles=s.cycles, m_iters=s.m_iters)


def sps_two_pass(X, y, C, prior_mean, prior_sd, J, N, seed, kind=RW, **kw):
    """Algorithm 3: an adaptive pass records (t_l, R_l, Sigma_lr); its
    particles are discarded and a second, nonadaptive pass reruns with it."""
    p1 = sps_run(X, y, C, prior_mean, prior_sd, J, N, seed, kind=kind, record_sigma=20000, **kw)
    p2 = sps_run_fixed(X, y, C, prior_mean, prior_sd, J, N, seed, p1["t"], p1["R"], p1["sigma"],
                       kind=kind, scheme=kw.get("scheme", RESIDUAL), prior_cov=kw.get("prior_cov"))
    return p1, p2
