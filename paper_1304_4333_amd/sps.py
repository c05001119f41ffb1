"""Python binding of libsps (include/sps.h): argument marshalling only.

Each function carries the name of the C entry point it calls and takes torch
tensors on the context's GPU.  Shapes, dtypes, devices and contiguity are
checked here; every computation runs in the HIP library.  There is no CPU
fallback: if libsps.so cannot be loaded the first call raises.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsps.so")

SPS_OK, SPS_ERR_ARG, SPS_ERR_HIP, SPS_ERR_NOT_PD = 0, -1, -2, -3
SPS_ERR_NONFINITE, SPS_ERR_DEGENERATE, SPS_ERR_NOMEM, SPS_ERR_STATE = -4, -5, -6, -7
SPS_FP64, SPS_FP32, SPS_BF16X3 = 0, 1, 2
SPS_RESIDUAL, SPS_MULTINOMIAL = 0, 1
SPS_RW, SPS_MALA = 0, 1
SPS_KT_LOGLIK, SPS_KT_LOGLIK_GRAD, SPS_KT_PEROBS = 0, 1, 2

PREC = {"fp64": SPS_FP64, "fp32": SPS_FP32, "bf16x3": SPS_BF16X3}
KIND = {"rw": SPS_RW, "mala": SPS_MALA}
SCHEME = {"residual": SPS_RESIDUAL, "multinomial": SPS_MULTINOMIAL}

_lib = None
_vp = ct.c_void_p
_i64 = ct.c_int64
_i32 = ct.c_int32
_u64 = ct.c_uint64
_dbl = ct.c_double

# name -> argtypes (restype int unless listed in _RESTYPE)
_SIGS = {
    "sps_create": [ct.POINTER(_vp), ct.c_int, _vp],
    "sps_destroy": [_vp],
    "sps_last_error": [_vp],
    "sps_set_stream": [_vp, _vp],
    "sps_set_data": [_vp, _vp, _vp, _i64, _i32, _i32],
    "sps_set_prior": [_vp, _vp, _vp],
    "sps_set_prior_cov": [_vp, _vp, _vp],
    "sps_set_prior_g": [_vp, _dbl, _vp],
    "sps_get_prior_cov": [_vp, _vp],
    "sps_random": [_vp, ct.c_int, _u64, _u64, _i64, _i32, _vp],
    "sps_init_prior": [_vp, _vp, _i64, _u64, _u64],
    "sps_loglik": [_vp, _vp, _i64, _i64, _i64, ct.c_int, _vp],
    "sps_loglik_grad": [_vp, _vp, _i64, _i64, _i64, ct.c_int, _vp, _vp],
    "sps_loglik_noalloc": [_vp, _vp, _i64, _i64, _i64, ct.c_int, _vp],
    "sps_correct": [_vp, _vp, _vp, _i32, _i32, _i64, _dbl, ct.c_int, _vp,
                    ct.POINTER(_i64), ct.POINTER(_dbl)],
    "sps_logml": [_vp, _vp, _i32, _i32, _vp, ct.POINTER(_dbl), ct.POINTER(_dbl)],
    "sps_resample": [_vp, _vp, _i32, _i32, ct.c_int, _vp, _u64, _u64, _vp, _vp, _vp, _vp, _vp,
                     _vp, _vp],
    "sps_resample_fixed": [_vp, _vp, _i32, _i32, ct.c_int, _vp, _vp],
    "sps_mutate": [_vp, _vp, _vp, _vp, _i32, _i32, _i64, _dbl, ct.c_int, ct.c_int, _vp, _vp,
                   _u64, _u64, ct.POINTER(_dbl)],
    "sps_monitor": [_vp, _vp, _i64, _vp],
    "sps_moments": [_vp, _vp, _i32, _i32, _i32, ct.POINTER(_dbl), ct.POINTER(_dbl),
                    ct.POINTER(_dbl), ct.POINTER(_dbl)],
    "sps_mutate_cov": [_vp, _vp, _vp, _vp, _i32, _i32, _i64, _vp, ct.c_int, ct.c_int, _vp, _vp,
                       _u64, _u64, ct.POINTER(_dbl)],
    "sps_last_sigma": [_vp, _vp],
    "sps_mphase": [_vp, _vp, _vp, _vp, _i32, _i32, _i64, ct.c_int, ct.c_int, ct.POINTER(_dbl), _dbl,
                   _dbl, _dbl, _dbl, _dbl, _i32, ct.c_int, _u64, _u64, _u64, _vp, _vp,
                   ct.POINTER(_i32), ct.POINTER(_dbl), ct.POINTER(_dbl)],
    "sps_correct_fixed": [_vp, _vp, _vp, _i32, _i32, _i64, _i64, ct.c_int, _vp],
    "sps_timing_enable": [_vp, ct.c_int],
    "sps_timing_read": [_vp, ct.c_int, ct.POINTER(_i64), ct.POINTER(_dbl)],
}
_RESTYPE = {"sps_destroy": None, "sps_last_error": ct.c_char_p}
ABI_NAMES = tuple(_SIGS)


class SpsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libsps status {status}: {msg}")
        self.status = status


def lib():
    """Load libsps.so (building it first only if no library exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _build
            _build.build(incremental=True)
        L = ct.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)  # AttributeError: the library lacks an entry point
            f.argtypes = args
            f.restype = _RESTYPE.get(name, ct.c_int)
        _lib = L
    return _lib


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ct.c_void_p(t.data_ptr())


class Context:
    """An sps_ctx bound to one GPU and a HIP stream (default: torch's current)."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None):
        self.device = torch.device("cuda", device)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = s
        h = _vp()
        st = lib().sps_create(ct.byref(h), device, _vp(s.cuda_stream))
        if st != SPS_OK:
            raise SpsError(st, "sps_create failed")
        self.handle = h
        self.T = self.k = self.C = self.d = 0

    def close(self):
        if getattr(self, "handle", None):
            lib().sps_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, status: int):
        if status != SPS_OK:
            msg = lib().sps_last_error(self.handle)
            raise SpsError(status, msg.decode() if msg else "")

    # --- tensor checks -------------------------------------------------
    def _t(self, t, dtype, shape, name, allow_none=False):
        if t is None:
            if allow_none:
                return None
            raise ValueError(f"{name} is required")
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}, got {t.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        return t


# ------------------------------------------------------------------ entry points
def sps_set_data(ctx: Context, X: torch.Tensor, y: torch.Tensor, C: int):
    T, k = X.shape
    ctx._t(X, torch.float64, (T, k), "X")
    ctx._t(y, torch.int32, (T,), "y")
    ctx.check(lib().sps_set_data(ctx.handle, _ptr(X), _ptr(y), T, k, C))
    ctx.T, ctx.k, ctx.C, ctx.d = T, k, C, k * (C - 1)


def sps_set_prior(ctx: Context, mean, sd):
    import numpy as np
    m = np.ascontiguousarray(np.broadcast_to(np.asarray(mean, dtype=np.float64), (ctx.d,)))
    s = np.ascontiguousarray(np.broadcast_to(np.asarray(sd, dtype=np.float64), (ctx.d,)))
    ctx.check(lib().sps_set_prior(ctx.handle, m.ctypes.data_as(_vp), s.ctypes.data_as(_vp)))


def sps_set_prior_cov(ctx: Context, mean, cov):
    """Full-covariance Gaussian prior N(mean, cov) on the free parameters."""
    import numpy as np
    m = np.ascontiguousarray(np.broadcast_to(np.asarray(mean, dtype=np.float64), (ctx.d,)))
    S = np.ascontiguousarray(np.asarray(cov, dtype=np.float64))
    if S.shape != (ctx.d, ctx.d):
        raise ValueError(f"cov must be {ctx.d} x {ctx.d}")
    ctx.check(lib().sps_set_prior_cov(ctx.handle, m.ctypes.data_as(_vp), S.ctypes.data_as(_vp)))


def sps_set_prior_g(ctx: Context, g: float, mean=None):
    """The normalised g-prior (covariance built from the data on the device)."""
    import numpy as np
    m = None
    if mean is not None:
        m = np.ascontiguousarray(np.broadcast_to(np.asarray(mean, dtype=np.float64), (ctx.d,)))
    ctx.check(lib().sps_set_prior_g(ctx.handle, float(g), None if m is None else m.ctypes.data_as(_vp)))


def sps_get_prior_cov(ctx: Context):
    import numpy as np
    out = np.zeros((ctx.d, ctx.d))
    ctx.check(lib().sps_get_prior_cov(ctx.handle, out.ctypes.data_as(_vp)))
    return out


def sps_random(ctx: Context, kind: int, seed: int, stream: int, count: int, d: int = 1,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    if kind == 0:
        shape, dt = (count,), torch.uint64
    elif kind == 1:
        shape, dt = (count,), torch.float64
    else:
        shape, dt = (count, d), torch.float64
    if out is None:
        out = torch.empty(shape, dtype=dt, device=ctx.device)
    ctx._t(out, dt, shape, "out")
    ctx.check(lib().sps_random(ctx.handle, kind, seed, stream, count, d, _ptr(out)))
    return out


def sps_init_prior(ctx: Context, theta: torch.Tensor, seed: int, stream: int):
    P = theta.shape[0]
    ctx._t(theta, torch.float64, (P, ctx.d), "theta")
    ctx.check(lib().sps_init_prior(ctx.handle, _ptr(theta), P, seed, stream))


def sps_loglik(ctx: Context, theta: torch.Tensor, t0: int, t1: int, prec: int,
               ll: Optional[torch.Tensor] = None) -> torch.Tensor:
    P = theta.shape[0]
    ctx._t(theta, torch.float64, (P, ctx.d), "theta")
    if ll is None:
        ll = torch.empty(P, dtype=torch.float64, device=ctx.device)
    ctx._t(ll, torch.float64, (P,), "ll")
    ctx.check(lib().sps_loglik(ctx.handle, _ptr(theta), P, t0, t1, prec, _ptr(ll)))
    return ll


def sps_loglik_noalloc(ctx: Context, theta: torch.Tensor, t0: int, t1: int, prec: int,
                       ll: torch.Tensor) -> torch.Tensor:
    """sps_loglik with no device allocation in the call (the caller passes
    ll; the library's per-GPU scratch array holds the partial sums)."""
    P = theta.shape[0]
    ctx._t(theta, torch.float64, (P, ctx.d), "theta")
    ctx._t(ll, torch.float64, (P,), "ll")
    ctx.check(lib().sps_loglik_noalloc(ctx.handle, _ptr(theta), P, t0, t1, prec, _ptr(ll)))
    return ll


def sps_loglik_grad(ctx: Context, theta: torch.Tensor, t0: int, t1: int, prec: int,
                    ll: Optional[torch.Tensor] = None, grad: Optional[torch.Tensor] = None):
    P = theta.shape[0]
    ctx._t(theta, torch.float64, (P, ctx.d), "theta")
    if ll is None:
        ll = torch.empty(P, dtype=torch.float64, device=ctx.device)
    if grad is None:
        grad = torch.empty(P, ctx.d, dtype=torch.float64, device=ctx.device)
    ctx._t(ll, torch.float64, (P,), "ll")
    ctx._t(grad, torch.float64, (P, ctx.d), "grad")
    ctx.check(lib().sps_loglik_grad(ctx.handle, _ptr(theta), P, t0, t1, prec, _ptr(ll), _ptr(grad)))
    return ll, grad


def sps_correct(ctx: Context, theta: torch.Tensor, ll: torch.Tensor, J: int, N: int, s0: int,
                ess_frac: float, prec: int, log_w: Optional[torch.Tensor] = None):
    P = J * N
    ctx._t(theta, torch.float64, (P, ctx.d), "theta")
    ctx._t(ll, torch.float64, (P,), "ll")
    if log_w is None:
        log_w = torch.empty(P, dtype=torch.float64, device=ctx.device)
    ctx._t(log_w, torch.float64, (P,), "log_w")
    t_end = _i64(0)
    ess = _dbl(0.0)
    ctx.check(lib().sps_correct(ctx.handle, _ptr(theta), _ptr(ll), J, N, s0, ess_frac, prec,
                                _ptr(log_w), ct.byref(t_end), ct.byref(ess)))
    return log_w, t_end.value, ess.value


def sps_logml(ctx: Context, log_w: torch.Tensor, J: int, N: int, logml_j: torch.Tensor,
              want_total: bool = True):
    ctx._t(log_w, torch.float64, (J * N,), "log_w")
    ctx._t(logml_j, torch.float64, (J,), "logml_j")
    if want_total:
        a, b = _dbl(), _dbl()
        ctx.check(lib().sps_logml(ctx.handle, _ptr(log_w), J, N, _ptr(logml_j), ct.byref(a), ct.byref(b)))
        return a.value, b.value
    ctx.check(lib().sps_logml(ctx.handle, _ptr(log_w), J, N, _ptr(logml_j), None, None))
    return None


def sps_resample(ctx: Context, log_w: torch.Tensor, J: int, N: int, scheme: int,
                 u53: Optional[torch.Tensor] = None, seed: int = 0, stream: int = 0,
                 ancestor: Optional[torch.Tensor] = None,
                 theta_in=None, theta_out=None, ll_in=None, ll_out=None, grad_in=None,
                 grad_out=None) -> torch.Tensor:
    P = J * N
    ctx._t(log_w, torch.float64, (P,), "log_w")
    ctx._t(u53, torch.uint64, (P,), "u53", allow_none=True)
    if ancestor is None:
        ancestor = torch.empty(P, dtype=torch.int32, device=ctx.device)
    ctx._t(ancestor, torch.int32, (P,), "ancestor")
    for t, n, shp in ((theta_in, "theta_in", (P, ctx.d)), (theta_out, "theta_out", (P, ctx.d)),
                      (ll_in, "ll_in", (P,)), (ll_out, "ll_out", (P,)),
                      (grad_in, "grad_in", (P, ctx.d)), (grad_out, "grad_out", (P, ctx.d))):
        ctx._t(t, torch.float64, shp, n, allow_none=True)
    ctx.check(lib().sps_resample(ctx.handle, _ptr(log_w), J, N, scheme, _ptr(u53), seed, stream,
                                 _ptr(ancestor), _ptr(theta_in), _ptr(theta_out), _ptr(ll_in),
                                 _ptr(ll_out), _ptr(grad_in), _ptr(grad_out)))
    return ancestor


def sps_resample_fixed(ctx: Context, W: torch.Tensor, J: int, N: int, scheme: int,
                     u53: torch.Tensor, ancestor: Optional[torch.Tensor] = None) -> torch.Tensor:
    P = J * N
    ctx._t(W, torch.uint64, (P,), "W")
    ctx._t(u53, torch.uint64, (P,), "u53")
    if ancestor is None:
        ancestor = torch.empty(P, dtype=torch.int32, device=ctx.device)
    ctx._t(ancestor, torch.int32, (P,), "ancestor")
    ctx.check(lib().sps_resample_fixed(ctx.handle, _ptr(W), J, N, scheme, _ptr(u53), _ptr(ancestor)))
    return ancestor


def sps_mutate(ctx: Context, theta: torch.Tensor, ll: torch.Tensor, grad: Optional[torch.Tensor],
               J: int, N: int, t: int, h: float, kind: int, prec: int,
               z: Optional[torch.Tensor] = None, u: Optional[torch.Tensor] = None,
               seed: int = 0, stream: int = 0, want_rate: bool = True):
    P = J * N
    ctx._t(theta, torch.float64, (P, ctx.d), "theta")
    ctx._t(ll, torch.float64, (P,), "ll")
    ctx._t(grad, torch.float64, (P, ctx.d), "grad", allow_none=True)
    ctx._t(z, torch.float64, (P, ctx.d), "z", allow_none=True)
    ctx._t(u, torch.float64, (P,), "u", allow_none=True)
    rate = _dbl(-1.0)
    ctx.check(lib().sps_mutate(ctx.handle, _ptr(theta), _ptr(ll), _ptr(grad), J, N, t, h, kind,
                               prec, _ptr(z), _ptr(u), seed, stream,
                               ct.byref(rate) if want_rate else None))
    return rate.value if want_rate else None


def sps_mutate_cov(ctx: Context, theta: torch.Tensor, ll: torch.Tensor, grad: Optional[torch.Tensor],
                   J: int, N: int, t: int, Sigma: torch.Tensor, kind: int, prec: int,
                   z: Optional[torch.Tensor] = None, u: Optional[torch.Tensor] = None,
                   seed: int = 0, stream: int = 0, want_rate: bool = True):
    P = J * N
    ctx._t(theta, torch.float64, (P, ctx.d), "theta")
    ctx._t(ll, torch.float64, (P,), "ll")
    ctx._t(grad, torch.float64, (P, ctx.d), "grad", allow_none=True)
    ctx._t(Sigma, torch.float64, (ctx.d, ctx.d), "Sigma")
    ctx._t(z, torch.float64, (P, ctx.d), "z", allow_none=True)
    ctx._t(u, torch.float64, (P,), "u", allow_none=True)
    rate = _dbl(-1.0)
    ctx.check(lib().sps_mutate_cov(ctx.handle, _ptr(theta), _ptr(ll), _ptr(grad), J, N, t, _ptr(Sigma),
                                   kind, prec, _ptr(z), _ptr(u), seed, stream,
                                   ct.byref(rate) if want_rate else None))
    return rate.value if want_rate else None


def sps_mphase(ctx: Context, theta: torch.Tensor, ll: torch.Tensor, grad: Optional[torch.Tensor],
               J: int, N: int, t: int, kind: int, prec: int, h: float, h_step: float, h_min: float,
               h_max: float, acc_target: float, K: float, R_max: int, rne_rule: int, seed: int,
               stream0: int, stream_step: int, g_work: torch.Tensor,
               sigma_out: Optional[torch.Tensor] = None):
    """One cycle's M phase.  Returns (R, h after the last update, aggregate
    RNE, acceptance rate of the last step)."""
    P, d = J * N, ctx.d
    ctx._t(theta, torch.float64, (P, d), "theta")
    ctx._t(ll, torch.float64, (P,), "ll")
    ctx._t(grad, torch.float64, (P, d), "grad", allow_none=True)
    ctx._t(g_work, torch.float64, (P, d + ctx.C - 1), "g_work")
    ctx._t(sigma_out, torch.float64, (R_max, d, d), "sigma_out", allow_none=True)
    hh, R, rne, rate = _dbl(h), _i32(0), _dbl(), _dbl()
    ctx.check(lib().sps_mphase(ctx.handle, _ptr(theta), _ptr(ll), _ptr(grad), J, N, t, kind, prec,
                               ct.byref(hh), h_step, h_min, h_max, acc_target, K, R_max, rne_rule, seed,
                               stream0, stream_step, _ptr(g_work), _ptr(sigma_out), ct.byref(R),
                               ct.byref(rne), ct.byref(rate)))
    return R.value, hh.value, rne.value, rate.value


def sps_last_sigma(ctx: Context, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    if out is None:
        out = torch.empty(ctx.d, ctx.d, dtype=torch.float64, device=ctx.device)
    ctx._t(out, torch.float64, (ctx.d, ctx.d), "Sigma")
    ctx.check(lib().sps_last_sigma(ctx.handle, _ptr(out)))
    return out


def sps_correct_fixed(ctx: Context, theta: torch.Tensor, ll: torch.Tensor, J: int, N: int, s0: int,
                      s1: int, prec: int, log_w: Optional[torch.Tensor] = None) -> torch.Tensor:
    P = J * N
    ctx._t(theta, torch.float64, (P, ctx.d), "theta")
    ctx._t(ll, torch.float64, (P,), "ll")
    if log_w is None:
        log_w = torch.empty(P, dtype=torch.float64, device=ctx.device)
    ctx._t(log_w, torch.float64, (P,), "log_w")
    ctx.check(lib().sps_correct_fixed(ctx.handle, _ptr(theta), _ptr(ll), J, N, s0, s1, prec, _ptr(log_w)))
    return log_w


def sps_monitor(ctx: Context, theta: torch.Tensor, g: Optional[torch.Tensor] = None) -> torch.Tensor:
    P = theta.shape[0]
    m = ctx.d + ctx.C - 1
    ctx._t(theta, torch.float64, (P, ctx.d), "theta")
    if g is None:
        g = torch.empty(P, m, dtype=torch.float64, device=ctx.device)
    ctx._t(g, torch.float64, (P, m), "g")
    ctx.check(lib().sps_monitor(ctx.handle, _ptr(theta), P, _ptr(g)))
    return g


def sps_moments(ctx: Context, g: torch.Tensor, J: int, N: int):
    import numpy as np
    P, m = g.shape
    ctx._t(g, torch.float64, (J * N, m), "g")
    outs = [np.zeros(m) for _ in range(4)]
    ptrs = [o.ctypes.data_as(ct.POINTER(_dbl)) for o in outs]
    ctx.check(lib().sps_moments(ctx.handle, _ptr(g), J, N, m, *ptrs))
    return tuple(outs)  # mean, sd, nse, rne


def sps_timing_enable(ctx: Context, enable: bool = True):
    ctx.check(lib().sps_timing_enable(ctx.handle, 1 if enable else 0))


def sps_timing_read(ctx: Context, which: int):
    """(launches, total milliseconds) of one kernel class since the last enable."""
    n, ms = _i64(0), _dbl(0.0)
    ctx.check(lib().sps_timing_read(ctx.handle, which, ct.byref(n), ct.byref(ms)))
    return n.value, ms.value


# ------------------------------------------------------------------ autograd
class LogLik(torch.autograd.Function):
    """ll = sps_loglik(theta); backward uses the hand-written adjoint kernel
    (sps_loglik_grad), dL/dtheta = grad_out[:, None] * G."""

    @staticmethod
    def forward(ctx_, theta: torch.Tensor, sctx: Context, t0: int, t1: int, prec: int):
        th = theta.detach().contiguous()
        if theta.requires_grad:
            ll, g = sps_loglik_grad(sctx, th, t0, t1, prec)
            ctx_.save_for_backward(g)
        else:
            ll = sps_loglik(sctx, th, t0, t1, prec)
            ctx_.save_for_backward(None)
        return ll

    @staticmethod
    def backward(ctx_, grad_out: torch.Tensor):
        (g,) = ctx_.saved_tensors
        return grad_out[:, None] * g, None, None, None, None
