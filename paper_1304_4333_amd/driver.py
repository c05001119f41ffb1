"""Adaptive sequential posterior simulator (Algorithm 2 of Geweke, Durham &
Xu 2013) driven through the libsps C ABI.

Every numerical step runs in the HIP library: C phase with the ESS rule
(sps_correct), log marginal likelihood increments (sps_logml), S phase
(sps_resample), M phase steps (sps_mutate), monitored functions and
NSE/RNE (sps_monitor, sps_moments).  This module holds only the control
flow: the cycle loop, the RNE stopping rule and the step-size rule.

Random streams (shared convention with the oracle's driver):
stream(pass, cycle, step, phase) = pass << 60 | cycle << 32 | step << 4 | phase,
phase 1 = initial particles, 2 = resampling integers, 3 = proposal normals,
4 = acceptance uniforms; pass 0 = adaptive run, 1 = the second pass of the
two-pass algorithm (Algorithm 3).
"""
from __future__ import annotations

import dataclasses
import time
from typing import Optional

import numpy as np
import torch

from . import sps


@dataclasses.dataclass
class SpsConfig:
    """Design constants of Algorithm 2 (all user-changeable, Section 2.3)."""
    J: int
    N: int
    precision: str = "fp64"      # likelihood arithmetic: fp64, fp32, bf16x3
    kind: str = "rw"             # M-phase proposal: rw (the paper) or mala
    scheme: str = "residual"     # S phase: residual or multinomial
    rne_rule: str = "mean"       # aggregate of the monitored RNEs: mean or min
    R_max: int = 100             # cap on M steps per cycle
    ess_frac: float = 0.5        # C phase stops when ESS < ess_frac J N
    K_mid: float = 0.35          # RNE target before the last cycle
    K_final: float = 0.9         # RNE target in the last cycle
    h_init: float = 0.5
    h_step: float = 0.01
    h_min: float = 0.1
    h_max: float = 1.0
    acc_target: float = 0.25
    seed: int = 0

    @staticmethod
    def mala_defaults(**kw) -> "SpsConfig":
        """MALA tuning: target acceptance 0.574, h in [0.01, 2]."""
        base = dict(kind="mala", h_min=0.01, h_max=2.0, acc_target=0.574)
        base.update(kw)
        return SpsConfig(**base)


def stream_id(cycle: int, step: int, phase: int, pass_: int = 0) -> int:
    return (pass_ << 60) | (cycle << 32) | (step << 4) | phase


@dataclasses.dataclass
class Design:
    """What the first pass of Algorithm 3 retains: the cycle ends t_l, the
    number of M steps R_l and the proposal covariances Sigma_lr (device
    tensors, in step order)."""
    t: list
    R: list
    sigma: list


def run_sps(ctx: sps.Context, cfg: SpsConfig, log=None, record: bool = False,
            fused: bool = True) -> dict:
    """One pass of the adaptive SPS (Algorithm 2) on the data and prior set in
    ctx.  record=True also returns the Design of Algorithm 3's first pass.
    fused=True runs each cycle's M phase in one library call (sps_mphase: the
    step-size and stopping rules on the device, a small state record read per
    step); False takes it step by step from here (same arithmetic, more host
    round trips)."""
    J, N = cfg.J, cfg.N
    P, d, C, T = J * N, ctx.d, ctx.C, ctx.T
    m = d + C - 1
    dev = ctx.device
    prec = sps.PREC[cfg.precision]
    kind = sps.KIND[cfg.kind]
    scheme = sps.SCHEME[cfg.scheme]
    mala = kind == sps.SPS_MALA
    f64 = dict(dtype=torch.float64, device=dev)

    theta = torch.empty(P, d, **f64)
    theta_b = torch.empty(P, d, **f64)
    ll = torch.zeros(P, **f64)
    ll_b = torch.empty(P, **f64)
    grad = torch.zeros(P, d, **f64) if mala else None
    grad_b = torch.empty(P, d, **f64) if mala else None
    log_w = torch.empty(P, **f64)
    logml_j = torch.zeros(J, **f64)
    inc_j = torch.empty(J, **f64)
    g = torch.empty(P, m, **f64)
    anc = torch.empty(P, dtype=torch.int32, device=dev)

    t_start = time.perf_counter()
    sps.sps_init_prior(ctx, theta, cfg.seed, stream_id(0, 0, 1))
    h = cfg.h_init
    t = 0
    cycle = 0
    m_iters = 0
    hit_R_max = 0
    records = []
    sigmas = []
    logml = nse_logml = float("nan")
    while t < T:
        cycle += 1
        t_prev = t
        log_w, t_end, ess = sps.sps_correct(ctx, theta, ll, J, N, t, cfg.ess_frac, prec, log_w)
        t = t_end
        # log predictive likelihood of y_{t_prev+1 .. t} given y_{1 .. t_prev} (Section 3):
        # the same estimator as the log marginal likelihood, on this cycle's weights alone
        inc_j.zero_()
        pred, pred_nse = sps.sps_logml(ctx, log_w, J, N, inc_j)
        logml, nse_logml = sps.sps_logml(ctx, log_w, J, N, logml_j)
        sps.sps_resample(ctx, log_w, J, N, scheme, seed=cfg.seed, stream=stream_id(cycle, 0, 2),
                         ancestor=anc, theta_in=theta, theta_out=theta_b, ll_in=ll, ll_out=ll_b)
        theta, theta_b = theta_b, theta
        ll, ll_b = ll_b, ll
        if mala:
            # the cached gradient must cover y_{1:t_l}: evaluate it afresh
            sps.sps_loglik_grad(ctx, theta, 0, t, prec, ll, grad)
        K = cfg.K_mid if t < T else cfg.K_final
        r = 0
        rate = 0.0
        if fused:
            sig = torch.empty(cfg.R_max, d, d, **f64) if record else None
            r, h, agg, rate = sps.sps_mphase(ctx, theta, ll, grad, J, N, t, kind, prec, h, cfg.h_step,
                                             cfg.h_min, cfg.h_max, cfg.acc_target, K, cfg.R_max,
                                             1 if cfg.rne_rule == "min" else 0, cfg.seed,
                                             stream_id(cycle, 0, 3), 1 << 4, g, sig)
            if record:
                sigmas.extend(sig[i].clone() for i in range(r))
            if agg < K:
                hit_R_max += 1
        while not fused:
            r += 1
            rate = sps.sps_mutate(ctx, theta, ll, grad, J, N, t, h, kind, prec,
                                  seed=cfg.seed, stream=stream_id(cycle, r, 3))
            if record:
                sigmas.append(sps.sps_last_sigma(ctx))
            h = min(h + cfg.h_step, cfg.h_max) if rate > cfg.acc_target else max(h - cfg.h_step, cfg.h_min)
            sps.sps_monitor(ctx, theta, g)
            _, _, _, rne = sps.sps_moments(ctx, g, J, N)
            agg = float(np.min(rne)) if cfg.rne_rule == "min" else float(np.mean(rne))
            if agg >= K:
                break
            if r >= cfg.R_max:
                hit_R_max += 1
                break
        m_iters += r
        rec = dict(cycle=cycle, t_prev=t_prev, t=t, ess=ess, R=r, h=h, acc=rate, rne=agg, logml=logml,
                   pred=pred, pred_nse=pred_nse)
        records.append(rec)
        if log is not None:
            log(rec)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t_start
    sps.sps_monitor(ctx, theta, g)
    mean, sd, nse, rne = sps.sps_moments(ctx, g, J, N)
    out = dict(theta=theta, ll=ll, mean=mean, sd=sd, nse=nse, rne=rne, logml=logml,
               logml_nse=nse_logml, logml_j=logml_j.cpu().numpy(), cycles=cycle,
               m_iters=m_iters, hit_R_max=hit_R_max, records=records, wall=wall)
    if record:
        out["design"] = Design(t=[r["t"] for r in records], R=[r["R"] for r in records], sigma=sigmas)
    return out


def run_fixed(ctx: sps.Context, cfg: SpsConfig, design: Design, pass_: int = 1) -> dict:
    """Algorithm 1 with a fixed design (the second pass of Algorithm 3): the C
    phase runs to the recorded t_l, the M phase takes the recorded R_l steps
    with the recorded proposal covariances.  Fresh random streams (pass 1)."""
    J, N = cfg.J, cfg.N
    P, d, C = J * N, ctx.d, ctx.C
    m = d + C - 1
    dev = ctx.device
    prec = sps.PREC[cfg.precision]
    kind = sps.KIND[cfg.kind]
    scheme = sps.SCHEME[cfg.scheme]
    mala = kind == sps.SPS_MALA
    f64 = dict(dtype=torch.float64, device=dev)
    theta, theta_b = torch.empty(P, d, **f64), torch.empty(P, d, **f64)
    ll, ll_b = torch.zeros(P, **f64), torch.empty(P, **f64)
    grad = torch.zeros(P, d, **f64) if mala else None
    log_w = torch.empty(P, **f64)
    logml_j = torch.zeros(J, **f64)
    g = torch.empty(P, m, **f64)
    anc = torch.empty(P, dtype=torch.int32, device=dev)
    t_start = time.perf_counter()
    sps.sps_init_prior(ctx, theta, cfg.seed, stream_id(0, 0, 1, pass_))
    step = 0
    t_prev = 0
    logml = nse_logml = float("nan")
    for li, (t, R) in enumerate(zip(design.t, design.R)):
        cycle = li + 1
        sps.sps_correct_fixed(ctx, theta, ll, J, N, t_prev, t, prec, log_w)
        logml, nse_logml = sps.sps_logml(ctx, log_w, J, N, logml_j)
        sps.sps_resample(ctx, log_w, J, N, scheme, seed=cfg.seed, stream=stream_id(cycle, 0, 2, pass_),
                         ancestor=anc, theta_in=theta, theta_out=theta_b, ll_in=ll, ll_out=ll_b)
        theta, theta_b = theta_b, theta
        ll, ll_b = ll_b, ll
        if mala:
            sps.sps_loglik_grad(ctx, theta, 0, t, prec, ll, grad)
        for r in range(1, R + 1):
            sps.sps_mutate_cov(ctx, theta, ll, grad, J, N, t, design.sigma[step], kind, prec,
                               seed=cfg.seed, stream=stream_id(cycle, r, 3, pass_), want_rate=True)
            step += 1
        t_prev = t
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t_start
    sps.sps_monitor(ctx, theta, g)
    mean, sd, nse, rne = sps.sps_moments(ctx, g, J, N)
    return dict(theta=theta, ll=ll, mean=mean, sd=sd, nse=nse, rne=rne, logml=logml,
                logml_nse=nse_logml, cycles=len(design.t), m_iters=step, wall=wall)


def run_two_pass(ctx: sps.Context, cfg: SpsConfig) -> tuple:
    """Algorithm 3: an adaptive pass whose particles are discarded, then the
    nonadaptive pass with its design.  Returns (pass 1, pass 2) results."""
    p1 = run_sps(ctx, cfg, record=True)
    p2 = run_fixed(ctx, cfg, p1["design"])
    return p1, p2


def setup(X: np.ndarray, y: np.ndarray, C: int, prior_mean=0.0, prior_sd=1.0,
          device: int = 0, stream: Optional[torch.cuda.Stream] = None,
          prior_cov: Optional[np.ndarray] = None, g: Optional[float] = None) -> sps.Context:
    """A context with the data set and its prior: the iid
    N(prior_mean, prior_sd^2) prior by default, N(prior_mean, prior_cov) when
    prior_cov is given, or the normalised g-prior (eqs. (g-prior_def),
    (prior_norm)) when g is given."""
    ctx = sps.Context(device, stream)
    Xg = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float64)).to(ctx.device)
    yg = torch.from_numpy(np.ascontiguousarray(y, dtype=np.int32)).to(ctx.device)
    sps.sps_set_data(ctx, Xg, yg, C)
    if g is not None:
        sps.sps_set_prior_g(ctx, g, prior_mean)
    elif prior_cov is not None:
        sps.sps_set_prior_cov(ctx, prior_mean, prior_cov)
    else:
        sps.sps_set_prior(ctx, prior_mean, prior_sd)
    return ctx
