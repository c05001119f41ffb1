#!/usr/bin/env python3
"""Throughput of the SPS hot path on one MI355X.

Metric: particle x observation log-likelihood(+gradient) evaluations per
second over whole SPS cycles.  One step is one pass of every stage of the
hot path on the benchmark workload, the way a late cycle of Algorithm 2 runs
it:
  C phase from observation T - 1000 with the ESS rule (sps_correct),
  log marginal likelihood increment (sps_logml),
  residual resampling with gathers (sps_resample),
  one Gaussian random-walk M step at t = t_end (sps_mutate, RW),
  the gradient refresh at t_end (sps_loglik_grad, forward + adjoint),
  one MALA M step at t = t_end (sps_mutate, MALA).
Evaluations per step = P (t_end - s0) + 3 P t_end.  Inputs are resident on
the GPU before the timed region; each step first restores the particle state
(two device copies) so every step does the same work.

The JSON line also carries the roofline of the dominant kernel (timed live
with HIP events around each launch inside libsps) and the FP64 CPU oracle
timed on a particle subsample of the same step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "particle×obs loglik(+grad) evals/sec and SPS wall time at fixed NSE vs FP64"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16x3": 2500.0}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}
C_BLOCK = 1000


def _workload_desc(w):
    return (f"{w.name}: multinomial logit C={w.C}, T={w.T} observations, k={w.k} covariates "
            f"(d={w.d}), J={w.J} groups x N={w.N} particles, prior N(0,{w.prior_sd**2:g} I), "
            f"{w.precision} likelihood")


def gpu_bench(w, steps, warmup, seed=1):
    import torch
    from paper_1304_4333_amd import driver, sps, synth

    X, y, B = synth.make_data(w)
    ctx = driver.setup(X, y, w.C, 0.0, w.prior_sd)
    prec = sps.PREC[w.precision]
    J, N, P, d, T = w.J, w.N, w.P, w.d, w.T
    s0 = max(0, T - C_BLOCK)
    f64 = dict(dtype=torch.float64, device="cuda")
    # particle cloud at posterior scale around the generating coefficients
    th_np = synth.make_particles(P, d, scale=0.02, seed=seed, center=B.reshape(-1))
    theta0 = torch.from_numpy(th_np).cuda()
    ll0 = sps.sps_loglik(ctx, theta0, 0, s0, prec)
    theta, theta_b = torch.empty(P, d, **f64), torch.empty(P, d, **f64)
    ll, ll_b = torch.empty(P, **f64), torch.empty(P, **f64)
    grad = torch.empty(P, d, **f64)
    log_w = torch.empty(P, **f64)
    logml_j = torch.zeros(J, **f64)
    anc = torch.empty(P, dtype=torch.int32, device="cuda")

    def step(i):
        theta.copy_(theta0)
        ll.copy_(ll0)
        _, t_end, _ = sps.sps_correct(ctx, theta, ll, J, N, s0, 0.5, prec, log_w)
        sps.sps_logml(ctx, log_w, J, N, logml_j)
        sps.sps_resample(ctx, log_w, J, N, sps.SPS_RESIDUAL, seed=seed, stream=(i << 32) | 2,
                         ancestor=anc, theta_in=theta, theta_out=theta_b, ll_in=ll, ll_out=ll_b)
        sps.sps_mutate(ctx, theta_b, ll_b, None, J, N, t_end, 0.3, sps.SPS_RW, prec,
                       seed=seed, stream=(i << 32) | 3)
        sps.sps_loglik_grad(ctx, theta_b, 0, t_end, prec, ll_b, grad)
        sps.sps_mutate(ctx, theta_b, ll_b, grad, J, N, t_end, 0.3, sps.SPS_MALA, prec,
                       seed=seed, stream=(i << 32) | 5)
        return P * (t_end - s0) + 3 * P * t_end, t_end

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    sps.sps_timing_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evals = 0
    t_ends = []
    for i in range(steps):
        e, te = step(warmup + i)
        evals += e
        t_ends.append(te)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = {name: sps.sps_timing_read(ctx, which) for name, which in
          (("loglik", sps.SPS_KT_LOGLIK), ("loglik_grad", sps.SPS_KT_LOGLIK_GRAD),
           ("perobs", sps.SPS_KT_PEROBS))}
    sps.sps_timing_enable(ctx, False)
    return dict(evals=evals, elapsed=elapsed, kt=kt, t_ends=t_ends, P=P, s0=s0)


def _progress(tag):
    def log(rec):
        if rec["cycle"] % 25 == 0:
            print(f"{tag} cycle {rec['cycle']} t={rec['t']} R={rec['R']} h={rec['h']:.3f}",
                  file=sys.stderr, flush=True)
    return log


def sps_fixed_nse(w, seeds, rw_hmin=0.1):
    """Whole adaptive SPS runs on the workload: (A) the paper's Gaussian
    random walk with the FP64 likelihood, (B) the split-precision likelihood
    with the MALA M phase.  Efficiency per monitored moment e = wall * NSE^2
    (proportional to the paper's efficiency-adjusted time, since
    NSE^2 = var / (J N RNE)); reported: median over moments of e_A / e_B
    (> 1 means B needs less time for the same NSE), averaged over seeds."""
    import torch
    from paper_1304_4333_amd import driver, synth

    X, y, _ = synth.make_data(w)
    ctx = driver.setup(X, y, w.C, 0.0, w.prior_sd)
    fast = "bf16x3" if w.precision != "fp64" else "fp64"
    out = {"A": [], "B": []}
    for seed in seeds:
        ra = driver.run_sps(ctx, driver.SpsConfig(J=w.J, N=w.N, precision="fp64", kind="rw", seed=seed,
                                                  h_min=rw_hmin), log=_progress(f"A seed {seed}"))
        rb = driver.run_sps(ctx, driver.SpsConfig.mala_defaults(J=w.J, N=w.N, precision=fast, seed=seed),
                            log=_progress(f"B seed {seed}"))
        out["A"].append(ra)
        out["B"].append(rb)
    torch.cuda.synchronize()

    def summary(rs):
        return dict(wall_s=round(float(np.mean([r["wall"] for r in rs])), 4),
                    cycles=float(np.mean([r["cycles"] for r in rs])),
                    m_steps=float(np.mean([r["m_iters"] for r in rs])),
                    logml=round(float(np.mean([r["logml"] for r in rs])), 4),
                    logml_nse=round(float(np.mean([r["logml_nse"] for r in rs])), 5))

    ratios = []
    for ra, rb in zip(out["A"], out["B"]):
        ea = ra["wall"] * ra["nse"] ** 2
        eb = rb["wall"] * rb["nse"] ** 2
        ratios.append(float(np.median(ea / eb)))
    # agreement of the two estimates of every monitored posterior mean
    za = np.mean([r["mean"] for r in out["A"]], axis=0)
    zb = np.mean([r["mean"] for r in out["B"]], axis=0)
    sa = np.sqrt(np.mean([r["nse"] ** 2 for r in out["A"]], axis=0) / len(seeds))
    sb = np.sqrt(np.mean([r["nse"] ** 2 for r in out["B"]], axis=0) / len(seeds))
    z = np.abs(za - zb) / np.sqrt(sa ** 2 + sb ** 2)
    # mixing gain per likelihood call: (M steps of RW / M steps of MALA) over
    # the cost of a gradient call relative to a plain call, both at full data
    # in the precision of run B
    t_ll, t_gr = _call_times(ctx, w, fast)
    steps_ratio = float(np.mean([r["m_iters"] for r in out["A"]]) / np.mean([r["m_iters"] for r in out["B"]]))
    return {"A": dict(summary(out["A"]), precision="fp64", kernel="rw", h_min=rw_hmin),
            "B": dict(summary(out["B"]), precision=fast, kernel="mala"),
            "efficiency_ratio_A_over_B": round(float(np.mean(ratios)), 3),
            "max_mean_z_A_vs_B": round(float(z.max()), 2), "seeds": list(seeds),
            "m_steps_ratio_rw_over_mala": round(steps_ratio, 3),
            "grad_over_loglik_time": round(t_gr / t_ll, 3),
            "mixing_gain_per_call": round(steps_ratio / (t_gr / t_ll), 3)}


def sps_run_counts(w, seed=1):
    """One whole adaptive SPS run (Algorithm 2) on the workload with its own
    precision and M-phase kernel: GPU wall time, cycles, M steps, and the
    particle x observation likelihood evaluations the run made (C phases:
    P (t_l - t_{l-1}); M steps: P t_l each, as gradient evaluations with
    MALA, which also refreshes the gradient once per cycle).  With a CPU rate
    in evals/s for the same mix, evals / rate estimates the oracle's wall
    time for the same run."""
    import torch
    from paper_1304_4333_amd import driver
    X, y, _ = synth_data(w)
    ctx = driver.setup(X, y, w.C, 0.0, w.prior_sd)
    base = dict(J=w.J, N=w.N, precision=w.precision, seed=seed)
    cfg = driver.SpsConfig.mala_defaults(**base) if w.kernel == "mala" else driver.SpsConfig(**base)
    r = driver.run_sps(ctx, cfg, log=_progress(f"{w.name} seed {seed}"))
    torch.cuda.synchronize()
    P = w.P
    c_evals = sum(P * (rec["t"] - rec["t_prev"]) for rec in r["records"])
    m_evals = sum(P * rec["t"] * rec["R"] for rec in r["records"])
    refresh = sum(P * rec["t"] for rec in r["records"]) if w.kernel == "mala" else 0
    row = dict(study="sps_run", workload=w.name, precision=w.precision, kernel=w.kernel, seed=seed,
               wall_s=round(r["wall"], 3), cycles=r["cycles"], m_steps=r["m_iters"],
               hit_R_max=r["hit_R_max"], logml=round(float(r["logml"]), 4),
               c_phase_evals=c_evals, m_step_evals=m_evals, gradient_refresh_evals=refresh,
               m_steps_are_gradient_evals=w.kernel == "mala")
    print(json.dumps(row), flush=True)
    del ctx
    return row


def design_sweep(w, seeds, ess_fracs=(0.3, 0.5, 0.7), k_mids=(0.35, 0.9), kind="rw"):
    """Algorithm 2 with other design constants (Section 2.3 discusses them):
    the ESS threshold of the C phase and the RNE target K of the cycles before
    the last.  One JSON line per setting: cycles, M steps, wall time, logML,
    its reported NSE and the spread of logML over the seeds."""
    import torch
    from paper_1304_4333_amd import driver
    X, y, _ = synth_data(w)
    ctx = driver.setup(X, y, w.C, 0.0, w.prior_sd)
    rows = []
    for ef in ess_fracs:
        for km in k_mids:
            rs = []
            for seed in seeds:
                base = dict(J=w.J, N=w.N, precision=w.precision, seed=seed, ess_frac=ef, K_mid=km)
                cfg = driver.SpsConfig.mala_defaults(**base) if kind == "mala" else driver.SpsConfig(**base)
                rs.append(driver.run_sps(ctx, cfg))
            torch.cuda.synchronize()
            lm = np.array([r["logml"] for r in rs])
            row = dict(workload=w.name, kind=kind, precision=w.precision, ess_frac=ef, K_mid=km,
                       seeds=len(seeds), cycles=float(np.mean([r["cycles"] for r in rs])),
                       m_steps=float(np.mean([r["m_iters"] for r in rs])),
                       wall_s=round(float(np.mean([r["wall"] for r in rs])), 4),
                       logml=round(float(lm.mean()), 4),
                       logml_nse=round(float(np.mean([r["logml_nse"] for r in rs])), 4),
                       logml_sd_over_seeds=round(float(lm.std(ddof=1)), 4) if len(rs) > 1 else None)
            rows.append(row)
            print(json.dumps(row), flush=True)
    return rows


def _logodds_row(r, C):
    """The log-odds moments theta_c' xbar (c = 1 .. C-1; the last C-1
    monitored functions) with their NSE and RNE, and the logML with its NSE."""
    q = slice(len(r["mean"]) - (C - 1), None)
    return dict(logodds=[round(float(v), 5) for v in r["mean"][q]],
                logodds_nse=[round(float(v), 5) for v in r["nse"][q]],
                logodds_rne=[round(float(v), 3) for v in r["rne"][q]],
                logml=round(float(r["logml"]), 4), logml_nse=round(float(r["logml_nse"]), 4))


def reliability_study(w, g=0.25, sizes=((10, 1000), (40, 2500)), runs=("A", "B", "C")):
    """The one- and two-pass reliability study (Section 4.1, Table 2) on a
    synthetic data set: for each J x N, independent runs of Algorithm 3, with
    the log-odds moments, the log marginal likelihood and their NSEs at the
    end of each pass.  Summary per J x N and pass: the spread of each estimate
    over the runs against the mean reported NSE, and the largest within-run
    pass 1 / pass 2 difference in units of sqrt(NSE_1^2 + NSE_2^2).  One JSON
    line per pass and one per summary."""
    import torch
    from paper_1304_4333_amd import driver
    X, y, _ = synth_data(w)
    ctx = driver.setup(X, y, w.C, 0.0, g=g)
    rows = []
    for J, N in sizes:
        per = {1: [], 2: []}
        for i, run in enumerate(runs):
            cfg = driver.SpsConfig(J=J, N=N, precision=w.precision, kind=w.kernel, seed=300 + i)
            p1, p2 = driver.run_two_pass(ctx, cfg)
            for pas, r in ((1, p1), (2, p2)):
                row = dict(study="reliability", workload=w.name, g=g, J=J, N=N, run=run, pass_=pas,
                           cycles=r["cycles"], m_steps=r["m_iters"], wall_s=round(r["wall"], 3),
                           **_logodds_row(r, w.C))
                per[pas].append(row)
                rows.append(row)
                print(json.dumps(row), flush=True)
        torch.cuda.synchronize()
        summ = dict(study="reliability_summary", workload=w.name, g=g, J=J, N=N, runs=len(runs))
        for pas in (1, 2):
            est = np.array([r["logodds"] + [r["logml"]] for r in per[pas]])
            nse = np.array([r["logodds_nse"] + [r["logml_nse"]] for r in per[pas]])
            summ[f"pass{pas}_sd_over_runs"] = np.round(est.std(axis=0, ddof=1), 5).tolist()
            summ[f"pass{pas}_mean_nse"] = np.round(nse.mean(axis=0), 5).tolist()
        z = [(np.array(a["logodds"] + [a["logml"]]) - np.array(b["logodds"] + [b["logml"]])) /
             np.hypot(np.array(a["logodds_nse"] + [a["logml_nse"]]), np.array(b["logodds_nse"] + [b["logml_nse"]]))
             for a, b in zip(per[1], per[2])]
        summ["max_abs_z_pass1_vs_pass2"] = round(float(np.abs(np.array(z)).max()), 3)
        summ["wall_ratio_two_pass_over_one"] = round(
            float(sum(r["wall_s"] for r in per[1] + per[2]) / sum(r["wall_s"] for r in per[1])), 3)
        rows.append(summ)
        print(json.dumps(summ), flush=True)
    return rows


def g_sweep(w, gs=(1 / 64, 1 / 16, 1 / 4, 1.0, 4.0), sizes=((10, 1000), (40, 2500)), seeds=(1, 2, 3)):
    """Adaptation against prior tightness (Section 4.2, Table 3) on a
    synthetic data set: for each g of the g-prior (eq. (g-prior_def)) and
    each J x N, Algorithm 2's cycles, M iterations, wall time relative to the
    tightest prior, RNE of the log-odds moments, the logML and its NSE
    (means over the seeds; the logML spread over seeds beside the NSE).  One
    JSON line per g and J x N."""
    import torch
    from paper_1304_4333_amd import driver
    X, y, _ = synth_data(w)
    rows = []
    for J, N in sizes:
        base_wall = None
        for g in gs:
            ctx = driver.setup(X, y, w.C, 0.0, g=g)
            rs = [driver.run_sps(ctx, driver.SpsConfig(J=J, N=N, precision=w.precision, kind=w.kernel, seed=s))
                  for s in seeds]
            torch.cuda.synchronize()
            q = slice(w.d, None)
            wall = float(np.mean([r["wall"] for r in rs]))
            base_wall = base_wall or wall
            lm = np.array([r["logml"] for r in rs])
            row = dict(study="g_sweep", workload=w.name, g=g, J=J, N=N, seeds=len(seeds),
                       cycles=float(np.mean([r["cycles"] for r in rs])),
                       m_steps=float(np.mean([r["m_iters"] for r in rs])),
                       wall_s=round(wall, 4), relative_time=round(wall / base_wall, 3),
                       logodds_rne=np.round(np.mean([r["rne"][q] for r in rs], axis=0), 3).tolist(),
                       logml=round(float(lm.mean()), 4),
                       logml_nse=round(float(np.mean([r["logml_nse"] for r in rs])), 4),
                       logml_sd_over_seeds=round(float(lm.std(ddof=1)), 4) if len(rs) > 1 else None)
            rows.append(row)
            print(json.dumps(row), flush=True)
            del ctx
    return rows


def synth_data(w):
    from paper_1304_4333_amd import synth
    return synth.make_data(w)


def _call_times(ctx, w, precision, reps=5):
    """Mean seconds of one full-data sps_loglik and sps_loglik_grad call."""
    import torch
    from paper_1304_4333_amd import sps, synth
    _, _, B = synth.make_data(w)
    th = torch.from_numpy(synth.make_particles(w.P, w.d, scale=0.02, seed=3, center=B.reshape(-1))).cuda()
    ll = torch.empty(w.P, dtype=torch.float64, device="cuda")
    g = torch.empty(w.P, w.d, dtype=torch.float64, device="cuda")
    prec = sps.PREC[precision]
    out = []
    for grad in (False, True):
        call = (lambda: sps.sps_loglik_grad(ctx, th, 0, w.T, prec, ll, g)) if grad else \
            (lambda: sps.sps_loglik(ctx, th, 0, w.T, prec, ll))
        call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            call()
        torch.cuda.synchronize()
        out.append((time.perf_counter() - t0) / reps)
    return out[0], out[1]


PREC_SOURCES = {"fp64": ("loglik_fp64.hip",), "fp32": ("loglik_fp32.hip",),
                "bf16x3": ("loglik_pipe.h", "loglik_pipe_grad.hip", "loglik_bf16.hip", "loglik_bf16_wide.hip",
                           "loglik_bf16_c8.hip") + tuple(f"loglik_pipe_fwd_{g}.hip" for g in "abcd")}


def kernel_digest(precision):
    """Digest of the likelihood kernel sources and compile flags of one
    precision: HBM traffic counters taken on other sources do not describe
    the current kernel."""
    import hashlib
    from paper_1304_4333_amd import build
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in ("loglik_kernel.h", "loglik.hip", "sps_internal.h") + PREC_SOURCES[precision]:
        with open(os.path.join(root, "paper_1304_4333_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
        h.update(" ".join(build.CFLAGS[:-2] + build.FILE_FLAGS.get(f, [])).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel, precision):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, if it was taken on the current
    kernel sources; otherwise None."""
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_digest") != kernel_digest(precision):
        return None
    try:
        return int(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# MI355X published peaks: dense MFMA per input type (TFLOP/s), HBM3E (GB/s),
# and the FP32 vector rate, 157.3 TFLOP/s = 78.6 T lane FMAs/s.  The
# transcendental unit (exp2, log2, rcp) runs at a quarter of the FP32 lane
# rate: 78.6 / 4 = 19.66 T ops/s (a microbenchmark of v_exp_f32 on one
# MI355X measured 19.2 T/s).
PEAK_HBM_GBS = 8000.0
PEAK_TRANS_TOPS = 157.3 / 2 / 4
MFMA_MULT = {"fp64": 1, "fp32": 1, "bf16x3": 3}  # MFMA products per multiply-add


def work_per_po(w, grad):
    """Algorithmic work per particle x observation of one likelihood launch:
    MFMA flops as issued (the BF16x3 split issues three products per
    multiply-add; 2 k (C-1) flops per product, twice with the adjoint), and
    transcendentals (C - 1 exponentials and one logarithm, one reciprocal
    more with the adjoint)."""
    flops = MFMA_MULT[w.precision] * 2 * w.k * (w.C - 1) * (2 if grad else 1)
    trans = w.C + (1 if grad else 0)
    return flops, trans


def alg_bytes(w, t_end, grad):
    """Algorithmic HBM bytes of one full-range launch: X (and X^T for the
    adjoint) once in the kernel's format, theta once, ll (and grad) out."""
    xb = {"fp64": 8, "fp32": 4, "bf16x3": 4}[w.precision]
    x = t_end * w.k * xb * (2 if grad else 1)
    return x + w.P * w.d * 8 + w.P * 8 + (w.P * w.d * 8 if grad else 0)


def roofline(w, res):
    """Dominant likelihood kernel: its per-launch time bounds from the MFMA
    peak of its input type, the transcendental rate and HBM, over its
    average HIP-event duration; `bound` is the largest of the three."""
    kt = res["kt"]
    name = max(("loglik", "loglik_grad"), key=lambda n: kt[n][1])
    n, ms = kt[name]
    if n == 0:
        return None, None
    grad = name == "loglik_grad"
    t_end = int(np.median(res["t_ends"]))
    units = res["P"] * t_end
    flops_po, trans_po = work_per_po(w, grad)
    flops, trans, nbytes = flops_po * units, trans_po * units, alg_bytes(w, t_end, grad)
    avg_s = ms / n * 1e-3
    peak_mfma = PEAK_TFLOPS[DTYPE[w.precision]]
    bounds = {"mfma": flops / (peak_mfma * 1e12), "alu": trans / (PEAK_TRANS_TOPS * 1e12),
              "hbm": nbytes / (PEAK_HBM_GBS * 1e9)}
    bound = max(bounds, key=bounds.get)
    if bound == "mfma":
        achieved, peak, unit = flops / avg_s / 1e12, peak_mfma, "TFLOP/s"
    elif bound == "alu":
        achieved, peak, unit = trans / avg_s / 1e12, PEAK_TRANS_TOPS, "TFLOP/s"
    else:
        achieved, peak, unit = nbytes / avg_s / 1e9, PEAK_HBM_GBS, "GB/s"
    info = dict(kernel=name, launches=n, avg_us=round(ms / n * 1e3, 2), units_per_launch=units,
                mfma_flops_per_po=flops_po, transcendentals_per_po=trans_po,
                alg_bytes_per_launch=nbytes,
                time_bounds_us={k: round(v * 1e6, 1) for k, v in bounds.items()})
    return dict(bound=bound, achieved=round(achieved, 3), peak=peak, unit=unit,
                frac=round(achieved / peak, 4), traffic=measured_traffic(w.name, name, w.precision)), info


def cpu_info():
    """CPU model, sockets x cores x threads per core and online CPUs of this host."""
    info = {"nproc": os.cpu_count()}
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        kv = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        info.update(model=kv.get("Model name"), sockets=kv.get("Socket(s)"),
                    cores_per_socket=kv.get("Core(s) per socket"), threads_per_core=kv.get("Thread(s) per core"))
    except Exception as e:  # lscpu missing: report what os gives
        info["lscpu"] = f"unavailable ({e.__class__.__name__})"
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    return info


def _oracle_steps(w, J, N, seconds, seed):
    """The oracle on the benchmark step for J groups of N particles, repeated
    for about `seconds` (at least once); returns (evals, elapsed, steps)."""
    from oracle import oracle as O
    from paper_1304_4333_amd import synth

    X, y, B = synth.make_data(w)
    P, d, T = J * N, w.d, w.T
    s0 = max(0, T - C_BLOCK)
    th0 = synth.make_particles(w.P, d, scale=0.02, seed=seed, center=B.reshape(-1))[:P]
    ll0 = O.loglik(X, y, w.C, th0, 0, s0)
    evals = 0
    t0 = time.perf_counter()
    steps = 0
    while True:
        lw, ll, t_end, _ = O.correct(X, y, w.C, th0, ll0, J, N, s0, 0.5)
        O.logml_update(lw, J, N, np.zeros(J))
        anc, _ = O.resample(lw, J, N, 0, O.u53(seed, (steps << 32) | 2, P))
        th, ll = th0[anc], ll[anc]
        z = O.normals(seed, (steps << 32) | 3, P, d)
        u = O.uniforms(seed, (steps << 32) | 4, P)
        th, ll, _, _, _, _ = O.mutate(X, y, w.C, 0.0, w.prior_sd, th, ll, None, J, N, t_end, 0.3, 0, z, u)
        ll, gr = O.loglik(X, y, w.C, th, 0, t_end, grad=True)
        z = O.normals(seed, (steps << 32) | 5, P, d)
        u = O.uniforms(seed, (steps << 32) | 6, P)
        O.mutate(X, y, w.C, 0.0, w.prior_sd, th, ll, gr, J, N, t_end, 0.3, 1, z, u)
        evals += P * (t_end - s0) + 3 * P * t_end
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            return evals, el, steps


def _oracle_loglik_rate(w, P, seconds, seed):
    """Full-data oracle log-likelihood evaluations on P particles, repeated
    for about `seconds` (at least once): particle-obs evals per second."""
    from oracle import oracle as O
    from paper_1304_4333_amd import synth

    X, y, B = synth.make_data(w)
    th = synth.make_particles(w.P, w.d, scale=0.02, seed=seed, center=B.reshape(-1))[:P]
    n = 0
    t0 = time.perf_counter()
    while True:
        O.loglik(X, y, w.C, th, 0, w.T)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            return n * P * w.T / el, n, el


def cpu_baseline(w, seconds, seed=1):
    """The FP64 oracle on the same step as the GPU benchmark, on a particle
    subsample (its cost is linear in the particle count), timed on all cores
    of this host; and, on one core, its full-data log-likelihood evaluation
    (the step's dominant part) on 16 particles."""
    from oracle import oracle as O

    # the subsample's pooled covariance must stay positive definite after
    # resampling (which repeats particles): at least four particles per
    # parameter, in 16 groups of 32, or 4 groups of a multiple of 32 for large d
    if 16 * 32 >= 4 * w.d:
        J_all, N_all = 16, 32
    else:
        J_all, N_all = 4, -(-w.d // 32) * 32
    cores_all = O.threads(int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1))
    e_all, t_all, s_all = _oracle_steps(w, J_all, N_all, seconds, seed)
    O.threads(1)
    r_one, n_one, t_one = _oracle_loglik_rate(w, 16, seconds / 3, seed)
    O.threads(cores_all)
    return dict(value=round(e_all / t_all, 1), unit="particle-obs evals/s", cores=cores_all, kind="oracle",
                sample=f"{s_all} steps of the benchmark step on {J_all * N_all} of the {w.P} particles "
                       f"({J_all} groups x {N_all}), {t_all:.1f} s, OpenMP over particles on {cores_all} "
                       f"threads; one thread: {n_one} full-data log-likelihood evaluations of 16 particles, "
                       f"{r_one:.4g} evals/s, {t_one:.1f} s",
                one_thread_loglik_value=round(r_one, 1), host=cpu_info())


def kernel_table(names, reps=5, precisions=("fp64", "fp32", "bf16x3")):
    """Full-data sps_loglik and sps_loglik_grad throughput through the ABI
    (main kernel + split reduction + sufficient-statistic terms), per
    workload and precision, with particles at posterior scale."""
    import torch
    from paper_1304_4333_amd import driver, sps, synth
    rows = []
    for name in names:
        w = synth.workload(name)
        X, y, B = synth.make_data(w)
        ctx = driver.setup(X, y, w.C, 0.0, w.prior_sd)
        th = torch.from_numpy(synth.make_particles(w.P, w.d, scale=0.02, seed=1, center=B.reshape(-1))).cuda()
        ll = torch.empty(w.P, dtype=torch.float64, device="cuda")
        g = torch.empty(w.P, w.d, dtype=torch.float64, device="cuda")
        for prec_name in precisions:
            prec = sps.PREC[prec_name]
            for grad in (False, True):
                def call():
                    if grad:
                        sps.sps_loglik_grad(ctx, th, 0, w.T, prec, ll, g)
                    else:
                        sps.sps_loglik(ctx, th, 0, w.T, prec, ll)
                call()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    call()
                e1.record()
                torch.cuda.synchronize()
                us = e0.elapsed_time(e1) * 1e3 / reps
                flops = 2.0 * w.k * (w.C - 1) * (2 if grad else 1) * w.P * w.T
                rows.append(dict(workload=name, precision=prec_name, call="loglik_grad" if grad else "loglik",
                                 us=round(us, 1), evals_per_s=float(f"{w.P * w.T / us * 1e6:.4g}"),
                                 mfma_tflops=round(flops / us * 1e-6, 2)))
                print(json.dumps(rows[-1]), flush=True)
        del ctx
    return rows


def copy_calibration(mib=1024, reps=3):
    """A plain device-to-device copy of known size (reads and writes `mib`
    MiB per launch): the reference that scales the FETCH_SIZE / WRITE_SIZE
    counters of the likelihood kernel to bytes."""
    import torch
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": src.numel() * 4, "launches": reps}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="multi6")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sps", action="store_true", help="skip the fixed-NSE SPS comparison")
    ap.add_argument("--sps-workload", default="ar100",
                    help="workload of the fixed-NSE SPS comparison (FP64 RW against BF16x3 MALA)")
    ap.add_argument("--sps-seeds", type=int, default=1)
    ap.add_argument("--rw-hmin", type=float, default=0.01,
                    help="lower bound of the RW step-size factor in the fixed-NSE comparison "
                         "(the paper's 0.1 is above the RW optimum 2.38^2/d at d = 100)")
    ap.add_argument("--kernel-table", default=None,
                    help="comma-separated workloads: print full-data loglik/grad rates instead")
    ap.add_argument("--table-precisions", default="fp64,fp32,bf16x3",
                    help="precisions of the kernel table (comma-separated)")
    ap.add_argument("--table-reps", type=int, default=5, help="timed calls per kernel-table entry")
    ap.add_argument("--design-sweep", action="store_true",
                    help="run Algorithm 2 over ESS thresholds and RNE targets and print one line each")
    ap.add_argument("--sweep-kind", default="rw", choices=["rw", "mala"])
    ap.add_argument("--reliability", action="store_true",
                    help="one- and two-pass reliability study (Table 2 design) on the cars3 workload")
    ap.add_argument("--sps-run", default=None,
                    help="comma-separated workloads: one whole adaptive SPS run each, with its evaluation counts")
    ap.add_argument("--g-sweep", action="store_true",
                    help="prior-tightness study (Table 3 design) over g = 1/64 .. 4 on the cars3 workload")
    ap.add_argument("--sps-only", action="store_true",
                    help="run only the fixed-NSE SPS comparison and print it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a device copy of 1 GiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.kernel_table:
        kernel_table(args.kernel_table.split(","), reps=args.table_reps,
                     precisions=tuple(args.table_precisions.split(",")))
        return
    if args.sps_run:
        from paper_1304_4333_amd import synth
        for name in args.sps_run.split(","):
            sps_run_counts(synth.workload(name))
        return
    if args.reliability or args.g_sweep:
        from paper_1304_4333_amd import synth
        w = synth.workload("cars3")
        if args.reliability:
            reliability_study(w)
        if args.g_sweep:
            g_sweep(w)
        return
    if args.design_sweep:
        from paper_1304_4333_amd import synth
        design_sweep(synth.workload(args.workload), list(range(1, 1 + args.sps_seeds)), kind=args.sweep_kind)
        return
    if args.sps_only:
        from paper_1304_4333_amd import synth
        print(json.dumps(sps_fixed_nse(synth.workload(args.sps_workload), list(range(1, 1 + args.sps_seeds)),
                                       rw_hmin=args.rw_hmin)))
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the particle-group "
              "sharding across GPUs is a design note only.", file=sys.stderr)
        sys.exit(2)
    from paper_1304_4333_amd import synth
    w = synth.workload(args.workload)
    res = gpu_bench(w, args.steps, args.warmup)
    value = res["evals"] / res["elapsed"]
    roof, kinfo = roofline(w, res)
    sps_cmp = None
    if not args.no_sps:
        ws = synth.workload(args.sps_workload)
        sps_cmp = dict(sps_fixed_nse(ws, list(range(1, 1 + args.sps_seeds)), rw_hmin=args.rw_hmin),
                       workload=_workload_desc(ws))
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_seconds)
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "particle-obs evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["elapsed"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[w.precision],
        "data": "synthetic",
        "config": {"workload": _workload_desc(w), "step": "C phase (last 1000 obs) + logML + "
                   "resample + RW step + gradient refresh + MALA step",
                   "evals_per_step": int(res["evals"] / args.steps),
                   "dominant_kernel": kinfo,
                   "kernel_ms": {k: [v[0], round(v[1], 3)] for k, v in res["kt"].items()}},
        "roofline": roof,
        "cpu_baseline": cpu,
        "sps_fixed_nse": sps_cmp,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
