#!/usr/bin/env python3
"""Write the oracle's end-to-end SPS results that the GPU parity test
(tests/test_gpu_sps_parity.py) compares against.

Only the FP64 CPU oracle (oracle/) and the seeded input generator
(paper_1304_4333_amd/synth.py) are used: no value here comes from the HIP
path.  For every case the oracle's own adaptive driver (Algorithm 2, the
paper's design constants; the MALA proposal with its own tuning) runs on
seeds 1000, 1001, ...; the GPU test uses seeds 2000, 2001, ..., disjoint
from these.  The cars3 cases use the g-prior of eq. (g-prior_def) (covariance
from the oracle's own X'X) at the five values of g of Table 3, and Algorithm 3
(two passes; both passes are stored) at g = 1/4.  Stored per run: the monitored posterior means (every free
parameter and the log-odds theta_c' xbar at the covariate means), their
posterior sds, NSEs (eq. (NSE_def), reading in the oracle's header) and
RNEs, the log marginal likelihood with its delta-method NSE, the numbers
of cycles and M steps, and the run's wall time on this host with the
OpenMP thread count (the CPU SPS baseline).

Usage (repository root):  python tests/golden/make_sps_goldens.py [case ...]
"""
from __future__ import annotations

import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1304_4333_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# name: (workload, overrides, kind, runs[, options]); options: g (g-prior),
# two_pass (Algorithm 3), J, N
CASES = {
    # the first benchmark configuration exactly: binary logit, T = 500, k = 5,
    # J = 4 groups of N = 256, FP64 random-walk Metropolis
    "small_rw": ("small", {}, "rw", 24),
    # the binary30 and multi4 designs (k, C, J x N, covariate recipes, priors)
    # with T = 200 observations (the oracle's runs take minutes each there)
    "binary30_T200_rw": ("binary30", {"T": 200}, "rw", 6),
    "binary30_T200_mala": ("binary30", {"T": 200}, "mala", 6),
    "multi4_T200_rw": ("multi4", {"T": 200}, "rw", 4),
    # the shape of Table 1's cars data (T = 263, k = 4, C = 3), J x N = 10 x 1000
    **{f"cars3_g{tag}_rw": ("cars3", {}, "rw", 4, dict(g=g)) for tag, g in
       (("1_64", 1 / 64), ("1_16", 1 / 16), ("1_4", 1 / 4), ("1", 1.0), ("4", 4.0))},
    "cars3_g1_4_two_pass": ("cars3", {}, "rw", 4, dict(g=1 / 4, two_pass=True)),
}

MALA = dict(h_min=0.01, h_max=2.0, acc_target=0.574)


def case_data(name):
    wname, over, kind, runs = CASES[name][:4]
    opts = CASES[name][4] if len(CASES[name]) > 4 else {}
    w = synth.workload(wname, **over)
    X, y, _ = synth.make_data(w)
    return w, X, y, kind, runs, opts


def _record(seed, r, wall):
    return dict(seed=seed, mean=r["mean"].tolist(), sd=r["sd"].tolist(), nse=r["nse"].tolist(),
                rne=r["rne"].tolist(), logml=r["logml"], logml_nse=r["logml_nse"],
                cycles=int(r["cycles"]), m_iters=int(r["m_iters"]), hit_R_max=int(r.get("hit_R_max", 0)),
                wall_s=round(wall, 3))


def run_case(name):
    w, X, y, kind, runs, opts = case_data(name)
    J, N = opts.get("J", w.J), opts.get("N", w.N)
    cov = O.gprior_cov(X, w.C, opts["g"]) if "g" in opts else None
    out, out2 = [], []
    for i in range(runs):
        seed = 1000 + i
        kw = dict(kind=O.MALA, **MALA) if kind == "mala" else dict(kind=O.RW)
        t0 = time.perf_counter()
        if opts.get("two_pass"):
            r, r2 = O.sps_two_pass(X, y, w.C, 0.0, w.prior_sd, J, N, seed, prior_cov=cov, **kw)
            out2.append(_record(seed, r2, 0.0))
        else:
            r = O.sps_run(X, y, w.C, 0.0, w.prior_sd, J, N, seed=seed, prior_cov=cov, **kw)
        wall = time.perf_counter() - t0
        out.append(_record(seed, r, wall))
        print(f"{name} seed {seed}: cycles {r['cycles']} M steps {r['m_iters']} logml {r['logml']:.4f} "
              f"wall {wall:.1f} s", flush=True)
    doc = dict(case=name, workload=w.name, overrides=CASES[name][1], kind=kind, C=w.C, T=w.T, k=w.k,
               J=J, N=N, prior_sd=w.prior_sd, g=opts.get("g"), two_pass=bool(opts.get("two_pass")),
               runs=out, pass2_runs=out2 or None,
               host=dict(machine=platform.machine(), processor=platform.processor(),
                         omp_threads=O.threads(), cpus=os.cpu_count()),
               note="written by tests/golden/make_sps_goldens.py from the FP64 oracle only")
    path = os.path.join(HERE, f"sps_{name}.json")
    with open(path, "w") as fh:
        json.dump(doc, fh, indent=1)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for n in names:
        run_case(n)
