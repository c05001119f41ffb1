"""GPU parity at the benchmark shapes and in the reduced-precision corner
cases, against the FP64 oracle on the same seeded inputs.

- The binary fast epilogue (FP32 / BF16x3) multiplies several factors
  1 + 2^z and takes one log2.  When that product overflows, the step is
  redone with the max-shifted form.  Prior-scale particles (|eta| ~ 10^2)
  force the redo; it is checked element by element, forward and adjoint, on
  ragged particle counts and observation ranges, in both likelihood kernels
  (k <= 32 and k > 32).
- The C phase at the multi4 and multi6 shapes (32768 / 65536 particles,
  BF16x3, from observation T - 1000).
- One M step at the ar100 and multi6 shapes (d = 100 / 250: covariance on
  tiles, blocked Cholesky, FP64 VALU proposal contractions), RW and MALA.
  Both sides take their own precision's log-likelihood of the current
  particles, as they do inside a run, so an acceptance decision can differ
  only where |log alpha - log u| is within the error of what the MH test
  uses.  That error is at most 0.05 nats for LL(theta') - LL(theta)
  (test_gpu_loglik.py, full-size difference test).  MALA adds the
  reduced-precision gradient at theta' in the reverse proposal density: a
  relative gradient error e (at most 1e-3) moves |u'|^2 / 2 by about
  e sqrt(h d) |u'|, which is bounded here by 1e-3 sqrt(h d) (sqrt(d) + 3)
  nats.
"""
import math

import numpy as np
import pytest

from gpu_common import dataset, make_ctx, need_gpu, rel_err, to_gpu
from paper_1304_4333_amd import synth

pytestmark = pytest.mark.gpu

TOL = {1: 1e-4, 2: 1e-4}
GTOL = 1e-3
DLL_BAR = 0.05


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("k", [20, 60, 100])
def test_binary_fast_form_fallback(orc, prec, k):
    """Binary likelihood with prior-scale particles: the products of the fast
    epilogue overflow FP32 in most steps, so the shifted redo runs."""
    need_gpu()
    from paper_1304_4333_amd import sps
    T, t0, t1, P = 777, 13, 771, 300
    X, y, _ = dataset(T, k, 2, seed=400 + k)
    th = synth.make_particles(P, k, scale=5.0, seed=401)
    th[1::3] *= 0.06  # posterior-scale particles in the same waves
    eta = X[t0:t1] @ th.T
    assert np.abs(eta).max() > 100.0  # 2^(100 log2 e) overflows any product of factors
    print(f"fallback k={k} prec={prec} max|eta| {np.abs(eta).max():.1f}", flush=True)
    ctx = make_ctx(X, y, 2)
    ll = sps.sps_loglik(ctx, to_gpu(th), t0, t1, prec).cpu().numpy()
    llg, g = sps.sps_loglik_grad(ctx, to_gpu(th), t0, t1, prec)
    ref_ll, ref_g = orc.loglik(X, y, 2, th, t0, t1, grad=True)
    assert np.all(np.isfinite(ll))
    assert rel_err(ll, ref_ll).max() <= TOL[prec]
    assert rel_err(llg.cpu().numpy(), ref_ll).max() <= TOL[prec]
    g = g.cpu().numpy()
    nrm = np.linalg.norm(g - ref_g, axis=1) / np.maximum(1.0, np.linalg.norm(ref_g, axis=1))
    assert nrm.max() <= GTOL


@pytest.mark.parametrize("name", ["multi4", "multi6"])
def test_correct_full_size(orc, name):
    """The C phase at the full multinomial shapes, BF16x3, from T - 1000, with
    the benchmark's posterior-scale particles: the same crossing t_l, ESS and
    log-weights as the oracle."""
    need_gpu()
    from paper_1304_4333_amd import sps
    w = synth.workload(name)
    X, y, B = synth.make_data(w)
    P, s0 = w.P, w.T - 1000
    th = synth.make_particles(P, w.d, scale=0.02, seed=81, center=B.reshape(-1))
    ll0 = synth.make_normals(P, 1, seed=82)[:, 0]
    print(f"correct full size {name}: P={P} d={w.d} s0={s0}", flush=True)
    ctx = make_ctx(X, y, w.C, w.prior_sd)
    llg = to_gpu(ll0.copy())
    lw, t_end, ess = sps.sps_correct(ctx, to_gpu(th), llg, w.J, w.N, s0, 0.5, 2)
    lw_o, ll_o, t_o, ess_o = orc.correct(X, y, w.C, th, ll0, w.J, w.N, s0, 0.5)
    print(f"  t_end {t_end} (oracle {t_o}), ESS {ess:.2f} (oracle {ess_o:.2f})")
    assert s0 < t_o < w.T  # the crossing lies inside the block
    assert t_end == t_o
    assert ess == pytest.approx(ess_o, rel=1e-3)
    assert rel_err(lw.cpu().numpy(), lw_o).max() <= 1e-4
    assert rel_err(llg.cpu().numpy(), ll_o).max() <= 1e-4


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("name,t", [("ar100", 5000), ("multi6", 2000)])
def test_mutate_full_shape(orc, kind, name, t):
    """One M step with every particle of the workload (d > 64 path), at an
    observation count t of an early cycle, BF16x3 likelihood."""
    need_gpu()
    from paper_1304_4333_amd import sps
    w = synth.workload(name)
    X, y, B = synth.make_data(w)
    P, d, h, prec = w.P, w.d, 0.3, 2
    th = synth.make_particles(P, d, scale=0.02, seed=91, center=B.reshape(-1))
    ll_o0, gr_o0 = orc.loglik(X, y, w.C, th, 0, t, grad=True)
    z = synth.make_normals(P, d, seed=92)
    u = synth.make_uniforms(P, seed=93)
    print(f"mutate full shape {name}: P={P} d={d} t={t} kind={kind}", flush=True)
    ctx = make_ctx(X, y, w.C, w.prior_sd)
    thg = to_gpu(th)
    # the GPU's own log-likelihood of the current particles; the oracle's
    # gradient (so both sides draw the same proposals)
    llg = sps.sps_loglik(ctx, thg, 0, t, prec)
    grg = to_gpu(gr_o0) if kind == 1 else None
    rate = sps.sps_mutate(ctx, thg, llg, grg, w.J, w.N, t, h, kind, prec, z=to_gpu(z), u=to_gpu(u))
    th_o, ll_o, gr_o, rate_o, la_o, acc_o = orc.mutate(X, y, w.C, 0.0, w.prior_sd, th, ll_o0,
                                                       gr_o0 if kind else None, w.J, w.N, t, h, kind, z, u)
    th_g = thg.cpu().numpy()
    acc_g = np.any(th_g != th, axis=1)
    assert 0.0 < acc_g.mean() < 1.0
    assert rate == acc_g.sum() / P
    bound = DLL_BAR + (1e-3 * math.sqrt(h * d) * (math.sqrt(d) + 3.0) if kind == 1 else 0.0)
    margin = np.abs(np.log(u) - la_o)
    diff = acc_g != acc_o
    print(f"  acceptance {acc_g.mean():.4f} (oracle {rate_o:.4f}); {int(diff.sum())} decisions differ, "
          f"largest margin among them {margin[diff].max() if diff.any() else 0:.3g}; bound {bound:.3g}")
    assert np.all(margin[diff] < bound), f"{diff.sum()} decisions differ beyond {bound} nats"
    same = ~diff
    assert rel_err(th_g[same], th_o[same]).max() <= 1e-9
    assert rel_err(llg.cpu().numpy()[same], ll_o[same]).max() <= 1e-4
