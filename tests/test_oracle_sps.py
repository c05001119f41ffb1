"""End-to-end pins of the oracle's adaptive SPS (Algorithm 2) on models whose
posterior and marginal likelihood are known by quadrature or in closed form."""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

from paper_1304_4333_amd import synth


def _intercept_model(T, frac, seed):
    X = np.ones((T, 1))
    y = (synth.rng(seed).random(T) < frac).astype(np.int32)
    return X, y


def _intercept_truth(y, s):
    T, m = len(y), int(y.sum())
    f = lambda a: math.exp(stats.norm.logpdf(a, 0, s) + m * special.log_expit(a) + (T - m) * special.log_expit(-a))
    lo, hi = -12.0, 12.0
    Z = integrate.quad(f, lo, hi, epsabs=0, epsrel=1e-12, limit=400)[0]
    m1 = integrate.quad(lambda a: a * f(a), lo, hi, epsabs=0, epsrel=1e-12, limit=400)[0] / Z
    m2 = integrate.quad(lambda a: a * a * f(a), lo, hi, epsabs=0, epsrel=1e-12, limit=400)[0] / Z
    return math.log(Z), m1, math.sqrt(m2 - m1 * m1)


def test_single_observation_logml_is_minus_log2(orc):
    """T = 1, binary, prior symmetric about 0: the marginal likelihood is 1/2
    exactly (theta'x is symmetric and sigmoid(-u) = 1 - sigmoid(u))."""
    w = synth.workload("small", T=1)
    X, y, _ = synth.make_data(w)
    r = orc.sps_run(X, y, 2, 0.0, 5.0, J=16, N=2048, seed=1)
    assert r["cycles"] == 1
    assert abs(r["logml"] + math.log(2.0)) < 4 * r["logml_nse"] + 1e-12
    assert r["logml_nse"] < 0.02


@pytest.mark.parametrize("kind", [0, 1])
def test_intercept_only_against_quadrature(orc, kind):
    X, y = _intercept_model(60, 0.75, seed=2)
    logZ, m1, sd = _intercept_truth(y, 5.0)
    kw = dict(kind=kind)
    if kind == 1:
        kw.update(h_min=0.01, h_max=2.0, acc_target=0.574)
    r = orc.sps_run(X, y, 2, 0.0, 5.0, J=16, N=1024, seed=3, **kw)
    assert r["hit_R_max"] == 0
    assert abs(r["mean"][0] - m1) < 4 * r["nse"][0] + 1e-4
    assert abs(r["sd"][0] - sd) < 0.03 * sd
    assert abs(r["logml"] - logZ) < 4 * r["logml_nse"] + 0.01


def test_two_parameter_model_against_grid(orc):
    """k = 2 binary logit (intercept + slope): posterior moments and marginal
    likelihood by a dense 2-D grid."""
    T, s = 80, 2.0
    g = synth.rng(4)
    X = np.stack([np.ones(T), g.standard_normal(T)], axis=1)
    y = (g.random(T) < special.expit(0.5 + 1.0 * X[:, 1])).astype(np.int32)
    a = np.linspace(-4, 5, 901)
    b = np.linspace(-4, 6, 1001)
    A, B = np.meshgrid(a, b, indexing="ij")
    eta = A[..., None] + B[..., None] * X[:, 1]
    ll = (y * eta - np.logaddexp(0, eta)).sum(-1)
    lp = ll + stats.norm.logpdf(A, 0, s) + stats.norm.logpdf(B, 0, s)
    M = lp.max()
    dA, dB = a[1] - a[0], b[1] - b[0]
    Z = np.exp(lp - M).sum() * dA * dB
    logZ = M + math.log(Z)
    Pm = np.exp(lp - M) * dA * dB / Z
    mA, mB = (Pm * A).sum(), (Pm * B).sum()
    r = orc.sps_run(X, y, 2, 0.0, s, J=16, N=1024, seed=5)
    assert abs(r["mean"][0] - mA) < 4 * r["nse"][0] + 2e-3
    assert abs(r["mean"][1] - mB) < 4 * r["nse"][1] + 2e-3
    assert abs(r["logml"] - logZ) < 4 * r["logml_nse"] + 0.02


def test_multinomial_relabel_moments(orc):
    """C = 3 run: the monitored log-odds theta_c' xbar equal the corresponding
    parameter combinations of the same particles (internal consistency of the
    report), and the cycle record is increasing and ends at T."""
    w = synth.workload("multi4", T=300, k=3, n_dummy=1, J=4, N=256)
    X, y, _ = synth.make_data(w)
    r = orc.sps_run(X, y, 4, 0.0, 5.0, J=4, N=256, seed=6)
    t = r["t"]
    assert np.all(np.diff(t) > 0) and t[-1] == w.T
    xbar = X.mean(0)
    th = r["theta"]
    for c in range(3):
        g = th[:, c * 3:(c + 1) * 3] @ xbar
        assert r["mean"][9 + c] == pytest.approx(g.mean(), rel=1e-10, abs=1e-12)


def test_tstat_calibration_over_runs(orc):
    """Eq. (gbar_tstat): over independent runs, (gbar - E[g|y]) / NSE is
    close to t(J - 1) (KS test on 40 runs)."""
    X, y = _intercept_model(25, 0.6, seed=7)
    _, m1, _ = _intercept_truth(y, 5.0)
    J = 8
    z = []
    for seed in range(40):
        r = orc.sps_run(X, y, 2, 0.0, 5.0, J=J, N=256, seed=1000 + seed)
        z.append((r["mean"][0] - m1) / r["nse"][0])
    assert stats.kstest(z, stats.t(J - 1).cdf).pvalue > 1e-3


def test_deterministic_given_seed(orc):
    X, y = _intercept_model(20, 0.5, seed=8)
    a = orc.sps_run(X, y, 2, 0.0, 5.0, J=4, N=128, seed=9)
    b = orc.sps_run(X, y, 2, 0.0, 5.0, J=4, N=128, seed=9)
    assert np.array_equal(a["theta"], b["theta"]) and a["logml"] == b["logml"]


@pytest.mark.parametrize("kind", [0, 1])
def test_two_pass_against_quadrature(orc, kind):
    """Algorithm 3: the second pass (fixed design, fresh randomness) agrees
    with quadrature, and replays the first pass's cycles and M steps."""
    X, y = _intercept_model(60, 0.75, seed=2)
    logZ, m1, sd = _intercept_truth(y, 5.0)
    kw = dict(kind=kind)
    if kind == 1:
        kw.update(h_min=0.01, h_max=2.0, acc_target=0.574)
    p1, p2 = orc.sps_two_pass(X, y, 2, 0.0, 5.0, J=16, N=1024, seed=13, **kw)
    assert p2["cycles"] == p1["cycles"] and p2["m_iters"] == p1["m_iters"]
    assert p1["sigma"].shape == (p1["m_iters"], 1, 1)
    assert abs(p2["mean"][0] - m1) < 4 * p2["nse"][0] + 1e-4
    assert abs(p2["logml"] - logZ) < 4 * p2["logml_nse"] + 0.01
    # the second pass draws fresh variates: its particles differ from the first pass's
    assert not np.allclose(p1["theta"], p2["theta"])


def test_mutate_cov_log_alpha_independent(orc):
    """Given proposal covariance: log alpha rebuilt with scipy."""
    w = synth.workload("small", T=80)
    X, y, _ = synth.make_data(w)
    J, N, d, t = 2, 16, w.d, 60
    th = synth.make_particles(J * N, d, scale=0.3, seed=11, center=[-0.7, 1, 0.3, -1.4, 0.4])
    ll, gr = orc.loglik(X, y, 2, th, 0, t, grad=True)
    A = synth.rng(3).standard_normal((d, d))
    S = 0.01 * (A @ A.T + d * np.eye(d))
    z = synth.make_normals(J * N, d, seed=12)
    u = synth.make_uniforms(J * N, seed=13)
    _, _, _, _, la, _ = orc.mutate_cov(X, y, 2, 0.0, 5.0, th, ll, gr, J, N, t, S, 1, z, u)
    L = np.linalg.cholesky(S)
    prior = lambda a: stats.norm.logpdf(a, 0.0, 5.0).sum(axis=-1)
    mu0 = th + 0.5 * (gr - th / 25.0) @ S.T
    prop = mu0 + z @ L.T
    llp, grp = orc.loglik(X, y, 2, prop, 0, t, grad=True)
    mu1 = prop + 0.5 * (grp - prop / 25.0) @ S.T
    ref = llp + prior(prop) - ll - prior(th)
    for p in range(J * N):
        ref[p] += (stats.multivariate_normal.logpdf(th[p], mu1[p], S)
                   - stats.multivariate_normal.logpdf(prop[p], mu0[p], S))
    assert np.allclose(la, ref, rtol=1e-9, atol=1e-9)
