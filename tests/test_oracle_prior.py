"""Pins of the oracle's Gaussian prior with a full covariance and of the
normalised g-prior (eqs. (prior_Gauss), (prior_norm), (g-prior_def)).

Each check compares with something other than the oracle's own arithmetic:
scipy's multivariate normal density, numpy's matrix inverse, the algebraic
identity for the average prior log-odds variance, invariance of the prior of
all log-odds ratios to the choice of the base outcome, and moments of draws."""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

from paper_1304_4333_amd import synth


def _spd(d, seed):
    A = synth.rng(seed).standard_normal((d, d))
    return A @ A.T / d + 0.5 * np.eye(d)


def test_logprior_full_cov_matches_scipy(orc):
    d = 7
    cov = _spd(d, 1)
    mean = synth.rng(2).standard_normal(d)
    th = synth.rng(3).standard_normal((11, d)) * 2.0
    lp, g = orc.logprior(th, mean, cov=cov)
    ref = stats.multivariate_normal(mean, cov).logpdf(th)
    assert np.allclose(lp, ref, rtol=1e-12, atol=1e-12)
    gref = -np.linalg.solve(cov, (th - mean).T).T
    assert np.allclose(g, gref, rtol=1e-10, atol=1e-12)


def test_logprior_diagonal_case_is_independent_normals(orc):
    d = 5
    sd = np.array([0.5, 1.0, 2.0, 3.0, 5.0])
    th = synth.rng(4).standard_normal((6, d)) * 3
    lp, g = orc.logprior(th, 0.0, sd)
    assert np.allclose(lp, stats.norm.logpdf(th, 0.0, sd).sum(1), rtol=1e-13)
    assert np.allclose(g, -th / sd ** 2, rtol=1e-13)


def test_init_prior_full_cov_moments(orc):
    d = 4
    cov = _spd(d, 5)
    mean = np.array([1.0, -2.0, 0.5, 0.0])
    P = 200_000
    th = orc.init_prior(mean, 1.0, P, seed=9, stream=1, cov=cov)
    se = np.sqrt(np.diag(cov) / P)
    assert np.all(np.abs(th.mean(0) - mean) < 5 * se)
    # sample covariance within a few standard errors (Wishart sd ~ sqrt((s_ii s_jj + s_ij^2)/P))
    S = np.cov(th.T)
    sd_S = np.sqrt((np.outer(np.diag(cov), np.diag(cov)) + cov ** 2) / P)
    assert np.all(np.abs(S - cov) < 5 * sd_S)


def test_gprior_cov_blocks_against_numpy_inverse(orc):
    w = synth.workload("small", T=300)
    X, _, _ = synth.make_data(w)
    C, g = 4, 0.25
    k = X.shape[1]
    cov = orc.gprior_cov(X, C, g)
    Sig = g * X.shape[0] * np.linalg.inv(X.T @ X)
    for i in range(C - 1):
        for j in range(C - 1):
            blk = cov[i * k:(i + 1) * k, j * k:(j + 1) * k]
            assert np.allclose(blk, (2.0 if i == j else 1.0) * Sig, rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("C", [2, 3, 5])
def test_gprior_average_log_odds_variance(orc, C):
    """With Sigma = g T (X'X)^-1, the prior variance of any log-odds ratio
    (theta_i - theta_j)' x_t averaged over the T data rows is
    (1/T) tr(2 g T I_k) = 2 g k (the identity behind eq. (g-prior_def))."""
    w = synth.workload("small", T=250)
    X, _, _ = synth.make_data(w)
    T, k = X.shape
    g = 0.5
    cov = orc.gprior_cov(X, C, g)
    # log-odds of outcome c against the base: beta_c' x; of c against c': (beta_c - beta_c')' x
    for c in range(C - 1):
        Bc = cov[c * k:(c + 1) * k, c * k:(c + 1) * k]
        v = np.einsum("ti,ij,tj->t", X, Bc, X).mean()
        assert math.isclose(v, 2 * g * k, rel_tol=1e-10)
    if C > 2:
        D = np.zeros((k, (C - 1) * k))
        D[:, 0:k] = np.eye(k)
        D[:, k:2 * k] = -np.eye(k)
        Bd = D @ cov @ D.T
        v = np.einsum("ti,ij,tj->t", X, Bd, X).mean()
        assert math.isclose(v, 2 * g * k, rel_tol=1e-10)


def test_gprior_invariant_to_base_outcome(orc):
    """Eq. (prior_norm): re-normalising on another outcome leaves the prior of
    the free parameters in the same block form (the prior is the same)."""
    w = synth.workload("small", T=200)
    X, _, _ = synth.make_data(w)
    k = X.shape[1]
    C = 4
    cov = orc.gprior_cov(X, C, 1.0)
    m = C - 1
    # beta_c = theta_c - theta_0 (c = 1..3) -> gamma_c = theta_c - theta_1 (c = 0, 2, 3):
    # gamma_0 = -beta_1, gamma_2 = beta_2 - beta_1, gamma_3 = beta_3 - beta_1
    M1 = np.array([[-1, 0, 0], [-1, 1, 0], [-1, 0, 1]], dtype=float)
    M = np.kron(M1, np.eye(k))
    assert np.allclose(M @ cov @ M.T, cov, rtol=1e-10, atol=1e-12)
    assert m == 3


def test_sps_gprior_intercept_model_vs_quadrature(orc):
    """Intercept-only binary model: X'X = T, so the normalised g-prior on the
    intercept is N(0, 2 g).  The oracle SPS matches quadrature."""
    T = 60
    X = np.ones((T, 1))
    y = (synth.rng(12).random(T) < 0.3).astype(np.int32)
    m = int(y.sum())
    g = 0.5
    cov = orc.gprior_cov(X, 2, g)
    assert math.isclose(cov[0, 0], 2 * g, rel_tol=1e-14)
    s = math.sqrt(2 * g)
    f = lambda a: math.exp(stats.norm.logpdf(a, 0, s) + m * special.log_expit(a) + (T - m) * special.log_expit(-a))
    Z = integrate.quad(f, -10, 10, epsabs=0, epsrel=1e-12, limit=400)[0]
    m1 = integrate.quad(lambda a: a * f(a), -10, 10, epsabs=0, epsrel=1e-12, limit=400)[0] / Z
    r = orc.sps_run(X, y, 2, 0.0, 1.0, 8, 512, seed=5, prior_cov=cov)
    assert abs(r["mean"][0] - m1) < 4 * r["nse"][0] + 1e-4
    assert abs(r["logml"] - math.log(Z)) < 4 * r["logml_nse"] + 0.01
