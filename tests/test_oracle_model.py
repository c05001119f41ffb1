"""Pins of the oracle's model functions (eq. (plogit), Section 2.1) against
values fixed by the mathematics: closed forms, 50-digit brute force, a library
routine for the binary case, symmetry invariants and finite differences."""
import math

import mpmath
import numpy as np
import pytest
from scipy import special, stats

from paper_1304_4333_amd import synth

mpmath.mp.dps = 50


def _tiny(T, k, C, seed, scale=1.0):
    g = synth.rng(seed)
    X = g.standard_normal((T, k))
    y = g.integers(0, C, size=T).astype(np.int32)
    th = scale * g.standard_normal((3, k * (C - 1)))
    return X, y, th


def _mp_loglik(X, y, C, th, t0, t1):
    """log prod_t P(Y_t = y_t) straight from eq. (plogit): ratio of exponentials,
    multiplied over observations, logged once, at 50 digits."""
    T, k = X.shape
    L = mpmath.mpf(1)
    for t in range(t0, t1):
        e = [mpmath.mpf(0)]
        for c in range(1, C):
            e.append(mpmath.fsum(mpmath.mpf(float(X[t, i])) * mpmath.mpf(float(th[(c - 1) * k + i]))
                                 for i in range(k)))
        L *= mpmath.exp(e[int(y[t])]) / mpmath.fsum(mpmath.exp(v) for v in e)
    return mpmath.log(L)


@pytest.mark.parametrize("C", [2, 3, 4])
def test_loglik_at_zero_is_minus_T_log_C(orc, C):
    X, y, _ = _tiny(37, 4, C, seed=1)
    th = np.zeros((5, 4 * (C - 1)))
    ll = orc.loglik(X, y, C, th)
    assert np.allclose(ll, -37 * math.log(C), rtol=0, atol=1e-12)
    ll = orc.loglik(X, y, C, th, 5, 19)
    assert np.allclose(ll, -14 * math.log(C), rtol=0, atol=1e-12)


@pytest.mark.parametrize("C,k,T", [(2, 1, 4), (2, 2, 3), (3, 2, 4), (3, 1, 2), (4, 2, 3)])
def test_loglik_brute_force_50_digits(orc, C, k, T):
    X, y, th = _tiny(T, k, C, seed=10 * C + k, scale=2.0)
    ll = orc.loglik(X, y, C, th)
    for p in range(th.shape[0]):
        ref = float(_mp_loglik(X, y, C, th[p], 0, T))
        assert abs(ll[p] - ref) <= 1e-13 * max(1.0, abs(ref))
    ll = orc.loglik(X, y, C, th, 1, T)
    ref = float(_mp_loglik(X, y, C, th[0], 1, T))
    assert abs(ll[0] - ref) <= 1e-13 * max(1.0, abs(ref))


def test_loglik_brute_force_large_predictors(orc):
    """|eta| of order 10^2 (prior draws with sd 5): no overflow, exact to 1e-13."""
    X, y, th = _tiny(4, 3, 3, seed=3, scale=30.0)
    ll = orc.loglik(X, y, 3, th)
    for p in range(th.shape[0]):
        ref = float(_mp_loglik(X, y, 3, th[p], 0, 4))
        assert abs(ll[p] - ref) <= 1e-13 * max(1.0, abs(ref))


def test_binary_equals_library_log_sigmoid(orc):
    """C = 2: log P(y|x) = log sigmoid((2y-1) x'theta), via scipy.special.log_expit."""
    X, y, th = _tiny(200, 6, 2, seed=4, scale=3.0)
    ll = orc.loglik(X, y, 2, th)
    eta = X @ th.T
    ref = special.log_expit((2.0 * y[:, None] - 1.0) * eta).sum(axis=0)
    assert np.allclose(ll, ref, rtol=1e-12, atol=1e-10)


def test_loglik_permutation_invariance(orc):
    X, y, th = _tiny(64, 5, 4, seed=5, scale=1.0)
    th = np.concatenate([th, th[::-1]])
    ll = orc.loglik(X, y, 4, th)
    perm = synth.rng(6).permutation(64)
    ll2 = orc.loglik(X[perm], y[perm], 4, th)
    assert np.allclose(ll, ll2, rtol=1e-13)
    assert np.allclose(ll[:3], ll[3:][::-1], rtol=0, atol=0)


def test_loglik_outcome_relabelling(orc):
    """Swapping which outcome is the base is the affine reparametrisation
    theta_c -> theta_c - theta_b of Section 3.1; the likelihood is unchanged."""
    X, y, th = _tiny(40, 3, 3, seed=7, scale=1.5)
    k = 3
    # base 0 -> base 1: outcomes relabelled (0,1,2) -> (1,0,2)
    y2 = np.where(y == 0, 1, np.where(y == 1, 0, y)).astype(np.int32)
    th1, th2 = th[:, :k], th[:, k:]
    # new params: outcome "1" is old 0 (theta = -th1), outcome "2" is old 2 (th2 - th1)
    th_new = np.concatenate([-th1, th2 - th1], axis=1)
    assert np.allclose(orc.loglik(X, y, 3, th), orc.loglik(X, y2, 3, th_new), rtol=1e-12)


def test_gradient_closed_form_at_zero(orc):
    X, y, _ = _tiny(50, 4, 3, seed=8)
    th = np.zeros((2, 8))
    _, g = orc.loglik(X, y, 3, th, grad=True)
    ref = np.concatenate([X.T @ ((y == c) - 1.0 / 3.0) for c in (1, 2)])
    assert np.allclose(g[0], ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("C,k,T", [(2, 2, 3), (3, 2, 3)])
def test_gradient_brute_force_50_digits(orc, C, k, T):
    X, y, th = _tiny(T, k, C, seed=20 + C, scale=1.0)
    _, g = orc.loglik(X, y, C, th, grad=True)
    d = k * (C - 1)
    for i in range(d):
        def f(v, i=i):
            t = [mpmath.mpf(float(a)) for a in th[0]]
            t[i] = v
            return _mp_loglik_mp(X, y, C, t, T)
        ref = float(mpmath.diff(f, mpmath.mpf(float(th[0, i]))))
        assert abs(g[0, i] - ref) <= 1e-12 * max(1.0, abs(ref))


def _mp_loglik_mp(X, y, C, t, T):
    k = X.shape[1]
    L = mpmath.mpf(1)
    for s in range(T):
        e = [mpmath.mpf(0)] + [mpmath.fsum(mpmath.mpf(float(X[s, i])) * t[(c - 1) * k + i]
                                           for i in range(k)) for c in range(1, C)]
        L *= mpmath.exp(e[int(y[s])]) / mpmath.fsum(mpmath.exp(v) for v in e)
    return mpmath.log(L)


def test_gradient_finite_differences(orc):
    X, y, th = _tiny(120, 5, 4, seed=9, scale=0.7)
    ll, g = orc.loglik(X, y, 4, th, 10, 100, grad=True)
    assert np.allclose(ll, orc.loglik(X, y, 4, th, 10, 100), rtol=0, atol=0)
    d = th.shape[1]
    for i in range(d):
        e = np.zeros(d)
        hstep = 1e-5
        e[i] = hstep
        fd = (orc.loglik(X, y, 4, th + e, 10, 100) - orc.loglik(X, y, 4, th - e, 10, 100)) / (2 * hstep)
        assert np.allclose(g[:, i], fd, rtol=1e-6, atol=1e-6)


def test_gradient_residuals_sum_to_zero_over_all_outcomes(orc):
    """With an intercept column, sum over outcomes c=0..C-1 of (1{y=c} - pi_c) = 0
    per observation, so the intercept gradient over the C-1 free outcomes equals
    minus the base-outcome residual sum: sum_t (pi_0 - 1{y_t=0}); at theta = 0
    that is T/C - #{y=0}."""
    X, y, _ = _tiny(60, 3, 4, seed=11)
    X[:, 0] = 1.0
    _, g = orc.loglik(X, y, 4, np.zeros((1, 9)), grad=True)
    intercepts = g[0, [0, 3, 6]]
    assert abs(intercepts.sum() - (60 / 4 - np.sum(y == 0))) < 1e-12


def test_logprior_matches_scipy(orc):
    th = synth.make_particles(7, 6, scale=2.0, seed=12)
    mean = np.linspace(-1, 1, 6)
    sd = np.linspace(0.5, 3, 6)
    lp, g = orc.logprior(th, mean, sd)
    assert np.allclose(lp, stats.norm.logpdf(th, mean, sd).sum(axis=1), rtol=1e-13)
    assert np.allclose(g, -(th - mean) / sd ** 2, rtol=1e-13)
