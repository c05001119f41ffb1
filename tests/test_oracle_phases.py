"""Pins of the oracle's C, S and M phases and accuracy measures
(Algorithms 1-2, eqs. (C_phase_compute), (ESS_rule), (partial_g)-(RNE_def))."""
import math
import os

import mpmath
import numpy as np
import pytest
from scipy import stats

from paper_1304_4333_amd import synth

mpmath.mp.dps = 40


# --------------------------------------------------------------- ESS / C phase
def test_ess_equal_weights_is_P(orc):
    assert orc.ess(np.full(1000, -3.7)) == pytest.approx(1000, rel=1e-14)


def test_ess_one_hot_is_one(orc):
    lw = np.full(100, -np.inf)
    lw[17] = 4.0
    assert orc.ess(lw) == 1.0


def test_ess_shift_invariant_and_two_level(orc):
    # a particles of weight 1 and b of weight w: ESS = (a + b w)^2 / (a + b w^2)
    a, b, w = 30, 70, 0.25
    lw = np.array([0.0] * a + [math.log(w)] * b)
    ref = (a + b * w) ** 2 / (a + b * w * w)
    assert orc.ess(lw) == pytest.approx(ref, rel=1e-14)
    assert orc.ess(lw + 1234.5) == pytest.approx(ref, rel=1e-12)


def _mp_logprob(X, y, C, th, t):
    k = X.shape[1]
    e = [mpmath.mpf(0)] + [mpmath.fsum(mpmath.mpf(float(X[t, i])) * mpmath.mpf(float(th[(c - 1) * k + i]))
                                       for i in range(k)) for c in range(1, C)]
    return mpmath.log(mpmath.exp(e[int(y[t])]) / mpmath.fsum(mpmath.exp(v) for v in e))


def test_correct_brute_force(orc):
    """Brute force of the C phase: weights multiplied observation by observation
    at 40 digits, ESS from its definition, first s with ESS < 0.5 P."""
    g = synth.rng(21)
    T, k, C, J, N = 12, 2, 3, 2, 4
    X = g.standard_normal((T, k))
    y = g.integers(0, C, T).astype(np.int32)
    th = 2.0 * g.standard_normal((J * N, k * (C - 1)))
    ll0 = g.standard_normal(J * N)
    for s0 in (0, 3):
        w = [mpmath.mpf(1)] * (J * N)
        s = s0
        while True:
            s += 1
            w = [w[p] * mpmath.exp(_mp_logprob(X, y, C, th[p], s - 1)) for p in range(J * N)]
            ess = mpmath.fsum(w) ** 2 / mpmath.fsum(v * v for v in w)
            if ess < 0.5 * J * N or s == T:
                break
        lw, ll, t_end, ess_o = orc.correct(X, y, C, th, ll0, J, N, s0, 0.5)
        assert t_end == s
        assert ess_o == pytest.approx(float(ess), rel=1e-12)
        assert np.allclose(lw, [float(mpmath.log(v)) for v in w], rtol=1e-12, atol=1e-12)
        assert np.allclose(ll, ll0 + lw, rtol=0, atol=1e-14)


def test_correct_sums_to_loglik_increment(orc):
    """log w(t_end) equals the log-likelihood of observations s0+1..t_end."""
    w = synth.workload("small")
    X, y, _ = synth.make_data(w)
    th = synth.make_particles(64, w.d, scale=1.0, seed=3)
    lw, ll, t_end, _ = orc.correct(X, y, 2, th, np.zeros(64), 4, 16, 100, 0.5)
    assert 100 < t_end <= w.T
    assert np.allclose(lw, orc.loglik(X, y, 2, th, 100, t_end), rtol=1e-12, atol=1e-12)


def test_correct_equal_particles_runs_to_T(orc):
    """Identical particles keep ESS = P, so the C phase runs to s = T."""
    X = np.ones((20, 1))
    y = np.zeros(20, dtype=np.int32)
    th = np.full((8, 1), 0.3)
    lw, _, t_end, ess = orc.correct(X, y, 2, th, np.zeros(8), 2, 4, 5, 0.5)
    assert t_end == 20 and ess == pytest.approx(8.0)


def test_correct_rejects_bad_args(orc):
    X = np.ones((5, 1))
    y = np.zeros(5, dtype=np.int32)
    th = np.zeros((4, 1))
    for s0, ef in ((5, 0.5), (-1, 0.5), (0, 0.0), (0, 1.0)):
        with pytest.raises(orc.OracleError):
            orc.correct(X, y, 2, th, np.zeros(4), 2, 2, s0, ef)


# --------------------------------------------------------------- logML
def test_logml_update_equal_weights(orc):
    """Equal weights w: each group's increment is exactly log w."""
    lj = orc.logml_update(np.full(12, -2.5), 3, 4, np.zeros(3))
    assert np.allclose(lj, -2.5, rtol=0, atol=1e-15)


def test_logml_update_brute_force(orc):
    lw = synth.make_log_weights(40, seed=5, spread=4.0)
    lj = orc.logml_update(lw, 4, 10, np.ones(4))
    for j in range(4):
        ref = mpmath.log(mpmath.fsum(mpmath.exp(mpmath.mpf(v)) for v in lw[j * 10:(j + 1) * 10]) / 10)
        assert lj[j] == pytest.approx(1.0 + float(ref), rel=1e-14)


def test_logml_total_closed_forms(orc):
    L, nse, ml, mlnse = orc.logml_total(np.full(5, -17.25))
    assert L == pytest.approx(-17.25, abs=1e-14) and nse == 0.0 and mlnse == 0.0
    # two groups at log 1 and log 3: mean ML 2, r = (0.5, 1.5), sd(r) = 1/sqrt(2)
    L, nse, ml, mlnse = orc.logml_total(np.log([1.0, 3.0]))
    assert L == pytest.approx(math.log(2.0), rel=1e-14)
    assert nse == pytest.approx(math.sqrt(0.5) / math.sqrt(2.0), rel=1e-14)
    assert ml == pytest.approx(0.5 * math.log(3.0), rel=1e-14)


def test_logml_degenerate_group(orc):
    lw = np.zeros(8)
    lw[4:] = -np.inf
    with pytest.raises(orc.OracleError) as e:
        orc.logml_update(lw, 2, 4, np.zeros(2))
    assert e.value.status == orc.ORC_ERR_DEGENERATE


# --------------------------------------------------------------- S phase
def _ref_resample(W, J, N, scheme, U):
    """Independent reference on Python integers with numpy.searchsorted as the
    inverse CDF (library routine)."""
    out = []
    for j in range(J):
        w = [int(v) for v in W[j * N:(j + 1) * N]]
        u = [int(v) for v in U[j * N:(j + 1) * N]]
        S = sum(w)
        if scheme == 1:
            cum = np.cumsum(np.array(w, dtype=np.uint64))
            for i in range(N):
                tgt = (u[i] * S) >> 53
                out.append(j * N + int(np.searchsorted(cum, np.uint64(tgt), side="right")))
        else:
            copies = [(N * v) // S for v in w]
            for n, c in enumerate(copies):
                out.extend([j * N + n] * c)
            R = N - sum(copies)
            res = [N * v - c * S for v, c in zip(w, copies)]
            cum = np.cumsum(np.array(res, dtype=np.uint64))
            tot = sum(res)
            assert tot == R * S
            for i in range(R):
                tgt = (u[i] * tot) >> 53
                out.append(j * N + int(np.searchsorted(cum, np.uint64(tgt), side="right")))
    return np.array(out, dtype=np.int32)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("J,N", [(1, 1), (3, 7), (4, 256), (2, 4096)])
def test_resample_int_matches_searchsorted(orc, scheme, J, N):
    W = synth.make_int_weights(J, N, seed=J * 100 + N)
    U = synth.make_u53(J * N, seed=N)
    anc = orc.resample_int(W, J, N, scheme, U)
    assert np.array_equal(anc, _ref_resample(W, J, N, scheme, U))
    # ancestors stay inside their group and have positive weight
    assert np.all(anc // N == np.repeat(np.arange(J), N))
    assert np.all(W[anc] > 0)


def test_resample_residual_copies(orc):
    J, N = 2, 64
    W = synth.make_int_weights(J, N, seed=3)
    U = synth.make_u53(J * N, seed=4)
    anc = orc.resample_int(W, J, N, 0, U)
    for j in range(J):
        w = W[j * N:(j + 1) * N].astype(object)
        S = sum(w)
        counts = np.bincount(anc[j * N:(j + 1) * N] - j * N, minlength=N)
        floor_ = np.array([(N * v) // S for v in w])
        assert np.all(counts >= floor_) and np.all(counts <= floor_ + (N - floor_.sum()))
        assert counts.sum() == N


def test_resample_multinomial_counts_chi_square(orc):
    """Counts over many independent draws follow the weights (chi-square)."""
    N, reps = 8, 4000
    w = np.array([1, 2, 3, 4, 5, 6, 7, 12], dtype=np.uint64) << np.uint64(30)
    W = np.tile(w, reps)
    U = synth.make_u53(N * reps, seed=9)
    anc = orc.resample_int(W, reps, N, 1, U) % N
    counts = np.bincount(anc, minlength=N)
    expect = N * reps * w.astype(float) / w.astype(float).sum()
    assert stats.chisquare(counts, expect).pvalue > 1e-3


def test_resample_from_log_weights(orc):
    J, N = 3, 50
    lw = synth.make_log_weights(J * N, seed=6, spread=2.0, n_neg_inf=10)
    U = synth.make_u53(J * N, seed=7)
    anc, W = orc.resample(lw, J, N, 0, U)
    for j in range(J):
        seg = lw[j * N:(j + 1) * N]
        m = seg.max()
        ref = [int(mpmath.floor(mpmath.exp(mpmath.mpf(v) - mpmath.mpf(m)) * 2 ** 40)) if np.isfinite(v) else 0
               for v in seg]
        assert [int(v) for v in W[j * N:(j + 1) * N]] == ref
    assert np.array_equal(anc, orc.resample_int(W, J, N, 0, U))
    assert np.all(np.isfinite(lw[anc]))


# --------------------------------------------------------------- M phase
def test_cov_and_cholesky_match_numpy(orc):
    th = synth.make_particles(500, 7, seed=8) @ synth.rng(9).standard_normal((7, 7))
    mean, V = orc.cov(th)
    assert np.allclose(mean, th.mean(0), rtol=1e-13, atol=1e-14)
    assert np.allclose(V, np.cov(th.T, ddof=1), rtol=1e-12, atol=1e-13)
    L = orc.cholesky(V)
    assert np.allclose(L, np.linalg.cholesky(V), rtol=1e-10, atol=1e-12)


def test_cholesky_not_pd_for_collapsed_particles(orc):
    """Section 4.2: with one unique particle per group the sample variance has
    rank min(J, dim theta) and the M phase must fail."""
    J, d = 3, 5
    base = synth.make_particles(J, d, seed=10)
    th = np.repeat(base, 16, axis=0)
    _, V = orc.cov(th)
    with pytest.raises(orc.OracleError) as e:
        orc.cholesky(V)
    assert e.value.status == orc.ORC_ERR_NOT_PD


@pytest.mark.parametrize("kind", [0, 1])
def test_mutate_log_alpha_independent(orc, kind):
    """log alpha rebuilt with numpy/scipy: proposal from numpy's Cholesky,
    prior from scipy.stats.norm, MALA densities from scipy.stats.multivariate_normal."""
    w = synth.workload("small", T=80)
    X, y, _ = synth.make_data(w)
    J, N, d, t, h = 2, 16, w.d, 60, 0.4
    th = synth.make_particles(J * N, d, scale=0.3, seed=11, center=[-0.7, 1, 0.3, -1.4, 0.4])
    if kind == 1:
        ll, gr = orc.loglik(X, y, 2, th, 0, t, grad=True)
    else:
        ll, gr = orc.loglik(X, y, 2, th, 0, t), None
    z = synth.make_normals(J * N, d, seed=12)
    u = synth.make_uniforms(J * N, seed=13)
    th2, ll2, gr2, rate, la, acc = orc.mutate(X, y, 2, 0.0, 5.0, th, ll, gr, J, N, t, h, kind, z, u)
    V = np.cov(th.T, ddof=1)
    L = np.linalg.cholesky(V)
    prior = lambda a: stats.norm.logpdf(a, 0.0, 5.0).sum(axis=-1)
    if kind == 0:
        prop = th + math.sqrt(h) * z @ L.T
        la_ref = orc.loglik(X, y, 2, prop, 0, t) + prior(prop) - ll - prior(th)
    else:
        mu0 = th + 0.5 * h * (gr - th / 25.0) @ V.T
        prop = mu0 + math.sqrt(h) * z @ L.T
        llp, grp = orc.loglik(X, y, 2, prop, 0, t, grad=True)
        mu1 = prop + 0.5 * h * (grp - prop / 25.0) @ V.T
        la_ref = llp + prior(prop) - ll - prior(th)
        for p in range(J * N):
            la_ref[p] += (stats.multivariate_normal.logpdf(th[p], mu1[p], h * V)
                          - stats.multivariate_normal.logpdf(prop[p], mu0[p], h * V))
    assert np.allclose(la, la_ref, rtol=1e-9, atol=1e-9)
    assert np.array_equal(acc, np.log(u) < la_ref)
    assert rate == acc.mean()
    assert np.allclose(th2[acc], prop[acc], rtol=1e-12) and np.array_equal(th2[~acc], th[~acc])
    if kind == 1:
        assert np.allclose(gr2[acc], orc.loglik(X, y, 2, th2[acc], 0, t, grad=True)[1], rtol=1e-12)


def _posterior_grid(y_sum, T, s, lo=-6, hi=6, n=20001):
    """Intercept-only binary logit with prior N(0, s^2): posterior on a grid."""
    a = np.linspace(lo, hi, n)
    logp = stats.norm.logpdf(a, 0, s) + y_sum * -np.logaddexp(0, -a) + (T - y_sum) * -np.logaddexp(0, a)
    p = np.exp(logp - logp.max())
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    return a, cdf


@pytest.mark.parametrize("kind", [0, 1])
def test_mutate_leaves_posterior_invariant(orc, kind):
    """Eq. (M_invariant): exact posterior draws (inverse CDF on a quadrature
    grid) keep their distribution after repeated M steps (KS test)."""
    T = 30
    X = np.ones((T, 1))
    y = (synth.rng(14).random(T) < 0.7).astype(np.int32)
    a, cdf = _posterior_grid(int(y.sum()), T, 5.0)
    J, N = 8, 512
    th = np.interp(synth.make_uniforms(J * N, seed=15), cdf, a)[:, None]
    if kind == 1:
        ll, gr = orc.loglik(X, y, 2, th, grad=True)
    else:
        ll, gr = orc.loglik(X, y, 2, th), None
    for r in range(8):
        z = synth.make_normals(J * N, 1, seed=100 + r)
        u = synth.make_uniforms(J * N, seed=200 + r)
        th, ll, gr, rate, _, _ = orc.mutate(X, y, 2, 0.0, 5.0, th, ll, gr, J, N, T, 0.8, kind, z, u)
        assert 0.2 < rate < 1.0
    F = lambda v: np.interp(v, a, cdf)
    assert stats.kstest(th[:, 0], F).pvalue > 1e-3


# --------------------------------------------------------------- NSE / RNE
def test_moments_worked_example(orc):
    path = os.path.join(os.path.dirname(__file__), "golden", "moments_worked_example.txt")
    with open(path) as f:
        line = [l for l in f if not l.startswith("#")][0]
    lhs, rhs = line.split("->")
    v = [float(a) for a in lhs.split()]
    J, N, g = int(v[0]), int(v[1]), np.array(v[2:])
    mean, sd, nse, rne = orc.moments(g, J, N)
    exp = [float(a) for a in rhs.split()]
    assert [mean[0], sd[0], nse[0], rne[0]] == pytest.approx(exp, rel=1e-15)


def test_rne_near_one_for_iid(orc):
    g = synth.rng(16).standard_normal((64 * 200, 50))
    _, _, _, rne = orc.moments(g, 64, 200)
    # v_hat/v ~ chi2(63)/63 per function: mean of 1/that ~ 63/61
    assert abs(rne.mean() - 63 / 61) < 0.1


def test_rne_for_group_dependence(orc):
    """Group effects of variance tau^2 on top of unit noise: the true v is
    1 + N tau^2, so RNE concentrates around (1 + tau^2)/(1 + N tau^2)."""
    J, N, tau = 400, 50, 0.2
    g0 = synth.rng(17)
    g = g0.standard_normal((J, N)) + tau * g0.standard_normal((J, 1))
    _, _, _, rne = orc.moments(g.reshape(-1), J, N)
    assert rne[0] == pytest.approx((1 + tau ** 2) / (1 + N * tau ** 2), rel=0.15)


def test_nse_t_calibration(orc):
    """Eq. (gbar_tstat): (gbar - g) / NSE ~ t(J - 1) over independent repetitions."""
    J, N, reps = 6, 40, 3000
    g = synth.rng(18).standard_normal((reps, J * N)).T.copy()
    mean, _, nse, _ = orc.moments(g, J, N)
    tstat = mean / nse
    assert stats.kstest(tstat, stats.t(J - 1).cdf).pvalue > 1e-3
