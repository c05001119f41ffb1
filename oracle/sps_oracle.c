/*
 * sps_oracle.c -- plain FP64 CPU oracle of the sequential posterior simulator
 * (SPS) for multinomial logit models, written from Geweke, Durham & Xu (2013).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * CPU baseline of the benchmark; the product library never calls it.  It
 * shares no source with the HIP path.
 *
 * Style: the slowest obvious code.  Every quantity is computed in double in
 * the order the paper states it; the only parallelism is an OpenMP loop over
 * independent particles (each particle's arithmetic is serial and unchanged).
 *
 * Points the paper leaves open are marked READING where the reading is
 * applied; the comment there states the reading taken.
 */
#include "sps_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of the 4x32 Philox S-box with the    */
/* published multipliers and Weyl key increments.                            */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One Philox block for element index e of a stream: counter (e, stream),
 * key = seed.  Two 53-bit integers from the four output words. */
static void philox_pair(uint64_t seed, uint64_t stream, uint64_t e, uint64_t* a, uint64_t* b)
{
    uint32_t ctr[4] = { (uint32_t)e, (uint32_t)(e >> 32), (uint32_t)stream, (uint32_t)(stream >> 32) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    *a = ((((uint64_t)o[0]) << 32) | o[1]) >> 11;
    *b = ((((uint64_t)o[2]) << 32) | o[3]) >> 11;
}

void orc_u53(uint64_t seed, uint64_t stream, int64_t count, uint64_t* out)
{
    for (int64_t e = 0; e < count; ++e) {
        uint64_t a, b;
        philox_pair(seed, stream, (uint64_t)e, &a, &b);
        out[e] = a;
    }
}

void orc_uniforms(uint64_t seed, uint64_t stream, int64_t count, double* out)
{
    for (int64_t e = 0; e < count; ++e) {
        uint64_t a, b;
        philox_pair(seed, stream, (uint64_t)e, &a, &b);
        out[e] = ((double)a + 0.5) * 0x1p-53;
    }
}

/* Standard normals by the Box-Muller transform; element (p, i) of a P x d
 * array takes output i mod 2 of block e = p ceil(d/2) + floor(i/2). */
void orc_normals(uint64_t seed, uint64_t stream, int64_t P, int32_t d, double* out)
{
    int64_t half = (d + 1) / 2;
    for (int64_t p = 0; p < P; ++p) {
        for (int32_t i = 0; i < d; ++i) {
            uint64_t a, b;
            philox_pair(seed, stream, (uint64_t)(p * half + i / 2), &a, &b);
            double u1 = ((double)a + 0.5) * 0x1p-53;
            double u2 = ((double)b + 0.5) * 0x1p-53;
            double r = sqrt(-2.0 * log(u1));
            out[p * d + i] = (i % 2 == 0) ? r * cos(2.0 * M_PI * u2) : r * sin(2.0 * M_PI * u2);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Model: eq. (plogit), normalised by theta_0 = 0 (Section 2.1 and the        */
/* normalisation discussion of Section 3.1).                                  */
/* ------------------------------------------------------------------------ */

/* log P(Y_t = yt | x_t, theta) = eta_yt - log sum_c exp(eta_c), with
 * eta_0 = 0 and eta_c = theta_c' x_t.  The log-sum-exp is evaluated with the
 * largest eta factored out (an exact identity).  eta has room for C values. */
static double obs_logprob(const double* x, int32_t k, int32_t C, int32_t yt,
                          const double* th, double* eta)
{
    eta[0] = 0.0;
    for (int32_t c = 1; c < C; ++c) {
        double s = 0.0;
        for (int32_t i = 0; i < k; ++i) s += x[i] * th[(int64_t)(c - 1) * k + i];
        eta[c] = s;
    }
    double m = eta[0];
    for (int32_t c = 1; c < C; ++c) if (eta[c] > m) m = eta[c];
    double s = 0.0;
    for (int32_t c = 0; c < C; ++c) s += exp(eta[c] - m);
    return eta[yt] - m - log(s);
}

static int data_ok(int64_t T, int32_t k, int32_t C, int64_t t0, int64_t t1)
{
    return T >= 0 && k >= 1 && C >= 2 && C <= 64 && t0 >= 0 && t0 <= t1 && t1 <= T;
}

/* Log-likelihood of observations t0+1..t1 (rows t0..t1-1): the product form
 * of the likelihood (Section 2.1) summed in logs, left to right. */
int orc_loglik(const double* X, const int32_t* y, int64_t T, int32_t k, int32_t C,
               const double* theta, int64_t P, int64_t t0, int64_t t1, double* ll)
{
    if (!data_ok(T, k, C, t0, t1) || P < 0) return ORC_ERR_ARG;
    int64_t d = (int64_t)k * (C - 1);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
        double eta[64];
        double acc = 0.0;
        for (int64_t t = t0; t < t1; ++t)
            acc += obs_logprob(X + t * k, k, C, y[t], theta + p * d, eta);
        ll[p] = acc;
    }
    return ORC_OK;
}

/* Gradient of the log-likelihood with respect to the free parameters:
 * d/d theta_{c,i} sum_t log P(Y_t=y_t) = sum_t x_{t,i} (1{y_t=c} - pi_{t,c}),
 * pi_{t,c} = exp(eta_c) / sum_c' exp(eta_c'). */
int orc_loglik_grad(const double* X, const int32_t* y, int64_t T, int32_t k, int32_t C,
                    const double* theta, int64_t P, int64_t t0, int64_t t1,
                    double* ll, double* grad)
{
    if (!data_ok(T, k, C, t0, t1) || P < 0) return ORC_ERR_ARG;
    int64_t d = (int64_t)k * (C - 1);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
        double eta[64];
        const double* th = theta + p * d;
        double* g = grad + p * d;
        for (int64_t i = 0; i < d; ++i) g[i] = 0.0;
        double acc = 0.0;
        for (int64_t t = t0; t < t1; ++t) {
            const double* x = X + t * k;
            acc += obs_logprob(x, k, C, y[t], th, eta);
            double m = eta[0];
            for (int32_t c = 1; c < C; ++c) if (eta[c] > m) m = eta[c];
            double s = 0.0;
            for (int32_t c = 0; c < C; ++c) s += exp(eta[c] - m);
            for (int32_t c = 1; c < C; ++c) {
                double pi_c = exp(eta[c] - m) / s;
                double r = (y[t] == c ? 1.0 : 0.0) - pi_c;
                for (int32_t i = 0; i < k; ++i) g[(int64_t)(c - 1) * k + i] += x[i] * r;
            }
        }
        ll[p] = acc;
    }
    return ORC_OK;
}

static void lower_solve(const double* L, int32_t d, const double* r, double* v);

/* Gaussian prior on the free parameters, theta ~ N(mean, S) with S = L L'
 * (L lower triangular, row-major d x d).  Eq. (prior_Gauss) with independent
 * components gives a diagonal L; the normalised form of eq. (prior_norm),
 * e.g. with the g-prior of eq. (g-prior_def), gives a full one.
 *   log p = -d/2 log(2 pi) - sum_i log L_ii - |r|^2 / 2,  L r = theta - mean,
 *   grad log p = -S^-1 (theta - mean) = -L'^-1 r.
 * glp may be NULL. */
void orc_logprior(const double* theta, int64_t P, int32_t d, const double* mean,
                  const double* L, double* lp, double* glp)
{
    double logdet = 0.0;
    for (int32_t i = 0; i < d; ++i) logdet += log(L[i * d + i]);
#pragma omp parallel
    {
    double* r = (double*)malloc(sizeof(double) * (d > 0 ? d : 1));
#pragma omp for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
        const double* th = theta + p * d;
        /* forward substitution L r = theta - mean */
        double q = 0.0;
        for (int32_t i = 0; i < d; ++i) {
            double s = th[i] - mean[i];
            for (int32_t j = 0; j < i; ++j) s -= L[i * d + j] * r[j];
            r[i] = s / L[i * d + i];
            q += r[i] * r[i];
        }
        lp[p] = -0.5 * d * log(2.0 * M_PI) - logdet - 0.5 * q;
        if (glp) {
            /* back substitution L' w = r, grad = -w */
            double* g = glp + p * d;
            for (int32_t i = d - 1; i >= 0; --i) {
                double s = r[i];
                for (int32_t j = i + 1; j < d; ++j) s -= L[j * d + i] * g[j];
                g[i] = s / L[i * d + i];
            }
            for (int32_t i = 0; i < d; ++i) g[i] = -g[i];
        }
    }
    free(r);
    }
}

/* Algorithm 1 step 1: particles iid from the prior, theta = mean + L z. */
void orc_init_prior(const double* mean, const double* L, int32_t d, int64_t P,
                    uint64_t seed, uint64_t stream, double* theta)
{
    double* z = (double*)malloc(sizeof(double) * (size_t)(P > 0 ? P : 1) * (d > 0 ? d : 1));
    orc_normals(seed, stream, P, d, z);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p)
        for (int32_t i = 0; i < d; ++i) {
            double s = mean[i];
            for (int32_t j = 0; j <= i; ++j) s += L[i * d + j] * z[p * d + j];
            theta[p * d + i] = s;
        }
    free(z);
}

/* The prior covariance of eq. (prior_norm) for the model normalised on
 * outcome 0, when theta_c ~ iid N(0, Sigma) for all C outcomes before
 * normalisation and Sigma = g T (X'X)^-1 (eq. (g-prior_def)): the free
 * vectors beta_c = theta_c - theta_0 (c = 1..C-1) have var 2 Sigma and
 * pairwise covariance Sigma, i.e. block (i, j) of the d x d covariance is
 * (1 + [i == j]) Sigma.  X'X is inverted through its Cholesky factor. */
int orc_gprior_cov(const double* X, int64_t T, int32_t k, int32_t C, double g, double* cov)
{
    if (!data_ok(T, k, C, 0, 0) || T < 1 || !(g > 0.0)) return ORC_ERR_ARG;
    int32_t d = k * (C - 1);
    double* S = (double*)malloc(sizeof(double) * (size_t)k * k);
    double* Ls = (double*)malloc(sizeof(double) * (size_t)k * k);
    double* Sig = (double*)malloc(sizeof(double) * (size_t)k * k);
    double* e = (double*)malloc(sizeof(double) * k);
    double* v = (double*)malloc(sizeof(double) * k);
    int status = ORC_OK;
    if (!S || !Ls || !Sig || !e || !v) { status = ORC_ERR_NOMEM; goto done; }
    for (int32_t a = 0; a < k; ++a)
        for (int32_t b = 0; b < k; ++b) {
            double s = 0.0;
            for (int64_t t = 0; t < T; ++t) s += X[t * k + a] * X[t * k + b];
            S[a * k + b] = s;
        }
    status = orc_cholesky(S, k, Ls);
    if (status != ORC_OK) goto done;
    /* column b of S^-1: solve Ls Ls' x = e_b */
    for (int32_t b = 0; b < k; ++b) {
        for (int32_t i = 0; i < k; ++i) e[i] = (i == b) ? 1.0 : 0.0;
        lower_solve(Ls, k, e, v);
        for (int32_t i = k - 1; i >= 0; --i) {
            double s = v[i];
            for (int32_t j = i + 1; j < k; ++j) s -= Ls[j * k + i] * e[j];
            e[i] = s / Ls[i * k + i];
        }
        for (int32_t i = 0; i < k; ++i) Sig[i * k + b] = g * (double)T * e[i];
    }
    for (int32_t ci = 0; ci < C - 1; ++ci)
        for (int32_t cj = 0; cj < C - 1; ++cj)
            for (int32_t a = 0; a < k; ++a)
                for (int32_t b = 0; b < k; ++b)
                    cov[((int64_t)ci * k + a) * d + (int64_t)cj * k + b] =
                        (ci == cj ? 2.0 : 1.0) * Sig[a * k + b];
done:
    free(S); free(Ls); free(Sig); free(e); free(v);
    return status;
}

/* ------------------------------------------------------------------------ */
/* C phase (Algorithm 1 step 2(a), eq. (C_phase_compute)) with the adaptive  */
/* stopping rule of Algorithm 2 step 1 (eq. (ESS_rule)).                      */
/* ------------------------------------------------------------------------ */

/* ESS = (sum w)^2 / sum w^2 over all particles, w = exp(log_w); the common
 * factor exp(max log_w) cancels and is divided out first. */
double orc_ess(const double* log_w, int64_t P)
{
    double m = -INFINITY;
    for (int64_t p = 0; p < P; ++p) if (log_w[p] > m) m = log_w[p];
    if (!(m > -INFINITY)) return 0.0;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t p = 0; p < P; ++p) {
        double w = exp(log_w[p] - m);
        s1 += w;
        s2 += w * w;
    }
    return s1 * s1 / s2;
}

/* Starting from w = 1 at s0, multiply in p(y_s | theta) for s = s0+1, ...;
 * stop at the first s with ESS(s) < ess_frac J N (strict, READING) or s = T.
 * On return log_w holds log w(t_end), ll has log_w added (the cached
 * log-likelihood over y_{1:t_end}, READING), *t_end = t_l. */
int orc_correct(const double* X, const int32_t* y, int64_t T, int32_t k, int32_t C,
                const double* theta, double* ll, int32_t J, int32_t N, int64_t s0,
                double ess_frac, double* log_w, int64_t* t_end, double* ess_end)
{
    if (!data_ok(T, k, C, 0, T) || J < 1 || N < 1 || s0 < 0 || s0 >= T ||
        !(ess_frac > 0.0 && ess_frac < 1.0))
        return ORC_ERR_ARG;
    int64_t P = (int64_t)J * N;
    int64_t d = (int64_t)k * (C - 1);
    for (int64_t p = 0; p < P; ++p) log_w[p] = 0.0;
    int64_t s = s0;
    double ess = (double)P;
    for (;;) {
        s += 1;
        const double* x = X + (s - 1) * k;
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < P; ++p) {
            double eta[64];
            log_w[p] += obs_logprob(x, k, C, y[s - 1], theta + p * d, eta);
        }
        for (int64_t p = 0; p < P; ++p)
            if (isnan(log_w[p]) || log_w[p] == INFINITY) return ORC_ERR_NONFINITE;
        ess = orc_ess(log_w, P);
        if (ess < ess_frac * (double)P || s == T) break;
    }
    for (int64_t p = 0; p < P; ++p) ll[p] += log_w[p];
    *t_end = s;
    if (ess_end) *ess_end = ess;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Log marginal likelihood (READING of the estimator the paper defers to     */
/* Durham and Geweke 2012): each group's running product over cycles of its  */
/* mean unnormalised weight, logml_j += log(N^-1 sum_n w_jn).                */
/* ------------------------------------------------------------------------ */
int orc_logml_update(const double* log_w, int32_t J, int32_t N, double* logml_j)
{
    for (int32_t j = 0; j < J; ++j) {
        const double* lw = log_w + (int64_t)j * N;
        double m = -INFINITY;
        for (int32_t n = 0; n < N; ++n) if (lw[n] > m) m = lw[n];
        if (!(m > -INFINITY)) return ORC_ERR_DEGENERATE;
        double s = 0.0;
        for (int32_t n = 0; n < N; ++n) s += exp(lw[n] - m);
        logml_j[j] += m + log(s) - log((double)N);
    }
    return ORC_OK;
}

/* Combine the J group estimates: logml = log(J^-1 sum_j exp(logml_j)); its
 * NSE by the delta method is sd_j(exp(logml_j - logml)) / sqrt(J).  The mean
 * of the group logs and its NSE are returned as a secondary summary. */
void orc_logml_total(const double* logml_j, int32_t J, double* logml, double* nse,
                     double* meanlog, double* meanlog_nse)
{
    double m = -INFINITY;
    for (int32_t j = 0; j < J; ++j) if (logml_j[j] > m) m = logml_j[j];
    double s = 0.0;
    for (int32_t j = 0; j < J; ++j) s += exp(logml_j[j] - m);
    double L = m + log(s / (double)J);
    double v = 0.0, ml = 0.0, vl = 0.0;
    for (int32_t j = 0; j < J; ++j) {
        double r = exp(logml_j[j] - L) - 1.0;
        v += r * r;
        ml += logml_j[j];
    }
    ml /= (double)J;
    for (int32_t j = 0; j < J; ++j) vl += (logml_j[j] - ml) * (logml_j[j] - ml);
    *logml = L;
    *nse = J > 1 ? sqrt(v / (double)(J - 1) / (double)J) : 0.0;
    if (meanlog) *meanlog = ml;
    if (meanlog_nse) *meanlog_nse = J > 1 ? sqrt(vl / (double)(J - 1) / (double)J) : 0.0;
}

/* ------------------------------------------------------------------------ */
/* S phase (Algorithm 1 step 2(b)), independently in each group, on integer  */
/* weights (READING: exact integer arithmetic so that draws are reproducible */
/* bit for bit).                                                             */
/* ------------------------------------------------------------------------ */

/* Inverse CDF on an integer cumulative table: the smallest n with cum[n] >
 * target (cum is inclusive and strictly reaches the total). */
static int32_t first_above(const uint64_t* cum, int32_t N, uint64_t target)
{
    for (int32_t n = 0; n < N; ++n)
        if (cum[n] > target) return n;
    return N - 1; /* unreachable when target < cum[N-1] */
}

/* W: J x N integer weights, each group having a positive total below 2^52
 * and N <= 4096.  u53: J x N integers in [0, 2^53).
 * Multinomial: draw i of group j takes target floor(U_i S / 2^53).
 * Residual: floor(N W_n / S) copies of particle n in increasing n, then the
 * R remaining draws multinomially on N W_n - copies_n S, appended in draw
 * order, using U_0..U_{R-1} of the group. */
int orc_resample_int(const uint64_t* W, int32_t J, int32_t N, int32_t scheme,
                     const uint64_t* u53, int32_t* ancestor)
{
    if (J < 1 || N < 1 || N > 4096 || (scheme != ORC_RESIDUAL && scheme != ORC_MULTINOMIAL))
        return ORC_ERR_ARG;
    uint64_t* cum = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)N);
    if (!cum) return ORC_ERR_NOMEM;
    int status = ORC_OK;
    for (int32_t j = 0; j < J && status == ORC_OK; ++j) {
        const uint64_t* w = W + (int64_t)j * N;
        const uint64_t* U = u53 + (int64_t)j * N;
        int32_t* anc = ancestor + (int64_t)j * N;
        unsigned __int128 S = 0;
        for (int32_t n = 0; n < N; ++n) S += w[n];
        if (S == 0 || S >= ((unsigned __int128)1 << 52)) { status = ORC_ERR_DEGENERATE; break; }
        uint64_t S64 = (uint64_t)S;
        if (scheme == ORC_MULTINOMIAL) {
            uint64_t run = 0;
            for (int32_t n = 0; n < N; ++n) { run += w[n]; cum[n] = run; }
            for (int32_t i = 0; i < N; ++i) {
                uint64_t target = (uint64_t)(((unsigned __int128)U[i] * S64) >> 53);
                anc[i] = j * N + first_above(cum, N, target);
            }
        } else {
            int32_t pos = 0;
            for (int32_t n = 0; n < N; ++n) {
                uint64_t copies = ((uint64_t)N * w[n]) / S64;
                for (uint64_t c = 0; c < copies; ++c) anc[pos++] = j * N + n;
            }
            int32_t R = N - pos;
            if (R > 0) {
                uint64_t run = 0;
                for (int32_t n = 0; n < N; ++n) {
                    uint64_t copies = ((uint64_t)N * w[n]) / S64;
                    run += (uint64_t)N * w[n] - copies * S64;
                    cum[n] = run;
                }
                /* run == R * S < 2^64 */
                for (int32_t i = 0; i < R; ++i) {
                    uint64_t target = (uint64_t)(((unsigned __int128)U[i] * run) >> 53);
                    anc[pos++] = j * N + first_above(cum, N, target);
                }
            }
        }
    }
    free(cum);
    return status;
}

/* Integer weights from log-weights: W_n = floor(exp(log_w_n - max_n log_w) 2^40)
 * (weights below 2^-40 of the group maximum become 0, READING). */
int orc_resample(const double* log_w, int32_t J, int32_t N, int32_t scheme,
                 const uint64_t* u53, int32_t* ancestor, uint64_t* W_out)
{
    if (J < 1 || N < 1 || N > 4096) return ORC_ERR_ARG;
    int64_t P = (int64_t)J * N;
    uint64_t* W = W_out ? W_out : (uint64_t*)malloc(sizeof(uint64_t) * (size_t)P);
    if (!W) return ORC_ERR_NOMEM;
    int status = ORC_OK;
    for (int32_t j = 0; j < J; ++j) {
        const double* lw = log_w + (int64_t)j * N;
        double m = -INFINITY;
        for (int32_t n = 0; n < N; ++n) {
            if (isnan(lw[n]) || lw[n] == INFINITY) status = ORC_ERR_NONFINITE;
            if (lw[n] > m) m = lw[n];
        }
        if (status == ORC_OK && !(m > -INFINITY)) status = ORC_ERR_DEGENERATE;
        if (status != ORC_OK) break;
        for (int32_t n = 0; n < N; ++n)
            W[(int64_t)j * N + n] = (uint64_t)floor(exp(lw[n] - m) * 0x1p40);
    }
    if (status == ORC_OK) status = orc_resample_int(W, J, N, scheme, u53, ancestor);
    if (!W_out) free(W);
    return status;
}

void orc_gather(const int32_t* ancestor, int64_t P, int32_t m, const double* src, double* dst)
{
    for (int64_t p = 0; p < P; ++p)
        for (int32_t i = 0; i < m; ++i)
            dst[p * m + i] = src[(int64_t)ancestor[p] * m + i];
}

/* ------------------------------------------------------------------------ */
/* M phase (Algorithm 2 step 2(c)).                                           */
/* ------------------------------------------------------------------------ */

/* Sample mean and sample variance of all J N particles pooled, divisor
 * P - 1 (READING). */
void orc_cov(const double* theta, int64_t P, int32_t d, double* mean, double* V)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < d; ++i) {
        double s = 0.0;
        for (int64_t p = 0; p < P; ++p) s += theta[p * d + i];
        mean[i] = s / (double)P;
    }
#pragma omp parallel for schedule(dynamic)
    for (int32_t a = 0; a < d; ++a)
        for (int32_t b = 0; b < d; ++b) {
            double s = 0.0;
            for (int64_t p = 0; p < P; ++p)
                s += (theta[p * d + a] - mean[a]) * (theta[p * d + b] - mean[b]);
            V[a * d + b] = s / (double)(P - 1);
        }
}

/* Lower-triangular L with L L' = V; fails (the failure of Algorithm 2
 * step 2(c)i discussed in Section 4.2) when V is not positive definite. */
int orc_cholesky(const double* V, int32_t d, double* L)
{
    for (int64_t i = 0; i < (int64_t)d * d; ++i) L[i] = 0.0;
    for (int32_t j = 0; j < d; ++j) {
        double s = V[j * d + j];
        for (int32_t q = 0; q < j; ++q) s -= L[j * d + q] * L[j * d + q];
        if (!(s > 0.0) || !isfinite(s)) return ORC_ERR_NOT_PD;
        double Ljj = sqrt(s);
        L[j * d + j] = Ljj;
        for (int32_t i = j + 1; i < d; ++i) {
            double t = V[i * d + j];
            for (int32_t q = 0; q < j; ++q) t -= L[i * d + q] * L[j * d + q];
            L[i * d + j] = t / Ljj;
        }
    }
    return ORC_OK;
}

/* Solve L v = r (forward substitution). */
static void lower_solve(const double* L, int32_t d, const double* r, double* v)
{
    for (int32_t i = 0; i < d; ++i) {
        double s = r[i];
        for (int32_t q = 0; q < i; ++q) s -= L[i * d + q] * v[q];
        v[i] = s / L[i * d + i];
    }
}

/* MALA mean (extension beyond the paper): theta + (1/2) Sigma grad log pi,
 * Sigma the proposal covariance. */
static void mala_mean(const double* th, const double* glp, const double* Sigma, int32_t d,
                      double* mu)
{
    for (int32_t a = 0; a < d; ++a) {
        double s = 0.0;
        for (int32_t b = 0; b < d; ++b) s += Sigma[a * d + b] * glp[b];
        mu[a] = th[a] + 0.5 * s;
    }
}

/* One Metropolis step for every particle with proposal covariance Sigma
 * (Algorithm 1 step 2(c) with lambda = Sigma, as replayed by Algorithm 3).
 * RW (the paper): theta' = theta + L z, L L' = Sigma.
 * MALA: theta' = mu(theta) + L z, with the Hastings correction
 * log q(theta|theta') - log q(theta'|theta), log q(a|b) = -|L^-1 (a - mu(b))|^2 / 2.
 * Accept iff log u < log alpha (strict).  ll (and for MALA grad, the gradient
 * of the log-likelihood over the same observations) are cached per particle
 * and updated on acceptance.  Observations 1..t are used. */
int orc_mutate_cov(const double* X, const int32_t* y, int64_t T, int32_t k, int32_t C,
                   const double* prior_mean, const double* prior_L,
                   double* theta, double* ll, double* grad, int32_t J, int32_t N,
                   int64_t t, const double* Sigma, int32_t kind, const double* z, const double* u,
                   double* accept_rate, double* log_alpha_out, int8_t* accepted_out)
{
    if (!data_ok(T, k, C, 0, t) || J < 1 || N < 1 ||
        (kind != ORC_RW && kind != ORC_MALA) || (kind == ORC_MALA && !grad))
        return ORC_ERR_ARG;
    int64_t P = (int64_t)J * N;
    int32_t d = k * (C - 1);
    double* L = (double*)malloc(sizeof(double) * (size_t)d * d);
    double* prop = (double*)malloc(sizeof(double) * (size_t)P * d);
    double* llp = (double*)malloc(sizeof(double) * (size_t)P);
    double* gp = (double*)malloc(sizeof(double) * (size_t)P * d);
    double* lp0 = (double*)malloc(sizeof(double) * (size_t)P);
    double* lp1 = (double*)malloc(sizeof(double) * (size_t)P);
    double* glp0 = (double*)malloc(sizeof(double) * (size_t)P * d);
    double* glp1 = (double*)malloc(sizeof(double) * (size_t)P * d);
    int status = ORC_OK;
    if (!L || !prop || !llp || !gp || !lp0 || !lp1 || !glp0 || !glp1) {
        status = ORC_ERR_NOMEM;
        goto done;
    }
    status = orc_cholesky(Sigma, d, L);
    if (status != ORC_OK) goto done;
    orc_logprior(theta, P, d, prior_mean, prior_L, lp0, glp0);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
        const double* th = theta + p * d;
        double* q = prop + p * d;
        if (kind == ORC_MALA) {
            double* g = (double*)malloc(sizeof(double) * d);
            for (int32_t i = 0; i < d; ++i) g[i] = grad[p * d + i] + glp0[p * d + i];
            mala_mean(th, g, Sigma, d, q);
            free(g);
        } else {
            for (int32_t i = 0; i < d; ++i) q[i] = th[i];
        }
        for (int32_t a = 0; a < d; ++a) {
            double s = 0.0;
            for (int32_t b = 0; b <= a; ++b) s += L[a * d + b] * z[p * d + b];
            q[a] += s;
        }
    }
    if (kind == ORC_MALA)
        status = orc_loglik_grad(X, y, T, k, C, prop, P, 0, t, llp, gp);
    else
        status = orc_loglik(X, y, T, k, C, prop, P, 0, t, llp);
    if (status != ORC_OK) goto done;
    orc_logprior(prop, P, d, prior_mean, prior_L, lp1, glp1);
    int64_t acc = 0;
#pragma omp parallel for schedule(static) reduction(+ : acc)
    for (int64_t p = 0; p < P; ++p) {
        double la = (llp[p] + lp1[p]) - (ll[p] + lp0[p]);
        if (kind == ORC_MALA) {
            double* g = (double*)malloc(sizeof(double) * d);
            double* mu = (double*)malloc(sizeof(double) * d);
            double* r = (double*)malloc(sizeof(double) * d);
            double* v = (double*)malloc(sizeof(double) * d);
            /* log q(theta | theta') */
            for (int32_t i = 0; i < d; ++i) g[i] = gp[p * d + i] + glp1[p * d + i];
            mala_mean(prop + p * d, g, Sigma, d, mu);
            for (int32_t i = 0; i < d; ++i) r[i] = theta[p * d + i] - mu[i];
            lower_solve(L, d, r, v);
            double qb = 0.0;
            for (int32_t i = 0; i < d; ++i) qb += v[i] * v[i];
            /* log q(theta' | theta) */
            for (int32_t i = 0; i < d; ++i) g[i] = grad[p * d + i] + glp0[p * d + i];
            mala_mean(theta + p * d, g, Sigma, d, mu);
            for (int32_t i = 0; i < d; ++i) r[i] = prop[p * d + i] - mu[i];
            lower_solve(L, d, r, v);
            double qf = 0.0;
            for (int32_t i = 0; i < d; ++i) qf += v[i] * v[i];
            la += -0.5 * qb + 0.5 * qf;
            free(g); free(mu); free(r); free(v);
        }
        if (isnan(la)) la = -INFINITY;
        int take = log(u[p]) < la;
        if (log_alpha_out) log_alpha_out[p] = la;
        if (accepted_out) accepted_out[p] = (int8_t)take;
        if (take) {
            ++acc;
            for (int32_t i = 0; i < d; ++i) theta[p * d + i] = prop[p * d + i];
            ll[p] = llp[p];
            if (kind == ORC_MALA)
                for (int32_t i = 0; i < d; ++i) grad[p * d + i] = gp[p * d + i];
        }
    }
    *accept_rate = (double)acc / (double)P;
done:
    free(L); free(prop); free(llp); free(gp);
    free(lp0); free(lp1); free(glp0); free(glp1);
    return status;
}

/* Algorithm 2 step 2(c)i-ii: proposal covariance Sigma = h V with V the
 * sample variance of all particles, then one Metropolis step.  The Sigma
 * used is returned in sigma_out (d x d, may be NULL). */
int orc_mutate(const double* X, const int32_t* y, int64_t T, int32_t k, int32_t C,
               const double* prior_mean, const double* prior_L,
               double* theta, double* ll, double* grad, int32_t J, int32_t N,
               int64_t t, double h, int32_t kind, const double* z, const double* u,
               double* accept_rate, double* log_alpha_out, int8_t* accepted_out,
               double* sigma_out)
{
    if (J < 1 || N < 1 || !(h > 0.0) || (int64_t)J * N < 2 || k < 1 || C < 2) return ORC_ERR_ARG;
    int64_t P = (int64_t)J * N;
    int32_t d = k * (C - 1);
    double* mean = (double*)malloc(sizeof(double) * d);
    double* V = (double*)malloc(sizeof(double) * (size_t)d * d);
    int status = ORC_ERR_NOMEM;
    if (mean && V) {
        orc_cov(theta, P, d, mean, V);
        for (int64_t i = 0; i < (int64_t)d * d; ++i) V[i] *= h;
        if (sigma_out) memcpy(sigma_out, V, sizeof(double) * (size_t)d * d);
        status = orc_mutate_cov(X, y, T, k, C, prior_mean, prior_L, theta, ll, grad, J, N, t, V,
                                kind, z, u, accept_rate, log_alpha_out, accepted_out);
    }
    free(mean);
    free(V);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Numerical accuracy from the group structure, eqs. (partial_g), (whole_g), */
/* (v-hat), (NSE_def), (RNE_def).  g: P x m function values.                 */
/* READING: NSE = sqrt(v_hat / (J N)), the standard error of the grand mean  */
/* implied by the central limit theorem (basic_CLT).                         */
/* ------------------------------------------------------------------------ */
void orc_moments(const double* g, int32_t J, int32_t N, int32_t m,
                 double* mean, double* sd, double* nse, double* rne)
{
    int64_t P = (int64_t)J * N;
#pragma omp parallel
    {
    double* gm = (double*)malloc(sizeof(double) * (size_t)J);
#pragma omp for schedule(dynamic)
    for (int32_t f = 0; f < m; ++f) {
        for (int32_t j = 0; j < J; ++j) {
            double s = 0.0;
            for (int32_t n = 0; n < N; ++n) s += g[((int64_t)j * N + n) * m + f];
            gm[j] = s / (double)N;
        }
        double gbar = 0.0;
        for (int32_t j = 0; j < J; ++j) gbar += gm[j];
        gbar /= (double)J;
        double vb = 0.0;
        for (int32_t j = 0; j < J; ++j) vb += (gm[j] - gbar) * (gm[j] - gbar);
        double vhat = J > 1 ? (double)N / (double)(J - 1) * vb : 0.0;
        double var = 0.0;
        for (int64_t p = 0; p < P; ++p) var += (g[p * m + f] - gbar) * (g[p * m + f] - gbar);
        var /= (double)P;
        mean[f] = gbar;
        if (sd) sd[f] = sqrt(var);
        if (nse) nse[f] = sqrt(vhat / (double)P);
        if (rne) rne[f] = vhat > 0.0 ? var / vhat : INFINITY;
    }
    free(gm);
    }
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2, the adaptive SPS.                                             */
/* Random streams: stream = (cycle << 32) | (step << 4) | phase, phase 1 =   */
/* initial particles, 2 = resampling integers, 3 = proposal normals,          */
/* 4 = acceptance uniforms.                                                   */
/* Monitored functions (READING): each free parameter and the log-odds       */
/* theta_c' xbar at the sample mean of the covariates (as in Tables 2 and 5); */
/* the stopping test uses their mean RNE (rne_rule 0) or minimum (1).         */
/* ------------------------------------------------------------------------ */
static uint64_t stream_id(int pass, int64_t cycle, int64_t step, int phase)
{
    return ((uint64_t)pass << 60) | ((uint64_t)cycle << 32) | ((uint64_t)step << 4) | (uint64_t)phase;
}

static void monitored(const double* theta, int64_t P, int32_t k, int32_t C,
                      const double* xbar, double* g)
{
    int32_t d = k * (C - 1), m = d + C - 1;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
        for (int32_t i = 0; i < d; ++i) g[p * m + i] = theta[p * d + i];
        for (int32_t c = 1; c < C; ++c) {
            double s = 0.0;
            for (int32_t i = 0; i < k; ++i) s += theta[p * d + (c - 1) * k + i] * xbar[i];
            g[p * m + d + c - 1] = s;
        }
    }
}

int orc_sps_run(const double* X, const int32_t* y, int64_t T, int32_t k, int32_t C,
                const double* prior_mean, const double* prior_L, const orc_config* cfg,
                double* theta_out, double* ll_out,
                double* mom_mean, double* mom_sd, double* mom_nse, double* mom_rne,
                int64_t* rec_t, int32_t* rec_R, double* rec_h, double* rec_acc,
                double* rec_sigma, int64_t sigma_cap, orc_summary* summary)
{
    int32_t J = cfg->J, N = cfg->N;
    int64_t P = (int64_t)J * N;
    int32_t d = k * (C - 1), m = d + C - 1;
    if (T < 1 || J < 2 || N < 1 || C < 2) return ORC_ERR_ARG;
    memset(summary, 0, sizeof(*summary));
    double* theta = theta_out;
    double* ll = ll_out;
    double* th2 = (double*)malloc(sizeof(double) * (size_t)P * d);
    double* grad = (double*)calloc((size_t)P * d, sizeof(double));
    double* grad2 = (double*)calloc((size_t)P * d, sizeof(double));
    double* ll2 = (double*)malloc(sizeof(double) * (size_t)P);
    double* lw = (double*)malloc(sizeof(double) * (size_t)P);
    double* z = (double*)malloc(sizeof(double) * (size_t)P * d);
    double* u = (double*)malloc(sizeof(double) * (size_t)P);
    uint64_t* u53 = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)P);
    int32_t* anc = (int32_t*)malloc(sizeof(int32_t) * (size_t)P);
    double* g = (double*)malloc(sizeof(double) * (size_t)P * m);
    double* rne = (double*)malloc(sizeof(double) * (size_t)m);
    double* logml_j = (double*)calloc((size_t)J, sizeof(double));
    double* xbar = (double*)calloc((size_t)k, sizeof(double));
    int status = ORC_OK;
    if (!th2 || !grad || !grad2 || !ll2 || !lw || !z || !u || !u53 || !anc || !g || !rne ||
        !logml_j || !xbar) {
        status = ORC_ERR_NOMEM;
        goto out;
    }
    for (int64_t t = 0; t < T; ++t)
        for (int32_t i = 0; i < k; ++i) xbar[i] += X[t * k + i];
    for (int32_t i = 0; i < k; ++i) xbar[i] /= (double)T;

    orc_init_prior(prior_mean, prior_L, d, P, cfg->seed, stream_id(0, 0, 0, 1), theta);
    for (int64_t p = 0; p < P; ++p) ll[p] = 0.0;
    double h = cfg->h_init;
    int64_t t = 0;
    int32_t cycle = 0;
    while (t < T) {
        ++cycle;
        int64_t t_end = 0;
        double ess = 0.0;
        status = orc_correct(X, y, T, k, C, theta, ll, J, N, t, cfg->ess_frac, lw, &t_end, &ess);
        if (status != ORC_OK) goto out;
        t = t_end;
        status = orc_logml_update(lw, J, N, logml_j);
        if (status != ORC_OK) goto out;
        orc_u53(cfg->seed, stream_id(0, cycle, 0, 2), P, u53);
        status = orc_resample(lw, J, N, cfg->scheme, u53, anc, NULL);
        if (status != ORC_OK) goto out;
        orc_gather(anc, P, d, theta, th2);
        memcpy(theta, th2, sizeof(double) * (size_t)P * d);
        orc_gather(anc, P, 1, ll, ll2);
        memcpy(ll, ll2, sizeof(double) * (size_t)P);
        if (cfg->kind == ORC_MALA) {
            status = orc_loglik_grad(X, y, T, k, C, theta, P, 0, t, ll, grad);
            if (status != ORC_OK) goto out;
        }
        double K = (t < T) ? cfg->K_mid : cfg->K_final;
        int32_t r = 0;
        double rate = 0.0;
        for (;;) {
            ++r;
            orc_normals(cfg->seed, stream_id(0, cycle, r, 3), P, d, z);
            orc_uniforms(cfg->seed, stream_id(0, cycle, r, 4), P, u);
            double* sig = NULL;
            if (rec_sigma && summary->m_iters + r <= sigma_cap)
                sig = rec_sigma + (size_t)(summary->m_iters + r - 1) * d * d;
            status = orc_mutate(X, y, T, k, C, prior_mean, prior_L, theta, ll,
                                cfg->kind == ORC_MALA ? grad : NULL, J, N, t, h, cfg->kind,
                                z, u, &rate, NULL, NULL, sig);
            if (status != ORC_OK) goto out;
            h = rate > cfg->acc_target ? fmin(h + cfg->h_step, cfg->h_max)
                                       : fmax(h - cfg->h_step, cfg->h_min);
            monitored(theta, P, k, C, xbar, g);
            orc_moments(g, J, N, m, mom_mean, mom_sd, mom_nse, rne);
            double agg = cfg->rne_rule == 1 ? INFINITY : 0.0;
            for (int32_t f = 0; f < m; ++f)
                agg = cfg->rne_rule == 1 ? fmin(agg, rne[f]) : agg + rne[f] / (double)m;
            if (agg >= K) break;
            if (r >= cfg->R_max) { summary->hit_R_max += 1; break; }
        }
        summary->m_iters += r;
        if (cycle <= cfg->max_cycles) {
            rec_t[cycle - 1] = t;
            rec_R[cycle - 1] = r;
            rec_h[cycle - 1] = h;
            rec_acc[cycle - 1] = rate;
        }
    }
    summary->cycles = cycle;
    monitored(theta, P, k, C, xbar, g);
    orc_moments(g, J, N, m, mom_mean, mom_sd, mom_nse, mom_rne);
    orc_logml_total(logml_j, J, &summary->logml, &summary->logml_nse, &summary->meanlog,
                    &summary->meanlog_nse);
out:
    summary->status = status;
    free(th2); free(grad); free(grad2); free(ll2); free(lw); free(z); free(u); free(u53);
    free(anc); free(g); free(rne); free(logml_j); free(xbar);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 with a fixed design, as run by the second pass of Algorithm 3: */
/* cycle ends t_1..t_L, R_l M steps per cycle and proposal covariances       */
/* Sigma_lr (sum_l R_l matrices, d x d each) recorded by a first adaptive   */
/* pass.  Random streams carry pass = 1.                                     */
/* ------------------------------------------------------------------------ */
int orc_sps_run_fixed(const double* X, const int32_t* y, int64_t T, int32_t k, int32_t C,
                      const double* prior_mean, const double* prior_L, const orc_config* cfg,
                      int32_t L, const int64_t* t_l, const int32_t* R_l, const double* Sigma,
                      double* theta_out, double* ll_out,
                      double* mom_mean, double* mom_sd, double* mom_nse, double* mom_rne,
                      orc_summary* summary)
{
    int32_t J = cfg->J, N = cfg->N;
    int64_t P = (int64_t)J * N;
    int32_t d = k * (C - 1), m = d + C - 1;
    if (T < 1 || J < 2 || N < 1 || C < 2 || L < 1 || t_l[L - 1] != T) return ORC_ERR_ARG;
    for (int32_t l = 0; l < L; ++l)
        if (R_l[l] < 1 || t_l[l] <= (l ? t_l[l - 1] : 0)) return ORC_ERR_ARG;
    memset(summary, 0, sizeof(*summary));
    double* theta = theta_out;
    double* ll = ll_out;
    double* th2 = (double*)malloc(sizeof(double) * (size_t)P * d);
    double* grad = (double*)calloc((size_t)P * d, sizeof(double));
    double* ll2 = (double*)malloc(sizeof(double) * (size_t)P);
    double* lw = (double*)malloc(sizeof(double) * (size_t)P);
    double* z = (double*)malloc(sizeof(double) * (size_t)P * d);
    double* u = (double*)malloc(sizeof(double) * (size_t)P);
    uint64_t* u53 = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)P);
    int32_t* anc = (int32_t*)malloc(sizeof(int32_t) * (size_t)P);
    double* g = (double*)malloc(sizeof(double) * (size_t)P * m);
    double* logml_j = (double*)calloc((size_t)J, sizeof(double));
    double* xbar = (double*)calloc((size_t)k, sizeof(double));
    int status = ORC_OK;
    if (!th2 || !grad || !ll2 || !lw || !z || !u || !u53 || !anc || !g || !logml_j || !xbar) {
        status = ORC_ERR_NOMEM;
        goto out;
    }
    for (int64_t t = 0; t < T; ++t)
        for (int32_t i = 0; i < k; ++i) xbar[i] += X[t * k + i];
    for (int32_t i = 0; i < k; ++i) xbar[i] /= (double)T;

    orc_init_prior(prior_mean, prior_L, d, P, cfg->seed, stream_id(1, 0, 0, 1), theta);
    for (int64_t p = 0; p < P; ++p) ll[p] = 0.0;
    int64_t step = 0;
    for (int32_t l = 0; l < L; ++l) {
        int32_t cycle = l + 1;
        int64_t t0 = l ? t_l[l - 1] : 0, t1 = t_l[l];
        /* C phase over observations t0+1..t1 (fixed cycle end) */
        status = orc_loglik(X, y, T, k, C, theta, P, t0, t1, lw);
        if (status != ORC_OK) goto out;
        for (int64_t p = 0; p < P; ++p) ll[p] += lw[p];
        status = orc_logml_update(lw, J, N, logml_j);
        if (status != ORC_OK) goto out;
        orc_u53(cfg->seed, stream_id(1, cycle, 0, 2), P, u53);
        status = orc_resample(lw, J, N, cfg->scheme, u53, anc, NULL);
        if (status != ORC_OK) goto out;
        orc_gather(anc, P, d, theta, th2);
        memcpy(theta, th2, sizeof(double) * (size_t)P * d);
        orc_gather(anc, P, 1, ll, ll2);
        memcpy(ll, ll2, sizeof(double) * (size_t)P);
        if (cfg->kind == ORC_MALA) {
            status = orc_loglik_grad(X, y, T, k, C, theta, P, 0, t1, ll, grad);
            if (status != ORC_OK) goto out;
        }
        for (int32_t r = 1; r <= R_l[l]; ++r, ++step) {
            double rate = 0.0;
            orc_normals(cfg->seed, stream_id(1, cycle, r, 3), P, d, z);
            orc_uniforms(cfg->seed, stream_id(1, cycle, r, 4), P, u);
            status = orc_mutate_cov(X, y, T, k, C, prior_mean, prior_L, theta, ll,
                                    cfg->kind == ORC_MALA ? grad : NULL, J, N, t1,
                                    Sigma + (size_t)step * d * d, cfg->kind, z, u, &rate, NULL, NULL);
            if (status != ORC_OK) goto out;
        }
        summary->m_iters += R_l[l];
    }
    summary->cycles = L;
    monitored(theta, P, k, C, xbar, g);
    orc_moments(g, J, N, m, mom_mean, mom_sd, mom_nse, mom_rne);
    orc_logml_total(logml_j, J, &summary->logml, &summary->logml_nse, &summary->meanlog,
                    &summary->meanlog_nse);
out:
    summary->status = status;
    free(th2); free(grad); free(ll2); free(lw); free(z); free(u); free(u53); free(anc); free(g);
    free(logml_j); free(xbar);
    return status;
}

/* Threads of the OpenMP loops over particles: n > 0 sets the count; the
 * count in use is returned.  (Used to time the oracle on one core and on
 * all cores; no arithmetic of the method depends on it.) */
int orc_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}
