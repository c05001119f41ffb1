/*
 * sps.h -- C ABI of libsps, the MI355X (gfx950) hot path of the sequential
 * posterior simulator (SPS) for multinomial logit models of Geweke, Durham &
 * Xu, "Bayesian Inference for Logistic Regression Models using Sequential
 * Posterior Simulation" (2013).
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Status: 0 (SPS_OK) on success, a negative SPS_ERR_* code on failure, with
 *    a message available from sps_last_error().  No exception or abort crosses
 *    the ABI.  Arguments are validated before anything is launched; on an
 *    argument error no output is touched.
 *  - Memory: pointers documented "device" are HIP device memory owned by the
 *    caller (contiguous, row-major, of the stated type); pointers documented
 *    "host" are host memory.  The library keeps no pointer to caller memory
 *    after a call returns, except the data and prior it copies.
 *  - Asynchrony: work is enqueued on the context's stream.  A call returns
 *    before the GPU finishes unless it has a host output.  A call with host
 *    outputs ("waits" below) returns once the stream has run everything up
 *    to those outputs; it reads them from pinned host memory that a small
 *    kernel fills, without a stream synchronisation, so launches queued
 *    after that point (device outputs, empty look-ahead launches) may still
 *    be in flight.  Device outputs are complete in stream order, as for any
 *    launch; reading them from another stream needs an event.
 *  - Model layout: X is T x k covariates (FP64), y holds T outcomes in
 *    [0, C), outcome 0 is the base outcome whose coefficients are fixed at 0
 *    (the normalisation theta_c = 0 of Section 2.1).  A particle is the
 *    vector of d = k (C - 1) free coefficients; entry (c - 1) k + i is the
 *    coefficient of covariate i for outcome c.  theta is P x d FP64.
 *  - Particles form J groups of N (Section 2.2): particle p = j N + n.
 *  - Observation s (1-based, as the paper counts) is row s - 1 of X.  An
 *    observation range [t0, t1) means rows t0..t1-1.
 *  - Random numbers: every entry point that draws takes explicit variates
 *    (z, u, u53) or, when they are NULL, draws them from Philox4x32-10 with
 *    key = seed and counter = (element index, stream).
 *  - One context per host thread; a context holds no global state, and two
 *    contexts may be used concurrently on different streams.
 */
#ifndef SPS_H
#define SPS_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SPS_OK = 0,
    SPS_ERR_ARG = -1,        /* invalid argument or unsupported shape          */
    SPS_ERR_HIP = -2,        /* a HIP runtime call failed                       */
    SPS_ERR_NOT_PD = -3,     /* particle sample variance not positive definite */
    SPS_ERR_NONFINITE = -4,  /* NaN or +inf in a log-likelihood or log-weight   */
    SPS_ERR_DEGENERATE = -5, /* every weight of a group is zero                */
    SPS_ERR_NOMEM = -6,      /* device allocation failed                        */
    SPS_ERR_STATE = -7       /* data or prior not set                           */
};

/* Arithmetic of the likelihood kernels. */
enum {
    SPS_FP64 = 0,   /* FP64 MFMA contraction, FP64 log-sum-exp and sums           */
    SPS_FP32 = 1,   /* FP32 MFMA contraction, FP32 log-sum-exp, FP64 running sums */
    SPS_BF16X3 = 2  /* BF16 hi/lo split of both operands, three BF16 MFMAs with
                       FP32 accumulation; FP32 log-sum-exp; FP64 running sums  */
};
enum { SPS_RESIDUAL = 0, SPS_MULTINOMIAL = 1 }; /* S phase schemes            */
enum { SPS_RW = 0, SPS_MALA = 1 };              /* M phase proposals          */

typedef struct sps_ctx sps_ctx;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the context. */
int sps_create(sps_ctx** out, int device, void* hip_stream);

/* Release the context and every device buffer it owns.  NULL is a no-op. */
void sps_destroy(sps_ctx* ctx);

/* Message of the last failing call on ctx ("" if none).  The string is owned
 * by ctx and valid until the next call on it. */
const char* sps_last_error(const sps_ctx* ctx);

/* Replace the stream that subsequent calls enqueue on. */
int sps_set_stream(sps_ctx* ctx, void* hip_stream);

/* Copy the data set into the context and build the kernel copies of X:
 * FP64, FP32 and a BF16 hi/lo pair (hi = bf16(x), lo = bf16(x - hi)), row
 * major and transposed, zero padded.  For C = 2 each row is multiplied by
 * 1 - 2 y_t, so that log P(Y_t = y_t) = -softplus(x~_t' theta) needs no y.
 * X: device, T x k FP64; y: device, T int32 in [0, C).  Requires
 * 1 <= T < 2^31, 1 <= k <= 128, 2 <= C <= 8.  Checks the data on the
 * device: SPS_ERR_ARG if any y is outside [0, C), SPS_ERR_NONFINITE if X
 * holds NaN or inf.  Synchronises the stream. */
int sps_set_data(sps_ctx* ctx, const double* X, const int32_t* y, int64_t T,
                 int32_t k, int32_t C);

/* Prior of the free parameters: independent N(mean_i, sd_i^2), i < d, the
 * diagonal case of eq. (prior_Gauss).  mean, sd: host, d FP64 each, sd > 0.
 * Requires sps_set_data first (d is taken from it). */
int sps_set_prior(sps_ctx* ctx, const double* mean, const double* sd);

/* Prior of the free parameters: N(mean, cov) with a full covariance, e.g.
 * the normalised prior of eq. (prior_norm).  mean: host, d FP64 (NULL:
 * zero); cov: host, d x d FP64 row-major, symmetric (to 1e-12 relative)
 * and positive definite.  The library keeps its own copy (Cholesky factor
 * and inverse on the device).  SPS_ERR_NOT_PD if cov is not positive
 * definite, SPS_ERR_ARG if not symmetric or not finite.  Requires
 * sps_set_data first.  Synchronises the stream. */
int sps_set_prior_cov(sps_ctx* ctx, const double* mean, const double* cov);

/* The normalised g-prior: theta_c ~ iid N(0, Sigma) for all C outcomes
 * before normalisation on outcome 0, Sigma = g T (X'X)^-1 (eq.
 * (g-prior_def)); the free vectors theta_c - theta_0 then have variance
 * 2 Sigma and pairwise covariance Sigma (eq. (prior_norm)).  X'X is formed
 * on the device in FP64 from the data of sps_set_data.  g > 0; mean: host,
 * d FP64 or NULL (zero).  SPS_ERR_NOT_PD if X'X is singular.
 * Synchronises the stream. */
int sps_set_prior_g(sps_ctx* ctx, double g, const double* mean);

/* Copy the d x d prior covariance in use (diagonal after sps_set_prior)
 * into cov (host, row-major). */
int sps_get_prior_cov(sps_ctx* ctx, double* cov);

/* ------------------------------------------------------- random numbers */

/* Philox4x32-10 variates of a stream (the same definitions as used inside
 * the phases).  out: device.  kind 0: `count` 53-bit integers (uint64),
 * kind 1: `count` uniforms (U + 1/2) 2^-53 (FP64), kind 2: a count x d array
 * of standard normals by Box-Muller (FP64). */
int sps_random(sps_ctx* ctx, int kind, uint64_t seed, uint64_t stream,
               int64_t count, int32_t d, void* out);

/* Algorithm 1 step 1: theta (device, P x d) <- iid draws from the prior. */
int sps_init_prior(sps_ctx* ctx, double* theta, int64_t P, uint64_t seed,
                   uint64_t stream);

/* -------------------------------------------------------- likelihood */

/* ll[p] = sum over observations t0 <= t < t1 of log P(Y_t = y_t | x_t,
 * theta_p), eq. (plogit) summed over the product form of the likelihood
 * (Section 2.1).  theta: device P x d FP64; ll: device P FP64.
 * prec: SPS_FP64, SPS_FP32 or SPS_BF16X3.  0 <= t0 <= t1 <= T.  Results are
 * deterministic (fixed-order reductions, no float atomics). */
int sps_loglik(sps_ctx* ctx, const double* theta, int64_t P, int64_t t0,
               int64_t t1, int prec, double* ll);

/* As sps_loglik, plus grad (device, P x d FP64): the gradient of ll[p] with
 * respect to theta_p, sum_t x_t (1{y_t = c} - pi_{t,c}) for outcome c
 * (the adjoint of the likelihood; an extension beyond the paper). */
int sps_loglik_grad(sps_ctx* ctx, const double* theta, int64_t P, int64_t t0,
                    int64_t t1, int prec, double* ll, double* grad);

/* As sps_loglik, for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): no
 * hipMalloc, hipFree or other allocation happens in this call.
 * - Its scratch (observation-split partial sums, multinomial sufficient
 *   statistics) is one fixed device array per GPU: 2^21 + 1024 doubles
 *   (16 MiB), held from the first sps_create on that GPU until the process
 *   ends.
 * - The observation split is limited so that its partials fit.
 * - Nothing in the scratch needs to start at zero: every call writes what it
 *   reads, and the array keeps the last call's contents.
 * - Calls that overlap on one GPU (other streams or contexts) race on the
 *   scratch: serialise them.
 * - Not timed by sps_timing_enable.
 * - Errors: those of sps_loglik, and SPS_ERR_ARG when d exceeds the 1024
 *   doubles kept for the sufficient statistics. */
int sps_loglik_noalloc(sps_ctx* ctx, const double* theta, int64_t P, int64_t t0,
                       int64_t t1, int prec, double* ll);

/* ------------------------------------------------------------ phases */

/* C phase of cycle l (Algorithm 1 step 2(a), eq. (C_phase_compute)) with the
 * adaptive stopping rule of Algorithm 2 step 1 (eq. (ESS_rule)): starting at
 * w = 1 after observation s0, multiply in p(y_s | theta) for s = s0+1, ...
 * and stop at the first s with ESS(s) < ess_frac J N (ESS pooled over all
 * J N particles) or s = T.  Outputs: log_w (device, P FP64) = log w(t_end);
 * ll (device, P FP64, in/out) += log_w; *t_end, *ess_end (host) = t_l and
 * ESS(t_l).  0 <= s0 < T, 0 < ess_frac < 1.  Waits (for t_end and ESS). */
int sps_correct(sps_ctx* ctx, const double* theta, double* ll, int32_t J,
                int32_t N, int64_t s0, double ess_frac, int prec,
                double* log_w, int64_t* t_end, double* ess_end);

/* Log marginal likelihood by-product (Section 3): each group keeps the
 * running product over cycles of its mean unnormalised C-phase weight,
 * logml_j (device, J FP64, in/out) += log(N^-1 sum_n exp(log_w[j N + n])).
 * The combined estimate log(J^-1 sum_j exp(logml_j)) and its delta-method
 * NSE, sd_j(exp(logml_j - logml)) / sqrt(J), are returned in *logml, *nse
 * (host, each may be NULL).  Waits.  SPS_ERR_DEGENERATE if a group has
 * every log_w = -inf, SPS_ERR_NONFINITE on NaN or +inf; such a group's
 * logml_j is left unchanged (the other groups' are updated). */
int sps_logml(sps_ctx* ctx, const double* log_w, int32_t J, int32_t N,
              double* logml_j, double* logml, double* nse);

/* S phase (Algorithm 1 step 2(b)), independently in each group, on exact
 * integer weights W_n = floor(exp(log_w_n - max_n log_w) 2^40).
 * scheme: SPS_RESIDUAL (copies floor(N W_n / S), then the remainder drawn
 * multinomially on the residual weights, appended in draw order) or
 * SPS_MULTINOMIAL.  u53: device J x N uint64 in [0, 2^53) or NULL (Philox
 * from seed, stream).  ancestor: device P int32, global index j N + a.
 * The gathers dst[p] = src[ancestor[p]] are done for each non-NULL pair
 * (theta P x d, ll P, grad P x d); a destination must not alias its source.
 * N <= 4096.  Waits (for the error flags).  SPS_ERR_NONFINITE on a NaN or
 * +inf log_w, SPS_ERR_DEGENERATE if a group has every log_w = -inf: such a
 * group's ancestors are its own indices, and no gather is done. */
int sps_resample(sps_ctx* ctx, const double* log_w, int32_t J, int32_t N,
                 int scheme, const uint64_t* u53, uint64_t seed, uint64_t stream,
                 int32_t* ancestor, const double* theta_in, double* theta_out,
                 const double* ll_in, double* ll_out, const double* grad_in,
                 double* grad_out);

/* The S phase on given integer weights W (device, J x N uint64, each group's
 * total in (0, 2^52)); the bit-exactness entry point of sps_resample. */
int sps_resample_fixed(sps_ctx* ctx, const uint64_t* W, int32_t J, int32_t N,
                       int scheme, const uint64_t* u53, int32_t* ancestor);

/* M phase, one Metropolis step for every particle (Algorithm 2 step 2(c)):
 * V = sample variance of all J N particles (divisor P - 1), L = chol(V),
 * proposal covariance h V.
 *   kind SPS_RW  : theta' = theta + sqrt(h) L z                     (paper)
 *   kind SPS_MALA: theta' = theta + (h/2) V grad log pi(theta) + sqrt(h) L z
 *                  with the Hastings correction                 (extension)
 * log pi = log-likelihood over observations [0, t) + log prior.
 * theta (device P x d), ll (device P: log-likelihood over [0, t) of theta)
 * and, for MALA, grad (device P x d: its gradient) are updated in place for
 * accepted particles; accept iff log u < log alpha.  z: device P x d
 * normals, u: device P uniforms in (0, 1), or NULL for Philox draws from
 * (seed, stream) and (seed, stream + 1).  *accept_rate (host, may be NULL)
 * = accepted / P.  The call waits (the accepted count and the
 * positive-definiteness flag are read back).  SPS_ERR_NOT_PD if V is not
 * positive definite (the failure of Section 4.2); then nothing is modified.
 * The log-likelihood of the proposal uses precision prec. */
int sps_mutate(sps_ctx* ctx, double* theta, double* ll, double* grad, int32_t J,
               int32_t N, int64_t t, double h, int kind, int prec, const double* z,
               const double* u, uint64_t seed, uint64_t stream, double* accept_rate);

/* Algorithm 3, second pass: one M step exactly as sps_mutate but with the
 * proposal covariance given instead of h V: Sigma (device, d x d FP64,
 * symmetric positive definite), typically recorded by sps_last_sigma in an
 * adaptive first pass.  RW: theta' = theta + L z (L L' = Sigma); MALA:
 * theta' = theta + (1/2) Sigma grad log pi + L z.  SPS_ERR_NOT_PD if Sigma
 * is not positive definite (nothing is modified). */
int sps_mutate_cov(sps_ctx* ctx, double* theta, double* ll, double* grad,
                   int32_t J, int32_t N, int64_t t, const double* Sigma, int kind,
                   int prec, const double* z, const double* u, uint64_t seed,
                   uint64_t stream, double* accept_rate);

/* The M phase of one cycle, Algorithm 2 step 2(c), in one call.  Step
 * r = 1, 2, ... is the step of sps_mutate with the current h and Philox
 * streams stream0 + r stream_step (normals) and that + 1 (uniforms); after it
 * the monitored functions (sps_monitor) and their RNEs (sps_moments) are
 * formed on the device and aggregated (rne_rule 0: mean, 1: minimum).  A
 * control kernel applies the step-size rule (h += h_step if the acceptance
 * rate exceeds acc_target, else h -= h_step, kept in [h_min, h_max]) and the
 * stopping rule (aggregate RNE >= K, or R_max steps) on the device; h and the
 * stop word stay in device memory.  The host reads each step's small state
 * record asynchronously, with the next step already queued when the steps
 * are short, so the device does not wait for the host between steps; a step
 * queued after the stop leaves every output unchanged.  theta, ll, grad: as
 * sps_mutate.  h: host, in: the step-size factor of the first step, out:
 * after the last update.  g_work: device scratch of P x (d + C - 1) FP64.
 * sigma_out: device, R_max x d x d FP64, or NULL; rows 0 .. R_out - 1
 * receive the proposal covariance of every step taken (the record of
 * Algorithm 3's first pass), later rows are unspecified.  *R_out: steps
 * taken; *rne_out, *rate_out (host, may be NULL): aggregate RNE and
 * acceptance rate of the last step.  Errors as sps_mutate (SPS_ERR_NOT_PD
 * stops the loop; the steps before it stand). */
int sps_mphase(sps_ctx* ctx, double* theta, double* ll, double* grad, int32_t J,
               int32_t N, int64_t t, int kind, int prec, double* h, double h_step,
               double h_min, double h_max, double acc_target, double K, int32_t R_max,
               int rne_rule, uint64_t seed, uint64_t stream0, uint64_t stream_step,
               double* g_work, double* sigma_out, int32_t* R_out, double* rne_out,
               double* rate_out);

/* Copy of the proposal covariance (h V, or the given Sigma) used by the last
 * sps_mutate / sps_mutate_cov call on ctx into Sigma (device, d x d FP64):
 * the lambda_l of Algorithm 3's record. */
int sps_last_sigma(sps_ctx* ctx, double* Sigma);

/* Algorithm 1 step 2(a) with a fixed cycle end (Algorithm 3, second pass):
 * log_w (device, P FP64) = log-likelihood of observations s0+1..s1 (the
 * log of the product of the C-phase weight increments), ll (in/out) +=
 * log_w.  0 <= s0 < s1 <= T.  Asynchronous. */
int sps_correct_fixed(sps_ctx* ctx, const double* theta, double* ll, int32_t J,
                      int32_t N, int64_t s0, int64_t s1, int prec, double* log_w);

/* ------------------------------------------------ accuracy measures */

/* Monitored functions of each particle: g (device, P x m FP64, m = d + C - 1)
 * = (theta_1..theta_d, theta_c' xbar for c = 1..C-1), xbar the mean of the
 * rows of X (the log-odds at the sample mean reported in Tables 2 and 5). */
int sps_monitor(sps_ctx* ctx, const double* theta, int64_t P, double* g);

/* Eqs. (partial_g)-(RNE_def) for each of m functions: g device P x m FP64;
 * mean, sd, nse, rne: host, m FP64 each (any may be NULL).
 * NSE = sqrt(v_hat / (J N)).  Waits. */
int sps_moments(sps_ctx* ctx, const double* g, int32_t J, int32_t N, int32_t m,
                double* mean, double* sd, double* nse, double* rne);

/* ------------------------------------------------------ instrumentation */

/* Kernel classes timed by sps_timing_read. */
enum { SPS_KT_LOGLIK = 0,       /* forward likelihood kernel (sps_loglik, M-phase proposals) */
       SPS_KT_LOGLIK_GRAD = 1,  /* fused forward + adjoint kernel                          */
       SPS_KT_PEROBS = 2 };     /* per-observation terms of the C phase                      */

/* enable != 0: from now on bracket every launch of the likelihood kernels
 * with HIP events on the context stream; enable == 0: stop.  Either way the
 * accumulated counts are reset. */
int sps_timing_enable(sps_ctx* ctx, int enable);

/* Synchronises the stream and returns, for kernel class `which`, the number
 * of timed launches and their summed GPU duration in milliseconds (host). */
int sps_timing_read(sps_ctx* ctx, int which, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* SPS_H */
