/*
 * sps_oracle.h -- plain FP64 CPU oracle of the sequential posterior simulator
 * (SPS) for multinomial logit models (Geweke, Durham & Xu, "Bayesian
 * Inference for Logistic Regression Models using Sequential Posterior
 * Simulation", 2013).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test suite, the smoke check and the CPU
 * baseline of the benchmark use it.  It shares no code with the HIP path.
 *
 * Conventions (all pointers are host memory, all arrays row-major):
 *   X        T x k covariates, y T outcomes in [0, C), outcome 0 is the base.
 *   theta    P x d particles, d = k (C-1); entry (c-1) k + i is the
 *            coefficient of covariate i for outcome c (c = 1..C-1).
 *   P = J N  particles in J groups of N, particle p = j N + n.
 *   Observation s (1-based, as in Algorithms 1-2) is row s-1 of X.
 */
#ifndef SPS_ORACLE_H
#define SPS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_NOT_PD = -3,
       ORC_ERR_NONFINITE = -4, ORC_ERR_DEGENERATE = -5, ORC_ERR_NOMEM = -6 };
enum { ORC_RW = 0, ORC_MALA = 1 };
enum { ORC_RESIDUAL = 0, ORC_MULTINOMIAL = 1 };

/* Counter-based random numbers (Philox4x32-10, Salmon et al. SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* OpenMP thread count: n > 0 sets it; returns the count in use. */
int orc_threads(int n);
void orc_u53(uint64_t seed, uint64_t stream, int64_t count, uint64_t* out);
void orc_uniforms(uint64_t seed, uint64_t stream, int64_t count, double* out);
void orc_normals(uint64_t seed, uint64_t stream, int64_t P, int32_t d, double* out);

/* Model, eq. (plogit). */
int orc_loglik(const double* X, const int32_t* y, int64_t T, int32_t k, int32_t C,
               const double* theta, int64_t P, int64_t t0, int64_t t1, double* ll);
int orc_loglik_grad(const double* X, const int32_t* y, int64_t T, int32_t k, int32_t C,
                    const double* theta, int64_t P, int64_t t0, int64_t t1,
                    double* ll, double* grad);
/* Gaussian prior N(mean, L L'), L lower triangular d x d (diagonal for
 * independent components, eq. (prior_Gauss); full for eq. (prior_norm)). */
void orc_logprior(const double* theta, int64_t P, int32_t d, const double* mean,
                  const double* L, double* lp, double* glp);
void orc_init_prior(const double* mean, const double* L, int32_t d, int64_t P,
                    uint64_t seed, uint64_t stream, double* theta);
/* Normalised g-prior covariance, eqs. (g-prior_def) and (prior_norm). */
int orc_gprior_cov(const double* X, int64_t T, int32_t k, int32_t C, double g, double* cov);

/* C phase, Algorithm 1 step 2(a) with the ESS stopping rule of Algorithm 2. */
int orc_correct(const double* X, const int32_t* y, int64_t T, int32_t k, int32_t C,
                const double* theta, double* ll, int32_t J, int32_t N, int64_t s0,
                double ess_frac, double* log_w, int64_t* t_end, double* ess_end);
double orc_ess(const double* log_w, int64_t P);

/* Marginal likelihood by-product, Section 2.3 / Section 3. */
int orc_logml_update(const double* log_w, int32_t J, int32_t N, double* logml_j);
void orc_logml_total(const double* logml_j, int32_t J, double* logml, double* nse,
                     double* meanlog, double* meanlog_nse);

/* S phase, Algorithm 1 step 2(b). */
int orc_resample_int(const uint64_t* W, int32_t J, int32_t N, int32_t scheme,
                     const uint64_t* u53, int32_t* ancestor);
int orc_resample(const double* log_w, int32_t J, int32_t N, int32_t scheme,
                 const uint64_t* u53, int32_t* ancestor, uint64_t* W_out);
void orc_gather(const int32_t* ancestor, int64_t P, int32_t m, const double* src,
                double* dst);

/* M phase, Algorithm 2 step 2(c). */
void orc_cov(const double* theta, int64_t P, int32_t d, double* mean, double* V);
int orc_cholesky(const double* V, int32_t d, double* L);
int orc_mutate_cov(const double* X, const int32_t* y, int64_t T, int32_t k, int32_t C,
                   const double* prior_mean, const double* prior_L,
                   double* theta, double* ll, double* grad, int32_t J, int32_t N,
                   int64_t t, const double* Sigma, int32_t kind, const double* z, const double* u,
                   double* accept_rate, double* log_alpha_out, int8_t* accepted_out);
int orc_mutate(const double* X, const int32_t* y, int64_t T, int32_t k, int32_t C,
               const double* prior_mean, const double* prior_L,
               double* theta, double* ll, double* grad, int32_t J, int32_t N,
               int64_t t, double h, int32_t kind, const double* z, const double* u,
               double* accept_rate, double* log_alpha_out, int8_t* accepted_out,
               double* sigma_out);

/* Numerical accuracy, eqs. (partial_g)-(RNE_def). */
void orc_moments(const double* g, int32_t J, int32_t N, int32_t m,
                 double* mean, double* sd, double* nse, double* rne);

/* Whole adaptive SPS, Algorithm 2. */
typedef struct {
    int32_t J, N;
    int32_t kind;        /* ORC_RW or ORC_MALA */
    int32_t scheme;      /* ORC_RESIDUAL or ORC_MULTINOMIAL */
    int32_t rne_rule;    /* 0: mean RNE over monitored functions, 1: minimum */
    int32_t R_max;       /* cap on M steps per cycle */
    int32_t max_cycles;  /* capacity of the per-cycle record arrays */
    int32_t pad_;
    double ess_frac, K_mid, K_final, h_init, h_step, h_min, h_max, acc_target;
    uint64_t seed;
} orc_config;

typedef struct {
    double logml, logml_nse, meanlog, meanlog_nse;
    int32_t cycles, m_iters, hit_R_max, status;
} orc_summary;

int orc_sps_run(const double* X, const int32_t* y, int64_t T, int32_t k, int32_t C,
                const double* prior_mean, const double* prior_L, const orc_config* cfg,
                double* theta_out, double* ll_out,
                double* mom_mean, double* mom_sd, double* mom_nse, double* mom_rne,
                int64_t* rec_t, int32_t* rec_R, double* rec_h, double* rec_acc,
                double* rec_sigma, int64_t sigma_cap, orc_summary* summary);

/* Algorithm 1 with the design recorded by a first adaptive pass (Algorithm 3). */
int orc_sps_run_fixed(const double* X, const int32_t* y, int64_t T, int32_t k, int32_t C,
                      const double* prior_mean, const double* prior_L, const orc_config* cfg,
                      int32_t L, const int64_t* t_l, const int32_t* R_l, const double* Sigma,
                      double* theta_out, double* ll_out,
                      double* mom_mean, double* mom_sd, double* mom_nse, double* mom_rne,
                      orc_summary* summary);

#ifdef __cplusplus
}
#endif
#endif
