// sps_internal.h -- context and shared helpers of libsps (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/sps.h"

namespace sps {

// Observations are processed in steps of 32 rows (two 16-row MFMA tiles);
// observation ranges are split across workgroups on 32-row boundaries.
constexpr int kObsStep = 32;

// A grow-only device buffer owned by the context.
struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace sps

struct sps_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    // ---- data set (sps_set_data) --------------------------------------
    bool has_data = false;
    bool has_prior = false;
    bool has_sigma = false;  // a proposal covariance is held in chol (sps_last_sigma)
    int64_t T = 0;       // observations
    int32_t k = 0;       // covariates
    int32_t C = 0;       // outcomes
    int32_t d = 0;       // free parameters k (C - 1)
    int64_t Tp = 0;      // padded row count (multiple of 32, plus one spare step)
    int32_t kp = 0;      // row stride of the FP64/FP32 copies (multiple of 16)
    int32_t kb = 0;      // row stride of the BF16 copies (multiple of 32)
    int32_t kt = 0;      // rows of the transposed copies, max(kp, kb)
    // Kernel copies of X.  For C == 2 row t is multiplied by (1 - 2 y_t)
    // ("sign folding"), so that the per-observation log-probability is
    // -softplus(x~_t' theta) without reading y.  Padding rows/cols are 0.
    double* Xd = nullptr;      // Tp x kp   FP64
    float* Xf = nullptr;       // Tp x kp   FP32
    uint16_t* Xh = nullptr;    // Tp x kb   BF16 high part
    uint16_t* Xl = nullptr;    // Tp x kb   BF16 low part (x - hi)
    double* XTd = nullptr;     // kt x Tp   FP64, transposed (adjoint operand)
    float* XTf = nullptr;      // kt x Tp   FP32, transposed
    uint16_t* XTh = nullptr;   // kt x Tp   BF16 high, transposed
    uint16_t* XTl = nullptr;   // kt x Tp   BF16 low, transposed
    int8_t* y8 = nullptr;      // Tp outcomes as bytes (padding 0)
    double* xbar = nullptr;    // k column means of X
    double* prior_mean = nullptr;  // d
    double* prior_isd = nullptr;   // d  1 / sd (independent components only)
    // Full prior covariance S = L L' (sps_set_prior_cov, sps_set_prior_g).
    bool prior_full = false;
    double* prior_L = nullptr;     // d x d lower Cholesky factor of S
    double* prior_Li = nullptr;    // d x d, L^-1 (lower)
    double* prior_LiT = nullptr;   // d x d, (L^-1)'
    std::vector<double> prior_cov_host;  // the prior covariance as set, d x d (either kind)

    // ---- scratch (grow-only; allocated on first use at a given size) ----
    sps::Buf part_ll;    // obs-split partial log-likelihoods
    sps::Buf part_g;     // obs-split partial gradients
    sps::Buf theta2;     // proposals
    sps::Buf ll2, grad2; // proposal log-likelihood / gradient
    sps::Buf cov;        // covariance partials
    sps::Buf chol;       // proposal covariance, its Cholesky factor and inverse (3 d x d)
    sps::Buf mean;       // d
    sps::Buf pstat;      // per-particle statistics of the M step
    sps::Buf z, u;       // Philox draws when the caller passes none
    sps::Buf u53;
    sps::Buf corr_lw;    // C phase block of running log-weights
    sps::Buf corr_red;   // C phase per-observation reductions
    sps::Buf small;      // small device results (status words, sums)
    sps::Buf mstat;      // device-resident state of the M phase (step size, stop word)
    sps::Buf hostbuf;    // pinned host staging for scalar read-back
    void* pub = nullptr;       // fine-grained pinned host memory written by publish_kernel
    size_t pub_bytes = 0;
    uint64_t pub_seq = 0;      // sequence number of the last read-back
    sps::Buf W;          // resampling integer weights
    sps::Buf gstat;      // moments partials
    sps::Buf suff;       // multinomial sufficient statistics for one observation range
    sps::Buf pw;         // full prior: centred and whitened particles (3 P d)
    bool suff_valid = false;
    int64_t suff_t0 = 0, suff_t1 = 0;
    int suff_prec = -1;

    // ---- optional kernel timing (sps_timing_enable) ----
    struct Timed {
        int which;
        hipEvent_t a, b;
    };
    bool timing = false;
    std::vector<hipEvent_t> evpool;
    std::vector<Timed> pending;
    double kt_ms[3] = {0, 0, 0};
    int64_t kt_n[3] = {0, 0, 0};
};

namespace sps {

int fail(sps_ctx* c, int code, const char* fmt, ...);
int hip_fail(sps_ctx* c, hipError_t e, const char* what);
// Ensure b holds at least `bytes` device bytes (grow-only).
int ensure(sps_ctx* c, Buf& b, size_t bytes, const char* what);
int ensure_host(sps_ctx* c, Buf& b, size_t bytes);

#define SPS_HIP(ctx, call)                                      \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return sps::hip_fail(ctx, e_, #call); \
    } while (0)

#define SPS_CHECK(expr)         \
    do {                        \
        int s_ = (expr);        \
        if (s_ != SPS_OK) return s_; \
    } while (0)

// Launch-error check after a kernel launch.
inline int launched(sps_ctx* c, const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, what);
    return SPS_OK;
}

// Likelihood entry used by the phases (defined in loglik.hip).
// Writes ll (and grad when non-null) for observations [t0, t1).
// skip (optional, device): the likelihood kernel does nothing when *skip is
// nonzero at the time it runs (the outputs are then left as they were).
int loglik_launch(sps_ctx* c, const double* theta, int64_t P, int64_t t0, int64_t t1,
                  int prec, double* ll, double* grad, const unsigned* skip = nullptr);
// As loglik_launch, but when the kernel leaves observation-split partials and
// no term is added after the sum (C = 2 or FP64), the sum is left to the
// caller: out->ll holds out->n slices of P, out->g (grad given) out->n
// slices of P x d, valid until the next likelihood launch on the context.
// Otherwise out = {ll, grad, 1}.
struct LoglikSplit {
    const double* ll;
    const double* g;
    int32_t n;
};
int loglik_launch_split(sps_ctx* c, const double* theta, int64_t P, int64_t t0, int64_t t1,
                        int prec, double* ll, double* grad, LoglikSplit* out,
                        const unsigned* skip = nullptr);
// Device scratch supplied by the caller instead of the context's grow-only
// buffers (sps_loglik_noalloc): part holds part_doubles doubles for the
// observation-split partials, suff at least d doubles.
struct LoglikScratch {
    double* part;
    int64_t part_doubles;
    double* suff;
};
// sps_loglik on that scratch: no device allocation (arguments checked).
int loglik_launch_scratch(sps_ctx* c, const double* theta, int64_t P, int64_t t0, int64_t t1, int prec,
                          double* ll, const LoglikScratch& ext);
// Once per device, with the device current (sps_create): resolve the device
// address of the no-allocation scratch array (noalloc.hip).
int noalloc_setup(sps_ctx* c, int device);
// Per-observation terms l_{p,t} for t0 <= t < t1 into perobs[(t - t0) * P + p]:
// FP64 natural-log values in SPS_FP64 mode, otherwise the kernel's FP32
// base-2 values (read them with perobs_value).  chunk_tot (optional):
// chunk_tot[q * P + p] = sum of the terms of particle p over the observations
// of [t0, t1) in the q-th 32-aligned row block counted from t0 rounded down to
// a multiple of 32 (the kernel's observation steps).  skip (optional, device):
// the launch does nothing when *skip is nonzero at the time it runs.
int loglik_perobs(sps_ctx* c, const double* theta, int64_t P, int64_t t0, int64_t t1,
                  int prec, void* perobs, double* chunk_tot, const unsigned* skip);
// Entry i of a per-observation buffer as an FP64 natural-log value.  Not
// contracted into a following add, so every kernel that sums these values
// in the same order gets the same bits.
__device__ __forceinline__ double perobs_value(const void* lw, int f32, int64_t i) {
#pragma clang fp contract(off)
    return f32 ? (double)((const float*)lw)[i] * 0.69314718055994530942 : ((const double*)lw)[i];
}
// Reads `bytes` of device memory at dsrc into host memory once every earlier
// launch on the context stream has finished, without a stream
// synchronisation: a one-wave kernel copies the bytes into fine-grained
// pinned host memory and then writes a sequence number there, on which the
// host spins (checking the stream for errors every 1024 spins; a stream that
// drains without the number appearing is an SPS_ERR_HIP failure).  Reads
// above kPublishBytes use a copy and a stream synchronisation instead.
// *host points at the bytes until the next read-back on the context.
int readback(sps_ctx* c, const void* dsrc, size_t bytes, const void** host);
// The same in two halves, for reads that overlap later launches: the copy is
// queued now (at most kPublishBytes, up to kPublishSlots in flight) and
// publish_wait returns its bytes, valid until kPublishSlots more publishes.
constexpr size_t kPublishBytes = 4096;
constexpr int kPublishSlots = 4;
struct PubTicket {
    int slot;
    uint64_t seq;
    const void* dsrc;
    size_t bytes;
};
int publish_async(sps_ctx* c, const void* dsrc, size_t bytes, PubTicket* t);
int publish_wait(sps_ctx* c, const PubTicket& t, const void** host);
// Event pair bracketing one timed launch (no-op unless timing is enabled).
int timing_begin(sps_ctx* c, int which, int* slot);
int timing_end(sps_ctx* c, int slot);
void timing_release(sps_ctx* c);
// p[0..n) = v on the context stream (a kernel, safe under graph capture).
int fill(sps_ctx* c, double* p, int64_t n, double v);
// Philox draws into out (kind 0: 53-bit integers, 1: uniforms, 2: normals).
int random_fill(sps_ctx* c, int kind, uint64_t seed, uint64_t stream, int64_t count, int32_t d,
                void* out);
// Out = Base + alpha A B' with A (P x d), B (d x d), all row-major FP64;
// Base may be null or alias Out.
int gemm_abt(sps_ctx* c, const double* A, const double* B, const double* Base, double* Out,
             int64_t P, int32_t d, double alpha);
// Monitored functions (theta and theta_c' xbar) of P particles into g (P x m).
int monitor_launch(sps_ctx* c, const double* theta, int64_t P, double* g);
// Moments of g (J groups of N, m functions) on the device; *out points at
// [mean | sd | NSE | RNE] (4 m doubles, context scratch).
int moments_launch(sps_ctx* c, const double* g, int32_t J, int32_t N, int32_t m, double** out);
// dst[0] = mean (rule 0) or minimum (rule 1) of the m RNEs in mom.
int rne_aggregate(sps_ctx* c, const double* mom, int32_t m, int rule, double* dst);
// Full prior: R = rows L^-1 (theta_p - mean); tmp (P x d) is scratch.
int prior_whiten(sps_ctx* c, const double* theta, int64_t P, double* tmp, double* R);

}  // namespace sps
