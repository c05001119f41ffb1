// loglik.hip -- launch logic of the likelihood kernels and the sps_loglik /
// sps_loglik_grad entry points.
#include <algorithm>

#include "loglik_kernel.h"
#include "loglik_pipe.h"

namespace sps {

__global__ void loglik_reduce_kernel(const double* __restrict__ part_ll,
                                     const double* __restrict__ part_g, int64_t P, int32_t d,
                                     int32_t nsplit, double* __restrict__ ll,
                                     double* __restrict__ grad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P) {
        double s = 0.0;
        for (int q = 0; q < nsplit; ++q) s += part_ll[(int64_t)q * P + i];
        ll[i] = s;
    }
    if (grad != nullptr && i < P * d) {
        double s = 0.0;
        for (int q = 0; q < nsplit; ++q) s += part_g[(int64_t)q * P * d + i];
        grad[i] = s;
    }
}

// Sufficient statistics of the multinomial likelihood over rows [t0, t1):
// S[(c - 1) k + i] = sum_{t0 <= t < t1, y_t = c} x_{t,i}, c = 1..C-1 (same
// layout as theta), with x as the likelihood kernel of precision prec sees it
// (the FP32 copy, or hi + lo of the BF16 pair), so that the eta_{y_t} term
// carries the same rounding as the normaliser the kernel computes.  One block
// per covariate, reading the transposed copy; fixed-order reduction.
__global__ void suffstat_kernel(const float* __restrict__ XTf, const uint16_t* __restrict__ XTh,
                                const uint16_t* __restrict__ XTl, int prec, const int8_t* __restrict__ y8,
                                int64_t Tp, int64_t t0, int64_t t1, int32_t k, int32_t C,
                                double* __restrict__ S) {
    __shared__ double red[8][256];
    const int32_t i = blockIdx.x;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t row = (int64_t)i * Tp;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += 256) {
        const int yt = y8[t];
        const double x = prec == SPS_FP32 ? (double)XTf[row + t]
                                          : (double)from_bf16(XTh[row + t]) + (double)from_bf16(XTl[row + t]);
#pragma unroll
        for (int c = 1; c < 8; ++c) acc[c] += (yt == c) ? x : 0.0;
    }
    for (int c = 1; c < C; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 1; c < C; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 1; c < C; ++c) S[(int64_t)(c - 1) * k + i] = red[c][0];
}

// ll[p] += ln 2 * theta~_p . S, the sum of eta_{y_t} with theta rounded exactly
// as the kernel's B operand (log2(e) theta in FP32, or its BF16 hi + lo);
// grad[p] += S.  Wave per particle.
__global__ __launch_bounds__(256) void suffstat_apply_kernel(const double* __restrict__ theta,
                                                             const double* __restrict__ S, int64_t P,
                                                             int32_t d, int prec, double* __restrict__ ll,
                                                             double* __restrict__ grad) {
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= P) return;
    double v = 0.0;
    for (int32_t e = lane; e < d; e += 64) {
        const double vd = theta[p * d + e] * kLog2e;
        double t2;
        if (prec == SPS_FP32) {
            t2 = (double)(float)vd;
        } else {
            const unsigned short h = to_bf16((float)vd);
            const unsigned short l = to_bf16((float)(vd - (double)from_bf16(h)));
            t2 = (double)from_bf16(h) + (double)from_bf16(l);
        }
        v += t2 * S[e];
        if (grad) grad[p * d + e] += S[e];
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    if (lane == 0) ll[p] += v * kLn2;
}

__global__ void fill_kernel(double* __restrict__ p, int64_t n, double v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int fill(sps_ctx* c, double* p, int64_t n, double v) {
    if (n <= 0) return SPS_OK;
    fill_kernel<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(p, n, v);
    return launched(c, "fill_kernel");
}

// BF16x3 full-range calls of the shapes in bf16_pipe_shape run the pipelined
// kernel (loglik_pipe.h); every other call runs loglik_kernel.h.
static LoglikEntry lookup(int prec, int nc, int ks, int mode) {
    switch (prec) {
        case SPS_FP64: return lookup_fp64(nc, ks, mode);
        case SPS_FP32: return lookup_fp32(nc, ks, mode);
        case SPS_BF16X3:
            return bf16_pipe_shape(nc, ks, mode) ? lookup_pipe(nc, ks, mode == MODE_GRAD) : lookup_bf16(nc, ks, mode);
        default: return LoglikEntry{};
    }
}

// Common launcher.  grad != nullptr -> forward + adjoint.  perobs != nullptr ->
// per-observation terms written to perobs[(t - t0) * P + p] (forward only).
// ext (optional): caller-provided device scratch instead of the context's
// grow-only buffers; the observation split is limited so its partials fit.
static int run_loglik(sps_ctx* c, const double* theta, int64_t P, int64_t t0, int64_t t1,
                      int prec, double* ll, double* grad, void* perobs, double* chunk_tot = nullptr,
                      const unsigned* skip = nullptr, LoglikSplit* keep = nullptr,
                      const LoglikScratch* ext = nullptr) {
    if (keep) *keep = LoglikSplit{ll, grad, 1};
    const int mode = grad ? MODE_GRAD : (perobs ? MODE_PEROBS : MODE_FWD);
    const int ks = (prec == SPS_BF16X3) ? c->kb / 32 : c->kp / 4;
    LoglikEntry e = lookup(prec, c->C - 1, ks, mode);
    if (!e.fn) return fail(c, SPS_ERR_ARG, "no likelihood kernel for C=%d k=%d prec=%d", c->C, c->k, prec);
    if (mode == MODE_FWD && (P + e.ppb - 1) / e.ppb < 64) {
        // few particles: more, narrower waves beat operand reuse (measured at
        // P = 1024: 13 us with one block of 16 particles per wave, 24 us with two)
        const LoglikEntry narrow = lookup(prec, c->C - 1, ks, MODE_PEROBS);
        if (narrow.fn) e = narrow;
    }
    if (P == 0) return SPS_OK;
    if (t1 == t0) {
        if (ll) SPS_CHECK(fill(c, ll, P, 0.0));
        if (grad) SPS_CHECK(fill(c, grad, P * c->d, 0.0));
        return SPS_OK;
    }
    LoglikArgs a{};
    switch (prec) {
        case SPS_FP64: a.X = c->Xd; a.XT = c->XTd; a.ldx = c->kp; break;
        case SPS_FP32: a.X = c->Xf; a.XT = c->XTf; a.ldx = c->kp; break;
        default: a.X = c->Xh; a.Xlo = c->Xl; a.XT = c->XTh; a.XTlo = c->XTl; a.ldx = c->kb; break;
    }
    a.y8 = c->y8;
    a.theta = theta;
    a.P = P;
    a.Tp = c->Tp;
    a.t0 = t0;
    a.t1 = t1;
    a.t0a = t0 & ~int64_t(kObsStep - 1);
    a.k = c->k;
    a.d = c->d;
    a.binary = c->C == 2;
    a.nsteps = (int32_t)((t1 - a.t0a + kObsStep - 1) / kObsStep);
    // Observation splits: the kernel's workgroup target (measured per kernel
    // shape), at least 4 steps of work per wave.  Up to four parts are taken
    // by the waves of one workgroup (a particle group per 1, 2 or 4 waves),
    // whose sums meet in LDS; further parts go to separate workgroups and
    // leave partial slices in memory (bounded storage), summed afterwards.
    const int64_t npt0 = (P + e.ppb - 1) / e.ppb;
    int64_t parts = std::max<int64_t>(1, (e.target + npt0 - 1) / npt0);
    parts = std::min<int64_t>(parts, std::max<int64_t>(1, a.nsteps / 4));
    const int ws = (!e.wsplit || perobs) ? 1 : parts >= 4 ? 4 : parts >= 2 ? 2 : 1;
    int64_t nsplit = (parts + ws - 1) / ws;
    if (grad) {
        const int64_t cap = std::max<int64_t>(1, (int64_t(512) << 20) / (P * c->d * 8));
        nsplit = std::min(nsplit, cap);
    }
    if (ext) nsplit = std::min<int64_t>(nsplit, std::max<int64_t>(1, ext->part_doubles / P));
    a.steps_per_split = (int32_t)((a.nsteps + nsplit * ws - 1) / (nsplit * ws));
    nsplit = ((a.nsteps + a.steps_per_split - 1) / a.steps_per_split + ws - 1) / ws;
    a.nsplit = (int32_t)nsplit;
    a.wsplit = ws;
    const int64_t npt = (P + e.ppb / ws - 1) / (e.ppb / ws);
    if (nsplit == 1 && ll) {
        a.out_ll = ll;
        a.out_g = grad;
    } else if (ext && !grad) {
        a.out_ll = ext->part;
    } else {
        SPS_CHECK(ensure(c, c->part_ll, sizeof(double) * nsplit * P, "partial log-likelihoods"));
        a.out_ll = (double*)c->part_ll.p;
        if (grad) {
            SPS_CHECK(ensure(c, c->part_g, sizeof(double) * nsplit * P * c->d, "partial gradients"));
            a.out_g = (double*)c->part_g.p;
        }
    }
    a.perobs = perobs;
    a.chunk_tot = perobs ? chunk_tot : nullptr;
    a.skip = skip;
    dim3 grid((unsigned)(npt * nsplit));
    int slot = -1;
    // (the no-allocation path is not timed: timing creates events)
    if (!ext) SPS_CHECK(timing_begin(c, grad ? SPS_KT_LOGLIK_GRAD : (perobs ? SPS_KT_PEROBS : SPS_KT_LOGLIK), &slot));
    hipError_t err = e.fn(a, grid, c->stream);
    if (err != hipSuccess) return hip_fail(c, err, "loglik_kernel launch");
    if (!ext) SPS_CHECK(timing_end(c, slot));
    const bool suff_term = ll && c->C > 2 && prec != SPS_FP64;
    if (ll && a.out_ll != ll && keep && !suff_term) {
        // the caller sums the observation-split partials itself
        *keep = LoglikSplit{a.out_ll, a.out_g, a.nsplit};
        return SPS_OK;
    }
    if (ll && a.out_ll != ll) {
        const int64_t n = grad ? P * c->d : P;
        loglik_reduce_kernel<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(
            a.out_ll, grad ? (const double*)c->part_g.p : nullptr, P, c->d, a.nsplit, ll, grad);
        SPS_CHECK(launched(c, "loglik_reduce_kernel"));
    }
    if (suff_term && ext) {
        // the eta_{y_t} / 1{y_t = c} terms the kernel leaves out, into the
        // caller's scratch (recomputed every call: the scratch is shared)
        suffstat_kernel<<<c->k, 256, 0, c->stream>>>(c->XTf, c->XTh, c->XTl, prec, c->y8, c->Tp, t0, t1, c->k,
                                                      c->C, ext->suff);
        SPS_CHECK(launched(c, "suffstat_kernel"));
        suffstat_apply_kernel<<<(unsigned)((P + 3) / 4), 256, 0, c->stream>>>(theta, ext->suff, P, c->d, prec,
                                                                              ll, grad);
        SPS_CHECK(launched(c, "suffstat_apply_kernel"));
    } else if (suff_term) {
        // the eta_{y_t} / 1{y_t = c} terms the kernel leaves out
        SPS_CHECK(ensure(c, c->suff, sizeof(double) * c->d, "sufficient statistics"));
        if (!(c->suff_valid && c->suff_t0 == t0 && c->suff_t1 == t1 && c->suff_prec == prec)) {
            suffstat_kernel<<<c->k, 256, 0, c->stream>>>(c->XTf, c->XTh, c->XTl, prec, c->y8, c->Tp, t0, t1,
                                                          c->k, c->C, (double*)c->suff.p);
            SPS_CHECK(launched(c, "suffstat_kernel"));
            c->suff_valid = true;
            c->suff_t0 = t0;
            c->suff_t1 = t1;
            c->suff_prec = prec;
        }
        suffstat_apply_kernel<<<(unsigned)((P + 3) / 4), 256, 0, c->stream>>>(theta, (const double*)c->suff.p,
                                                                              P, c->d, prec, ll, grad);
        SPS_CHECK(launched(c, "suffstat_apply_kernel"));
    }
    return SPS_OK;
}

static int check_loglik_args(sps_ctx* c, const char* who, const double* theta, int64_t P,
                             int64_t t0, int64_t t1, int prec) {
    if (!c->has_data) return fail(c, SPS_ERR_STATE, "%s: call sps_set_data first", who);
    if (!theta && P > 0) return fail(c, SPS_ERR_ARG, "%s: null theta", who);
    if (P < 0 || P > (int64_t(1) << 31)) return fail(c, SPS_ERR_ARG, "%s: P=%lld out of range", who, (long long)P);
    if (t0 < 0 || t1 < t0 || t1 > c->T)
        return fail(c, SPS_ERR_ARG, "%s: observation range [%lld, %lld) outside [0, %lld]", who,
                    (long long)t0, (long long)t1, (long long)c->T);
    if (prec != SPS_FP64 && prec != SPS_FP32 && prec != SPS_BF16X3)
        return fail(c, SPS_ERR_ARG, "%s: unknown precision %d", who, prec);
    return SPS_OK;
}

int loglik_launch(sps_ctx* c, const double* theta, int64_t P, int64_t t0, int64_t t1, int prec,
                  double* ll, double* grad, const unsigned* skip) {
    return run_loglik(c, theta, P, t0, t1, prec, ll, grad, nullptr, nullptr, skip);
}

int loglik_launch_split(sps_ctx* c, const double* theta, int64_t P, int64_t t0, int64_t t1, int prec,
                        double* ll, double* grad, LoglikSplit* out, const unsigned* skip) {
    return run_loglik(c, theta, P, t0, t1, prec, ll, grad, nullptr, nullptr, skip, out);
}

int loglik_perobs(sps_ctx* c, const double* theta, int64_t P, int64_t t0, int64_t t1, int prec,
                  void* perobs, double* chunk_tot, const unsigned* skip) {
    return run_loglik(c, theta, P, t0, t1, prec, nullptr, nullptr, perobs, chunk_tot, skip);
}

int loglik_launch_scratch(sps_ctx* c, const double* theta, int64_t P, int64_t t0, int64_t t1, int prec,
                          double* ll, const LoglikScratch& ext) {
    SPS_CHECK(check_loglik_args(c, "sps_loglik_noalloc", theta, P, t0, t1, prec));
    if (!ll && P > 0) return fail(c, SPS_ERR_ARG, "sps_loglik_noalloc: null ll");
    return run_loglik(c, theta, P, t0, t1, prec, ll, nullptr, nullptr, nullptr, nullptr, nullptr, &ext);
}

}  // namespace sps

using namespace sps;

extern "C" int sps_loglik(sps_ctx* c, const double* theta, int64_t P, int64_t t0, int64_t t1,
                          int prec, double* ll) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    SPS_CHECK(check_loglik_args(c, "sps_loglik", theta, P, t0, t1, prec));
    if (!ll && P > 0) return fail(c, SPS_ERR_ARG, "sps_loglik: null ll");
    return run_loglik(c, theta, P, t0, t1, prec, ll, nullptr, nullptr);
}

extern "C" int sps_loglik_grad(sps_ctx* c, const double* theta, int64_t P, int64_t t0, int64_t t1,
                               int prec, double* ll, double* grad) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    SPS_CHECK(check_loglik_args(c, "sps_loglik_grad", theta, P, t0, t1, prec));
    if ((!ll || !grad) && P > 0) return fail(c, SPS_ERR_ARG, "sps_loglik_grad: null ll or grad");
    return run_loglik(c, theta, P, t0, t1, prec, ll, grad, nullptr);
}
