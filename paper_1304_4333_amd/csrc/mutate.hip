// mutate.hip -- the M phase (Algorithm 2 step 2(c)): pooled sample variance
// of the particles, its Cholesky factor, Gaussian random-walk or MALA
// proposals, the proposals' log-likelihood on the MFMA kernels, and the
// Metropolis-Hastings accept step.  All of it in FP64 except the
// log-likelihood, which uses the requested precision.
#include <algorithm>
#include <cmath>

#include "philox.h"
#include "sps_internal.h"

namespace sps {

int random_fill(sps_ctx* c, int kind, uint64_t seed, uint64_t stream, int64_t count, int32_t d,
                void* out);

constexpr unsigned kFlagNotPD = 1u;

// mean[i] = P^-1 sum_p theta[p][i]; one block per coordinate, fixed order.
__global__ void col_mean_kernel(const double* __restrict__ theta, int64_t P, int32_t d,
                                double* __restrict__ mean) {
    __shared__ double red[256];
    const int32_t i = blockIdx.x;
    double s = 0.0;
    for (int64_t p = threadIdx.x; p < P; p += 256) s += theta[p * d + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) mean[i] = red[0] / (double)P;
}

// Partial centred cross products over one chunk of particles:
// part[chunk][a][b] = sum_{p in chunk} (theta[p][a] - m_a)(theta[p][b] - m_b).
// 64 x 64 tile per block, 4 x 4 per thread, particles in steps of 16.
constexpr int kCovChunk = 4096;
__global__ __launch_bounds__(256) void cov_partial_kernel(const double* __restrict__ theta,
                                                          const double* __restrict__ mean, int64_t P,
                                                          int32_t d, double* __restrict__ part) {
    __shared__ double As[16][65];
    __shared__ double Bs[16][65];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int a0 = blockIdx.x * 64, b0 = blockIdx.y * 64;
    const int64_t pbeg = (int64_t)blockIdx.z * kCovChunk;
    const int64_t pend = std::min<int64_t>(P, pbeg + kCovChunk);
    double acc[4][4] = {};
    for (int64_t p0 = pbeg; p0 < pend; p0 += 16) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int r = e >> 6, cc = e & 63;
            const int64_t p = p0 + r;
            const int a = a0 + cc, b = b0 + cc;
            As[r][cc] = (p < pend && a < d) ? theta[p * d + a] - mean[a] : 0.0;
            Bs[r][cc] = (p < pend && b < d) ? theta[p * d + b] - mean[b] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
        }
        __syncthreads();
    }
    double* out = part + (int64_t)blockIdx.z * d * d;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int a = a0 + ty * 4 + i, b = b0 + tx * 4 + j;
            if (a < d && b < d) out[(int64_t)a * d + b] = acc[i][j];
        }
}

__global__ void cov_reduce_kernel(const double* __restrict__ part, int32_t nchunk, int32_t d,
                                  int64_t P, double* __restrict__ V) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)d * d) return;
    double s = 0.0;
    for (int32_t q = 0; q < nchunk; ++q) s += part[(int64_t)q * d * d + e];
    V[e] = s / (double)(P - 1);
}

// Cholesky V = L L' in one workgroup (left-looking, one column per step).
// Sets flags |= kFlagNotPD and stops if a pivot is not positive and finite.
__global__ __launch_bounds__(1024) void cholesky_kernel(const double* __restrict__ V, int32_t d,
                                                        double* __restrict__ L, unsigned* flags) {
    __shared__ double col[1024];
    __shared__ int fail_s;
    const int t = threadIdx.x;
    if (t == 0) fail_s = 0;
    for (int64_t e = t; e < (int64_t)d * d; e += 1024) L[e] = 0.0;
    __syncthreads();
    for (int32_t j = 0; j < d; ++j) {
        // t_i = V[i][j] - sum_{q<j} L[i][q] L[j][q] for i >= j
        for (int32_t i = j + t; i < d; i += 1024) {
            double s = V[(int64_t)i * d + j];
            const double* Li = L + (int64_t)i * d;
            const double* Lj = L + (int64_t)j * d;
            for (int32_t q = 0; q < j; ++q) s -= Li[q] * Lj[q];
            col[i - j] = s;  // d <= 1024
        }
        __syncthreads();
        const double piv = col[0];
        if (!(piv > 0.0) || !isfinite(piv)) {
            if (t == 0) {
                fail_s = 1;
                atomicOr(flags, kFlagNotPD);
            }
        }
        __syncthreads();
        if (fail_s) return;
        const double ljj = sqrt(piv);
        for (int32_t i = j + t; i < d; i += 1024)
            L[(int64_t)i * d + j] = (i == j) ? ljj : col[i - j] / ljj;
        __syncthreads();
    }
}

// W = L^-1 (lower triangular), row by row in one workgroup.
__global__ __launch_bounds__(1024) void trinv_kernel(const double* __restrict__ L, int32_t d,
                                                     double* __restrict__ W, const unsigned* flags) {
    if (*flags & kFlagNotPD) return;
    const int t = threadIdx.x;
    for (int64_t e = t; e < (int64_t)d * d; e += 1024) W[e] = 0.0;
    __syncthreads();
    for (int32_t i = 0; i < d; ++i) {
        const double* Li = L + (int64_t)i * d;
        const double inv = 1.0 / Li[i];
        for (int32_t c = t; c <= i; c += 1024) {
            double s = (c == i) ? 1.0 : 0.0;
            for (int32_t q = c; q < i; ++q) s -= Li[q] * W[(int64_t)q * d + c];
            W[(int64_t)i * d + c] = s * inv;
        }
        __syncthreads();
    }
}

// Out[p][a] = Base[p][a] + alpha * sum_q A[p][q] B[a][q]  (A: P x d, B: d x d).
// Base may be null (treated as 0).  64 x 64 output tile per block.
__global__ __launch_bounds__(256) void gemm_abt_kernel(const double* __restrict__ A,
                                                       const double* __restrict__ B,
                                                       const double* Base,  // may alias Out
                                                       double* Out, int64_t P,
                                                       int32_t d, double alpha) {
    __shared__ double As[16][65];
    __shared__ double Bs[16][65];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t p0 = (int64_t)blockIdx.x * 64;
    const int a0 = blockIdx.y * 64;
    double acc[4][4] = {};
    for (int q0 = 0; q0 < d; q0 += 16) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int r = e >> 4, cc = e & 15;
            const int64_t p = p0 + r;
            const int q = q0 + cc;
            As[cc][r] = (p < P && q < d) ? A[p * d + q] : 0.0;
            Bs[cc][r] = (a0 + r < d && q < d) ? B[(int64_t)(a0 + r) * d + q] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t p = p0 + ty * 4 + i;
        if (p >= P) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int a = a0 + tx * 4 + j;
            if (a >= d) continue;
            const double b = Base ? Base[p * d + a] : 0.0;
            Out[p * d + a] = b + alpha * acc[i][j];
        }
    }
}

// gpi = grad + gradient of the log prior, -(theta - mu) / sd^2.
__global__ void grad_logpost_kernel(const double* __restrict__ grad, const double* __restrict__ theta,
                                    const double* __restrict__ mu, const double* __restrict__ isd,
                                    int64_t P, int32_t d, double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * d) return;
    const int32_t i = (int32_t)(e % d);
    out[e] = grad[e] - (theta[e] - mu[i]) * isd[i] * isd[i];
}

__global__ void sub_kernel(const double* __restrict__ a, const double* __restrict__ b,
                           double* __restrict__ out, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = a[e] - b[e];
}

// log alpha = [ll' + log p(theta')] - [ll + log p(theta)]
//             (+ MALA: -|v|^2 / (2h) + |z|^2 / 2, v = L^-1 (theta - mu(theta')));
// accept iff log u < log alpha; accepted particles take theta', ll' (grad').
__global__ void accept_kernel(double* __restrict__ theta, double* __restrict__ ll,
                              double* __restrict__ grad, const double* __restrict__ theta2,
                              const double* __restrict__ ll2, const double* __restrict__ grad2,
                              const double* __restrict__ z, const double* __restrict__ v,
                              const double* __restrict__ u, const double* __restrict__ mu,
                              const double* __restrict__ isd, int64_t P, int32_t d, double h,
                              int mala, const unsigned* flags, unsigned long long* count) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P || (*flags & kFlagNotPD)) return;
    const double* a = theta + p * d;
    const double* b = theta2 + p * d;
    double q0 = 0.0, q1 = 0.0;
    for (int32_t i = 0; i < d; ++i) {
        const double za = (a[i] - mu[i]) * isd[i];
        const double zb = (b[i] - mu[i]) * isd[i];
        q0 += za * za;
        q1 += zb * zb;
    }
    double la = (ll2[p] - 0.5 * q1) - (ll[p] - 0.5 * q0);
    if (mala) {
        double vv = 0.0, zz = 0.0;
        for (int32_t i = 0; i < d; ++i) {
            vv += v[p * d + i] * v[p * d + i];
            zz += z[p * d + i] * z[p * d + i];
        }
        la += -vv / (2.0 * h) + 0.5 * zz;
    }
    if (isnan(la)) la = -INFINITY;
    if (log(u[p]) < la) {
        for (int32_t i = 0; i < d; ++i) theta[p * d + i] = b[i];
        ll[p] = ll2[p];
        if (mala)
            for (int32_t i = 0; i < d; ++i) grad[p * d + i] = grad2[p * d + i];
        atomicAdd(count, 1ull);
    }
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace sps

using namespace sps;

extern "C" int sps_mutate(sps_ctx* c, double* theta, double* ll, double* grad, int32_t J, int32_t N,
                          int64_t t, double h, int kind, int prec, const double* z, const double* u,
                          uint64_t seed, uint64_t stream, double* accept_rate) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (!c->has_data || !c->has_prior) return fail(c, SPS_ERR_STATE, "sps_mutate: set data and prior first");
    if (J < 1 || N < 1 || (int64_t)J * N < 2 || !theta || !ll)
        return fail(c, SPS_ERR_ARG, "sps_mutate: bad arguments (need J N >= 2, theta, ll)");
    if (t < 0 || t > c->T) return fail(c, SPS_ERR_ARG, "sps_mutate: t=%lld outside [0, T]", (long long)t);
    if (!(h > 0.0) || !std::isfinite(h)) return fail(c, SPS_ERR_ARG, "sps_mutate: h must be positive");
    if (kind != SPS_RW && kind != SPS_MALA) return fail(c, SPS_ERR_ARG, "sps_mutate: unknown kind %d", kind);
    if (kind == SPS_MALA && !grad) return fail(c, SPS_ERR_ARG, "sps_mutate: MALA needs grad");
    if (prec != SPS_FP64 && prec != SPS_FP32 && prec != SPS_BF16X3)
        return fail(c, SPS_ERR_ARG, "sps_mutate: unknown precision %d", prec);
    const int64_t P = (int64_t)J * N;
    const int32_t d = c->d;
    if (d > 1024) return fail(c, SPS_ERR_ARG, "sps_mutate: d=%d above 1024", d);
    const bool mala = kind == SPS_MALA;
    const int64_t Pd = P * d;
    const int32_t nchunk = (int32_t)((P + kCovChunk - 1) / kCovChunk);

    SPS_CHECK(ensure(c, c->theta2, sizeof(double) * Pd, "proposals"));
    SPS_CHECK(ensure(c, c->ll2, sizeof(double) * P, "proposal log-likelihoods"));
    if (mala) {
        SPS_CHECK(ensure(c, c->grad2, sizeof(double) * Pd, "proposal gradients"));
        SPS_CHECK(ensure(c, c->pstat, sizeof(double) * 2 * Pd, "MALA work"));
    }
    SPS_CHECK(ensure(c, c->cov, sizeof(double) * ((size_t)nchunk + 3) * d * d, "covariance"));
    SPS_CHECK(ensure(c, c->mean, sizeof(double) * d, "mean"));
    SPS_CHECK(ensure(c, c->small, 4096, "small"));
    SPS_CHECK(ensure_host(c, c->hostbuf, 4096));
    double* part = (double*)c->cov.p;
    double* V = part + (size_t)nchunk * d * d;
    double* L = V + (size_t)d * d;
    double* W = L + (size_t)d * d;
    double* mean = (double*)c->mean.p;
    double* th2 = (double*)c->theta2.p;
    double* ll2 = (double*)c->ll2.p;
    unsigned* flags = (unsigned*)c->small.p;
    unsigned long long* count = (unsigned long long*)((char*)c->small.p + 8);
    SPS_CHECK(fill(c, (double*)c->small.p, 2, 0.0));

    if (!z) {
        SPS_CHECK(ensure(c, c->z, sizeof(double) * Pd, "normals"));
        SPS_CHECK(random_fill(c, 2, seed, stream, P, d, c->z.p));
        z = (const double*)c->z.p;
    }
    if (!u) {
        SPS_CHECK(ensure(c, c->u, sizeof(double) * P, "uniforms"));
        SPS_CHECK(random_fill(c, 1, seed, stream + 1, P, 1, c->u.p));
        u = (const double*)c->u.p;
    }

    // sample variance of all particles and its Cholesky factor
    col_mean_kernel<<<d, 256, 0, c->stream>>>(theta, P, d, mean);
    SPS_CHECK(launched(c, "col_mean_kernel"));
    cov_partial_kernel<<<dim3((d + 63) / 64, (d + 63) / 64, nchunk), 256, 0, c->stream>>>(theta, mean, P, d, part);
    SPS_CHECK(launched(c, "cov_partial_kernel"));
    cov_reduce_kernel<<<nblk((int64_t)d * d), 256, 0, c->stream>>>(part, nchunk, d, P, V);
    SPS_CHECK(launched(c, "cov_reduce_kernel"));
    cholesky_kernel<<<1, 1024, 0, c->stream>>>(V, d, L, flags);
    SPS_CHECK(launched(c, "cholesky_kernel"));

    const dim3 gg((unsigned)((P + 63) / 64), (unsigned)((d + 63) / 64));
    const double sh = std::sqrt(h);
    if (!mala) {
        gemm_abt_kernel<<<gg, 256, 0, c->stream>>>(z, L, theta, th2, P, d, sh);
        SPS_CHECK(launched(c, "gemm_abt_kernel"));
        SPS_CHECK(loglik_launch(c, th2, P, 0, t, prec, ll2, nullptr));
    } else {
        double* gpi = (double*)c->pstat.p;
        double* work = gpi + Pd;
        double* g2 = (double*)c->grad2.p;
        trinv_kernel<<<1, 1024, 0, c->stream>>>(L, d, W, flags);
        SPS_CHECK(launched(c, "trinv_kernel"));
        // mu(theta) = theta + (h/2) V grad log pi(theta); theta' = mu + sqrt(h) L z
        grad_logpost_kernel<<<nblk(Pd), 256, 0, c->stream>>>(grad, theta, c->prior_mean, c->prior_isd, P, d, gpi);
        SPS_CHECK(launched(c, "grad_logpost_kernel"));
        gemm_abt_kernel<<<gg, 256, 0, c->stream>>>(gpi, V, theta, work, P, d, 0.5 * h);
        SPS_CHECK(launched(c, "gemm_abt_kernel"));
        gemm_abt_kernel<<<gg, 256, 0, c->stream>>>(z, L, work, th2, P, d, sh);
        SPS_CHECK(launched(c, "gemm_abt_kernel"));
        SPS_CHECK(loglik_launch(c, th2, P, 0, t, prec, ll2, g2));
        // v = L^-1 (theta - mu(theta'))
        grad_logpost_kernel<<<nblk(Pd), 256, 0, c->stream>>>(g2, th2, c->prior_mean, c->prior_isd, P, d, gpi);
        SPS_CHECK(launched(c, "grad_logpost_kernel"));
        sub_kernel<<<nblk(Pd), 256, 0, c->stream>>>(theta, th2, work, Pd);
        SPS_CHECK(launched(c, "sub_kernel"));
        gemm_abt_kernel<<<gg, 256, 0, c->stream>>>(gpi, V, work, work, P, d, -0.5 * h);
        SPS_CHECK(launched(c, "gemm_abt_kernel"));
        gemm_abt_kernel<<<gg, 256, 0, c->stream>>>(work, W, nullptr, gpi, P, d, 1.0);
        SPS_CHECK(launched(c, "gemm_abt_kernel"));
    }
    accept_kernel<<<nblk(P), 256, 0, c->stream>>>(
        theta, ll, grad, th2, ll2, mala ? (const double*)c->grad2.p : nullptr, z,
        mala ? (const double*)c->pstat.p : nullptr, u, c->prior_mean, c->prior_isd, P, d, h, mala ? 1 : 0,
        flags, count);
    SPS_CHECK(launched(c, "accept_kernel"));
    SPS_HIP(c, hipMemcpyAsync(c->hostbuf.p, c->small.p, 16, hipMemcpyDeviceToHost, c->stream));
    SPS_HIP(c, hipStreamSynchronize(c->stream));
    const unsigned f = *(const unsigned*)c->hostbuf.p;
    const unsigned long long n_acc = *(const unsigned long long*)((const char*)c->hostbuf.p + 8);
    if (f & kFlagNotPD)
        return fail(c, SPS_ERR_NOT_PD, "sps_mutate: the particles' sample variance is not positive definite");
    if (accept_rate) *accept_rate = (double)n_acc / (double)P;
    return SPS_OK;
}
