// phases.hip -- random numbers, prior draws, the C phase with the ESS rule,
// the S phase on exact integer weights, the log marginal likelihood
// increments and the NSE/RNE reductions of libsps.
#include <algorithm>
#include <cmath>

#include "philox.h"
#include "sps_internal.h"

namespace sps {

// ------------------------------------------------------------------ block reductions
// 256-thread block sum / max in FP64 in a fixed order (deterministic): a
// butterfly inside each wave (a + b = b + a, so every lane ends with the same
// value), then (w0 + w1) + (w2 + w3) over the four waves; two barriers.
__device__ double block_sum256(double v, double* red) {
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) v += __shfl_xor(v, sh, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return r;
}
__device__ double block_max256(double v, double* red) {
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) v = fmax(v, __shfl_xor(v, sh, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    return r;
}

// ------------------------------------------------------------------ random numbers
__global__ void random_kernel(int kind, uint64_t seed, uint64_t stream, int64_t count, int32_t d,
                              void* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (kind == 2) {
        if (i >= count * d) return;
        ((double*)out)[i] = philox_normal(seed, stream, i / d, (int32_t)(i % d), d);
        return;
    }
    if (i >= count) return;
    uint64_t a, b;
    philox_u53x2(seed, stream, (uint64_t)i, a, b);
    if (kind == 0) ((uint64_t*)out)[i] = a;
    else ((double*)out)[i] = u53_to_uniform(a);
}

int random_fill(sps_ctx* c, int kind, uint64_t seed, uint64_t stream, int64_t count, int32_t d,
                void* out) {
    const int64_t n = kind == 2 ? count * d : count;
    if (n <= 0) return SPS_OK;
    random_kernel<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(kind, seed, stream, count, d, out);
    return launched(c, "random_kernel");
}

__global__ void init_prior_kernel(double* __restrict__ theta, int64_t P, int32_t d,
                                  const double* __restrict__ mean, const double* __restrict__ isd,
                                  uint64_t seed, uint64_t stream) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * d) return;
    const int32_t i = (int32_t)(e % d);
    theta[e] = mean[i] + philox_normal(seed, stream, e / d, i, d) / isd[i];
}

// ------------------------------------------------------------------ C phase
// Running log-weights over a block of nb observations s .. s + nb - 1 (u =
// observation - s).  The block is cut into chunks on the 32-aligned grid of
// the likelihood kernel's steps: chunk q holds rows r = u + off in
// [32 q, 32 q + 32), off = s mod 32, and the likelihood kernel writes the
// chunk totals tot[q][p] beside the per-observation terms.  A chunk is scanned
// as four runs of 8 rows.  The running value of particle p at u is
//   carry[p] + tot[0][p] + ... + tot[q-1][p]        (chunk_base)
//   + run sums of the earlier runs of the chunk      (run_sum)
//   + the terms of u's run up to u,
// added left to right in exactly that order by correct_scan_ess_kernel and
// correct_column_kernel, so both produce the same bits.  (Splitting the chunk
// totals over the scan's four waves, with an exchange through LDS, measured
// 6% slower on 22-chunk blocks: the loads are L2 hits issued together.)
constexpr int kScanChunk = 32;
constexpr int kScanRun = 8;

__device__ __forceinline__ double chunk_base(const double* __restrict__ carry, const double* __restrict__ tot,
                                             int64_t P, int64_t p, int32_t q) {
    double acc = carry ? carry[p] : 0.0;  // null carry: the first block (w = 1 before it)
#pragma unroll 8
    for (int32_t r = 0; r < q; ++r) acc += tot[(int64_t)r * P + p];
    return acc;
}

// Sum of the terms of particle p over rows u0 .. u0 + 7 that lie in [0, nb).
__device__ __forceinline__ double run_sum(const void* __restrict__ lw, int f32, int64_t P, int64_t p,
                                          int32_t u0, int32_t nb) {
    double sw = 0.0;
#pragma unroll
    for (int j = 0; j < kScanRun; ++j) {
        const int32_t u = u0 + j;
        if (u >= 0 && u < nb) sw += perobs_value(lw, f32, (int64_t)u * P + p);
    }
    return sw;
}

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// One workgroup per (64 particles, chunk q); wave w scans run w (rows
// 32 q + 8 w .. + 7), one particle per lane, and stages the running values in
// LDS.  Then 8 threads per row reduce over the 64 particles (thread j of a row
// takes particles j, j + 8, ...): m = max log w, s1 = sum exp(log w - m),
// s2 = sum exp(2 (log w - m)) into part[(u * npb + block) * 3 + {0, 1, 2}]
// (npb = workgroups per chunk); with FP32 terms the exponentials are FP32.
// The running value at u = nb - 1 goes to carry_out (the next block's carry).
// flags |= 1 on NaN or +inf.
constexpr int kScanLds = 72;  // row stride in doubles: rows 2i and 2i + 1 fall in different LDS banks
__global__ __launch_bounds__(256) void correct_scan_ess_kernel(const void* __restrict__ lw, int f32,
                                                               const double* __restrict__ carry,
                                                               const double* __restrict__ tot, int64_t P,
                                                               int32_t nb, int32_t off,
                                                               double* __restrict__ carry_out,
                                                               double* __restrict__ part, unsigned* flags,
                                                               const unsigned* skip) {
    __shared__ double S[kScanChunk / kScanRun][64];
    __shared__ double V[kScanChunk][kScanLds];
    if (*skip) return;  // the same value for the whole workgroup
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t p = (int64_t)blockIdx.x * 64 + lane;
    const int32_t q = blockIdx.y;
    const int32_t npb = gridDim.x;
    const bool pv = p < P;
    const int32_t u0 = q * kScanChunk - off + w * kScanRun;
    double val[kScanRun];
#pragma unroll
    for (int j = 0; j < kScanRun; ++j) {
        const int32_t u = u0 + j;
        val[j] = (pv && u >= 0 && u < nb) ? perobs_value(lw, f32, (int64_t)u * P + p) : 0.0;
    }
    double acc = pv ? chunk_base(carry, tot, P, p, q) : 0.0;
    {
        double sw = 0.0;  // run_sum's arithmetic on the loaded values
#pragma unroll
        for (int j = 0; j < kScanRun; ++j) {
            const int32_t u = u0 + j;
            if (u >= 0 && u < nb) sw += val[j];
        }
        S[w][lane] = sw;
    }
    __syncthreads();
    for (int w2 = 0; w2 < w; ++w2) acc += S[w2][lane];
    bool bad = false;
#pragma unroll
    for (int j = 0; j < kScanRun; ++j) {
        const int32_t u = u0 + j;
        double v = -INFINITY;
        if (u >= 0 && u < nb) {
            acc += val[j];
            if (pv) {
                v = acc;
                bad |= isnan(acc) || acc == INFINITY;
                if (u == nb - 1) carry_out[p] = acc;
            }
        }
        V[w * kScanRun + j][lane] = v;
    }
    if (bad) atomicOr(flags, 1u);
    __syncthreads();
    const int r = threadIdx.x >> 3, sg = threadIdx.x & 7;
    double m = -INFINITY;
#pragma unroll
    for (int i = 0; i < 8; ++i) m = fmax(m, V[r][sg + 8 * i]);
#pragma unroll
    for (int sh = 1; sh < 8; sh <<= 1) m = fmax(m, __shfl_xor(m, sh, 64));
    double s1 = 0.0, s2 = 0.0;
    // Reduced precision (FP32 terms): the weights' exponentials in FP32 too
    // (relative error ~1e-7, below that of the terms); FP64 otherwise.  The
    // sums stay FP64.  Two loops, so that the uniform branch is not turned
    // into evaluating both forms.
    if (m > -INFINITY && f32) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const double x = V[r][sg + 8 * i];
            if (x > -INFINITY) {
                const double e = (double)exp2f((float)((x - m) * 1.4426950408889634074));
                s1 += e;
                s2 += e * e;
            }
        }
    } else if (m > -INFINITY) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const double x = V[r][sg + 8 * i];
            if (x > -INFINITY) {
                const double e = exp(x - m);
                s1 += e;
                s2 += e * e;
            }
        }
    }
#pragma unroll
    for (int sh = 1; sh < 8; sh <<= 1) {
        s1 += __shfl_xor(s1, sh, 64);
        s2 += __shfl_xor(s2, sh, 64);
    }
    const int32_t u = q * kScanChunk - off + r;
    if (sg == 0 && u >= 0 && u < nb) {
        double* o = part + ((int64_t)u * npb + blockIdx.x) * 3;
        o[0] = m;
        o[1] = s1;
        o[2] = s2;
    }
}

// ESS(u) = S1^2 / S2 from the per-workgroup partials (max m, S1, S2 of
// exp(lw - m)).  One wave per observation.  Lane l loads partials l, l + 64,
// ... four at a time (all loads in flight together) and rescales them to its
// running maximum; the wave then takes the maximum over lanes and sums the
// lanes' rescaled S1, S2 in a fixed butterfly.  The exponentials of a lane are
// independent, so their latencies overlap.
__global__ __launch_bounds__(256) void correct_ess_combine_kernel(const double* __restrict__ part, int32_t npb,
                                                                  int32_t nb, double* __restrict__ ess,
                                                                  const unsigned* skip) {
    const int32_t u = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (u >= nb || *skip) return;
    const double* q = part + (int64_t)u * npb * 3;
    constexpr int kAhead = 4;
    double m = -INFINITY, s1 = 0.0, s2 = 0.0;
    for (int32_t b0 = lane; b0 < npb; b0 += 64 * kAhead) {
        double mk[kAhead], ak[kAhead], bk[kAhead];
#pragma unroll
        for (int k = 0; k < kAhead; ++k) {
            const int32_t b = b0 + 64 * k;
            const bool in = b < npb;
            mk[k] = in ? q[3 * b] : -INFINITY;
            ak[k] = in ? q[3 * b + 1] : 0.0;
            bk[k] = in ? q[3 * b + 2] : 0.0;
        }
        double M = m;
#pragma unroll
        for (int k = 0; k < kAhead; ++k) M = fmax(M, mk[k]);
        if (M == -INFINITY) continue;
        const double f = m > -INFINITY ? exp(m - M) : 0.0;
        s1 *= f;
        s2 *= f * f;
#pragma unroll
        for (int k = 0; k < kAhead; ++k) {
            const double g = mk[k] > -INFINITY ? exp(mk[k] - M) : 0.0;
            s1 += ak[k] * g;
            s2 += bk[k] * g * g;
        }
        m = M;
    }
    double W = m;
#pragma unroll
    for (int sh = 1; sh < 64; sh <<= 1) W = fmax(W, __shfl_xor(W, sh, 64));
    if (W == -INFINITY) {
        if (lane == 0) ess[u] = 0.0;
        return;
    }
    const double f = m > -INFINITY ? exp(m - W) : 0.0;
    s1 *= f;
    s2 *= f * f;
#pragma unroll
    for (int sh = 1; sh < 64; sh <<= 1) {  // a + b = b + a: every lane ends with the same sums
        s1 += __shfl_xor(s1, sh, 64);
        s2 += __shfl_xor(s2, sh, 64);
    }
    if (lane == 0) ess[u] = s1 * s1 / s2;
}

// C-phase header (doubles): [0] flags word (bit 0: NaN or +inf log-weight),
// [1] done word, [2] index found, [3] ESS there.
constexpr int kDoneWord = 2;  // the done word as an unsigned index (byte 8)

// eq. (ESS_rule): the first u in [0, nb) with ESS(u) < thr, or with
// s + u + 1 = T.  One workgroup.  hdr[2] = that u (-1 if none), hdr[3] = its
// ESS; the done word is set when a u is found or the NaN flag is up, which
// turns the launches of any later block into no-ops.
__global__ __launch_bounds__(256) void correct_find_kernel(const double* __restrict__ ess, int32_t nb, double thr,
                                                           int64_t s, int64_t T, double* hdr) {
    __shared__ int32_t red[4];
    unsigned* words = (unsigned*)hdr;
    if (words[kDoneWord] != 0u) return;  // the same value for the whole workgroup
    // thread t tests u = t, t + 256, ... with eight loads in flight (a block has
    // at most 2048 rows: one round); the first hit is its smallest u
    constexpr int kAhead = 8;
    int32_t first = INT32_MAX;
    for (int32_t u0 = threadIdx.x; u0 < nb && first == INT32_MAX; u0 += 256 * kAhead) {
        double e[kAhead];
#pragma unroll
        for (int k = 0; k < kAhead; ++k) e[k] = u0 + 256 * k < nb ? ess[u0 + 256 * k] : INFINITY;
#pragma unroll
        for (int k = 0; k < kAhead; ++k) {
            const int32_t u = u0 + 256 * k;
            if (first == INT32_MAX && u < nb && (e[k] < thr || s + u + 1 == T)) first = u;
        }
    }
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) first = min(first, __shfl_xor(first, sh, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = first;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int32_t f = min(min(red[0], red[1]), min(red[2], red[3]));
        hdr[2] = f == INT32_MAX ? -1.0 : (double)f;
        hdr[3] = f == INT32_MAX ? 0.0 : ess[f];
        if (f != INT32_MAX || (words[0] & 1u)) words[kDoneWord] = 1u;
    }
}

// Running log-weight at observation u of the block for every particle, in
// the order of correct_scan_ess_kernel.  Writes log_w (may alias carry) and
// adds it to ll if add_ll.
__global__ void correct_column_kernel(const void* __restrict__ lw, int f32, const double* carry,
                                      const double* __restrict__ tot, int64_t P, int32_t nb, int32_t off,
                                      int32_t u, double* log_w, double* __restrict__ ll, int add_ll) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int32_t r = u + off;
    const int32_t q = r / kScanChunk, w = (r % kScanChunk) / kScanRun;
    const int32_t c0 = q * kScanChunk - off;
    double acc = chunk_base(carry, tot, P, p, q);
    for (int32_t w2 = 0; w2 < w; ++w2) acc += run_sum(lw, f32, P, p, c0 + w2 * kScanRun, nb);
    for (int32_t v = c0 + w * kScanRun; v <= u; ++v)
        if (v >= 0) acc += perobs_value(lw, f32, (int64_t)v * P + p);
    log_w[p] = acc;
    if (add_ll) ll[p] += acc;
}

__global__ void add_kernel(double* __restrict__ a, const double* __restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] += b[i];
}

// ------------------------------------------------------------------ logML
// logml_j += log(N^-1 sum_n exp(log_w_jn)); flags |= 1 if a group is all -inf,
// |= 2 if a log-weight is NaN or +inf.  One block per group.
__global__ void logml_group_kernel(const double* __restrict__ log_w, int32_t N,
                                   double* __restrict__ logml_j, unsigned* flags) {
    __shared__ double red[256];
    const double* lw = log_w + (int64_t)blockIdx.x * N;
    // thread t takes n = t, t + 256, ... in that order, four loads in flight
    constexpr int kAhead = 4;
    double m = -INFINITY;
    bool bad = false;
    for (int32_t n0 = threadIdx.x; n0 < N; n0 += 256 * kAhead) {
        double v[kAhead];
#pragma unroll
        for (int k = 0; k < kAhead; ++k) v[k] = n0 + 256 * k < N ? lw[n0 + 256 * k] : -INFINITY;
#pragma unroll
        for (int k = 0; k < kAhead; ++k) {
            bad |= isnan(v[k]) || v[k] == INFINITY;
            m = fmax(m, v[k]);
        }
    }
    if (bad) atomicOr(flags, 2u);
    // any thread's bad weight voids the whole group's increment
    const bool any_bad = __syncthreads_or(bad) != 0;
    m = block_max256(m, red);
    double s = 0.0;
    if (m > -INFINITY && !any_bad) {
        for (int32_t n0 = threadIdx.x; n0 < N; n0 += 256 * kAhead) {
            double v[kAhead];
#pragma unroll
            for (int k = 0; k < kAhead; ++k) v[k] = n0 + 256 * k < N ? lw[n0 + 256 * k] : -INFINITY;
#pragma unroll
            for (int k = 0; k < kAhead; ++k)
                if (n0 + 256 * k < N) s += exp(v[k] - m);
        }
    }
    s = block_sum256(s, red);
    if (threadIdx.x == 0) {
        if (m > -INFINITY && !any_bad) logml_j[blockIdx.x] += m + log(s) - log((double)N);
        else if (!(m > -INFINITY)) atomicOr(flags, 1u);
    }
}

// logml = log(J^-1 sum_j exp(logml_j)); nse = sd_j(exp(logml_j - logml)) / sqrt(J).
__global__ void logml_total_kernel(const double* __restrict__ logml_j, int32_t J, double* out) {
    __shared__ double red[256];
    double m = -INFINITY;
    for (int32_t j = threadIdx.x; j < J; j += 256) m = fmax(m, logml_j[j]);
    m = block_max256(m, red);
    double s = 0.0;
    for (int32_t j = threadIdx.x; j < J; j += 256) s += exp(logml_j[j] - m);
    s = block_sum256(s, red);
    const double L = m + log(s / (double)J);
    double v = 0.0;
    for (int32_t j = threadIdx.x; j < J; j += 256) {
        const double r = exp(logml_j[j] - L) - 1.0;
        v += r * r;
    }
    v = block_sum256(v, red);
    if (threadIdx.x == 0) {
        out[0] = L;
        out[1] = J > 1 ? sqrt(v / (double)(J - 1) / (double)J) : 0.0;
    }
}

// ------------------------------------------------------------------ S phase
constexpr int kResThreads = 1024;
constexpr int kResMaxN = 4096;
constexpr int kResPer = kResMaxN / kResThreads;  // elements per thread

// Inclusive block scan of one uint64 per thread (1024 threads).
__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int off) {
    const unsigned lo = __shfl_up((unsigned)v, off, 64);
    const unsigned hi = __shfl_up((unsigned)(v >> 32), off, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive scan over the block's kResThreads threads (exact integers, so the
// grouping does not matter): a shuffle scan inside each wave, a scan of the
// 16 wave totals by wave 0, two barriers.  tmp holds at least 32 entries.
constexpr int kResWaves = kResThreads / 64;
__device__ uint64_t block_scan_u64(uint64_t v, uint64_t* tmp) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint64_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t y = shfl_up_u64(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) tmp[wv] = x;
    __syncthreads();
    if (wv == 0) {
        uint64_t s = lane < kResWaves ? tmp[lane] : 0;
#pragma unroll
        for (int off = 1; off < kResWaves; off <<= 1) {
            const uint64_t y = shfl_up_u64(s, off);
            if (lane >= off) s += y;
        }
        if (lane < kResWaves) tmp[kResWaves + lane] = s;
    }
    __syncthreads();
    const uint64_t r = x + (wv > 0 ? tmp[kResWaves + wv - 1] : 0);
    __syncthreads();  // tmp is free for the next call
    return r;
}

// floor(U * S / 2^53) for U < 2^53 and S < 2^64.
__device__ __forceinline__ uint64_t scaled_target(uint64_t U, uint64_t S) {
    const uint64_t hi = __umul64hi(U, S);
    const uint64_t lo = U * S;
    return (hi << 11) | (lo >> 53);
}

// Smallest n in [0, N) with cum[n] > target (cum inclusive, nondecreasing).
__device__ __forceinline__ int32_t search_cum(const uint64_t* cum, int32_t N, uint64_t target) {
    int32_t lo = 0, hi = N - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (cum[mid] > target) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// One block per group.  When log_w is non-null the integer weights are
// W_n = floor(exp(log_w_n - max log_w) 2^40); otherwise they are read from W.
// flags |= 1 degenerate group, |= 2 NaN/+inf log-weight, |= 4 bad W total.
__global__ __launch_bounds__(kResThreads) void resample_kernel(
    const double* __restrict__ log_w, const uint64_t* __restrict__ Win, int32_t N, int32_t scheme,
    const uint64_t* __restrict__ u53, int32_t* __restrict__ ancestor, unsigned* flags) {
    __shared__ uint64_t cum[kResMaxN];
    __shared__ uint64_t tmp[kResThreads];
    __shared__ int bad_s;
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * N;
    int32_t* anc = ancestor + base;
    const uint64_t* U = u53 + base;
    if (t == 0) bad_s = 0;
    __syncthreads();

    // ---- integer weights ----
    uint64_t w[kResPer];
    if (log_w != nullptr) {
        const double* lw = log_w + base;
        double m = -INFINITY;
        bool bad = false;
        for (int32_t n = t; n < N; n += kResThreads) {
            bad |= isnan(lw[n]) || lw[n] == INFINITY;
            m = fmax(m, lw[n]);
        }
        if (bad) atomicOr(flags, 2u);
        // a bad weight anywhere in the group sends it down the identity path
        const bool any_bad = __syncthreads_or(bad) != 0;
        // block max over the 1024 threads (fmax is exact: any order gives it)
        __shared__ double dred[kResWaves];
#pragma unroll
        for (int sh = 32; sh > 0; sh >>= 1) m = fmax(m, __shfl_xor(m, sh, 64));
        if ((t & 63) == 0) dred[t >> 6] = m;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kResWaves; ++q) m = fmax(m, dred[q]);
        __syncthreads();
        if (!(m > -INFINITY) || any_bad) {
            if (t == 0) atomicOr(flags, 1u);
            if (t == 0) bad_s = 1;
        }
        // weights only from a finite group maximum and no NaN / +inf anywhere
        // (exp of those would be converted to an integer below)
        const bool ok = m > -INFINITY && !any_bad;
#pragma unroll
        for (int q = 0; q < kResPer; ++q) {
            const int32_t n = t * kResPer + q;
            w[q] = (n < N && ok) ? (uint64_t)floor(exp(lw[n] - m) * 0x1p40) : 0;
        }
    } else {
#pragma unroll
        for (int q = 0; q < kResPer; ++q) {
            const int32_t n = t * kResPer + q;
            w[q] = n < N ? Win[base + n] : 0;
        }
    }
    __syncthreads();

    // ---- cumulative weights: each thread owns elements t*4 .. t*4+3 ----
    uint64_t local = 0;
#pragma unroll
    for (int q = 0; q < kResPer; ++q) local += w[q];
    uint64_t incl = block_scan_u64(local, tmp);
    uint64_t run = incl - local;
#pragma unroll
    for (int q = 0; q < kResPer; ++q) {
        run += w[q];
        const int32_t n = t * kResPer + q;
        if (n < N) cum[n] = run;
    }
    __syncthreads();
    const uint64_t S = cum[N - 1];
    if (S == 0 || S >= (uint64_t(1) << 52)) {
        if (t == 0) {
            atomicOr(flags, 4u);
            bad_s = 1;
        }
    }
    __syncthreads();
    if (bad_s) {
        // leave a valid (identity) ancestry so later gathers stay in bounds
        for (int32_t n = t; n < N; n += kResThreads) anc[n] = (int32_t)(base + n);
        return;
    }

    if (scheme == SPS_MULTINOMIAL) {
        for (int32_t i = t; i < N; i += kResThreads)
            anc[i] = (int32_t)(base + search_cum(cum, N, scaled_target(U[i], S)));
        return;
    }

    // ---- residual: deterministic copies, then multinomial on the remainders ----
    uint64_t cpy[kResPer];
    uint64_t ncpy = 0;
#pragma unroll
    for (int q = 0; q < kResPer; ++q) {
        cpy[q] = ((uint64_t)N * w[q]) / S;
        ncpy += cpy[q];
    }
    const uint64_t cincl = block_scan_u64(ncpy, tmp);
    uint64_t pos = cincl - ncpy;
    __shared__ uint64_t total_copies;
    if (t == kResThreads - 1) total_copies = cincl;
#pragma unroll
    for (int q = 0; q < kResPer; ++q) {
        const int32_t n = t * kResPer + q;
        for (uint64_t r = 0; r < cpy[q]; ++r) anc[pos + r] = (int32_t)(base + n);
        pos += cpy[q];
    }
    // residual weights N W_n - copies_n S, total R S < 2^64
    uint64_t rw[kResPer];
    uint64_t rloc = 0;
#pragma unroll
    for (int q = 0; q < kResPer; ++q) {
        rw[q] = (uint64_t)N * w[q] - cpy[q] * S;
        rloc += rw[q];
    }
    const uint64_t rincl = block_scan_u64(rloc, tmp);
    uint64_t rrun = rincl - rloc;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kResPer; ++q) {
        rrun += rw[q];
        const int32_t n = t * kResPer + q;
        if (n < N) cum[n] = rrun;
    }
    __syncthreads();
    const int32_t done = (int32_t)total_copies;
    const int32_t R = N - done;
    const uint64_t RS = cum[N - 1];
    for (int32_t i = t; i < R; i += kResThreads)
        anc[done + i] = (int32_t)(base + search_cum(cum, N, scaled_target(U[i], RS)));
}

__global__ void gather_kernel(const int32_t* __restrict__ anc, int64_t P, int32_t d,
                              const double* __restrict__ th_in, double* __restrict__ th_out,
                              const double* __restrict__ ll_in, double* __restrict__ ll_out,
                              const double* __restrict__ g_in, double* __restrict__ g_out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * d) return;
    const int64_t p = e / d;
    const int32_t i = (int32_t)(e % d);
    const int64_t a = anc[p];
    if (th_in) th_out[e] = th_in[a * d + i];
    if (g_in) g_out[e] = g_in[a * d + i];
    if (ll_in && i == 0) ll_out[p] = ll_in[a];
}

// ------------------------------------------------------------------ moments
// The monitored functions of a particle: theta itself, then theta_c' xbar
// for c = 0 .. C-2 (products in order i = 0 .. k-1).  One wave per particle:
// the wave copies theta's row, lanes 0 .. C-2 form the inner products (a flat
// index over P (d + C - 1) elements would need a 64-bit division per element,
// and waves holding an inner-product lane would wait on its 50-load chain).
__global__ __launch_bounds__(256) void monitor_kernel(const double* __restrict__ theta, int64_t P, int32_t k,
                                                      int32_t C, const double* __restrict__ xbar,
                                                      double* __restrict__ g) {
    const int32_t d = k * (C - 1), m = d + C - 1;
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= P) return;
    const double* th = theta + p * d;
    double* gp = g + p * m;
    for (int32_t f = lane; f < d; f += 64) gp[f] = th[f];
    for (int32_t c = lane; c < C - 1; c += 64) {
        double s = 0.0;
#pragma unroll 16
        for (int32_t i = 0; i < k; ++i) s += th[c * k + i] * xbar[i];  // loads issued 16 ahead
        gp[d + c] = s;
    }
}

// Sums of (g - g_0f) and its square over sub-blocks of kMomSub particles of
// a group, shifted by the first particle's value for stability:
// part[((j * nsub + s) * m + f) * 2 + {0, 1}].  Block (function tile of 64,
// group j, sub-block s); thread (f, lane q of 4) adds particles
// s kMomSub + q, + 4, ... in order, then the 4 lanes combine in order.
constexpr int kMomSub = 64;
__global__ __launch_bounds__(256) void moments_group_kernel(const double* __restrict__ g, int32_t N, int32_t m,
                                                            int32_t nsub, double* __restrict__ part) {
    __shared__ double r1[4][64], r2[4][64];
    const int fl = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int32_t f = blockIdx.x * 64 + fl;
    const int32_t j = blockIdx.y, sb = blockIdx.z;
    double s1 = 0.0, s2 = 0.0;
    if (f < m) {
        const double c = g[f];
        const int32_t n1 = min(N, (sb + 1) * kMomSub);
        for (int32_t n = sb * kMomSub + q; n < n1; n += 4) {
            const double v = g[((int64_t)j * N + n) * m + f] - c;
            s1 += v;
            s2 += v * v;
        }
    }
    r1[q][fl] = s1;
    r2[q][fl] = s2;
    __syncthreads();
    if (q == 0 && f < m) {
        const double a = ((r1[0][fl] + r1[1][fl]) + r1[2][fl]) + r1[3][fl];
        const double b = ((r2[0][fl] + r2[1][fl]) + r2[2][fl]) + r2[3][fl];
        part[(((int64_t)j * nsub + sb) * m + f) * 2 + 0] = a;
        part[(((int64_t)j * nsub + sb) * m + f) * 2 + 1] = b;
    }
}

// out[f] = mean, out[m+f] = sd, out[2m+f] = NSE, out[3m+f] = RNE.  One wave
// per function: lane l takes groups l, l + 64, ... (each group's sub-block
// sums added in order), then fixed butterflies combine the lanes.
__global__ __launch_bounds__(64) void moments_final_kernel(const double* __restrict__ g,
                                                           const double* __restrict__ part, int32_t J,
                                                           int32_t N, int32_t m, int32_t nsub,
                                                           double* __restrict__ out) {
    const int32_t f = blockIdx.x;
    const int lane = threadIdx.x;
    const double c = g[f];
    auto gsum = [&](int32_t j, int e) {  // group j's sum over its sub-blocks, in order
        double a = 0.0;
        for (int32_t sb = 0; sb < nsub; ++sb) a += part[(((int64_t)j * nsub + sb) * m + f) * 2 + e];
        return a;
    };
    double sg = 0.0;
    for (int32_t j = lane; j < J; j += 64) sg += gsum(j, 0) / (double)N;
    const double gb = wave_sum64(sg) / (double)J;  // grand mean minus c
    double vb = 0.0, ss = 0.0;
    for (int32_t j = lane; j < J; j += 64) {
        const double gj = gsum(j, 0) / (double)N;
        vb += (gj - gb) * (gj - gb);
        ss += gsum(j, 1);
    }
    vb = wave_sum64(vb);
    ss = wave_sum64(ss);
    if (lane != 0) return;
    const double P = (double)J * (double)N;
    const double vhat = J > 1 ? (double)N / (double)(J - 1) * vb : 0.0;
    double var = ss / P - gb * gb;
    var = var > 0.0 ? var : 0.0;
    out[f] = c + gb;
    out[m + f] = sqrt(var);
    out[2 * m + f] = sqrt(vhat / P);
    out[3 * m + f] = vhat > 0.0 ? var / vhat : INFINITY;
}

static int read_flags(sps_ctx* c, unsigned* dflags, unsigned* out) {
    const void* h = nullptr;
    SPS_CHECK(readback(c, dflags, sizeof(unsigned), &h));
    *out = *(const unsigned*)h;
    return SPS_OK;
}

static int zero_flags(sps_ctx* c) {
    SPS_CHECK(ensure(c, c->small, 4096, "small"));
    SPS_CHECK(ensure_host(c, c->hostbuf, 4096));
    SPS_CHECK(fill(c, (double*)c->small.p, 8, 0.0));
    return SPS_OK;
}

}  // namespace sps

using namespace sps;

extern "C" int sps_random(sps_ctx* c, int kind, uint64_t seed, uint64_t stream, int64_t count,
                          int32_t d, void* out) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (kind < 0 || kind > 2 || count < 0 || (kind == 2 && d < 1) || (!out && count > 0))
        return fail(c, SPS_ERR_ARG, "sps_random: bad arguments");
    return random_fill(c, kind, seed, stream, count, d, out);
}

// theta[p][i] = mean[i]
__global__ void rows_kernel(double* __restrict__ theta, const double* __restrict__ mean, int64_t P, int32_t d) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * d) return;
    theta[e] = mean[(int32_t)(e % d)];
}

extern "C" int sps_init_prior(sps_ctx* c, double* theta, int64_t P, uint64_t seed, uint64_t stream) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (!c->has_prior) return fail(c, SPS_ERR_STATE, "sps_init_prior: call sps_set_prior first");
    if (P < 0 || (!theta && P > 0)) return fail(c, SPS_ERR_ARG, "sps_init_prior: bad arguments");
    const int64_t n = P * c->d;
    if (n == 0) return SPS_OK;
    if (c->prior_full) {
        // theta = mean + L z, z the same Philox normals as in the independent case
        SPS_CHECK(ensure(c, c->z, sizeof(double) * n, "normals"));
        SPS_CHECK(random_fill(c, 2, seed, stream, P, c->d, c->z.p));
        rows_kernel<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(theta, c->prior_mean, P, c->d);
        SPS_CHECK(launched(c, "rows_kernel"));
        return gemm_abt(c, (const double*)c->z.p, c->prior_L, theta, theta, P, c->d, 1.0);
    }
    init_prior_kernel<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(
        theta, P, c->d, c->prior_mean, c->prior_isd, seed, stream);
    return launched(c, "init_prior_kernel");
}
extern "C" int sps_correct(sps_ctx* c, const double* theta, double* ll, int32_t J, int32_t N,
                           int64_t s0, double ess_frac, int prec, double* log_w, int64_t* t_end,
                           double* ess_end) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (!c->has_data) return fail(c, SPS_ERR_STATE, "sps_correct: call sps_set_data first");
    if (J < 1 || N < 1 || !theta || !ll || !log_w || !t_end)
        return fail(c, SPS_ERR_ARG, "sps_correct: bad arguments");
    if (s0 < 0 || s0 >= c->T) return fail(c, SPS_ERR_ARG, "sps_correct: s0=%lld outside [0, T)", (long long)s0);
    if (!(ess_frac > 0.0 && ess_frac < 1.0)) return fail(c, SPS_ERR_ARG, "sps_correct: ess_frac outside (0, 1)");
    if (prec != SPS_FP64 && prec != SPS_FP32 && prec != SPS_BF16X3)
        return fail(c, SPS_ERR_ARG, "sps_correct: unknown precision %d", prec);
    const int64_t P = (int64_t)J * N;
    // Observations per block: growing fourfold from 64 up to 2048, the block
    // buffer (P x block FP64) capped at 256 MiB.  A block's launches and
    // read-back cost about as much as a few hundred observations of
    // per-observation work, so fewer, larger blocks win once a cycle outlasts
    // the first.
    const int32_t kMaxBlock =
        (int32_t)std::max<int64_t>(kScanChunk, std::min<int64_t>(2048, (int64_t(32) << 20) / P / kScanChunk * kScanChunk));
    const int32_t nchmax = (kMaxBlock + 2 * kScanChunk - 1) / kScanChunk;  // chunks of a block at any alignment
    const int64_t npb = (P + 63) / 64;  // scan workgroups per chunk
    constexpr int kHdr = 8;             // doubles before ess: [0] = flags word
    SPS_CHECK(ensure(c, c->corr_lw, sizeof(double) * P * kMaxBlock, "C-phase block"));
    SPS_CHECK(ensure(c, c->corr_red,
                     sizeof(double) * (kHdr + kMaxBlock + (size_t)nchmax * P + (size_t)kMaxBlock * npb * 3 + P),
                     "C-phase ESS"));
    void* lwblk = c->corr_lw.p;  // per-observation terms: FP64, or FP32 base 2 (reduced precision)
    const int f32 = prec != SPS_FP64;
    double* hdr = (double*)c->corr_red.p;
    unsigned* flags = (unsigned*)hdr;  // sticky: the first NaN / +inf ends the call
    double* ess = hdr + kHdr;
    double* tot = ess + kMaxBlock;
    double* epart = tot + (size_t)nchmax * P;
    double* spare = epart + (size_t)kMaxBlock * npb * 3;  // the other carry column
    const unsigned pg = (unsigned)((P + 255) / 256);
    const double thr = ess_frac * (double)P;

    SPS_CHECK(fill(c, hdr, kHdr, 0.0));
    const unsigned* done = (const unsigned*)hdr + kDoneWord;
    // Blocks of observations grow fourfold.  The host queues block i + 1
    // before it reads block i's outcome; a block queued after the crossing
    // (or after a NaN) finds the done word set and its launches do nothing.
    // The running log-weights carried from one block to the next alternate
    // between log_w and spare; the final column is written into log_w.
    struct Block {
        int64_t s;
        int32_t nb, off;
        double* carry;
        double* next;
        PubTicket tk;
    };
    auto launch_block = [&](Block& b) -> int {
        const unsigned nch = (unsigned)((b.nb + b.off + kScanChunk - 1) / kScanChunk);
        SPS_CHECK(loglik_perobs(c, theta, P, b.s, b.s + b.nb, prec, lwblk, tot, done));
        correct_scan_ess_kernel<<<dim3((unsigned)npb, nch), 256, 0, c->stream>>>(lwblk, f32, b.carry, tot, P, b.nb,
                                                                                 b.off, b.next, epart, flags, done);
        SPS_CHECK(launched(c, "correct_scan_ess_kernel"));
        correct_ess_combine_kernel<<<(unsigned)((b.nb + 3) / 4), 256, 0, c->stream>>>(epart, (int32_t)npb, b.nb,
                                                                                      ess, done);
        SPS_CHECK(launched(c, "correct_ess_combine_kernel"));
        correct_find_kernel<<<1, 256, 0, c->stream>>>(ess, b.nb, thr, b.s, c->T, hdr);
        SPS_CHECK(launched(c, "correct_find_kernel"));
        return publish_async(c, hdr, 4 * sizeof(double), &b.tk);
    };
    auto make_block = [&](int64_t s, int32_t B, double* carry, double* next) {
        Block b{};
        b.s = s;
        b.nb = (int32_t)std::min<int64_t>(B, c->T - s);
        b.off = (int32_t)(s & (kScanChunk - 1));
        b.carry = carry;
        b.next = next;
        return b;
    };
    int32_t B = std::min<int32_t>(64, kMaxBlock);
    Block cur = make_block(s0, B, nullptr, spare);  // w = 1 after observation s0
    SPS_CHECK(launch_block(cur));
    for (;;) {
        const int64_t s1 = cur.s + cur.nb;
        const int32_t B1 = std::min(4 * B, kMaxBlock);
        Block nxt{};
        const bool ahead = s1 < c->T;
        if (ahead) {
            nxt = make_block(s1, B1, cur.next, cur.carry ? cur.carry : log_w);
            SPS_CHECK(launch_block(nxt));
        }
        const void* hv = nullptr;
        SPS_CHECK(publish_wait(c, cur.tk, &hv));
        const double* h = (const double*)hv;
        if (*(const unsigned*)h & 1u)
            return fail(c, SPS_ERR_NONFINITE, "sps_correct: NaN or +inf log-weight before observation %lld",
                        (long long)(cur.s + cur.nb));
        const int64_t idx = (int64_t)h[2];
        if (idx >= 0) {
            correct_column_kernel<<<pg, 256, 0, c->stream>>>(lwblk, f32, cur.carry, tot, P, cur.nb, cur.off,
                                                             (int32_t)idx, log_w, ll, 1);
            SPS_CHECK(launched(c, "correct_column_kernel"));
            *t_end = cur.s + idx + 1;
            if (ess_end) *ess_end = h[3];
            return SPS_OK;
        }
        if (!ahead) return fail(c, SPS_ERR_STATE, "sps_correct: no stopping point before T");  // unreachable
        cur = nxt;
        B = B1;
    }
}

extern "C" int sps_correct_fixed(sps_ctx* c, const double* theta, double* ll, int32_t J, int32_t N,
                                 int64_t s0, int64_t s1, int prec, double* log_w) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (!c->has_data) return fail(c, SPS_ERR_STATE, "sps_correct_fixed: call sps_set_data first");
    if (J < 1 || N < 1 || !theta || !ll || !log_w) return fail(c, SPS_ERR_ARG, "sps_correct_fixed: bad arguments");
    if (s0 < 0 || s1 <= s0 || s1 > c->T)
        return fail(c, SPS_ERR_ARG, "sps_correct_fixed: need 0 <= s0 < s1 <= T");
    if (prec != SPS_FP64 && prec != SPS_FP32 && prec != SPS_BF16X3)
        return fail(c, SPS_ERR_ARG, "sps_correct_fixed: unknown precision %d", prec);
    const int64_t P = (int64_t)J * N;
    SPS_CHECK(loglik_launch(c, theta, P, s0, s1, prec, log_w, nullptr));
    add_kernel<<<(unsigned)((P + 255) / 256), 256, 0, c->stream>>>(ll, log_w, P);
    return launched(c, "add_kernel");
}

extern "C" int sps_logml(sps_ctx* c, const double* log_w, int32_t J, int32_t N, double* logml_j,
                         double* logml, double* nse) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (J < 1 || N < 1 || !log_w || !logml_j) return fail(c, SPS_ERR_ARG, "sps_logml: bad arguments");
    SPS_CHECK(zero_flags(c));
    unsigned* flags = (unsigned*)c->small.p;
    double* res = (double*)c->small.p + 2;
    logml_group_kernel<<<J, 256, 0, c->stream>>>(log_w, N, logml_j, flags);
    SPS_CHECK(launched(c, "logml_group_kernel"));
    logml_total_kernel<<<1, 256, 0, c->stream>>>(logml_j, J, res);
    SPS_CHECK(launched(c, "logml_total_kernel"));
    const void* hv = nullptr;
    SPS_CHECK(readback(c, c->small.p, 4 * sizeof(double), &hv));
    const double* h = (const double*)hv;
    const unsigned f = *(const unsigned*)h;
    if (f & 2u) return fail(c, SPS_ERR_NONFINITE, "sps_logml: NaN or +inf log-weight");
    if (f & 1u) return fail(c, SPS_ERR_DEGENERATE, "sps_logml: a group has every weight zero");
    if (logml) *logml = h[2];
    if (nse) *nse = h[3];
    return SPS_OK;
}

static int resample_common(sps_ctx* c, const double* log_w, const uint64_t* W, int32_t J, int32_t N,
                           int scheme, const uint64_t* u53, int32_t* ancestor, const char* who) {
    if (J < 1 || N < 1 || N > kResMaxN || !ancestor || !u53)
        return fail(c, SPS_ERR_ARG, "%s: bad arguments (J>=1, 1<=N<=%d, non-null outputs)", who, kResMaxN);
    if (scheme != SPS_RESIDUAL && scheme != SPS_MULTINOMIAL)
        return fail(c, SPS_ERR_ARG, "%s: unknown scheme %d", who, scheme);
    SPS_CHECK(zero_flags(c));
    unsigned* flags = (unsigned*)c->small.p;
    resample_kernel<<<J, kResThreads, 0, c->stream>>>(log_w, W, N, scheme, u53, ancestor, flags);
    SPS_CHECK(launched(c, "resample_kernel"));
    unsigned f = 0;
    SPS_CHECK(read_flags(c, flags, &f));
    if (f & 2u) return fail(c, SPS_ERR_NONFINITE, "%s: NaN or +inf log-weight", who);
    if (f & 1u) return fail(c, SPS_ERR_DEGENERATE, "%s: a group has every weight zero", who);
    if (f & 4u) return fail(c, SPS_ERR_ARG, "%s: a group's integer weight total is 0 or >= 2^52", who);
    return SPS_OK;
}

extern "C" int sps_resample(sps_ctx* c, const double* log_w, int32_t J, int32_t N, int scheme,
                            const uint64_t* u53, uint64_t seed, uint64_t stream, int32_t* ancestor,
                            const double* theta_in, double* theta_out, const double* ll_in,
                            double* ll_out, const double* grad_in, double* grad_out) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (!log_w) return fail(c, SPS_ERR_ARG, "sps_resample: null log_w");
    if ((theta_in != nullptr) != (theta_out != nullptr) || (ll_in != nullptr) != (ll_out != nullptr) ||
        (grad_in != nullptr) != (grad_out != nullptr))
        return fail(c, SPS_ERR_ARG, "sps_resample: gather source and destination must both be given");
    if ((theta_in && theta_in == theta_out) || (ll_in && ll_in == ll_out) || (grad_in && grad_in == grad_out))
        return fail(c, SPS_ERR_ARG, "sps_resample: gather destination aliases its source");
    if ((theta_in || grad_in) && !c->has_data)
        return fail(c, SPS_ERR_STATE, "sps_resample: gathering theta needs sps_set_data (for d)");
    const int64_t P = (int64_t)J * N;
    if (!u53 && P > 0) {
        SPS_CHECK(ensure(c, c->u53, sizeof(uint64_t) * P, "resampling integers"));
        SPS_CHECK(random_fill(c, 0, seed, stream, P, 1, c->u53.p));
        u53 = (const uint64_t*)c->u53.p;
    }
    SPS_CHECK(resample_common(c, log_w, nullptr, J, N, scheme, u53, ancestor, "sps_resample"));
    if (theta_in || ll_in || grad_in) {
        const int32_t d = (theta_in || grad_in) ? c->d : 1;
        const int64_t n = P * d;
        gather_kernel<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(
            ancestor, P, d, theta_in, theta_out, ll_in, ll_out, grad_in, grad_out);
        SPS_CHECK(launched(c, "gather_kernel"));
    }
    return SPS_OK;
}

extern "C" int sps_resample_fixed(sps_ctx* c, const uint64_t* W, int32_t J, int32_t N, int scheme,
                                const uint64_t* u53, int32_t* ancestor) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (!W) return fail(c, SPS_ERR_ARG, "sps_resample_fixed: null W");
    return resample_common(c, nullptr, W, J, N, scheme, u53, ancestor, "sps_resample_fixed");
}

namespace sps {

int monitor_launch(sps_ctx* c, const double* theta, int64_t P, double* g) {
    const int64_t n = P * (c->d + c->C - 1);
    if (n == 0) return SPS_OK;
    monitor_kernel<<<(unsigned)((P + 3) / 4), 256, 0, c->stream>>>(theta, P, c->k, c->C, c->xbar, g);
    return launched(c, "monitor_kernel");
}

int moments_launch(sps_ctx* c, const double* g, int32_t J, int32_t N, int32_t m, double** out) {
    const int32_t nsub = (N + kMomSub - 1) / kMomSub;
    SPS_CHECK(ensure(c, c->gstat, sizeof(double) * ((size_t)J * nsub * m * 2 + 4 * (size_t)m), "moments"));
    double* part = (double*)c->gstat.p;
    double* o = part + (size_t)J * nsub * m * 2;
    moments_group_kernel<<<dim3((m + 63) / 64, J, nsub), 256, 0, c->stream>>>(g, N, m, nsub, part);
    SPS_CHECK(launched(c, "moments_group_kernel"));
    moments_final_kernel<<<m, 64, 0, c->stream>>>(g, part, J, N, m, nsub, o);
    SPS_CHECK(launched(c, "moments_final_kernel"));
    *out = o;
    return SPS_OK;
}

// dst = mean or minimum of the RNEs (mom[3m .. 4m)), lanes in a fixed order.
__global__ __launch_bounds__(64) void rne_aggregate_kernel(const double* __restrict__ mom, int32_t m, int rule,
                                                           double* __restrict__ dst) {
    const int lane = threadIdx.x;
    double s = 0.0, mn = INFINITY;
    for (int32_t f = lane; f < m; f += 64) {
        const double v = mom[3 * m + f];
        s += v;
        mn = fmin(mn, v);
    }
    s = wave_sum64(s);
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) mn = fmin(mn, __shfl_xor(mn, sh, 64));
    if (lane == 0) dst[0] = rule == 1 ? mn : s / (double)m;
}

int rne_aggregate(sps_ctx* c, const double* mom, int32_t m, int rule, double* dst) {
    rne_aggregate_kernel<<<1, 64, 0, c->stream>>>(mom, m, rule, dst);
    return launched(c, "rne_aggregate_kernel");
}

}  // namespace sps

extern "C" int sps_monitor(sps_ctx* c, const double* theta, int64_t P, double* g) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (!c->has_data) return fail(c, SPS_ERR_STATE, "sps_monitor: call sps_set_data first");
    if (P < 0 || ((!theta || !g) && P > 0)) return fail(c, SPS_ERR_ARG, "sps_monitor: bad arguments");
    return monitor_launch(c, theta, P, g);
}

extern "C" int sps_moments(sps_ctx* c, const double* g, int32_t J, int32_t N, int32_t m, double* mean,
                           double* sd, double* nse, double* rne) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (J < 1 || N < 1 || m < 1 || !g) return fail(c, SPS_ERR_ARG, "sps_moments: bad arguments");
    if (J > 65535 || (N + kMomSub - 1) / kMomSub > 65535)
        return fail(c, SPS_ERR_ARG, "sps_moments: J=%d or N=%d too large for the launch grid", J, N);
    double* out = nullptr;
    SPS_CHECK(moments_launch(c, g, J, N, m, &out));
    const void* hv = nullptr;
    SPS_CHECK(readback(c, out, sizeof(double) * 4 * m, &hv));
    const double* h = (const double*)hv;
    for (int32_t f = 0; f < m; ++f) {
        if (mean) mean[f] = h[f];
        if (sd) sd[f] = h[m + f];
        if (nse) nse[f] = h[2 * m + f];
        if (rne) rne[f] = h[3 * m + f];
    }
    return SPS_OK;
}
