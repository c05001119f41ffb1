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

constexpr unsigned kFlagNotPD = 1u;
constexpr int kSmallD = 64;  // d at or below this: the matrices of the M step fit one workgroup's LDS

// Status of an M step in the context's small buffer: the flags word at byte 0,
// the aggregate RNE at byte 16 (sps_mphase), and the accepted count split over
// kCountSlots 64-bit slots, kCountStride words apart from byte kCountOff.  One
// atomic per workgroup into a single address serialises over about a thousand
// workgroups (some 11 us at 16384 particles); spread over separate 128-byte
// lines the adds proceed in parallel.  The host sums the slots.
constexpr int kCountSlots = 28;
constexpr int kCountStride = 16;
constexpr size_t kCountOff = 512;
constexpr size_t kStatusBytes = kCountOff + (size_t)kCountSlots * kCountStride * 8;  // read back per step
static_assert(kStatusBytes <= 4096, "the status block fits the small buffer and one publish");

// Sample variance in one pass, shifted by the first particle c = theta[0]
// for stability: over each chunk of particles
//   part[chunk][a][b] = sum_p (theta_pa - c_a)(theta_pb - c_b),  a <= b,
//   psum[chunk][a]    = sum_p (theta_pa - c_a).
// 64 x 64 (a, b) tile per block on the FP64 matrix cores (16 x 16 x 4 over
// particles), particles staged in LDS 32 at a time in groups of four, laid
// out so that both the staging stores and the MFMA operand reads are free of
// bank conflicts.  Only tiles that reach the upper triangle run; the
// final kernel reads entry (min(a, b), max(a, b)), so V is exactly symmetric.
// psum comes from the diagonal tiles, summed in particle order.
constexpr int kCovK = 32;
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Optional outputs of the d > 64 contraction (gemm_abt_kernel): per particle
// p and 64-column output tile j, the sums over the tile's columns a of
// f(Base[p][a])^2 (sqb) and f(Out[p][a])^2 (sqo), at [j * P + p];
// f(x) = (x - mu_a) isd_a when mu is given, else x.  store = 0: Out itself
// is not written.
struct GemmSq {
    double* sqb = nullptr;
    double* sqo = nullptr;
    const double* mu = nullptr;
    const double* isd = nullptr;
    int store = 1;
};
// Grid: one workgroup per (chunk, upper tile), nblk in all, padded to a
// multiple of 8.  Workgroups are dealt to the 8 XCDs in turn, so workgroup g
// takes item (g % 8) * (grid / 8) + g / 8: the tiles of one chunk run on one
// XCD and share its L2, and every XCD gets the same number of items.
__global__ __launch_bounds__(256, 4) void cov_partial_kernel(const double* __restrict__ theta, int64_t P,
                                                          int32_t d, int64_t chunk, int64_t nblk,
                                                          double* __restrict__ part,
                                                          double* __restrict__ psum) {
    // [particle group of 4][pair in group][tile column][particle in pair]: a
    // wave's 16-byte stores are contiguous, and the 16 x 4 operand of one MFMA
    // is two runs of 32 consecutive doubles
    __shared__ double As[kCovK / 4][2][64][2];
    __shared__ double Bs[kCovK / 4][2][64][2];
    const int64_t item = (int64_t)(blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    if (item >= nblk) return;
    const int nt = (d + 63) / 64, ntiles = nt * (nt + 1) / 2;
    const int64_t z = item / ntiles;  // chunk
    int tx = (int)(item % ntiles), ty = 0;  // tile (tx, ty), tx <= ty, numbered ty (ty + 1) / 2 + tx
    while (tx > ty) {
        tx -= ty + 1;
        ++ty;
    }
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int m = lane & 15, kg = lane >> 4;
    const int a0 = tx * 64, b0 = ty * 64;
    const bool diag = tx == ty;
    const int64_t pbeg = z * chunk;
    const int64_t pend = std::min<int64_t>(P, pbeg + chunk);
    f64x4 acc[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[n] = f64x4{0, 0, 0, 0};
    double cs = 0.0;
    // thread t stages column t & 63 of the tile for particle groups j0 and
    // j0 + 4 (j0 = t >> 6); the next chunk is loaded into registers while this
    // chunk's MFMAs run
    constexpr int kGroups = kCovK / 4 / 4;  // groups of 4 particles per thread
    const int cc = t & 63, j0 = t >> 6;
    const int a = a0 + cc, b = b0 + cc;
    const double ca = a < d ? theta[a] : 0.0, cb = b < d ? theta[b] : 0.0;
    double va[4 * kGroups], vb[4 * kGroups];
    // reads past the chunk's last particle or the last column go to those
    // (in bounds) and are replaced by zero, so the loads need no branches
    const int ac = min(a, d - 1), bc = min(b, d - 1);
    auto load = [&](int64_t p0) __attribute__((always_inline)) {
#pragma unroll
        for (int h = 0; h < kGroups; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t p = p0 + 4 * (j0 + 4 * h) + i;
                const double* row = theta + std::min<int64_t>(p, pend - 1) * d;
                const double xa = row[ac], xb = row[bc];
                va[4 * h + i] = (p < pend && a < d) ? xa - ca : 0.0;
                vb[4 * h + i] = (p < pend && b < d) ? xb - cb : 0.0;
            }
    };
    load(pbeg);
    for (int64_t p0 = pbeg; p0 < pend; p0 += kCovK) {
#pragma unroll
        for (int h = 0; h < kGroups; ++h) {
            const int j = j0 + 4 * h;
            *reinterpret_cast<double2*>(&As[j][0][cc][0]) = double2{va[4 * h], va[4 * h + 1]};
            *reinterpret_cast<double2*>(&As[j][1][cc][0]) = double2{va[4 * h + 2], va[4 * h + 3]};
            *reinterpret_cast<double2*>(&Bs[j][0][cc][0]) = double2{vb[4 * h], vb[4 * h + 1]};
            *reinterpret_cast<double2*>(&Bs[j][1][cc][0]) = double2{vb[4 * h + 2], vb[4 * h + 3]};
        }
        __syncthreads();
        if (p0 + kCovK < pend) load(p0 + kCovK);
        if (diag && t < 64) {
#pragma unroll 8
            for (int r = 0; r < kCovK; ++r) cs += As[r >> 2][(r >> 1) & 1][t][r & 1];
        }
#pragma unroll
        for (int s = 0; s < kCovK / 4; ++s) {
            const double av = As[s][kg >> 1][16 * w + m][kg & 1];
#pragma unroll
            for (int n = 0; n < 4; ++n)
                acc[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Bs[s][kg >> 1][16 * n + m][kg & 1], acc[n], 0, 0, 0);
        }
        __syncthreads();
    }
    // element i of tile n: a = a0 + 16 w + kg + 4 i, b = b0 + 16 n + m
    double* out = part + z * d * d;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const int b = b0 + 16 * n + m;
        if (b >= d) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int a = a0 + 16 * w + kg + 4 * i;
            if (a < d && a <= b) out[(int64_t)a * d + b] = acc[n][i];
        }
    }
    if (diag && t < 64 && a0 + t < d) psum[z * d + a0 + t] = cs;
}

// Sigma = h V, V = (S - P m m') / (P - 1) with S, m the shifted sums over all
// chunks.  One wave per matrix element, lanes over chunks, butterfly sums.
// hdev (optional): h is read from device memory; stop (optional): nothing is
// written when *stop is nonzero.
__global__ __launch_bounds__(256) void cov_final_kernel(const double* __restrict__ part,
                                                        const double* __restrict__ psum, int32_t nchunk,
                                                        int32_t d, int64_t P, double h,
                                                        double* __restrict__ V, const double* hdev,
                                                        const unsigned* stop) {
    if (stop && *stop) return;  // the same value for the whole grid
    if (hdev) h = *hdev;
    const int lane = threadIdx.x & 63;
    const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= (int64_t)d * d) return;
    const int32_t a = (int32_t)(e / d), b = (int32_t)(e % d);
    const int64_t eu = a <= b ? e : (int64_t)b * d + a;  // the partials hold the upper triangle
    double s = 0.0, sa = 0.0, sb = 0.0;
    for (int32_t q = lane; q < nchunk; q += 64) {
        s += part[(int64_t)q * d * d + eu];
        sa += psum[(int64_t)q * d + a];
        sb += psum[(int64_t)q * d + b];
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        s += __shfl_xor(s, m, 64);
        sa += __shfl_xor(sa, m, 64);
        sb += __shfl_xor(sb, m, 64);
    }
    if (lane == 0) V[e] = h * ((s - sa * sb / (double)P) / (double)(P - 1));
}

// Lane l's value of v, read by every lane of the wave (two 32-bit readlanes).
__device__ inline double readlane_f64(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// d > 64: blocked Cholesky in one workgroup of 1024 threads, in place in L
// (which starts as the lower triangle of V).  Per panel of NB columns, staged
// in LDS:
//   1. one wave factors the NB x NB diagonal block with row i in lane i's
//      registers, column by column (entry (i, c) is its value minus the
//      products L_iq L_cq for q = 0 .. c-1 in that order, times 1 / L_cc, and
//      L_cc = sqrt of the pivot so reduced), other rows' L_cq read by lane;
//   2. every row below the block is solved against it, 8 columns at a time
//      (the earlier columns' products for all entries of the group in
//      parallel, then the group's own columns row by row), with the same
//      products in the same order, so each entry gets exactly the arithmetic
//      of the right-looking column sweep;
//   3. the panel is written back, rows k .. k+NB-1 of LT = L^T are written
//      from it, and the trailing lower triangle is updated with the panel's
//      rank-NB product on the FP64 matrix cores, one 16 x 16 tile per wave
//      at a time (tiles on or below the diagonal).
// A non-positive or non-finite pivot sets kFlagNotPD and stops.  Loops run
// over (row, column) thread grids, so no index is formed by a division.
template <int NB, int ROWS>
__global__ __launch_bounds__(1024) void cholesky_blocked_kernel(const double* __restrict__ V, int32_t d,
                                                                double* __restrict__ L, double* __restrict__ LT,
                                                                unsigned* flags) {
    __shared__ double Pn[ROWS][NB + 1];
    __shared__ double inv_s[NB];
    __shared__ int fail_s;
    const int t = threadIdx.x;
    const int ty32 = t >> 5, tx32 = t & 31;        // 32 x 32 grid
    const int tyn = t / NB, txn = t % NB;          // (1024 / NB) x NB grid
    constexpr int kRowsN = 1024 / NB;
    if (t == 0) fail_s = 0;
    for (int r = ty32; r < d; r += 32)
        for (int q = tx32; q < d; q += 32) L[(int64_t)r * d + q] = q <= r ? V[(int64_t)r * d + q] : 0.0;
    __syncthreads();
    for (int k = 0; k < d; k += NB) {
        const int kw = min(NB, d - k);  // panel width
        const int m = d - k;            // panel rows k .. d-1
        if (txn < kw)
            for (int i = tyn; i < m; i += kRowsN) Pn[i][txn] = L[(int64_t)(k + i) * d + k + txn];
        __syncthreads();
        if (t < 64) {  // 1. the diagonal block, row t in registers
            double r[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) r[q] = (t < kw && q < kw) ? Pn[t][q] : 0.0;
            bool fail = false;  // the same in every lane
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                if (c < kw && !fail) {
                    double x = r[c];
#pragma unroll
                    for (int q = 0; q < c; ++q) x -= r[q] * readlane_f64(r[q], c);
                    const double piv = readlane_f64(x, c);
                    if (!(piv > 0.0) || !isfinite(piv)) {
                        fail = true;
                    } else {
                        const double ljj = sqrt(piv);
                        const double inv = 1.0 / ljj;
                        r[c] = (t == c) ? ljj : x * inv;
                        if (t == 0) inv_s[c] = inv;
                    }
                }
            }
            if (fail) {
                if (t == 0) fail_s = 1;
            } else if (t < kw) {
#pragma unroll
                for (int q = 0; q < NB; ++q)
                    if (q <= t) Pn[t][q] = r[q];
            }
        }
        __syncthreads();
        if (fail_s) {
            if (t == 0) atomicOr(flags, kFlagNotPD);
            return;
        }
        // 2. rows below the block, 8 columns at a time: first every (row,
        //    column) entry of the group takes the products of the earlier
        //    groups' columns (one thread per entry), then each row finishes the
        //    group's columns in order (one thread per row)
        for (int cb = 0; cb < kw; cb += 8) {
            if (cb > 0) {
                for (int e = t; e < (m - kw) * 8; e += 1024) {
                    const int i = kw + (e >> 3), c = cb + (e & 7);
                    if (c < kw) {
                        double x = Pn[i][c];
                        for (int q = 0; q < cb; ++q) x -= Pn[i][q] * Pn[c][q];
                        Pn[i][c] = x;
                    }
                }
                __syncthreads();
            }
            for (int i = kw + t; i < m; i += 1024) {
#pragma unroll
                for (int cc = 0; cc < 8; ++cc) {
                    const int c = cb + cc;
                    if (c < kw) {
                        double x = Pn[i][c];
                        for (int q = cb; q < c; ++q) x -= Pn[i][q] * Pn[c][q];
                        Pn[i][c] = x * inv_s[c];
                    }
                }
            }
            __syncthreads();
        }
        // 3. write-back, rows of L^T, trailing update
        if (txn < kw)
            for (int i = tyn; i < m; i += kRowsN) L[(int64_t)(k + i) * d + k + txn] = i >= txn ? Pn[i][txn] : 0.0;
        for (int jj = ty32; jj < kw; jj += 32)
            for (int q = tx32; q < d; q += 32) {
                const int i = q - k;  // panel row of L entry (q, k + jj)
                LT[(int64_t)(k + jj) * d + q] = i >= jj ? Pn[i][jj] : 0.0;
            }
        // trailing tiles (bi, bc), bc <= bi, numbered bi (bi + 1) / 2 + bc; rows
        // past the panel are clamped for the reads and not written.  Lane
        // (lm, kg) supplies rows i0 + lm and c0 + lm at columns 4 s + kg;
        // element r of the result is entry (i0 + kg + 4 r, c0 + lm).
        {
            const int nb = (m - kw + 15) / 16, ntile = nb * (nb + 1) / 2;
            const int wave = t >> 6, lane = t & 63, lm = lane & 15, kg = lane >> 4;
            for (int tile = wave; tile < ntile; tile += 16) {
                int bc = tile, bi = 0;
                while (bc > bi) {
                    bc -= bi + 1;
                    ++bi;
                }
                const int i0 = kw + 16 * bi, c0 = kw + 16 * bc;
                const int ra = min(i0 + lm, m - 1), rb = min(c0 + lm, m - 1);
                f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < NB / 4; ++s)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Pn[ra][4 * s + kg], Pn[rb][4 * s + kg], acc, 0, 0, 0);
                const int c = c0 + lm;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + kg + 4 * r;
                    if (i < m && c <= i) L[(int64_t)(k + i) * d + k + c] -= acc[r];
                }
            }
        }
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
// Base may be null (treated as 0).  64 x 64 output tile per block on the FP64
// matrix cores (16 x 16 x 4): wave w takes particles 16 w .. 16 w + 15 and
// the four 16-wide output tiles; A and B are staged in LDS 32 columns at a
// time, rows padded to 33 doubles.  A lane supplies A[16 w + m][4 s + kg] and
// B[16 n + m][4 s + kg]; element i of tile n is row 16 w + kg + 4 i, column
// 16 n + m (the FP64 MFMA layout).  Grid: nblk = (particle tiles) x (output
// tiles) items, padded to a multiple of 8; workgroup g takes item
// (g % 8) * (grid / 8) + g / 8, so the output tiles of one particle tile,
// which read the same rows of A, run together on one XCD.  sq: the per-tile
// sums of squares (GemmSq), each row's over its 64 columns in tile order,
// then a butterfly over the 16 lanes that hold the columns.
constexpr int kGemmK = 32;
__global__ __launch_bounds__(256, 4) void gemm_abt_kernel(const double* __restrict__ A,
                                                       const double* __restrict__ B,
                                                       const double* Base,  // may alias Out
                                                       double* Out, int64_t P,
                                                       int32_t d, double alpha, int64_t nblk, GemmSq sq) {
    __shared__ double As[64][kGemmK + 1];
    __shared__ double Bs[64][kGemmK + 1];
    const int64_t item = (int64_t)(blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    if (item >= nblk) return;
    const int na = (d + 63) / 64;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int m = lane & 15, kg = lane >> 4;
    const int64_t p0 = item / na * 64;
    const int a0 = (int)(item % na) * 64;
    f64x4 acc[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[n] = f64x4{0, 0, 0, 0};
    // the next chunk's operands are loaded into registers while this chunk's
    // MFMAs run
    // Thread t reads rows t / 32 + 8 l of the chunk at column t % 32; reads
    // past the last row or column go to the last one (in bounds) and are
    // replaced by zero, so the loads need no branches.
    double va[64 * kGemmK / 256], vb[64 * kGemmK / 256];
    const int tr = t / kGemmK, tc = t % kGemmK;
    auto load = [&](int q0) __attribute__((always_inline)) {
        const int q = q0 + tc;
        const int qc = min(q, d - 1);
#pragma unroll
        for (int l = 0; l < 64 * kGemmK / 256; ++l) {
            const int64_t p = p0 + tr + 8 * l;
            const int a = a0 + tr + 8 * l;
            const double xa = A[std::min<int64_t>(p, P - 1) * d + qc];
            const double xb = B[(int64_t)min(a, d - 1) * d + qc];
            va[l] = (p < P && q < d) ? xa : 0.0;
            vb[l] = (a < d && q < d) ? xb : 0.0;
        }
    };
    load(0);
    for (int q0 = 0; q0 < d; q0 += kGemmK) {
#pragma unroll
        for (int l = 0; l < 64 * kGemmK / 256; ++l) {
            As[tr + 8 * l][tc] = va[l];
            Bs[tr + 8 * l][tc] = vb[l];
        }
        __syncthreads();
        if (q0 + kGemmK < d) load(q0 + kGemmK);
#pragma unroll
        for (int s = 0; s < kGemmK / 4; ++s) {
            const double av = As[16 * w + m][4 * s + kg];
#pragma unroll
            for (int n = 0; n < 4; ++n)
                acc[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Bs[16 * n + m][4 * s + kg], acc[n], 0, 0, 0);
        }
        __syncthreads();
    }
    const bool sums = sq.sqb || sq.sqo;  // the same for the whole grid
    double sb[4] = {0.0, 0.0, 0.0, 0.0}, so[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const int a = a0 + 16 * n + m;
        if (a >= d) continue;
        const double mua = sq.mu ? sq.mu[a] : 0.0, isa = sq.mu ? sq.isd[a] : 1.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t p = p0 + 16 * w + kg + 4 * i;
            if (p >= P) continue;
            const double b = Base ? Base[p * d + a] : 0.0;
            const double o = b + alpha * acc[n][i];
            if (sq.store) Out[p * d + a] = o;
            if (sums) {
                const double fb = sq.mu ? (b - mua) * isa : b;
                const double fo = sq.mu ? (o - mua) * isa : o;
                sb[i] += fb * fb;
                so[i] += fo * fo;
            }
        }
    }
    if (sums) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int x = 1; x < 16; x <<= 1) {
                sb[i] += __shfl_xor(sb[i], x, 64);
                so[i] += __shfl_xor(so[i], x, 64);
            }
        }
        if (m == 0) {
            const int64_t j = a0 / 64;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t p = p0 + 16 * w + kg + 4 * i;
                if (p >= P) continue;
                if (sq.sqb) sq.sqb[j * P + p] = sb[i];
                if (sq.sqo) sq.sqo[j * P + p] = so[i];
            }
        }
    }
}

// ---------------------------------------------------------------- d <= 64
// Partial sums of the shifted sample variance for d <= 64: one workgroup per
// chunk of particles, staged in LDS 64 particles at a time while the next 64
// are loaded into registers.  Thread (ty, tx) of a 16 x 16 grid owns the
// TILE x TILE block (a, b) = (ty TILE + i, tx TILE + j); every (a, b) and
// (b, a) run the same products in the same order (V exactly symmetric).
// zero2 (optional): the step's status block, cleared by workgroup 0 (the
// flags word and the accepted-count slots, which later kernels of the step
// update).
template <int TILE>
__global__ __launch_bounds__(256) void cov_partial_small_kernel(const double* __restrict__ theta, int64_t P,
                                                                int32_t d, int64_t chunk,
                                                                double* __restrict__ part,
                                                                double* __restrict__ psum,
                                                                unsigned long long* zero2) {
    if (zero2 != nullptr && blockIdx.x == 0) {
        if (threadIdx.x == 0) zero2[0] = 0ull;
        else if (threadIdx.x <= kCountSlots)
            zero2[kCountOff / 8 + (threadIdx.x - 1) * kCountStride] = 0ull;
    }
    constexpr int kSub = 64;
    constexpr int kW = 16 * TILE;           // covered width: 32 or 64 parameters
    constexpr int kPer = kSub * kW / 256;   // staged values per thread
    __shared__ double Xs[kSub][kW + 1];
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int64_t pbeg = (int64_t)blockIdx.x * chunk;
    const int64_t pend = std::min<int64_t>(P, pbeg + chunk);
    double pre[kPer];
    auto load = [&](int64_t p0) {
#pragma unroll
        for (int l = 0; l < kPer; ++l) {
            const int e = t + 256 * l;
            const int r = e / kW, a = e % kW;
            const int64_t p = p0 + r;
            pre[l] = (p < pend && a < d) ? theta[p * d + a] - theta[a] : 0.0;
        }
    };
    double acc[TILE][TILE] = {};
    double cs[TILE] = {};
    load(pbeg);
    for (int64_t p0 = pbeg; p0 < pend; p0 += kSub) {
        __syncthreads();  // the previous sub-chunk has been read
#pragma unroll
        for (int l = 0; l < kPer; ++l) {
            const int e = t + 256 * l;
            Xs[e / kW][e % kW] = pre[l];
        }
        __syncthreads();
        if (p0 + kSub < pend) load(p0 + kSub);
#pragma unroll 4
        for (int r = 0; r < kSub; ++r) {
            double av[TILE], bv[TILE];
#pragma unroll
            for (int i = 0; i < TILE; ++i) av[i] = Xs[r][ty * TILE + i];
#pragma unroll
            for (int j = 0; j < TILE; ++j) bv[j] = Xs[r][tx * TILE + j];
#pragma unroll
            for (int i = 0; i < TILE; ++i) {
                cs[i] += av[i];
#pragma unroll
                for (int j = 0; j < TILE; ++j) acc[i][j] += av[i] * bv[j];
            }
        }
    }
    double* out = part + (int64_t)blockIdx.x * d * d;
#pragma unroll
    for (int i = 0; i < TILE; ++i) {
        const int a = ty * TILE + i;
        if (a >= d) continue;
#pragma unroll
        for (int j = 0; j < TILE; ++j) {
            const int b = tx * TILE + j;
            if (b < d) out[(int64_t)a * d + b] = acc[i][j];
        }
        if (tx == 0) psum[(int64_t)blockIdx.x * d + a] = cs[i];
    }
}

// d <= 64: right-looking Cholesky in LDS with 256 threads, one barrier per
// column.  Column j stays unscaled in LDS: every thread forms the pivot's
// square root and reciprocal (same value), and thread (ty, tx) of a 16 x 16
// grid updates the trailing entries (j + 1 + ty + 16 a, j + 1 + tx + 16 b) on
// or below the diagonal with the scaled values A[r][j] / l_jj, A[q][j] / l_jj
// formed on the fly.  The update writes only columns above j, so no thread
// waits for the scaling; L takes the scaled columns at the end.  A
// non-positive or non-finite pivot sets kFlagNotPD.
__global__ __launch_bounds__(256) void cholesky_small_kernel(const double* __restrict__ V, int32_t d,
                                                             double* __restrict__ L, unsigned* flags) {
    __shared__ double A[kSmallD][kSmallD + 1];
    __shared__ double dl[kSmallD], di[kSmallD];
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    for (int r = ty; r < d; r += 16)
        for (int q = tx; q < d; q += 16) A[r][q] = (q <= r) ? V[r * d + q] : 0.0;
    __syncthreads();
    for (int j = 0; j < d; ++j) {
        const double piv = A[j][j];
        if (!(piv > 0.0) || !isfinite(piv)) {  // same value in every thread: uniform exit
            if (t == 0) atomicOr(flags, kFlagNotPD);
            return;
        }
        const double ljj = sqrt(piv);
        const double inv = 1.0 / ljj;
        if (t == 0) {
            dl[j] = ljj;
            di[j] = inv;
        }
        for (int r = j + 1 + ty; r < d; r += 16) {
            const double lr = A[r][j] * inv;
            for (int q = j + 1 + tx; q <= r; q += 16) A[r][q] -= lr * (A[q][j] * inv);
        }
        __syncthreads();
    }
    for (int r = ty; r < d; r += 16)
        for (int q = tx; q < d; q += 16)
            L[r * d + q] = q < r ? A[r][q] * di[q] : (q == r ? dl[q] : 0.0);
}

// d <= 64: W = L^-1 by forward substitution, one column per thread (the
// columns are independent), reciprocals of the diagonal formed once.
__global__ __launch_bounds__(64) void trinv_small_kernel(const double* __restrict__ L, int32_t d,
                                                         double* __restrict__ W, const unsigned* flags) {
    __shared__ double Ls[kSmallD][kSmallD + 1];
    __shared__ double Ws[kSmallD][kSmallD + 1];
    __shared__ double rd[kSmallD];
    if (*flags & kFlagNotPD) return;
    const int t = threadIdx.x;
    for (int r = 0; r < d; ++r)
        if (t < d) {
            Ls[r][t] = L[r * d + t];
            Ws[r][t] = 0.0;
        }
    if (t < d) rd[t] = 1.0 / L[t * d + t];
    __syncthreads();
    if (t < d) {
        for (int r = t; r < d; ++r) {
            double s = (r == t) ? 1.0 : 0.0;
            for (int q = t; q < r; ++q) s -= Ls[r][q] * Ws[q][t];
            Ws[r][t] = s * rd[r];
        }
    }
    __syncthreads();
    for (int r = 0; r < d; ++r)
        if (t < d) W[r * d + t] = Ws[r][t];
}
// d <= 64: small contractions on the FP64 matrix cores (16 x 16 x 4).  A
// workgroup takes 64 consecutive particles (a contiguous block in memory),
// wave w the tile of particles 16 w .. 16 w + 15 and every 16-wide tile of
// outputs.  Operands are staged in LDS with every load issued before the
// first store, and the result block goes back through LDS so that
// consecutive lanes write consecutive addresses.
//   GM_PLAIN:    Out = Base + alpha A B^T                     (A: P x d, B: d x d)
//   GM_MALA_FWD: u = z + L^T g(theta) / 2 -> U;  theta' = theta + L u -> Out
//   GM_MALA_REV: w = u + L^T g(theta') / 2 -> Out (Base = U; may alias Out)
// with g(x) = grad + the gradient of the independent normal prior,
// -(x - mu) / sd^2.  Since theta' - theta = L u, the MALA reverse term
// L^-1 (theta - mu(theta')) = -(u + L^T g(theta') / 2) = -w needs no inverse.
enum { GM_PLAIN = 0, GM_MALA_FWD = 1, GM_MALA_REV = 2 };
struct SmallGemm {
    const double* A;     // GM_PLAIN: P x d
    const double* B;     // GM_PLAIN: d x d
    const double* Base;  // GM_PLAIN (may be null), GM_MALA_REV: u
    double* Out;
    double* U;           // GM_MALA_FWD: u out
    const double* th;    // MALA_FWD: theta
    const double* th2;   // MALA_REV: theta'
    const double* g;     // MALA: likelihood gradient at theta (FWD) or theta' (REV)
    const double* z;     // MALA_FWD: standard normals
    const double* mu;    // prior mean and 1 / sd
    const double* isd;
    const double* L;     // lower factor of the proposal covariance
    int64_t P;
    int32_t d;
    double alpha;        // GM_PLAIN
    int32_t zgen;        // GM_PLAIN (A = z) and GM_MALA_FWD: draw z from Philox (seed, zstream)
    uint64_t seed;
    uint64_t zstream;
    int32_t gsplit;      // GM_MALA_REV: g holds gsplit slices of P x d, summed in slice order
    double* gout;        // GM_MALA_REV: receives the summed gradient (may equal g when gsplit = 1)
};
constexpr int kGemmRows = 64;
constexpr int kStagePer = kGemmRows * kSmallD / 256;  // elements of a 64 x d tile per thread

template <int MODE>
__global__ __launch_bounds__(256) void gemm_small_kernel(SmallGemm g) {
    extern __shared__ double lds[];
    const int d = g.d;
    const int ld = d + 1;
    const int NT = (d + 15) / 16;   // output tiles
    const int KS = (d + 3) / 4;     // contraction steps
    double* As = lds;               // [64][ld]: A operand, then u, then the result block
    double* Bs = lds + kGemmRows * ld;  // [d][ld]: B of the first contraction
    double* B2 = Bs + d * ld;       // [d][ld]: MALA_FWD: L
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t p0 = (int64_t)blockIdx.x * kGemmRows;
    const int64_t nA = std::min<int64_t>(kGemmRows, g.P - p0) * d;  // valid elements of the block
    const int64_t base = p0 * d;
    // element e = t + 256 l of a tile: row e / d, column e % d (updated incrementally)
    const int dr = 256 / d, dq = 256 % d;
    {
        double v0[kStagePer], v1[kStagePer];
#pragma unroll
        for (int l = 0; l < kStagePer; ++l) {
            const int64_t e = t + 256 * l;
            const bool ok = e < nA;
            if constexpr (MODE == GM_PLAIN) {
                v0[l] = (ok && !g.zgen) ? g.A[base + e] : 0.0;
            } else if constexpr (MODE == GM_MALA_FWD) {
                v0[l] = ok ? g.g[base + e] : 0.0;
                v1[l] = ok ? g.th[base + e] : 0.0;
            } else {
                double gs = 0.0;
                if (ok) {
#pragma unroll 4
                    for (int32_t q = 0; q < g.gsplit; ++q) gs += g.g[(int64_t)q * g.P * d + base + e];
                }
                v0[l] = gs;
                v1[l] = ok ? g.th2[base + e] : 0.0;
            }
        }
        int r = t / d, q = t % d;
#pragma unroll
        for (int l = 0; l < kStagePer; ++l) {
            if (r < kGemmRows) {
                if constexpr (MODE == GM_PLAIN) {
                    if (!g.zgen) As[r * ld + q] = v0[l];
                } else {
                    As[r * ld + q] = v0[l] - (v1[l] - g.mu[q]) * g.isd[q] * g.isd[q];
                    if constexpr (MODE == GM_MALA_REV) {
                        if (p0 + r < g.P) g.gout[(p0 + r) * d + q] = v0[l];
                    }
                }
            }
            r += dr;
            q += dq;
            if (q >= d) {
                q -= d;
                ++r;
            }
        }
    }
    // Drawn normals (PLAIN: the A operand; MALA_FWD: z of u = z + ...), one
    // Box-Muller pair per thread and element pair, into the A block or Zs.
    double* Zs = B2 + (MODE == GM_MALA_FWD ? d * ld : 0);  // [kGemmRows][ld], MALA_FWD only
    if constexpr (MODE != GM_MALA_REV) {
        if (g.zgen) {
            const int hd = (d + 1) / 2;
            double* dst = MODE == GM_PLAIN ? As : Zs;
            for (int e = t; e < kGemmRows * hd; e += 256) {
                const int r = e / hd, j = e % hd;
                double z0 = 0.0, z1 = 0.0;
                if (p0 + r < g.P) philox_normal_pair(g.seed, g.zstream, p0 + r, j, d, z0, z1);
                dst[r * ld + 2 * j] = z0;
                if (2 * j + 1 < d) dst[r * ld + 2 * j + 1] = z1;
            }
        }
    }
    {
        const int nB = d * d;
        double v0[kStagePer];
#pragma unroll
        for (int l = 0; l < kStagePer; ++l) {
            const int e = t + 256 * l;
            v0[l] = e < nB ? (MODE == GM_PLAIN ? g.B : g.L)[e] : 0.0;
        }
        int r = t / d, q = t % d;
#pragma unroll
        for (int l = 0; l < kStagePer; ++l) {
            if (r < d) {
                if constexpr (MODE == GM_PLAIN) {
                    Bs[r * ld + q] = v0[l];
                } else {
                    Bs[q * ld + r] = 0.5 * v0[l];  // L^T / 2
                    if constexpr (MODE == GM_MALA_FWD) B2[r * ld + q] = v0[l];
                }
            }
            r += dr;
            q += dq;
            if (q >= d) {
                q -= d;
                ++r;
            }
        }
    }
    __syncthreads();
    // A lane supplies A[16 w + m][4 s + kg] and B[16 n + m][4 s + kg]; result
    // element i of tile n sits at row 16 w + kg + 4 i, column 16 n + m.
    const int m = lane & 15, kg = lane >> 4;
    f64x4 acc[4];
    auto contract = [&](const double* Bm) {
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[n] = f64x4{0, 0, 0, 0};
        for (int s = 0; s < KS; ++s) {
            const int q = 4 * s + kg;
            const double a = q < d ? As[(16 * w + m) * ld + q] : 0.0;
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                if (n < NT) {  // uniform
                    const int an = 16 * n + m;
                    const double b = (q < d && an < d) ? Bm[an * ld + q] : 0.0;
                    acc[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[n], 0, 0, 0);
                }
            }
        }
    };
    contract(Bs);
    if constexpr (MODE == GM_MALA_FWD) {
        // u = z + acc, written out and kept in LDS as the A operand of L u
        __syncthreads();
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * w + kg + 4 * i, col = 16 * n + m;
                const int64_t p = p0 + row;
                if (n < NT && col < d) {
                    const double zz = p >= g.P ? 0.0 : (g.zgen ? Zs[row * ld + col] : g.z[p * d + col]);
                    const double u = zz + acc[n][i];
                    As[row * ld + col] = u;
                    if (p < g.P) g.U[p * d + col] = u;
                }
            }
        __syncthreads();
        contract(B2);
    }
    __syncthreads();
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = 16 * w + kg + 4 * i, col = 16 * n + m;
            if (n < NT && col < d) As[row * ld + col] = acc[n][i];
        }
    __syncthreads();
    const double* Bsrc = MODE == GM_MALA_FWD ? g.th : g.Base;
    const double al = MODE == GM_PLAIN ? g.alpha : 1.0;
    double bv[kStagePer];
#pragma unroll
    for (int l = 0; l < kStagePer; ++l) {
        const int64_t e = t + 256 * l;
        bv[l] = (Bsrc && e < nA) ? Bsrc[base + e] : 0.0;
    }
    int rr = t / d, qq = t % d;
#pragma unroll
    for (int l = 0; l < kStagePer; ++l) {
        const int64_t e = t + 256 * l;
        if (e < nA) g.Out[base + e] = bv[l] + al * As[rr * ld + qq];
        rr += dr;
        qq += dq;
        if (qq >= d) {
            qq -= d;
            ++rr;
        }
    }
}

template <int MODE>
static int gemm_small(sps_ctx* c, const SmallGemm& g) {
    constexpr int KM = MODE == GM_MALA_FWD ? 2 : 1;  // B matrices staged
    constexpr int AM = MODE == GM_MALA_FWD ? 2 : 1;  // row blocks staged (MALA_FWD: A and the normals)
    const size_t bytes = sizeof(double) * (size_t)(AM * kGemmRows + KM * g.d) * (g.d + 1);
    // the kernel's dynamic LDS limit (above the default for large d), set once per device
    constexpr int kMaxDev = 64;
    static bool attr_set[kMaxDev] = {};
    if (c->device < 0 || c->device >= kMaxDev || !attr_set[c->device]) {
        SPS_HIP(c, hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_small_kernel<MODE>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(sizeof(double) * (AM * kGemmRows + KM * kSmallD) * (kSmallD + 1))));
        if (c->device >= 0 && c->device < kMaxDev) attr_set[c->device] = true;
    }
    gemm_small_kernel<MODE><<<(unsigned)((g.P + kGemmRows - 1) / kGemmRows), 256, bytes, c->stream>>>(g);
    return launched(c, "gemm_small_kernel");
}

// gemm_abt with the optional sums of squares (d > 64 only).
static int gemm_abt_sq(sps_ctx* c, const double* A, const double* B, const double* Base, double* Out,
                       int64_t P, int32_t d, double alpha, const GemmSq* sq) {
    if (P <= 0 || d <= 0) return SPS_OK;
    if (d <= kSmallD) {
        if (sq) return fail(c, SPS_ERR_ARG, "gemm_abt: column sums need d > %d", kSmallD);
        SmallGemm g{};
        g.A = A;
        g.B = B;
        g.Base = Base;
        g.Out = Out;
        g.P = P;
        g.d = d;
        g.alpha = alpha;
        return gemm_small<GM_PLAIN>(c, g);
    }
    const int64_t nblk = (P + 63) / 64 * ((d + 63) / 64);
    gemm_abt_kernel<<<(unsigned)((nblk + 7) / 8 * 8), 256, 0, c->stream>>>(A, B, Base, Out, P, d, alpha, nblk,
                                                                           sq ? *sq : GemmSq{});
    return launched(c, "gemm_abt_kernel");
}

int gemm_abt(sps_ctx* c, const double* A, const double* B, const double* Base, double* Out,
             int64_t P, int32_t d, double alpha) {
    return gemm_abt_sq(c, A, B, Base, Out, P, d, alpha, nullptr);
}

// out[p][i] = theta[p][i] - mu[i]
__global__ void center_kernel(const double* __restrict__ theta, const double* __restrict__ mu,
                              int64_t P, int32_t d, double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * d) return;
    out[e] = theta[e] - mu[(int32_t)(e % d)];
}

int prior_whiten(sps_ctx* c, const double* theta, int64_t P, double* tmp, double* R) {
    const int32_t d = c->d;
    const int64_t n = P * d;
    if (n <= 0) return SPS_OK;
    center_kernel<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(theta, c->prior_mean, P, d, tmp);
    SPS_CHECK(launched(c, "center_kernel"));
    return gemm_abt(c, tmp, c->prior_Li, nullptr, R, P, d, 1.0);
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

// 16 lanes per particle (4 particles per wave, 16 per workgroup):
// log alpha = [ll' + log p(theta')] - [ll + log p(theta)]
//             (+ MALA: -|v|^2 / 2 + |z|^2 / 2, v = L^-1 (theta - mu(theta')), L L' = Sigma);
// accept iff log u < log alpha; accepted particles take theta', ll' (grad').
// The prior terms use the whitened particles w0, w1 when given (full prior),
// else (theta - mu) / sd.  Sums over the 16 lanes are fixed butterflies.
// Accepted particles are counted per workgroup and added with one atomic into
// count slot blockIdx mod kCountSlots.
// ll2 holds ll2n slices of P (the likelihood kernel's observation splits),
// summed here in slice order.
// z / u null: the normals (MALA) and uniforms are drawn here from Philox
// streams zstream / zstream + 1 (the values sps_random gives).
// sq (d > 64, independent prior): the sums of squares for |(theta - mu) / sd|^2,
// the same at theta', |v|^2 and |z|^2 come as n per-tile partials
// [j * P + p] from the contractions' epilogues (summed here in tile order)
// instead of from the rows; a null member keeps the row sum.
struct AccSq {
    const double* q0 = nullptr;
    const double* q1 = nullptr;
    const double* vv = nullptr;
    const double* zz = nullptr;
    int n = 0;
};
constexpr int kAccLanes = 16;
constexpr int kAccPerBlock = 256 / kAccLanes;
__device__ __forceinline__ double sum16(double v) {
#pragma unroll
    for (int m = kAccLanes / 2; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}
__global__ __launch_bounds__(256) void accept_kernel(
    double* __restrict__ theta, double* __restrict__ ll, double* __restrict__ grad,
    const double* __restrict__ theta2, const double* __restrict__ ll2,
    const double* __restrict__ grad2, const double* __restrict__ z, const double* __restrict__ v,
    const double* __restrict__ u, const double* __restrict__ mu, const double* __restrict__ isd,
    const double* __restrict__ w0, const double* __restrict__ w1,
    int64_t P, int32_t d, int mala, const unsigned* flags, unsigned long long* count,
    uint64_t seed, uint64_t zstream, int32_t ll2n, const unsigned* stop, AccSq sq) {
    __shared__ unsigned nacc[256 / kAccLanes];
    if (stop && *stop) return;  // the same value for the whole grid: theta, ll, grad stay
    const int sub = threadIdx.x & (kAccLanes - 1);
    const int slot = threadIdx.x / kAccLanes;
    const int64_t p = (int64_t)blockIdx.x * kAccPerBlock + slot;
    const bool ok = !(*flags & kFlagNotPD);
    unsigned taken = 0;
    if (ok && p < P) {  // the 16 lanes of a particle share p: no divergence inside a group
        const double* a = theta + p * d;
        const double* b = theta2 + p * d;
        // per-particle scalars first, so their loads overlap the loop's
        double l2 = 0.0;  // the proposal's log-likelihood: ll2n observation-split slices, in order
#pragma unroll 8
        for (int32_t q = 0; q < ll2n; ++q) l2 += ll2[(int64_t)q * P + p];
        const double l1 = ll[p];
        double up;
        if (u) {
            up = u[p];
        } else {  // the uniform of stream zstream + 1, as sps_random kind 1
            uint64_t ua, ub;
            philox_u53x2(seed, zstream + 1, (uint64_t)p, ua, ub);
            up = u53_to_uniform(ua);
        }
        double q0 = 0.0, q1 = 0.0, vv = 0.0, zz = 0.0;
        if (sq.q0) {  // lane 0 of the group sums the partials; the others add zeros
            if (sub == 0) {
                for (int j = 0; j < sq.n; ++j) {
                    q0 += sq.q0[(int64_t)j * P + p];
                    q1 += sq.q1[(int64_t)j * P + p];
                    if (mala) {
                        vv += sq.vv[(int64_t)j * P + p];
                        zz += sq.zz[(int64_t)j * P + p];
                    }
                }
            }
        } else {
#pragma unroll 4
            for (int32_t i = sub; i < d; i += kAccLanes) {
                const double za = w0 ? w0[p * d + i] : (a[i] - mu[i]) * isd[i];
                const double zb = w0 ? w1[p * d + i] : (b[i] - mu[i]) * isd[i];
                q0 += za * za;
                q1 += zb * zb;
                if (mala) vv += v[p * d + i] * v[p * d + i];
            }
        }
        if (mala && !sq.zz) {  // |z|^2 by Box-Muller pairs (elements 2 j, 2 j + 1), read or drawn alike
            for (int32_t j = sub; 2 * j < d; j += kAccLanes) {
                double z0, z1;
                if (z) {
                    z0 = z[p * d + 2 * j];
                    z1 = 2 * j + 1 < d ? z[p * d + 2 * j + 1] : 0.0;
                } else {
                    philox_normal_pair(seed, zstream, p, j, d, z0, z1);
                    if (2 * j + 1 >= d) z1 = 0.0;
                }
                zz += z0 * z0;
                zz += z1 * z1;
            }
        }
        q0 = sum16(q0);
        q1 = sum16(q1);
        double la = (l2 - 0.5 * q1) - (l1 - 0.5 * q0);
        if (mala) la += -0.5 * sum16(vv) + 0.5 * sum16(zz);
        if (isnan(la)) la = -INFINITY;
        if (log(up) < la) {
            for (int32_t i = sub; i < d; i += kAccLanes) {
                theta[p * d + i] = b[i];
                if (mala) grad[p * d + i] = grad2[p * d + i];
            }
            if (sub == 0) ll[p] = l2;
            taken = 1;
        }
    }
    if (sub == 0) nacc[slot] = taken;
    __syncthreads();
    if (threadIdx.x == 0 && ok) {
        unsigned tot = 0;
        for (int q = 0; q < kAccPerBlock; ++q) tot += nacc[q];
        if (tot) atomicAdd(count + (blockIdx.x % kCountSlots) * kCountStride, (unsigned long long)tot);
    }
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// One M step for every particle.  Sigma_in == nullptr: proposal covariance
// h V from the particles (Algorithm 2); otherwise the given matrix
// (Algorithm 3, second pass).  The Sigma used stays in the context for
// sps_last_sigma.
// All launches of one M step; the status flags and the accepted-count slots
// are left in the status block of c->small.  No synchronisation.
// h_dev (optional, device): the step size is read there when the covariance
// is formed, and h is not used.  stop (optional, device): when *stop is
// nonzero as the step runs, the step leaves theta, ll, grad and the context's
// Sigma unchanged (the likelihood launches do no work either).
static int mutate_launch(sps_ctx* c, const char* who, double* theta, double* ll, double* grad, int32_t J,
                         int32_t N, int64_t t, double h, const double* Sigma_in, int kind, int prec,
                         const double* z, const double* u, uint64_t seed, uint64_t stream,
                         const double* h_dev = nullptr, const unsigned* stop = nullptr) {
    if (!c->has_data || !c->has_prior) return fail(c, SPS_ERR_STATE, "%s: set data and prior first", who);
    if (J < 1 || N < 1 || (int64_t)J * N < 2 || !theta || !ll)
        return fail(c, SPS_ERR_ARG, "%s: bad arguments (need J N >= 2, theta, ll)", who);
    if (t < 0 || t > c->T) return fail(c, SPS_ERR_ARG, "%s: t=%lld outside [0, T]", who, (long long)t);
    if (!Sigma_in && !h_dev && (!(h > 0.0) || !std::isfinite(h)))
        return fail(c, SPS_ERR_ARG, "%s: h must be positive", who);
    if (kind != SPS_RW && kind != SPS_MALA) return fail(c, SPS_ERR_ARG, "%s: unknown kind %d", who, kind);
    if (kind == SPS_MALA && !grad) return fail(c, SPS_ERR_ARG, "%s: MALA needs grad", who);
    if (prec != SPS_FP64 && prec != SPS_FP32 && prec != SPS_BF16X3)
        return fail(c, SPS_ERR_ARG, "%s: unknown precision %d", who, prec);
    const int64_t P = (int64_t)J * N;
    const int32_t d = c->d;
    if (d > 1024) return fail(c, SPS_ERR_ARG, "%s: d=%d above 1024", who, d);
    const bool mala = kind == SPS_MALA;
    const int64_t Pd = P * d;
    const bool small = d <= kSmallD;
    // covariance chunks: d <= 64: at most 64 (one workgroup sums them before
    // the Cholesky); otherwise one round of resident blocks, at least 64
    // particles each
    int64_t chunk;
    if (small) {
        chunk = 64;  // one load round per workgroup; the partials are summed by cov_final_kernel
    } else {
        // the upper-triangle tiles times the chunks fill the chip's 1024
        // resident workgroups (4 per CU at 33 KB of LDS each) in one round
        const int64_t nt = (d + 63) / 64, tiles = nt * (nt + 1) / 2;
        const int64_t nch0 = std::max<int64_t>(1, std::min<int64_t>(1024 / tiles, (P + 63) / 64));
        chunk = (((P + nch0 - 1) / nch0) + 15) / 16 * 16;
    }
    const int32_t nchunk = (int32_t)((P + chunk - 1) / chunk);

    SPS_CHECK(ensure(c, c->theta2, sizeof(double) * Pd, "proposals"));
    SPS_CHECK(ensure(c, c->ll2, sizeof(double) * P, "proposal log-likelihoods"));
    // d > 64 with the independent prior: the MH test's sums of squares come
    // from the contractions' epilogues as na per-tile partials per particle
    // (in the first P d doubles of pstat, which MALA's v no longer needs)
    const bool fold = !small && !c->prior_full;
    const int na = (d + 63) / 64;
    if (mala) {
        SPS_CHECK(ensure(c, c->grad2, sizeof(double) * Pd, "proposal gradients"));
        SPS_CHECK(ensure(c, c->pstat, sizeof(double) * 3 * Pd, "MALA work"));
    } else if (fold) {
        SPS_CHECK(ensure(c, c->pstat, sizeof(double) * 2 * na * P, "MH-test partial sums"));
    }
    AccSq asq{};
    SPS_CHECK(ensure(c, c->chol, sizeof(double) * 4 * (size_t)d * d, "proposal covariance"));
    if (!Sigma_in) {
        SPS_CHECK(ensure(c, c->cov, sizeof(double) * (size_t)nchunk * d * d, "covariance partials"));
        SPS_CHECK(ensure(c, c->mean, sizeof(double) * (size_t)nchunk * d, "covariance sums"));
    }
    SPS_CHECK(ensure(c, c->small, 4096, "small"));
    SPS_CHECK(ensure_host(c, c->hostbuf, 4096));
    double* Sg = (double*)c->chol.p;  // Sigma, then its factor, its inverse and its transpose
    double* L = Sg + (size_t)d * d;
    double* W = L + (size_t)d * d;
    double* LT = W + (size_t)d * d;
    double* th2 = (double*)c->theta2.p;
    double* ll2 = (double*)c->ll2.p;
    unsigned* flags = (unsigned*)c->small.p;
    unsigned long long* count = (unsigned long long*)((char*)c->small.p + kCountOff);
    // status flags and accepted-count slots start at zero: cleared by the first
    // kernel of the step on the d <= 64 covariance path, by a fill otherwise
    const bool clear_in_cov = small && !Sigma_in;
    if (!clear_in_cov) SPS_CHECK(fill(c, (double*)c->small.p, (int64_t)(kStatusBytes / 8), 0.0));

    // Normals and uniforms that are not given come from Philox streams
    // (seed, stream) and (seed, stream + 1).  The d <= 64 proposal kernels and
    // the MH test draw them where they are used; the other proposal paths read
    // the normals from memory.
    const bool zgen = !z && small && (!mala || !c->prior_full);
    if (!z && !zgen) {
        SPS_CHECK(ensure(c, c->z, sizeof(double) * Pd, "normals"));
        SPS_CHECK(random_fill(c, 2, seed, stream, P, d, c->z.p));
        z = (const double*)c->z.p;
    }

    double* part = Sigma_in ? nullptr : (double*)c->cov.p;
    double* psum = Sigma_in ? nullptr : (double*)c->mean.p;
    if (small) {
        if (Sigma_in) {
            SPS_HIP(c, hipMemcpyAsync(Sg, Sigma_in, sizeof(double) * d * d, hipMemcpyDeviceToDevice, c->stream));
        } else {
            unsigned long long* z2 = (unsigned long long*)c->small.p;
            if (d <= 32)
                cov_partial_small_kernel<2><<<nchunk, 256, 0, c->stream>>>(theta, P, d, chunk, part, psum, z2);
            else
                cov_partial_small_kernel<4><<<nchunk, 256, 0, c->stream>>>(theta, P, d, chunk, part, psum, z2);
            SPS_CHECK(launched(c, "cov_partial_small_kernel"));
            cov_final_kernel<<<(unsigned)(((int64_t)d * d + 3) / 4), 256, 0, c->stream>>>(part, psum, nchunk, d,
                                                                                          P, h, Sg, h_dev, stop);
            SPS_CHECK(launched(c, "cov_final_kernel"));
        }
        cholesky_small_kernel<<<1, 256, 0, c->stream>>>(Sg, d, L, flags);
        SPS_CHECK(launched(c, "cholesky_small_kernel"));
        if (mala && c->prior_full) {  // the generic MALA path below uses L^-1
            trinv_small_kernel<<<1, 64, 0, c->stream>>>(L, d, W, flags);
            SPS_CHECK(launched(c, "trinv_small_kernel"));
        }
    } else {
        if (Sigma_in) {
            SPS_HIP(c, hipMemcpyAsync(Sg, Sigma_in, sizeof(double) * d * d, hipMemcpyDeviceToDevice, c->stream));
        } else {
            const int64_t nt = (d + 63) / 64, nblk = nt * (nt + 1) / 2 * nchunk;
            cov_partial_kernel<<<(unsigned)((nblk + 7) / 8 * 8), 256, 0, c->stream>>>(theta, P, d, chunk, nblk,
                                                                                   part, psum);
            SPS_CHECK(launched(c, "cov_partial_kernel"));
            cov_final_kernel<<<(unsigned)(((int64_t)d * d + 3) / 4), 256, 0, c->stream>>>(part, psum, nchunk, d,
                                                                                          P, h, Sg, h_dev, stop);
            SPS_CHECK(launched(c, "cov_final_kernel"));
        }
        if (d <= 512) cholesky_blocked_kernel<32, 512><<<1, 1024, 0, c->stream>>>(Sg, d, L, LT, flags);
        else cholesky_blocked_kernel<16, 1024><<<1, 1024, 0, c->stream>>>(Sg, d, L, LT, flags);
        SPS_CHECK(launched(c, "cholesky_blocked_kernel"));
        if (mala && c->prior_full) {  // the generic MALA path below uses L^-1
            trinv_kernel<<<1, 1024, 0, c->stream>>>(L, d, W, flags);
            SPS_CHECK(launched(c, "trinv_kernel"));
        }
    }

    // Full prior: whitened particles r = L^-1 (theta - mean) for the prior
    // terms of log alpha and, for MALA, its gradient -L^-T r.
    double* wtmp = nullptr;
    double* R0 = nullptr;
    double* R1 = nullptr;
    if (c->prior_full) {
        SPS_CHECK(ensure(c, c->pw, sizeof(double) * 3 * Pd, "whitened particles"));
        wtmp = (double*)c->pw.p;
        R0 = wtmp + Pd;
        R1 = R0 + Pd;
        SPS_CHECK(prior_whiten(c, theta, P, wtmp, R0));
    }
    auto grad_logpost = [&](const double* gl, const double* th, const double* R, double* out) -> int {
        if (c->prior_full) return gemm_abt(c, R, c->prior_LiT, gl, out, P, d, -1.0);
        grad_logpost_kernel<<<nblk(Pd), 256, 0, c->stream>>>(gl, th, c->prior_mean, c->prior_isd, P, d, out);
        return launched(c, "grad_logpost_kernel");
    };
    // The proposal's log-likelihood as the MH test reads it: ll2, or the
    // likelihood kernel's observation-split slices when the sum is left to it.
    const double* ll2s = ll2;
    int32_t ll2n = 1;
    if (!mala) {
        // theta' = theta + L z
        if (zgen) {
            SmallGemm g{};
            g.B = L;
            g.Base = theta;
            g.Out = th2;
            g.P = P;
            g.d = d;
            g.alpha = 1.0;
            g.zgen = 1;
            g.seed = seed;
            g.zstream = stream;
            SPS_CHECK(gemm_small<GM_PLAIN>(c, g));
        } else if (fold) {
            GemmSq g{};
            g.sqb = (double*)c->pstat.p;
            g.sqo = g.sqb + (size_t)na * P;
            g.mu = c->prior_mean;
            g.isd = c->prior_isd;
            SPS_CHECK(gemm_abt_sq(c, z, L, theta, th2, P, d, 1.0, &g));
            asq.q0 = g.sqb;
            asq.q1 = g.sqo;
            asq.n = na;
        } else {
            SPS_CHECK(gemm_abt(c, z, L, theta, th2, P, d, 1.0));
        }
        LoglikSplit sp;
        SPS_CHECK(loglik_launch_split(c, th2, P, 0, t, prec, ll2, nullptr, &sp, stop));
        ll2s = sp.ll;
        ll2n = sp.n;
        if (c->prior_full) SPS_CHECK(prior_whiten(c, th2, P, wtmp, R1));
    } else if (small && !c->prior_full) {
        // theta' = mu(theta) + L z through u = z + L^T g(theta) / 2 (theta' = theta + L u);
        // after the likelihood at theta', v = -(u + L^T g(theta') / 2) (only |v|^2 is used)
        double* v = (double*)c->pstat.p;
        double* g2 = (double*)c->grad2.p;
        SmallGemm f{};
        f.th = theta;
        f.g = grad;
        f.z = z;
        f.mu = c->prior_mean;
        f.isd = c->prior_isd;
        f.L = L;
        f.Out = th2;
        f.U = v;
        f.P = P;
        f.d = d;
        f.zgen = zgen ? 1 : 0;
        f.seed = seed;
        f.zstream = stream;
        SPS_CHECK(gemm_small<GM_MALA_FWD>(c, f));
        LoglikSplit sp;
        SPS_CHECK(loglik_launch_split(c, th2, P, 0, t, prec, ll2, g2, &sp, stop));
        ll2s = sp.ll;
        ll2n = sp.n;
        SmallGemm r{};
        r.th2 = th2;
        r.g = sp.g;          // the gradient slices, summed while staged
        r.gsplit = sp.n;
        r.gout = g2;         // the summed gradient at theta' (the MH test copies it)
        r.mu = c->prior_mean;
        r.isd = c->prior_isd;
        r.L = L;
        r.Base = v;
        r.Out = v;
        r.P = P;
        r.d = d;
        SPS_CHECK(gemm_small<GM_MALA_REV>(c, r));
    } else if (!c->prior_full) {
        // d > 64: the same u-form with FP64 VALU contractions and L^T from the factorisation:
        // u = z + L^T g(theta) / 2, theta' = theta + L u, after the likelihood w = u + L^T g(theta') / 2
        double* v = (double*)c->pstat.p;
        double* uu = v + Pd;
        double* gpi = uu + Pd;
        double* g2 = (double*)c->grad2.p;
        // partial sums in v's space: |z|^2, |(theta - mu) / sd|^2, the same at
        // theta', |v|^2 (v itself is not written)
        const size_t np = (size_t)na * P;
        GemmSq s0{}, s1{}, s2{};
        s0.sqb = v;
        s1.sqb = v + np;
        s1.sqo = v + 2 * np;
        s1.mu = c->prior_mean;
        s1.isd = c->prior_isd;
        s2.sqo = v + 3 * np;
        s2.store = 0;
        SPS_CHECK(grad_logpost(grad, theta, R0, gpi));
        SPS_CHECK(gemm_abt_sq(c, gpi, LT, z, uu, P, d, 0.5, &s0));
        SPS_CHECK(gemm_abt_sq(c, uu, L, theta, th2, P, d, 1.0, &s1));
        SPS_CHECK(loglik_launch(c, th2, P, 0, t, prec, ll2, g2, stop));
        SPS_CHECK(grad_logpost(g2, th2, R1, gpi));
        SPS_CHECK(gemm_abt_sq(c, gpi, LT, uu, v, P, d, 0.5, &s2));
        asq.q0 = s1.sqb;
        asq.q1 = s1.sqo;
        asq.vv = s2.sqo;
        asq.zz = s0.sqb;
        asq.n = na;
    } else {
        double* gpi = (double*)c->pstat.p;
        double* work = gpi + Pd;
        double* g2 = (double*)c->grad2.p;
        // mu(theta) = theta + (1/2) Sigma grad log pi(theta); theta' = mu + L z
        SPS_CHECK(grad_logpost(grad, theta, R0, gpi));
        SPS_CHECK(gemm_abt(c, gpi, Sg, theta, work, P, d, 0.5));
        SPS_CHECK(gemm_abt(c, z, L, work, th2, P, d, 1.0));
        SPS_CHECK(loglik_launch(c, th2, P, 0, t, prec, ll2, g2, stop));
        // v = L^-1 (theta - mu(theta'))
        if (c->prior_full) SPS_CHECK(prior_whiten(c, th2, P, wtmp, R1));
        SPS_CHECK(grad_logpost(g2, th2, R1, gpi));
        sub_kernel<<<nblk(Pd), 256, 0, c->stream>>>(theta, th2, work, Pd);
        SPS_CHECK(launched(c, "sub_kernel"));
        SPS_CHECK(gemm_abt(c, gpi, Sg, work, work, P, d, -0.5));
        SPS_CHECK(gemm_abt(c, work, W, nullptr, gpi, P, d, 1.0));
    }
    accept_kernel<<<(unsigned)((P + kAccPerBlock - 1) / kAccPerBlock), 256, 0, c->stream>>>(
        theta, ll, grad, th2, ll2s, mala ? (const double*)c->grad2.p : nullptr, z,
        mala ? (const double*)c->pstat.p : nullptr, u, c->prior_mean, c->prior_isd, R0, R1, P, d,
        mala ? 1 : 0, flags, count, seed, stream, ll2n, stop, asq);
    SPS_CHECK(launched(c, "accept_kernel"));
    c->has_sigma = true;
    return SPS_OK;
}

// Device-resident state of an M phase (sps_mphase).  The step size h is read
// by the covariance kernel of the next step; the stop word by every launch
// of a step that writes what the caller sees.
struct MState {
    double h;        // step size for the next step
    double agg;      // aggregate RNE after the last step taken
    double rate;     // acceptance rate of the last step taken
    int32_t r;       // steps taken
    unsigned stop;   // nonzero: the phase has ended; later queued steps do nothing
    unsigned notpd;  // the last step's proposal covariance was not positive definite
    unsigned pad;
};

__global__ void mstate_init_kernel(MState* s, double h) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *s = MState{h, 0.0, 0.0, 0, 0u, 0u, 0u};
}

// After each step: the acceptance rate from the count slots, the step-size
// rule of Algorithm 2 (h up by h_step when the rate is above the target, else
// down, within [h_min, h_max]) and the stopping rule (aggregate RNE at least
// K, or R_max steps), with the same expressions and order as a host loop
// would use, so the steps taken and the h they use do not change.
__global__ __launch_bounds__(64) void mstep_control_kernel(MState* s, const unsigned* flags, const double* agg,
                                                           const unsigned long long* count, int64_t P,
                                                           double h_step, double h_min, double h_max,
                                                           double acc_target, double K, int32_t R_max) {
    if (threadIdx.x != 0 || s->stop) return;
    const int32_t r = s->r + 1;
    s->r = r;
    if (*flags & kFlagNotPD) {
        s->notpd = 1u;
        s->stop = 1u;
        return;
    }
    unsigned long long n_acc = 0;
    for (int q = 0; q < kCountSlots; ++q) n_acc += count[q * kCountStride];
    const double rate = (double)n_acc / (double)P;
    const double a = *agg;
    const double h = s->h;
    const double up = h + h_step, dn = h - h_step;
    s->h = rate > acc_target ? (h_max < up ? h_max : up) : (dn < h_min ? h_min : dn);
    s->rate = rate;
    s->agg = a;
    if (a >= K || r >= R_max) s->stop = 1u;
}

// Read back the step's status block (flags, aggregate RNE, accepted-count
// slots) and check the flags.
static int mutate_readback(sps_ctx* c, const char* who, int64_t P, double* accept_rate,
                           const void** host_out = nullptr) {
    const void* h = nullptr;
    SPS_CHECK(readback(c, c->small.p, kStatusBytes, &h));
    if (host_out) *host_out = h;
    const unsigned f = *(const unsigned*)h;
    const unsigned long long* slots = (const unsigned long long*)((const char*)h + kCountOff);
    unsigned long long n_acc = 0;
    for (int q = 0; q < kCountSlots; ++q) n_acc += slots[q * kCountStride];
    if (f & kFlagNotPD)
        return fail(c, SPS_ERR_NOT_PD, "%s: the proposal covariance is not positive definite", who);
    if (accept_rate) *accept_rate = (double)n_acc / (double)P;
    return SPS_OK;
}

static int mutate_impl(sps_ctx* c, const char* who, double* theta, double* ll, double* grad, int32_t J,
                       int32_t N, int64_t t, double h, const double* Sigma_in, int kind, int prec,
                       const double* z, const double* u, uint64_t seed, uint64_t stream,
                       double* accept_rate) {
    SPS_CHECK(mutate_launch(c, who, theta, ll, grad, J, N, t, h, Sigma_in, kind, prec, z, u, seed, stream));
    return mutate_readback(c, who, (int64_t)J * N, accept_rate);
}

}  // namespace sps

using namespace sps;

extern "C" int sps_mutate(sps_ctx* c, double* theta, double* ll, double* grad, int32_t J, int32_t N,
                          int64_t t, double h, int kind, int prec, const double* z, const double* u,
                          uint64_t seed, uint64_t stream, double* accept_rate) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    return mutate_impl(c, "sps_mutate", theta, ll, grad, J, N, t, h, nullptr, kind, prec, z, u, seed,
                       stream, accept_rate);
}

extern "C" int sps_mutate_cov(sps_ctx* c, double* theta, double* ll, double* grad, int32_t J,
                              int32_t N, int64_t t, const double* Sigma, int kind, int prec,
                              const double* z, const double* u, uint64_t seed, uint64_t stream,
                              double* accept_rate) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (!Sigma) return fail(c, SPS_ERR_ARG, "sps_mutate_cov: null Sigma");
    return mutate_impl(c, "sps_mutate_cov", theta, ll, grad, J, N, t, 1.0, Sigma, kind, prec, z, u,
                       seed, stream, accept_rate);
}

extern "C" int sps_last_sigma(sps_ctx* c, double* Sigma) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (!Sigma) return fail(c, SPS_ERR_ARG, "sps_last_sigma: null output");
    if (!c->has_sigma) return fail(c, SPS_ERR_STATE, "sps_last_sigma: no M step has run");
    SPS_HIP(c, hipMemcpyAsync(Sigma, c->chol.p, sizeof(double) * c->d * c->d, hipMemcpyDeviceToDevice,
                              c->stream));
    return SPS_OK;
}

// The M phase of one cycle (Algorithm 2 step 2(c)) in one call: steps
// r = 1, 2, ... each take sps_mutate's step, then the monitored functions,
// their NSE/RNE and the aggregate RNE on the device, and a control kernel
// applies the step-size and stopping rules on the device (h and the stop word
// stay in device memory).  For launch-bound steps the host reads the state of
// step r asynchronously while step r + 1 is already queued (lookahead 1); a
// step queued after the stop leaves every output unchanged (its covariance,
// likelihood and accept launches test the stop word).  Other steps are read
// back one at a time.
extern "C" int sps_mphase(sps_ctx* c, double* theta, double* ll, double* grad, int32_t J, int32_t N,
                          int64_t t, int kind, int prec, double* h, double h_step, double h_min,
                          double h_max, double acc_target, double K, int32_t R_max, int rne_rule,
                          uint64_t seed, uint64_t stream0, uint64_t stream_step, double* g_work,
                          double* sigma_out, int32_t* R_out, double* rne_out, double* rate_out) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (!h || !g_work || !R_out || R_max < 1 || (rne_rule != 0 && rne_rule != 1) ||
        !(h_min > 0.0) || !(h_max >= h_min) || !(h_step >= 0.0) || !std::isfinite(K))
        return fail(c, SPS_ERR_ARG, "sps_mphase: bad arguments");
    if (!(*h > 0.0) || !std::isfinite(*h)) return fail(c, SPS_ERR_ARG, "sps_mphase: h must be positive");
    if (J > 65535 || (N + 63) / 64 > 65535) return fail(c, SPS_ERR_ARG, "sps_mphase: J or N too large");
    const int64_t P = (int64_t)J * N;
    const int32_t d = c->d, m = c->d + c->C - 1;
    SPS_CHECK(ensure(c, c->small, 4096, "small"));
    SPS_CHECK(ensure(c, c->mstat, sizeof(MState), "M phase state"));
    MState* ms = (MState*)c->mstat.p;
    const unsigned* stop = &ms->stop;
    mstate_init_kernel<<<1, 64, 0, c->stream>>>(ms, *h);
    SPS_CHECK(launched(c, "mstate_init_kernel"));
    // Queue a step ahead only where steps are launch-bound (little GPU work
    // per step): there the skipped step at the end of the phase runs while
    // the host is still launching the next phase.  Where the GPU is the
    // bottleneck, that step's covariance and proposal kernels would delay
    // the next phase by more than the read-back waits cost (measured at
    // binary30: 3.5 MALA steps per phase, 78 us lost per phase).
    const double step_work = (double)P * (double)std::max<int64_t>(t, 1) * d;
    const int look = (step_work <= (double)(1 << 26) && (double)P * d * d <= (double)(1 << 28)) ? 1 : 0;
    PubTicket tk[2];
    int head = 0, pending = 0;
    int32_t queued = 0;
    MState st{};
    for (;;) {
        while (queued < R_max && pending <= look) {
            ++queued;
            const uint64_t sid = stream0 + (uint64_t)queued * stream_step;
            SPS_CHECK(mutate_launch(c, "sps_mphase", theta, ll, grad, J, N, t, 0.0, nullptr, kind, prec, nullptr,
                                    nullptr, seed, sid, &ms->h, stop));
            if (sigma_out)
                SPS_HIP(c, hipMemcpyAsync(sigma_out + (size_t)(queued - 1) * d * d, c->chol.p,
                                          sizeof(double) * d * d, hipMemcpyDeviceToDevice, c->stream));
            SPS_CHECK(monitor_launch(c, theta, P, g_work));
            double* mom = nullptr;
            SPS_CHECK(moments_launch(c, g_work, J, N, m, &mom));
            double* agg = (double*)((char*)c->small.p + 16);
            SPS_CHECK(rne_aggregate(c, mom, m, rne_rule, agg));
            mstep_control_kernel<<<1, 64, 0, c->stream>>>(
                ms, (const unsigned*)c->small.p, agg, (const unsigned long long*)((char*)c->small.p + kCountOff),
                P, h_step, h_min, h_max, acc_target, K, R_max);
            SPS_CHECK(launched(c, "mstep_control_kernel"));
            SPS_CHECK(publish_async(c, ms, sizeof(MState), &tk[(head + pending) & 1]));
            ++pending;
        }
        const void* rec = nullptr;
        SPS_CHECK(publish_wait(c, tk[head], &rec));
        st = *(const MState*)rec;
        head ^= 1;
        --pending;
        if (st.stop) break;
        if (queued >= R_max && pending == 0)
            return fail(c, SPS_ERR_HIP, "sps_mphase: the M phase did not stop after R_max steps");
    }
    if (st.notpd)
        return fail(c, SPS_ERR_NOT_PD, "sps_mphase: the proposal covariance is not positive definite");
    *h = st.h;
    *R_out = st.r;
    if (rne_out) *rne_out = st.agg;
    if (rate_out) *rate_out = st.rate;
    return SPS_OK;
}
