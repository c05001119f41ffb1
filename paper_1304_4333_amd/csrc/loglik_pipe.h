// loglik_pipe.h -- the BF16x3 log-likelihood and adjoint kernels over full
// observation ranges, software-pipelined so that the matrix cores and the
// vector ALU work at the same time.
//
// What is computed is the same as in loglik_kernel.h (eq. (plogit) with
// theta_0 = 0, summed over the product form of the likelihood, and the
// adjoint G_{p,c} = sum_t x_t (1{y_t = c} - pi_{p,t,c})), with the same
// operands: X and theta split into BF16 hi + lo, eta ~ Xh Bh + Xh Bl + Xl Bh
// on MFMA with FP32 accumulation, the log-sum-exp in base 2 on the hardware
// exp/log, and per-tile sums carried into FP64.
//
// Why a second kernel.  On gfx950 a wave overlaps its own MFMAs with the
// independent VALU instructions it issues between them, but the epilogue of
// a 16-row tile needs that tile's MFMA results, so a wave that runs
// "contract, then epilogue" keeps one unit idle at a time (measured: MFMA
// busy 44-46% at the largest multinomial workload).  Here the contraction of
// tile tau + 1 is interleaved with the epilogue of tile tau (two accumulator
// sets), and the adjoint contraction of step st - 1 with the epilogues of
// step st.
//
// Operand staging.  The four waves of a workgroup share one copy of every X
// (and X^T) step tile in LDS, in a ring of four buffers: tile st + 2 is
// written at the top of step st from registers loaded during step st - 1, so
// a global load has a whole step to arrive, and one barrier per step orders
// the ring.  LDS rows are padded by 16 bytes so that the 16 rows a lane group
// reads together fall in distinct banks.
//
// Masking by zero rows.  Rows outside [t0, t1) are written to LDS as zeros.
// Such a row has eta = 0 for every outcome, so its log-probability is exactly
// -log2(C) in every form of the epilogue (binary: -log2(1 + 2^0) = -1) and
// its adjoint term x_t r_t is zero; the kernel adds the count of masked rows
// times log2(C) back to the sum.  Every step then runs the same unmasked
// body.
//
// Layouts (gfx950 MFMA lane layouts as in loglik_kernel.h):
//   X step tile in LDS: slot 16 h + m (h = tile, m = A row) holds X row
//     o + 8 (m >> 2) + 4 h + (m & 3), as [hi row | lo row | 16 B pad];
//     D row 4 g + i of tile h is then observation o + 8 g + 4 h + i.
//   X^T step tile in LDS: row i (covariate) holds observations o .. o + 31,
//     as [hi 64 B | lo 64 B | 16 B pad].
#pragma once

#include "loglik_kernel.h"

namespace sps {

template <int NC, int KS, bool GRAD>
struct PipeShape {
    // Particle blocks of 16 per wave: with one outcome column an X fragment
    // feeds PW chains (four in the forward kernel while the fragments are
    // short, two with the adjoint or at k > 64); with C > 2 the outcome
    // columns already give that reuse.
    static constexpr int PW = NC > 1 ? 1 : (GRAD || KS > 2) ? 2 : 4;
    static constexpr int KB = 32 * KS;             // BF16 row length of the X copies
    static constexpr int XRS = 4 * KB + 16;         // LDS bytes per X slot (hi, lo, pad)
    static constexpr int XTILE = 32 * XRS;          // one step of X
    static constexpr int TRS = 144;                 // LDS bytes per X^T row (32 obs hi, lo, pad)
    static constexpr int TTILE = GRAD ? KB * TRS : 0;
    static constexpr int BUF = XTILE + TTILE;       // one ring slot
    static constexpr int NBUF = 4;
    static constexpr int LDS = NBUF * BUF;
    static constexpr int KBT = 2 * KS;              // adjoint blocks of 16 covariates
};

// 16 bytes of LDS as an MFMA operand fragment.
__device__ __forceinline__ bf16x8 lds_frag(const unsigned char* p) {
    return __builtin_bit_cast(bf16x8, *(const u16x8*)p);
}

// Keep the 16-bit elements e of a 16-byte chunk (8 elements) with lo <= e < hi.
__device__ __forceinline__ uint4 keep_elems(uint4 v, int lo, int hi) {
    unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e0 = 2 * q, e1 = 2 * q + 1;
        const unsigned m0 = (e0 >= lo && e0 < hi) ? 0x0000FFFFu : 0u;
        const unsigned m1 = (e1 >= lo && e1 < hi) ? 0xFFFF0000u : 0u;
        w[q] &= (m0 | m1);
    }
    return uint4{w[0], w[1], w[2], w[3]};
}

template <int NC, int KS, bool GRAD>
__global__ __launch_bounds__(256) void loglik_pipe_kernel(LoglikArgs a) {
    using S = PipeShape<NC, KS, GRAD>;
    constexpr int PW = S::PW;
    constexpr int KB = S::KB;
    constexpr int KBT = S::KBT;
    constexpr int XRS = S::XRS;
    constexpr int TRS = S::TRS;
    // the binary epilogue hands the adjoint +sigmoid (the sign is applied at the fold)
    constexpr bool kNegRes = NC == 1;
    constexpr int kFoldSteps = 128;  // FP32 adjoint sums are added into FP64 every 4096 rows
    __shared__ __attribute__((aligned(16))) unsigned char lds[S::LDS];

    if (a.skip != nullptr && *a.skip != 0u) return;  // the same value for every wave
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int g = lane >> 4;
    const int r16 = lane & 15;
    const int split = blockIdx.x % a.nsplit;
    const int64_t ptile = blockIdx.x / a.nsplit;
    // Waves past the last particle still stage tiles and meet every barrier;
    // their theta is zero and they write nothing.
    const int64_t pbase = (ptile * 4 + wave) * (16 * PW);

    // ---- B operand: log2(e) theta of this wave's particles, BF16 hi + lo ----
    bf16x8 bh[PW][NC][KS], bl[PW][NC][KS];
#pragma unroll
    for (int b = 0; b < PW; ++b) {
        const int64_t p = pbase + b * 16 + r16;
        const bool pv = p < a.P;
        const double* th = a.theta + (pv ? p : 0) * a.d;
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                u16x8 hv, lv;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int kk = g * 8 * KS + 8 * s + j;
                    const double raw = th[c * a.k + min(kk, a.k - 1)];
                    const double vd = (pv && kk < a.k) ? raw * kLog2e : 0.0;
                    const unsigned short h = to_bf16((float)vd);
                    hv[j] = h;
                    lv[j] = to_bf16((float)(vd - (double)from_bf16(h)));
                }
                bh[b][c][s] = __builtin_bit_cast(bf16x8, hv);
                bl[b][c][s] = __builtin_bit_cast(bf16x8, lv);
            }
    }

    const int st_begin = split * a.steps_per_split;
    const int st_end = min(a.nsteps, st_begin + a.steps_per_split);
    const int64_t obase = a.t0a;

    // ---- staging of step tiles: KS chunks of X and KS of X^T per thread ----
    // Loads are issued a step before the tile is written to LDS; the masks are
    // applied at the write, so nothing waits for a load early.
    uint4 sx[KS], stt[GRAD ? KS : 1];
    auto stage_load = [&](int st) __attribute__((always_inline)) {
        const int64_t o = obase + (int64_t)st * 32;
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            const int c = tid + 256 * j;
            const int arr = c / (128 * KS);
            const int rem = c % (128 * KS);
            const int row = rem / (4 * KS);
            const int q = rem % (4 * KS);
            sx[j] = *(const uint4*)((const unsigned short*)(arr ? a.Xlo : a.X) + (o + row) * KB + 8 * q);
        }
        if constexpr (GRAD) {
#pragma unroll
            for (int j = 0; j < KS; ++j) {
                const int c = tid + 256 * j;
                const int arr = c / (128 * KS);
                const int rem = c % (128 * KS);
                const int row = rem / 4;
                const int q = rem % 4;
                stt[j] = *(const uint4*)((const unsigned short*)(arr ? a.XTlo : a.XT) + (int64_t)row * a.Tp + o + 8 * q);
            }
        }
    };
    auto stage_store = [&](int st) __attribute__((always_inline)) {
        const int64_t o = obase + (int64_t)st * 32;
        unsigned char* buf = lds + (st & 3) * S::BUF;
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            const int c = tid + 256 * j;
            const int arr = c / (128 * KS);
            const int rem = c % (128 * KS);
            const int row = rem / (4 * KS);
            const int q = rem % (4 * KS);
            const int64_t t = o + row;
            const bool keep = t >= a.t0 && t < a.t1;
            // row = 8 a + 4 h + b  ->  slot 16 h + 4 a + b
            const int slot = 16 * ((row >> 2) & 1) + 4 * (row >> 3) + (row & 3);
            *(uint4*)(buf + slot * XRS + arr * 2 * KB + 16 * q) = keep ? sx[j] : uint4{0, 0, 0, 0};
        }
        if constexpr (GRAD) {
#pragma unroll
            for (int j = 0; j < KS; ++j) {
                const int c = tid + 256 * j;
                const int arr = c / (128 * KS);
                const int rem = c % (128 * KS);
                const int row = rem / 4;
                const int q = rem % 4;
                const int64_t t = o + 8 * q;
                const int lo = (int)max<int64_t>(0, min<int64_t>(8, a.t0 - t));
                const int hi = (int)max<int64_t>(0, min<int64_t>(8, a.t1 - t));
                const uint4 v = (lo > 0 || hi < 8) ? keep_elems(stt[j], lo, hi) : stt[j];
                *(uint4*)(buf + S::XTILE + row * TRS + arr * 64 + 16 * q) = v;
            }
        }
    };

    // ---- fragment blocks ----
    // A contraction block (tile h of a ring slot, k-step s) feeds PW * NC
    // chains of three MFMAs from one X fragment pair; an adjoint block
    // (covariates 16 q .. 16 q + 15) feeds PW * NC chains from one X^T pair.
    // Every block's fragments are read from LDS one block ahead, so the LDS
    // latency hides behind the MFMAs of the block before.
    struct Frags {
        bf16x8 h, l;  // X (or X^T) hi / lo fragment
    };
    const f32x4 zero4{0, 0, 0, 0};
    auto cload = [&](int slot, int h, int s) __attribute__((always_inline)) -> Frags {
        const unsigned char* xb = lds + slot * S::BUF + (16 * h + r16) * XRS + (g * KS + s) * 16;
        Frags f;
        f.h = lds_frag(xb);
        f.l = lds_frag(xb + 2 * KB);
        return f;
    };
    auto cmfma = [&](f32x4 (&acc)[PW][NC], const Frags& f, int s) __attribute__((always_inline)) {
#pragma unroll
        for (int b = 0; b < PW; ++b)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                f32x4 t = s == 0 ? zero4 : acc[b][c];
                t = mfma(f.h, bh[b][c][s], t);
                t = mfma(f.h, bl[b][c][s], t);
                acc[b][c] = mfma(f.l, bh[b][c][s], t);
            }
    };

    // ---- residuals of one step for the adjoint: BF16 hi / lo ----
    // Component w of (b, c) holds elements 2w, 2w + 1 of the 32-row step,
    // element j = 4 h + i; the four components are the MFMA B fragment.
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    u32x4 rh[GRAD ? 2 : 1][GRAD ? PW : 1][GRAD ? NC : 1];
    u32x4 rl[GRAD ? 2 : 1][GRAD ? PW : 1][GRAD ? NC : 1];
    // Split of a residual pair: hi = the upper 16 bits (truncation), packed
    // with one byte permute; lo = r - hi, exact in FP32, rounded to BF16 in
    // one packed conversion.  |lo| < 2^-7 |r|, so hi + bf16(lo) is within
    // 2^-16 |r| of r.
    auto put_res = [&](int set, int b, int c, int w, float r0, float r1) __attribute__((always_inline)) {
        if constexpr (GRAD) {
            const unsigned u0 = __float_as_uint(r0), u1 = __float_as_uint(r1);
            rh[set][b][c][w] = __builtin_amdgcn_perm(u1, u0, 0x07060302u);
            const float l0 = r0 - __uint_as_float(u0 & 0xFFFF0000u);
            const float l1 = r1 - __uint_as_float(u1 & 0xFFFF0000u);
            rl[set][b][c][w] = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){l0, l1}, bf16x2));
        }
    };

    // ---- epilogue of one tile: fast unshifted form, or the max-shifted form ----
    // Writes the tile's base-2 sum per particle block into tsum_t and its
    // residuals into residual set `set`; returns whether the fast form left
    // its safe range (the caller then reruns it with fast = false).  Elements
    // go in pairs, so that each pair's residuals are split and packed at once.
    auto epilogue = [&](const f32x4 (&acc)[PW][NC], int set, int h, float (&tsum_t)[PW], auto fast_c)
        __attribute__((always_inline)) -> bool {
        constexpr bool FAST = decltype(fast_c)::value;
        bool bad = false;
#pragma unroll
        for (int b = 0; b < PW; ++b) {
            if constexpr (NC == 1) {
                float r[4];
                if constexpr (FAST) {
                    // -sum_i log2(1 + 2^z_i) as -log2 of the product of the four factors
                    float prod = 1.f;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float z = acc[b][0][i];
                        const float e = fexp2(z);
                        const float sf = 1.f + e;
                        prod *= sf;
                        if constexpr (GRAD) r[i] = e * frcp(sf);  // sigmoid
                    }
                    tsum_t[b] = -flog2(prod);
                    bad |= !(tsum_t[b] > -INFINITY);  // product overflow or NaN
                } else {
                    float t = 0.f;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float z = acc[b][0][i];
                        const float mz = __int_as_float(max(__float_as_int(z), 0));
                        const float lp = -(mz + flog2(1.f + fexp2(-fabsf(z))));
                        t += lp;
                        if constexpr (GRAD) r[i] = fexp2(z + lp);
                    }
                    tsum_t[b] = t;
                }
                put_res(set, b, 0, 2 * h, r[0], r[1]);
                put_res(set, b, 0, 2 * h + 1, r[2], r[3]);
            } else {
                float t = 0.f;
#pragma unroll
                for (int i2 = 0; i2 < 2; ++i2) {
                    float r[NC][2];
#pragma unroll
                    for (int ii = 0; ii < 2; ++ii) {
                        const int i = 2 * i2 + ii;
                        float ec[NC];
                        float s;
                        float m = 0.f;
                        if constexpr (FAST) {
                            s = 1.f;
#pragma unroll
                            for (int c = 0; c < NC; ++c) {
                                ec[c] = fexp2(acc[b][c][i]);
                                s += ec[c];
                            }
                            bad |= !(s < 0x1p126f);
                        } else {
#pragma unroll
                            for (int c = 0; c < NC; ++c)
                                m = __int_as_float(max(__float_as_int(acc[b][c][i]), __float_as_int(m)));
                            s = fexp2(-m);
#pragma unroll
                            for (int c = 0; c < NC; ++c) {
                                ec[c] = fexp2(acc[b][c][i] - m);
                                s += ec[c];
                            }
                        }
                        t -= FAST ? flog2(s) : m + flog2(s);
                        if constexpr (GRAD) {
                            const float inv = frcp(s);
#pragma unroll
                            for (int c = 0; c < NC; ++c) r[c][ii] = -ec[c] * inv;
                        }
                    }
                    if constexpr (GRAD) {
#pragma unroll
                        for (int c = 0; c < NC; ++c) put_res(set, b, c, 2 * h + i2, r[c][0], r[c][1]);
                    }
                }
                tsum_t[b] = t;
            }
        }
        return bad;
    };

    // ---- adjoint: G += X~^T R over one step ----
    f32x4 gacc[GRAD ? PW : 1][GRAD ? NC : 1][GRAD ? KBT : 1];
    if constexpr (GRAD) {
#pragma unroll
        for (int b = 0; b < PW; ++b)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int q = 0; q < KBT; ++q) gacc[b][c][q] = f32x4{0, 0, 0, 0};
    }
    auto aload = [&](int slot, int q) __attribute__((always_inline)) -> Frags {
        const unsigned char* tb = lds + slot * S::BUF + S::XTILE + (q * 16 + r16) * TRS + g * 16;
        Frags f;
        f.h = lds_frag(tb);
        f.l = lds_frag(tb + 64);
        return f;
    };
    auto amfma = [&](int set, const Frags& f, int q) __attribute__((always_inline)) {
        if constexpr (GRAD) {
#pragma unroll
            for (int b = 0; b < PW; ++b)
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const bf16x8 Rh = __builtin_bit_cast(bf16x8, rh[set][b][c]);
                    const bf16x8 Rl = __builtin_bit_cast(bf16x8, rl[set][b][c]);
                    gacc[b][c][q] = mfma(f.h, Rh, gacc[b][c][q]);
                    gacc[b][c][q] = mfma(f.h, Rl, gacc[b][c][q]);
                    gacc[b][c][q] = mfma(f.l, Rh, gacc[b][c][q]);
                }
        }
    };
    double* const g_out = GRAD ? a.out_g + (int64_t)split * a.P * a.d : nullptr;
    bool g_first = true;
    auto fold = [&]() __attribute__((always_inline)) {
        if constexpr (GRAD) {
#pragma unroll
            for (int b = 0; b < PW; ++b) {
                const int64_t p = pbase + b * 16 + r16;
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int q = 0; q < KBT; ++q) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int kk = q * 16 + 4 * g + i;
                            if (p < a.P && kk < a.k) {
                                double* dst = g_out + p * a.d + c * a.k + kk;
                                const double gv = (double)gacc[b][c][q][i];
                                *dst = (g_first ? 0.0 : *dst) + (kNegRes ? -gv : gv);
                            }
                        }
                        gacc[b][c][q] = f32x4{0, 0, 0, 0};
                    }
            }
            g_first = false;
        }
    };

    double acc64[PW];
#pragma unroll
    for (int b = 0; b < PW; ++b) acc64[b] = 0.0;

    // Interleave the MFMAs of a half-step with its VALU work.  Per block: the
    // LDS reads of the next block's fragments, then the block's MFMAs, each
    // followed by a few VALU instructions, so that the matrix pipe and the
    // vector ALU work at the same time.  NBLK blocks; TAIL: another block
    // follows the last one (its reads are issued during the last one).
    // VALU instructions per tile to spread over the MFMAs.  Measured for the
    // binary adjoint (ar100, one box, kernel table): 8 per element 3.25-3.35
    // ms, 16 3.18 ms, 24 3.06-3.17 ms, 32 and 48 no better than 24; twice the
    // forward counts gave nothing (binary) or lost 2% (C = 6).
    constexpr int kMfmaBlk = PW * NC * 3;  // MFMAs per block
    constexpr int kValuTile = NC == 1 ? PW * 4 * (GRAD ? 24 : 3) : PW * 4 * (2 * NC + 3 + (GRAD ? 4 * NC + 1 : 0));
    auto interleave = [&](auto nblk_c, auto tail_c) __attribute__((always_inline)) {
        constexpr int NBLK = decltype(nblk_c)::value;
        constexpr bool TAIL = decltype(tail_c)::value;
        constexpr int NB1 = NBLK > 0 ? NBLK : 1;
        constexpr int per = (kValuTile + NB1 * kMfmaBlk - 1) / (NB1 * kMfmaBlk);
#pragma unroll
        for (int blk = 0; blk < NBLK; ++blk) {
            if (blk + 1 < NBLK || TAIL) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);  // next block's fragments
#pragma unroll
            for (int i = 0; i < kMfmaBlk; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);    // MFMA
                __builtin_amdgcn_sched_group_barrier(0x002, per, 0);  // VALU
            }
        }
    };

    f32x4 accA[PW][NC], accB[PW][NC];
    const bconst<true> fast{};
    const bconst<false> slow{};
    const bconst<true> yes{};
    const bconst<false> no{};
    const std::integral_constant<int, 0> zero_c{};
    const std::integral_constant<int, KS> ks_c{};
    const std::integral_constant<int, KS + KBT> ksa_c{};

    // One step st: half A contracts tile 1 of st and runs the adjoint of step
    // st - 1 (PREV; residual set 1 - CUR) while the epilogue runs on tile 0;
    // half B contracts tile 0 of st + 1 (NEXT) while the epilogue runs on
    // tile 1.  The residuals of st go to set CUR.  `pre` holds the fragments
    // of the step's first block on entry and of the next step's on exit.
    Frags pre;
    auto step = [&](int st, auto cur_c, auto prev_c, auto next_c) __attribute__((always_inline)) {
        constexpr int CUR = decltype(cur_c)::value;
        constexpr bool PREV = decltype(prev_c)::value && GRAD;
        constexpr bool NEXT = decltype(next_c)::value;
        __syncthreads();  // ring slot (st + 2) & 3 is free; tile st + 1 is visible
        if (st + 2 < st_end) stage_store(st + 2);
        if (st + 3 < st_end) stage_load(st + 3);
        const int slot = st & 3, nslot = (st + 1) & 3, pslot = (st + 3) & 3;  // pslot: step st - 1
        float tA[PW], tB[PW];
        // half A
        Frags f = pre;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            Frags nf = f;
            if (s + 1 < KS) nf = cload(slot, 1, s + 1);
            else if (PREV) nf = aload(pslot, 0);
            else if (NEXT) nf = cload(nslot, 0, 0);
            cmfma(accB, f, s);
            f = nf;
        }
        if constexpr (PREV) {
#pragma unroll
            for (int q = 0; q < KBT; ++q) {
                Frags nf = f;
                if (q + 1 < KBT) nf = aload(pslot, q + 1);
                else if (NEXT) nf = cload(nslot, 0, 0);
                amfma(1 - CUR, f, q);
                f = nf;
            }
        }
        const bool badA = epilogue(accA, CUR, 0, tA, fast);
        if constexpr (PREV) interleave(ksa_c, bconst<NEXT>{});
        else interleave(ks_c, bconst<NEXT>{});
        if (__any(badA)) epilogue(accA, CUR, 0, tA, slow);
        // half B
        if constexpr (NEXT) {
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                // the last block prefetches the next step's first block
                const Frags nf = s + 1 < KS ? cload(nslot, 0, s + 1) : cload(nslot, 1, 0);
                cmfma(accA, f, s);
                f = nf;
            }
            pre = f;
        }
        const bool badB = epilogue(accB, CUR, 1, tB, fast);
        if constexpr (NEXT) interleave(ks_c, yes);
        else interleave(zero_c, no);
        if (__any(badB)) epilogue(accB, CUR, 1, tB, slow);
#pragma unroll
        for (int b = 0; b < PW; ++b) acc64[b] += (double)tA[b] + (double)tB[b];
    };

    // ---- prologue: tiles st_begin and st_begin + 1 in LDS, st_begin + 2 in flight ----
    stage_load(st_begin);
    stage_store(st_begin);
    if (st_begin + 1 < st_end) {
        stage_load(st_begin + 1);
        stage_store(st_begin + 1);
    }
    if (st_begin + 2 < st_end) stage_load(st_begin + 2);
    __syncthreads();
    {
        const int slot0 = st_begin & 3;
        Frags f = cload(slot0, 0, 0);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const Frags nf = s + 1 < KS ? cload(slot0, 0, s + 1) : cload(slot0, 1, 0);
            cmfma(accA, f, s);
            f = nf;
        }
        pre = f;
    }

    // Steps alternate the residual sets 0, 1, 0, ...; a step's adjoint runs
    // during the next step, the last one after the loop.
    const std::integral_constant<int, 0> set0{};
    const std::integral_constant<int, 1> set1{};
    int last_set = 0;
    if (st_end - st_begin == 1) {
        step(st_begin, set0, no, no);
    } else {
        step(st_begin, set0, no, yes);
        int st = st_begin + 1;
        int since_fold = 1;
        while (st + 2 < st_end) {  // steps st and st + 1 both have a successor
            step(st, set1, yes, yes);
            step(st + 1, set0, yes, yes);
            st += 2;
            since_fold += 2;
            if (GRAD && since_fold >= kFoldSteps) {
                fold();
                since_fold = 0;
            }
        }
        if (st + 1 < st_end) {
            step(st, set1, yes, yes);
            step(st + 1, set0, yes, no);
        } else {
            step(st, set1, yes, no);
            last_set = 1;
        }
    }
    if constexpr (GRAD) {
        // adjoint of the last step: its X^T tile is still in the ring, since
        // nothing past st_end is staged
        const int ls = (st_end - 1) & 3;
        Frags f = aload(ls, 0);
#pragma unroll
        for (int q = 0; q < KBT; ++q) {
            const Frags nf = q + 1 < KBT ? aload(ls, q + 1) : f;
            if (last_set == 0) amfma(0, f, q);
            else amfma(1, f, q);
            f = nf;
        }
        fold();
    }

    // ---- the log-likelihood partial ----
    const int64_t o_begin = obase + (int64_t)st_begin * 32;
    const int64_t o_end = obase + (int64_t)st_end * 32;
    const int64_t valid = max<int64_t>(0, min(a.t1, o_end) - max(a.t0, o_begin));
    const double masked = (double)((o_end - o_begin) - valid) * (double)flog2((float)(NC + 1));
    double* ll_out = a.out_ll + (int64_t)split * a.P;
#pragma unroll
    for (int b = 0; b < PW; ++b) {
        double v = acc64[b];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        const int64_t p = pbase + b * 16 + r16;
        if (g == 0 && p < a.P) ll_out[p] = (v + masked) * kLn2;
    }
}

template <int NC, int KS, bool GRAD>
hipError_t launch_loglik_pipe(const LoglikArgs& a, dim3 grid, hipStream_t s) {
    hipLaunchKernelGGL((loglik_pipe_kernel<NC, KS, GRAD>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int NC, int KS, bool GRAD>
LoglikEntry loglik_pipe_entry() {
    LoglikEntry e;
    e.fn = &launch_loglik_pipe<NC, KS, GRAD>;
    e.ppb = 4 * 16 * PipeShape<NC, KS, GRAD>::PW;
    // one workgroup per CU is resident at these register and LDS sizes; two
    // rounds of 256 keep every CU busy to the end
    e.target = 512;
    return e;
}

// BF16x3 instantiations, one lookup per translation unit: the forward
// kernel for k > 32 (loglik_pipe_fwd_{a,b,c,d}.hip: C = 2..3, 4..5, 6, 7..8,
// compiled in parallel) and the adjoint kernel for C = 2, k > 32
// (loglik_pipe_grad.hip); the shapes are those of bf16_pipe_shape.
LoglikEntry lookup_pipe_fwd_a(int nc, int ks);
LoglikEntry lookup_pipe_fwd_b(int nc, int ks);
LoglikEntry lookup_pipe_fwd_c(int nc, int ks);
LoglikEntry lookup_pipe_fwd_d(int nc, int ks);
LoglikEntry lookup_pipe_grad(int nc, int ks);
inline LoglikEntry lookup_pipe(int nc, int ks, bool grad) {
    if (grad) return lookup_pipe_grad(nc, ks);
    return nc <= 2 ? lookup_pipe_fwd_a(nc, ks) : nc <= 4 ? lookup_pipe_fwd_b(nc, ks)
           : nc == 5 ? lookup_pipe_fwd_c(nc, ks) : lookup_pipe_fwd_d(nc, ks);
}

}  // namespace sps
