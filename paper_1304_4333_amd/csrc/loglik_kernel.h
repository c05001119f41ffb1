// loglik_kernel.h -- the per-particle multinomial-logit log-likelihood and its
// adjoint on gfx950 matrix cores.
//
// What is computed (eq. (plogit), normalised by theta_0 = 0, summed over the
// product form of the likelihood): for particle p and observation t,
//     eta_{p,t,c} = x_t' theta_{p,c}   (c = 1..C-1),  eta_{p,t,0} = 0,
//     l_{p,t}     = eta_{p,t,y_t} - log sum_c exp(eta_{p,t,c}),
//     LL_p        = sum_{t0 <= t < t1} l_{p,t},
// and optionally G_{p,c} = sum_t x_t (1{y_t = c} - pi_{p,t,c}).
//
// Work decomposition.  A wave owns PW blocks of 16 particles and walks its
// share of the observations in steps of 32 rows.  The contraction eta = X B
// runs on MFMA with observations as rows and particles as columns, so the
// C-1 predictors of one (observation, particle) land in the same lane (one
// MFMA chain per outcome) and the log-sum-exp and the sum over observations
// need no lane exchange until the end.  theta is read once per wave and kept
// in registers as the B operand for the whole observation loop; X streams
// through L2 (it is re-read once per particle tile, never per particle).
//
// MFMA shapes (gfx950 lane layouts, measured with an in-bounds probe):
//   f32  16x16x4 : A lane l -> (row l%16, kslot l/16); B -> (kslot l/16, col l%16)
//   f64  16x16x4 : same A/B layout, FP64
//   bf16 16x16x32: A lane l -> (row l%16, kslots 8(l/16)..+7); B likewise
//   D of f32 and bf16: lane l holds rows 4(l/16)+i, i = 0..3, of column l%16;
//   D of f64         : lane l holds rows (l/16)+4i, i = 0..3, of column l%16.
// The contraction index may be assigned to (step, kslot) in any order as long
// as A and B agree; lane group g = l/16 takes a contiguous run of covariates,
// so each lane's A fragment is one contiguous piece of an X row.
//
// Row order inside a 32-row step: in MFMA tile h (0, 1) the D row that lane
// group g holds as value i covers observation o + 8g + 4h + i (the A-operand
// rows are permuted accordingly, which differs between the f64 and the other
// D layouts).  Lane group g then holds observations o + 8g .. o + 8g + 7 across
// the two tiles, which is exactly the contiguous K fragment the adjoint MFMA
// (X^T R) needs in its B operand.
//
// Precision modes: FP64 (parity anchor), FP32, and BF16x3 where each operand
// is split into hi + lo BF16 parts and eta ~ Xh Bh + Xh Bl + Xl Bh with FP32
// accumulation.  In the FP32/BF16 modes theta is pre-scaled by log2(e) so the
// log-sum-exp runs on the hardware base-2 exp/log; partial sums per 32-row
// step are carried into FP64 per lane.
#pragma once

#include <type_traits>

#include "sps_internal.h"

namespace sps {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.69314718055994530942;

// MODE_PEROBS: the forward kernel as launched for per-observation output (C
// phase): same arithmetic, tuned for short observation ranges.
enum { MODE_FWD = 0, MODE_GRAD = 1, MODE_PEROBS = 2 };

struct LoglikArgs {
    const void* X;      // row-major kernel copy of X (FP64 / FP32 / BF16 hi)
    const void* Xlo;    // BF16 lo part (BF16X3 only)
    const void* XT;     // transposed copy (kp x Tp) for the adjoint
    const void* XTlo;   // BF16 lo part of the transposed copy
    const int8_t* y8;   // outcomes as bytes
    const double* theta;
    double* out_ll;     // nsplit == 1: final ll[P]; else partials [nsplit][P]
    double* out_g;      // nsplit == 1: final grad[P][d]; else partials [nsplit][P][d]
    void* perobs;       // optional: per-observation terms [(t - t0) * P + p]:
                        // FP64 in natural log (FP64 mode), else FP32 in base 2
    double* chunk_tot;  // with perobs: per-particle total of every 32-row step,
                        // [step * P + p], natural log, FP64, summed in a fixed order
    const unsigned* skip;  // optional: the launch does nothing when *skip is nonzero
    int64_t P;
    int64_t Tp;
    int64_t t0, t1, t0a;  // t0a = t0 rounded down to a multiple of 32
    int32_t k, d, ldx;    // covariates, parameters, row stride of X
    int32_t nsteps, steps_per_split, nsplit;
    int32_t binary;       // C == 2: rows of X are sign-folded
    // Waves of a workgroup that share one particle group and split its
    // observations (1, 2 or 4; kernels with Shape::WSPLIT only): the
    // observation range has nsplit * wsplit parts, part (block split) * wsplit
    // + (wave % wsplit); the waves' sums are added in LDS in part order and
    // written once, to slice (block split) of the outputs.
    int32_t wsplit;
};

__device__ __forceinline__ f32x4 mfma(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Round-to-nearest-even FP32 -> BF16 bits.
__device__ __forceinline__ unsigned short to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) {
    return __uint_as_float(((unsigned)h) << 16);
}

__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float flog2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Precision traits.
template <int PREC> struct Prec;
template <> struct Prec<SPS_FP64> {
    using E = double;   // epilogue arithmetic
    using Acc = f64x4;
    static constexpr int KPS = 4;    // contraction length per MFMA
};
template <> struct Prec<SPS_FP32> {
    using E = float;
    using Acc = f32x4;
    static constexpr int KPS = 4;
};
template <> struct Prec<SPS_BF16X3> {
    using E = float;
    using Acc = f32x4;
    static constexpr int KPS = 32;
};

// PW, the particle blocks (of 16) per wave, chosen at compile time; the
// register counts (32-bit registers per lane) bound it.
template <int PREC, int NC, int KS, int MODE>
struct Shape {
    static constexpr bool BF = PREC == SPS_BF16X3;
    static constexpr int w = PREC == SPS_FP64 ? 2 : 1;           // registers per element
    static constexpr int breg = BF ? 8 * KS : w * KS;             // theta fragments per (block, outcome)
    static constexpr int accr = 2 * 4 * w;                        // one set: two tiles x 4 values
    static constexpr int kbt = BF ? 2 * KS : KS / 4;              // adjoint k blocks of 16
    static constexpr int grad = MODE == MODE_GRAD ? (4 * w * kbt + 8 * w) : 0;
    static constexpr int afrag = 2 * (BF ? 8 * KS : w * KS);      // one set: two tiles
    static constexpr int per1 = NC * (breg + accr + grad);
    // Measured on gfx950 (binary k=30 in all three precisions, BF16 with
    // k = 20/50/100 and C = 4/6): several particle blocks per wave pay off when
    // a wave has a single outcome column (each X fragment then feeds NC*PW
    // MFMA chains): four for the FP32/BF16 forward kernel, two with the
    // adjoint and for FP64; with C > 2 the outcome columns already give that
    // reuse and the extra registers cost occupancy.  The FP64 adjoint (64
    // registers per block) is the exception.  Over 256 live registers per lane,
    // use one.
    static constexpr int PW =
        MODE == MODE_PEROBS ? 1
        : (NC == 1 && PREC != SPS_FP64 && afrag + 4 * per1 <= 160) ? 4
        : (NC == 1 && !(PREC == SPS_FP64 && MODE == MODE_GRAD) && afrag + 2 * per1 <= 256) ? 2 : 1;
    // Workgroups per launch the observation split aims at.  Measured: the
    // FP32/BF16 kernels run fastest with few, long workgroups (about one or
    // two waves per SIMD; fewer split partials and prologues), the gradient
    // kernels with 256, the forward with 512, C > 2 gradients with 1024.  FP64,
    // the C > 2 forward kernels (multi4: 350 us at 2048 against 367 us at 1024)
    // and the per-observation launches keep more workgroups for latency hiding.
    static constexpr int TARGET =
        (PREC == SPS_FP64 || MODE == MODE_PEROBS || (NC > 1 && MODE == MODE_FWD)) ? 2048
        : NC > 1 ? 1024 : (MODE == MODE_GRAD ? 256 : 512);
    // The FP32/BF16 adjoint keeps each wave's FP64 gradient copy in LDS when
    // the four waves' copies fit (FP64 adds into the output slice instead).
    static constexpr int FOLDVALS = MODE == MODE_GRAD ? PW * NC * kbt * 4 : 1;
    static constexpr bool LFOLD = MODE == MODE_GRAD && PREC != SPS_FP64 && 4 * FOLDVALS * 64 * 8 <= 160 * 1024;
    // Whether waves may split a particle group's observations inside the
    // workgroup (wsplit > 1): the forward kernel, and the adjoint with its
    // gradient copy in LDS when the log-likelihood sums fit beside it.
    static constexpr bool WSPLIT =
        MODE == MODE_FWD || (LFOLD && 4 * FOLDVALS * 64 * 8 + 4 * PW * 16 * 8 <= 160 * 1024);
};

template <int PREC, int NC, int KS, int MODE>
constexpr int pick_pw() {
    return Shape<PREC, NC, KS, MODE>::PW;
}

template <bool V> using bconst = std::integral_constant<bool, V>;

template <int PREC, int NC, int KS, int MODE>
__global__ __launch_bounds__(256) void loglik_kernel(LoglikArgs a) {
    using P_ = Prec<PREC>;
    using E = typename P_::E;
    using Acc = typename P_::Acc;
    constexpr bool BF = (PREC == SPS_BF16X3);
    constexpr bool F64 = (PREC == SPS_FP64);
    constexpr int PW = Shape<PREC, NC, KS, MODE>::PW;
    constexpr int KBT = BF ? 2 * KS : KS / 4;  // adjoint k blocks of 16 (rows of XT)
    constexpr bool GRAD = (MODE == MODE_GRAD);
    // Multinomial FP32/BF16: the eta_{y_t} term of the log-likelihood is
    // linear in theta (sum_t eta_{y_t} = sum_c theta_c' S_c, S_c the sum of
    // the x_t with y_t = c over the range), and so is the 1{y_t = c} term of
    // the adjoint; both are added outside this kernel, which then evaluates
    // only -log sum_c exp(eta_c) and -pi_c (no outcome needed).  The outside
    // term uses x and theta rounded exactly as here, so the rounding errors of
    // the two parts cancel as they would in eta_y - LSE (otherwise the error
    // would grow with sum_t pi_t x_t, i.e. with T, instead of with the gradient).
    constexpr bool SUFF = (NC > 1) && !F64;
    // Steps take an unshifted fast form of the epilogue first and are redone
    // with the max-shifted form when a lane leaves its safe range (see body).
    constexpr bool FASTOK = SUFF || (NC == 1 && !F64);
    // The FP32 adjoint accumulators are added into the wave's FP64 output
    // slice every kFoldSteps steps (4096 observations), bounding the length
    // of any FP32 running sum; FP64 accumulates in registers throughout.
    constexpr int kFoldSteps = F64 ? (1 << 30) : 128;

    if (a.skip != nullptr && *a.skip != 0u) return;  // the same value for every wave
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int r16 = lane & 15;
    constexpr bool WS = Shape<PREC, NC, KS, MODE>::WSPLIT;
    const int ws = WS ? a.wsplit : 1;     // waves per particle group
    const int wpart = WS ? wave % ws : 0; // this wave's part of the group's observations
    const int oslice = blockIdx.x % a.nsplit;
    const int split = oslice * ws + wpart;
    const int64_t ptile = blockIdx.x / a.nsplit;
    const int64_t pbase = (ptile * (4 / ws) + wave / ws) * (16 * PW);
    // whole wave beyond the last particle: the waves of its group leave with
    // it, so the one barrier below (ws > 1) waits only for groups with work
    if (pbase >= a.P) return;

    // ---- B operand: theta of this wave's particles, kept in registers ----
    // f32/f64: step s, lane group g covers covariate g*KS + s.
    // bf16   : step s, lane group g covers covariates g*8*KS + 8 s + j.
    // Addresses are clamped into range and invalid entries zeroed afterwards,
    // so every load is unconditional and can be in flight together.
    using BReg = typename std::conditional<BF, bf16x8, E>::type;
    BReg bh[PW][NC][KS];
    BReg bl[BF ? PW : 1][BF ? NC : 1][BF ? KS : 1];
#pragma unroll
    for (int b = 0; b < PW; ++b) {
        const int64_t p = pbase + b * 16 + r16;
        const bool pv = p < a.P;
        const double* th = a.theta + (pv ? p : a.P - 1) * a.d;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                if constexpr (BF) {
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
                } else {
                    const int kk = g * KS + s;
                    const double raw = th[c * a.k + min(kk, a.k - 1)];
                    bh[b][c][s] = (pv && kk < a.k) ? (E)(F64 ? raw : raw * kLog2e) : E(0);
                }
            }
        }
    }

    double acc64[PW];
#pragma unroll
    for (int b = 0; b < PW; ++b) acc64[b] = 0.0;
    Acc gacc[GRAD ? PW : 1][GRAD ? NC : 1][GRAD ? KBT : 1];
    if constexpr (GRAD) {
#pragma unroll
        for (int b = 0; b < PW; ++b)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int q = 0; q < KBT; ++q) gacc[b][c][q] = Acc{0, 0, 0, 0};
    }
    // The binary FP32/BF16 epilogue hands the adjoint +sigmoid instead of the
    // residual -sigmoid (saves a sign flip per element); the sign is applied here.
    constexpr bool kNegRes = (NC == 1) && !F64;
    double* const g_out = GRAD ? a.out_g + (int64_t)oslice * a.P * a.d : nullptr;
    bool g_first = true;
    // The FP32 adjoint tiles are added into an FP64 copy every kFoldSteps
    // steps.  That copy lives in LDS (one slot per lane and value, private to
    // the wave) when the four waves' copies fit, and the gradient is written
    // to HBM once at the end; otherwise it is the wave's slice of the output
    // itself, read and written at every fold.
    constexpr int kFoldVals = Shape<PREC, NC, KS, MODE>::FOLDVALS;
    constexpr bool LFOLD = Shape<PREC, NC, KS, MODE>::LFOLD;
    __shared__ double fold_lds[LFOLD ? 4 * kFoldVals * 64 : 1];
    double* const fold_w = fold_lds + (LFOLD ? wave * kFoldVals * 64 + lane : 0);
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
                            const double gv = (double)gacc[b][c][q][i];
                            if constexpr (LFOLD) {
                                double* sl = fold_w + (((b * NC + c) * KBT + q) * 4 + i) * 64;
                                *sl = (g_first ? 0.0 : *sl) + gv;
                            } else {
                                const int kk = q * 16 + (F64 ? g + 4 * i : 4 * g + i);
                                if (p < a.P && kk < a.k) {
                                    double* dst = g_out + p * a.d + c * a.k + kk;
                                    *dst = (g_first ? 0.0 : *dst) + (kNegRes ? -gv : gv);
                                }
                            }
                        }
                        gacc[b][c][q] = Acc{0, 0, 0, 0};
                    }
            }
            g_first = false;
        }
    };
    // LDS copy -> output, once (the binary residual's sign applied here); with
    // ws > 1 the first wave of each group adds its group's copies in part order
    auto fold_out = [&]() __attribute__((always_inline)) {
        if constexpr (LFOLD) {
            if (wpart != 0) return;
#pragma unroll
            for (int b = 0; b < PW; ++b) {
                const int64_t p = pbase + b * 16 + r16;
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int q = 0; q < KBT; ++q)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int kk = q * 16 + 4 * g + i;
                            const int idx = (((b * NC + c) * KBT + q) * 4 + i) * 64;
                            double v = fold_w[idx];
                            for (int w2 = 1; w2 < ws; ++w2) v += fold_w[w2 * kFoldVals * 64 + idx];
                            if (p < a.P && kk < a.k) g_out[p * a.d + c * a.k + kk] = kNegRes ? -v : v;
                        }
            }
        }
    };

    const int st_begin = split * a.steps_per_split;
    const int st_end = min(a.nsteps, st_begin + a.steps_per_split);
    // A-operand row of this lane inside a 32-row step (tile h adds 4h): the
    // D row r = 4g+i (f32/bf16) or r = g+4i (f64) must map to o + 8g + i.
    const int arow = F64 ? 8 * (r16 & 3) + (r16 >> 2) : 8 * (r16 >> 2) + (r16 & 3);

    // A fragments (loaded one step ahead) and forward accumulators
    using AReg = typename std::conditional<BF, bf16x8, E>::type;
    AReg ah[2][KS];                       // [tile][k-step]
    AReg al[BF ? 2 : 1][BF ? KS : 1];
    Acc acc[2][PW][NC];                   // [tile][block][outcome]
    auto load_a = [&](int64_t o) __attribute__((always_inline)) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t row = o + arow + 4 * h;
            if constexpr (BF) {
                const unsigned short* xh = (const unsigned short*)a.X + row * a.ldx + g * 8 * KS;
                const unsigned short* xl = (const unsigned short*)a.Xlo + row * a.ldx + g * 8 * KS;
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    ah[h][s] = __builtin_bit_cast(bf16x8, *(const u16x8*)(xh + 8 * s));
                    al[h][s] = __builtin_bit_cast(bf16x8, *(const u16x8*)(xl + 8 * s));
                }
            } else {
                const E* xr = (const E*)a.X + row * a.ldx + g * KS;
#pragma unroll
                for (int s = 0; s < KS; ++s) ah[h][s] = xr[s];
            }
        }
    };
    // forward contraction of one step, independent chains interleaved
    auto mfma_fwd = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int b = 0; b < PW; ++b)
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[h][b][c] = Acc{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int b = 0; b < PW; ++b)
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        if constexpr (BF) {
                            acc[h][b][c] = mfma(ah[h][s], bh[b][c][s], acc[h][b][c]);
                            acc[h][b][c] = mfma(ah[h][s], bl[b][c][s], acc[h][b][c]);
                            acc[h][b][c] = mfma(al[h][s], bh[b][c][s], acc[h][b][c]);
                        } else {
                            acc[h][b][c] = mfma(ah[h][s], bh[b][c][s], acc[h][b][c]);
                        }
                    }
    };

    // One step: forward MFMAs, epilogue and adjoint of step st.
    // interior_c: the step is known to lie inside [t0, t1) with a successor,
    // so the unmasked epilogue is chosen at compile time (given one body with
    // both epilogues behind a runtime test, the compiler merges them into one
    // path that pays the masking selects on every step).
    auto body = [&](int st, bool has_next, auto interior_c) __attribute__((always_inline)) {
        constexpr bool INTERIOR = decltype(interior_c)::value;
        const int64_t o = a.t0a + (int64_t)st * 32;
        mfma_fwd();
        if (has_next) load_a(o + 32);  // the MFMAs have read this step's fragments
        // A operand of the adjoint (rows of the transposed X for this step),
        // requested before the epilogue so the load latency hides behind it.
        using XtReg = typename std::conditional<BF, bf16x8, E>::type;
        XtReg xth[GRAD ? KBT : 1][BF ? 1 : 8];
        XtReg xtl[GRAD && BF ? KBT : 1];
        if constexpr (GRAD) {
#pragma unroll
            for (int q = 0; q < KBT; ++q) {
                const int64_t xrow = (int64_t)(q * 16 + r16) * a.Tp + o + 8 * g;
                if constexpr (BF) {
                    xth[q][0] = __builtin_bit_cast(bf16x8, *(const u16x8*)((const unsigned short*)a.XT + xrow));
                    xtl[q] = __builtin_bit_cast(bf16x8, *(const u16x8*)((const unsigned short*)a.XTlo + xrow));
                } else {
                    const E* xt = (const E*)a.XT + xrow;
#pragma unroll
                    for (int j = 0; j < 8; ++j) xth[q][j] = xt[j];
                }
            }
        }

        unsigned ylo = 0, yhi = 0;
        if (NC > 1 && (!SUFF || a.perobs != nullptr)) {
            const uint2 yy = *(const uint2*)(a.y8 + o + 8 * g);
            ylo = yy.x;
            yhi = yy.y;
        }
        bool bad = false;  // the unshifted fast epilogue left its safe range
        E rres[GRAD ? 2 : 1][GRAD ? 4 : 1][GRAD ? PW : 1][GRAD ? NC : 1];
        E tsum[PW];
#pragma unroll
        for (int b = 0; b < PW; ++b) tsum[b] = E(0);
        double csum[MODE == MODE_PEROBS ? PW : 1];  // per-observation mode: this lane's share of the step total
#pragma unroll
        for (int b = 0; b < (MODE == MODE_PEROBS ? PW : 1); ++b) csum[b] = 0.0;

            auto epilogue = [&](auto masked_c, auto perobs_c, auto fast_c) __attribute__((always_inline)) {
                constexpr bool MASKED = decltype(masked_c)::value;
                constexpr bool PEROBS = decltype(perobs_c)::value;
                constexpr bool FAST = decltype(fast_c)::value;  // unshifted form, checked after the step
                constexpr bool NOY = SUFF && !PEROBS;           // eta_y via sufficient statistics
                // binary fast form: the 8 factors 1 + 2^z of a lane and particle block are
                // multiplied and their log2 taken once (one log instead of eight)
                [[maybe_unused]] E prod[(NC == 1 && FAST) ? PW : 1];
                if constexpr (NC == 1 && FAST) {
#pragma unroll
                    for (int b = 0; b < PW; ++b) prod[b] = E(1);
                }
    #pragma unroll
                for (int h = 0; h < 2; ++h) {
    #pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int64_t obs = o + 8 * g + 4 * h + i;
                        const bool ov = !MASKED || (obs >= a.t0 && obs < a.t1);
                        const int yt = NC > 1 ? (int)(((h ? yhi : ylo) >> (8 * i)) & 0xFFu) : 0;
    #pragma unroll
                        for (int b = 0; b < PW; ++b) {
                            E lp;
                            if constexpr (NC == 1 && FAST) {
                                // base 2, unshifted: l2 = -log2(1 + 2^z), summed as
                                // -log2 of the product of the factors (below).  Exact in
                                // range while the product is finite; otherwise tsum turns
                                // -inf or NaN and the step is redone with the shifted form.
                                const E z = acc[h][b][0][i];
                                const float e = fexp2(z);
                                const float sfac = 1.f + e;
                                prod[b] *= (MASKED && !ov) ? 1.f : sfac;
                                lp = E(0);
                                // sigmoid(z) = 2^z / (1 + 2^z)
                                if constexpr (GRAD) rres[h][i][b][0] = ov ? e * frcp(sfac) : 0.f;
                            } else if constexpr (NC == 1) {
                                // Binary with sign folding: l = -softplus(z), z = x~' theta.
                                const E z = acc[h][b][0][i];
                                if constexpr (F64) {
                                    const double e = exp(-fabs(z));
                                    const double q = 1.0 + e;
                                    lp = -(fmax(z, 0.0) + log1p(e));
                                    if constexpr (GRAD) rres[h][i][b][0] = ov ? -(z > 0.0 ? 1.0 : e) / q : 0.0;
                                } else {
                                    // base 2: softplus2(z) = max(z, 0) + log2(1 + 2^-|z|);
                                    // max via the signed-integer order of float bits
                                    const float mz = __int_as_float(max(__float_as_int(z), 0));
                                    lp = -(mz + flog2(1.f + fexp2(-fabsf(z))));
                                    // sigmoid(z) = 2^(z - softplus2(z)); the residual is its negative
                                    if constexpr (GRAD) rres[h][i][b][0] = ov ? fexp2(z + lp) : 0.f;
                                }
                            } else if constexpr (NOY && FAST) {
                                // base 2 without a shift: exact while the sum stays below 2^126
                                E ec[NC];
                                E s = E(1);
    #pragma unroll
                                for (int c = 0; c < NC; ++c) {
                                    ec[c] = fexp2(acc[h][b][c][i]);
                                    s += ec[c];
                                }
                                bad |= !(s < 0x1p126f);
                                lp = -flog2(s);
                                if constexpr (GRAD) {
                                    const E inv = frcp(s);
    #pragma unroll
                                    for (int c = 0; c < NC; ++c) rres[h][i][b][c] = ov ? -ec[c] * inv : E(0);
                                }
                            } else {
                                E m = E(0);
                                E ey = E(0);
    #pragma unroll
                                for (int c = 0; c < NC; ++c) {
                                    const E v = acc[h][b][c][i];
                                    if constexpr (F64) m = v > m ? v : m;
                                    else m = __int_as_float(max(__float_as_int(v), __float_as_int(m)));  // m >= 0
                                    if constexpr (!NOY) ey = (yt == c + 1) ? v : ey;
                                }
                                E ec[NC];
                                E s;
                                if constexpr (F64) {
                                    s = exp(-m);
    #pragma unroll
                                    for (int c = 0; c < NC; ++c) {
                                        ec[c] = exp(acc[h][b][c][i] - m);
                                        s += ec[c];
                                    }
                                    lp = ey - (m + log(s));
                                } else {
                                    s = fexp2(-m);
    #pragma unroll
                                    for (int c = 0; c < NC; ++c) {
                                        ec[c] = fexp2(acc[h][b][c][i] - m);
                                        s += ec[c];
                                    }
                                    lp = ey - (m + flog2(s));
                                }
                                if constexpr (GRAD) {
                                    const E inv = F64 ? E(1) / s : frcp(s);
    #pragma unroll
                                    for (int c = 0; c < NC; ++c)
                                        rres[h][i][b][c] =
                                            ov ? ((!NOY && yt == c + 1 ? E(1) : E(0)) - ec[c] * inv) : E(0);
                                }
                            }
                            if constexpr (!(NC == 1 && FAST)) tsum[b] += MASKED ? (ov ? lp : E(0)) : lp;
                            if constexpr (PEROBS) {
                                const int64_t p = pbase + b * 16 + r16;
                                if (ov && p < a.P)
                                {
                                    const int64_t at = (obs - a.t0) * a.P + p;
                                    if constexpr (F64) ((double*)a.perobs)[at] = (double)lp;
                                    else ((float*)a.perobs)[at] = (float)lp;
                                }
                                // the stored value as the scan reads it (natural log)
                                if (ov) csum[b] += F64 ? (double)lp : (double)(float)lp * kLn2;
                            }
                        }
                    }
                }
                if constexpr (NC == 1 && FAST) {
#pragma unroll
                    for (int b = 0; b < PW; ++b) tsum[b] -= flog2(prod[b]);
                }
            };

        const bool full = (o >= a.t0) && (o + 32 <= a.t1);
        // Non-per-observation steps; the per-observation output exists only in
        // the MODE_PEROBS instantiation, so the other kernels carry none of it.
        auto regular = [&]() __attribute__((always_inline)) {
            if constexpr (FASTOK) {
                if (INTERIOR || (full && has_next)) {
                    epilogue(bconst<false>{}, bconst<false>{}, bconst<true>{});
                } else {
                    epilogue(bconst<true>{}, bconst<false>{}, bconst<true>{});
                }
                if constexpr (NC == 1) {
    #pragma unroll
                    for (int b = 0; b < PW; ++b) bad |= !(tsum[b] > -INFINITY);  // -inf or NaN
                }
                if (__any(bad)) {  // wave-uniform: redo this step with the max shift
    #pragma unroll
                    for (int b = 0; b < PW; ++b) tsum[b] = E(0);
                    epilogue(bconst<true>{}, bconst<false>{}, bconst<false>{});
                }
            } else if (INTERIOR || (full && has_next)) {
                epilogue(bconst<false>{}, bconst<false>{}, bconst<false>{});
            } else {
                epilogue(bconst<true>{}, bconst<false>{}, bconst<false>{});
            }
        };
        if constexpr (MODE == MODE_PEROBS) {
            if (a.perobs != nullptr) {
                epilogue(bconst<true>{}, bconst<true>{}, bconst<false>{});
                if (a.chunk_tot != nullptr) {
                    // lane group g holds rows 8g .. 8g + 7 of the step: total = ((s0 + s1) + s2) + s3
    #pragma unroll
                    for (int b = 0; b < PW; ++b) {
                        const double v1 = __shfl(csum[b], lane + 16, 64);
                        const double v2 = __shfl(csum[b], lane + 32, 64);
                        const double v3 = __shfl(csum[b], lane + 48, 64);
                        const int64_t p = pbase + b * 16 + r16;
                        if (g == 0 && p < a.P) a.chunk_tot[(int64_t)st * a.P + p] = ((csum[b] + v1) + v2) + v3;
                    }
                }
            } else {
                regular();
            }
        } else {
            regular();
        }
#pragma unroll
        for (int b = 0; b < PW; ++b) acc64[b] += (double)tsum[b];

            // ---- adjoint: G += X~^T R over the 32 rows of this step ----
            if constexpr (GRAD) {
                if constexpr (BF) {
    #pragma unroll
                    for (int q = 0; q < KBT; ++q) {
                        const bf16x8 th8 = xth[q][0];
                        const bf16x8 tl8 = xtl[q];
    #pragma unroll
                        for (int b = 0; b < PW; ++b)
    #pragma unroll
                            for (int c = 0; c < NC; ++c) {
                                // hi = the upper 16 bits (truncation, one byte permute per
                                // pair); lo = v - hi, exact in FP32, rounded in one packed
                                // conversion per pair: hi + bf16(lo) is within 2^-16 |v| of v
                                typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
                                typedef float f32x2 __attribute__((ext_vector_type(2)));
                                typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
                                u32x4 wh, wl;
#pragma unroll
                                for (int w = 0; w < 4; ++w) {
                                    const float v0 = rres[(2 * w) >> 2][(2 * w) & 3][b][c];
                                    const float v1 = rres[(2 * w + 1) >> 2][(2 * w + 1) & 3][b][c];
                                    const unsigned u0 = __float_as_uint(v0), u1 = __float_as_uint(v1);
                                    wh[w] = __builtin_amdgcn_perm(u1, u0, 0x07060302u);
                                    const float l0 = v0 - __uint_as_float(u0 & 0xFFFF0000u);
                                    const float l1 = v1 - __uint_as_float(u1 & 0xFFFF0000u);
                                    wl[w] = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){l0, l1}, bf16x2));
                                }
                                const bf16x8 Rh = __builtin_bit_cast(bf16x8, wh);
                                const bf16x8 Rl = __builtin_bit_cast(bf16x8, wl);
                                gacc[b][c][q] = mfma(th8, Rh, gacc[b][c][q]);
                                gacc[b][c][q] = mfma(th8, Rl, gacc[b][c][q]);
                                gacc[b][c][q] = mfma(tl8, Rh, gacc[b][c][q]);
                            }
                    }
                } else {
    #pragma unroll
                    for (int j = 0; j < 8; ++j)
    #pragma unroll
                        for (int q = 0; q < KBT; ++q)
    #pragma unroll
                            for (int b = 0; b < PW; ++b)
    #pragma unroll
                                for (int c = 0; c < NC; ++c)
                                    gacc[b][c][q] = mfma(xth[q][j], rres[j >> 2][j & 3][b][c], gacc[b][c][q]);
                }
            if (((st - st_begin) % kFoldSteps) == kFoldSteps - 1) fold();
        }
    };

    if (st_begin < st_end) {
        load_a(a.t0a + (int64_t)st_begin * 32);
        // steps whose 32 rows all lie in [t0, t1) and that have a successor run
        // a body without the masked epilogue; the others (at most one at each
        // end of the split) run the general body
        const int lo = max(st_begin, a.t0 > a.t0a ? 1 : 0);
        const int hi = min(st_end - 1, (int)((a.t1 - a.t0a) / 32));
        int st = st_begin;
        for (; st < st_end && st < lo; ++st) body(st, st + 1 < st_end, bconst<false>{});
        for (; st < hi; ++st) body(st, true, bconst<true>{});
        for (; st < st_end; ++st) body(st, st + 1 < st_end, bconst<false>{});
    }
    if constexpr (GRAD) {
        if (g_first || ((st_end - st_begin) % kFoldSteps) != 0) fold();
    }
    const double lscale = F64 ? 1.0 : kLn2;
    double* ll_out = a.out_ll + (int64_t)oslice * a.P;
    if constexpr (WS) {
        // ---- the log-likelihood partial: lane group sums, then (ws > 1) the
        // group's waves in part order through LDS ----
        __shared__ double ll_lds[4 * PW * 16];
#pragma unroll
        for (int b = 0; b < PW; ++b) {
            acc64[b] += __shfl_xor(acc64[b], 16, 64);
            acc64[b] += __shfl_xor(acc64[b], 32, 64);
        }
        if (ws > 1) {
            if (g == 0) {
#pragma unroll
                for (int b = 0; b < PW; ++b) ll_lds[(wave * PW + b) * 16 + r16] = acc64[b];
            }
            __syncthreads();  // also orders the waves' final folds before fold_out
            if (wpart == 0) {
#pragma unroll
                for (int b = 0; b < PW; ++b)
                    for (int w2 = 1; w2 < ws; ++w2) acc64[b] += ll_lds[((wave + w2) * PW + b) * 16 + r16];
            }
        }
        if constexpr (GRAD) fold_out();
        if (wpart != 0) return;
#pragma unroll
        for (int b = 0; b < PW; ++b) {
            const int64_t p = pbase + b * 16 + r16;
            if (g == 0 && p < a.P) ll_out[p] = acc64[b] * lscale;
        }
    } else {
        if constexpr (GRAD) fold_out();
        // ---- write the log-likelihood partial ----
#pragma unroll
        for (int b = 0; b < PW; ++b) {
            double v = acc64[b];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            const int64_t p = pbase + b * 16 + r16;
            if (g == 0 && p < a.P) ll_out[p] = v * lscale;
        }
    }
}

// Fixed-order sum of the observation-split partials.
__global__ void loglik_reduce_kernel(const double* __restrict__ part_ll,
                                     const double* __restrict__ part_g, int64_t P, int32_t d,
                                     int32_t nsplit, double* __restrict__ ll,
                                     double* __restrict__ grad);

// Host-side launcher for one (PREC, NC, KS, MODE) instantiation.
template <int PREC, int NC, int KS, int MODE>
hipError_t launch_loglik(const LoglikArgs& a, dim3 grid, hipStream_t s) {
    hipLaunchKernelGGL((loglik_kernel<PREC, NC, KS, MODE>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int PREC, int NC, int KS, int MODE>
constexpr int particles_per_block() {
    return 4 * 16 * pick_pw<PREC, NC, KS, MODE>();
}

typedef hipError_t (*LoglikLaunchFn)(const LoglikArgs&, dim3, hipStream_t);
struct LoglikEntry {
    LoglikLaunchFn fn = nullptr;
    int ppb = 0;     // particles per 256-thread block
    int target = 0;  // workgroups per launch the observation split aims at
    bool wsplit = false;  // the kernel takes LoglikArgs::wsplit > 1
};

template <int PREC, int NC, int KS, int MODE>
LoglikEntry loglik_entry() {
    LoglikEntry e;
    e.fn = &launch_loglik<PREC, NC, KS, MODE>;
    e.ppb = particles_per_block<PREC, NC, KS, MODE>();
    e.target = Shape<PREC, NC, KS, MODE>::TARGET;
    e.wsplit = Shape<PREC, NC, KS, MODE>::WSPLIT;
    return e;
}

// Full-range BF16x3 shapes run by the software-pipelined kernel
// (loglik_pipe.h) instead of this one: the forward kernel at k > 32 (KS >= 2)
// and the adjoint kernel for C = 2 at k > 32.  Measured on MI355X, the
// pipelined kernel is faster there (multi6 forward 17.3 against 21.7 ms,
// ar100 forward 1.4 against 2.8 ms and adjoint 3.0 against 5.6 ms); with
// C > 2 the adjoint's registers exceed one wave's budget and this kernel is
// faster (multi6 45.9 against 56.8 ms), as it is at k <= 32 (multi4,
// binary30), where a step is too short for the per-step LDS staging.
constexpr bool bf16_pipe_shape(int nc, int ks, int mode) {
    return mode == MODE_FWD ? ks >= 2 : mode == MODE_GRAD ? (nc == 1 && ks >= 2) : false;
}
template <int NC, int KS, int MODE>
LoglikEntry loglik_entry_bf16() {
    if constexpr (bf16_pipe_shape(NC, KS, MODE)) return LoglikEntry{};
    else return loglik_entry<SPS_BF16X3, NC, KS, MODE>();
}

// One lookup per precision, each defined in its own translation unit.
LoglikEntry lookup_fp64(int nc, int ks, int mode);
LoglikEntry lookup_fp32(int nc, int ks, int mode);
LoglikEntry lookup_bf16(int nc, int ks, int mode);
LoglikEntry lookup_bf16_wide(int nc, int ks, int mode);  // C = 6, 7
LoglikEntry lookup_bf16_c8(int nc, int ks, int mode);    // C = 8

}  // namespace sps
