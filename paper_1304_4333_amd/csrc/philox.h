// philox.h -- Philox4x32-10 counter-based generator (Salmon, Moraes, Dror &
// Shaw, SC'11) and the variate mappings used by libsps.
//
// Stream convention: block counter = (e_lo, e_hi, stream_lo, stream_hi) for
// element index e, key = (seed_lo, seed_hi).  A block gives two 53-bit
// integers a = (w0:w1) >> 11 and b = (w2:w3) >> 11.
//   u53(e)      = a
//   uniform(e)  = (a + 1/2) 2^-53
//   normal(p,i) : Box-Muller on block e = p ceil(d/2) + floor(i/2);
//                 i even -> r cos(2 pi u_b), i odd -> r sin(2 pi u_b),
//                 r = sqrt(-2 log u_a).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace sps {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

__device__ __forceinline__ void philox_u53x2(uint64_t seed, uint64_t stream, uint64_t e,
                                             uint64_t& a, uint64_t& b) {
    const uint4 w = philox4x32_10(make_uint4((uint32_t)e, (uint32_t)(e >> 32), (uint32_t)stream,
                                             (uint32_t)(stream >> 32)),
                                  (uint32_t)seed, (uint32_t)(seed >> 32));
    a = ((((uint64_t)w.x) << 32) | w.y) >> 11;
    b = ((((uint64_t)w.z) << 32) | w.w) >> 11;
}

__device__ __forceinline__ double u53_to_uniform(uint64_t a) {
    return ((double)a + 0.5) * 0x1p-53;
}

// Standard normal for element (p, i) of a P x d array.
__device__ __forceinline__ double philox_normal(uint64_t seed, uint64_t stream, int64_t p,
                                                int32_t i, int32_t d) {
    const int64_t half = (d + 1) / 2;
    uint64_t a, b;
    philox_u53x2(seed, stream, (uint64_t)(p * half + i / 2), a, b);
    const double r = sqrt(-2.0 * log(u53_to_uniform(a)));
    double s, c;
    sincospi(2.0 * u53_to_uniform(b), &s, &c);
    return (i & 1) ? r * s : r * c;
}

// Elements 2 j and 2 j + 1 of row p of a P x d array (the two values of one
// Box-Muller pair, as philox_normal gives them); z1 is meaningless when
// 2 j + 1 = d.
__device__ __forceinline__ void philox_normal_pair(uint64_t seed, uint64_t stream, int64_t p, int32_t j,
                                                   int32_t d, double& z0, double& z1) {
    const int64_t half = (d + 1) / 2;
    uint64_t a, b;
    philox_u53x2(seed, stream, (uint64_t)(p * half + j), a, b);
    const double r = sqrt(-2.0 * log(u53_to_uniform(a)));
    double s, c;
    sincospi(2.0 * u53_to_uniform(b), &s, &c);
    z0 = r * c;
    z1 = r * s;
}

}  // namespace sps
