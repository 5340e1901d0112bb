// Philox4x32-10 counter-based generator on the device, and the maps from its
// words to uniforms and normals.
//
// The paper (Section 5, RNG discussion) recommends Philox (Salmon et al.
// 2011) because every thread can jump to its own stream in constant time and
// draw a varying number of values.  Here no generator state is stored at all:
// every draw is Philox(counter, key) with
//   key     = (seed low 32 bits, seed high 32 bits)
//   counter = (row or coordinate index, sweep number k, tag << 24 | round, chain)
// so a lane that needs another proposal just increments "round".
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hsp {

enum : uint32_t {
    kTagZ = 1,
    kTagLambda = 2,
    kTagTau = 3,
    kTagBetaS = 4,
    kTagNu = 5,
    kTagXi = 6,
};

struct Words4 {
    uint32_t w0, w1, w2, w3;
};

// Ten Philox rounds (Salmon et al. 2011, Philox4x32 with R = 10).  Each round
// takes the full 64-bit products of counter words 0 and 2 with two odd
// multipliers; the high halves are xored with the remaining words and the
// round key, and the round key advances by the two Weyl constants.
__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each product whole, in one 32 x 32 -> 64-bit multiply
        const uint64_t pa = (uint64_t)0xD2511F53u * c0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
        c0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        c1 = (uint32_t)pb;
        c2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        c3 = (uint32_t)pa;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words4{c0, c1, c2, c3};
}

__device__ __forceinline__ Words4 draw_words(uint64_t seed, uint32_t idx, uint32_t sweep,
                                             uint32_t tag, uint32_t round, uint32_t chain) {
    return philox4x32_10(idx, sweep, (tag << 24) | (round & 0x00FFFFFFu), chain,
                         (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Uniform strictly inside (0,1): an odd 24-bit integer times 2^-24.  The
// value is exact in float and in double, so both precisions see it alike.
__device__ __forceinline__ float u01f(uint32_t w) {
    return (float)((w >> 8) | 1u) * 0x1p-24f;
}
__device__ __forceinline__ double u01d(uint32_t w) {
    return (double)((w >> 8) | 1u) * 0x1p-24;
}

// Box-Muller (1958) normal from two uniforms, float64.
__device__ __forceinline__ double box_muller_d(double u1, double u2) {
    return sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

}  // namespace hsp
