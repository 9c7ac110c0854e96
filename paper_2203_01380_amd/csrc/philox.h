// Philox4x32 counter-based generator (Salmon, Moraes, Dror & Shaw, SC'11)
// for gfx950, with R rounds: 10 (the published Philox4x32-10, draw
// specification v1) or 7 (v2; its authors report that seven rounds already
// pass their statistical test batteries).  Each round multiplies counter
// words 0 and 2 by the two Philox multipliers (full 32x32 -> 64-bit
// products, one v_mad_u64_u32 each), then
//   (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// and the key advances by the two Weyl increments between rounds.  The key
// words are wave-uniform, so their schedule stays in scalar registers; each
// three-way xor is one v_bitop3_b32, so a round is four VALU instructions.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace ilg {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// a ^ b ^ c in one gfx950 v_bitop3_b32 (truth table 0x96): the compiler
// leaves the round's two-step xor chain as two instructions otherwise.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

template <int R>
__device__ __forceinline__ uint4 philox4x32(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1)
{
    static_assert(R == 7 || R == 10, "draw specifications use 10 or 7 rounds");
#pragma unroll
    for (int round = 0; round < R; ++round) {
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
    return philox4x32<10>(c0, c1, c2, c3, k0, k1);
}

}  // namespace ilg
