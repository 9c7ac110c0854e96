// Philox4x32 counter-based generator (Salmon, Moraes, Dror & Shaw, SC'11)
// for gfx950, with R rounds: 10 (the published Philox4x32-10, draw
// specification v1) or 7 (v2; its authors report that seven rounds already
// pass their statistical test batteries).  Each round multiplies counter
// words 0 and 2 by the two Philox multipliers (full 32x32 -> 64-bit
// products, one v_mad_u64_u32 each), then
//   (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// and the key advances by the two Weyl increments between rounds (round i
// uses k0 + i W0, k1 + i W1).  The key words are wave-uniform, so their
// schedule stays in scalar registers; each three-way xor is one
// v_bitop3_b32, so a round is four VALU instructions.
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

// Key of the generator: the two key words, the round keys (k0 + i W0,
// k1 + i W1) formed round by round.
struct PhiloxKey {
    uint32_t k0, k1;
    __device__ __forceinline__ uint32_t a(int i) const { return k0 + (uint32_t)i * kPhiloxW0; }
    __device__ __forceinline__ uint32_t b(int i) const { return k1 + (uint32_t)i * kPhiloxW1; }
};

// The same key with its ten round keys formed beforehand (the serving
// descriptors carry them, so a tile of a request does not rebuild them).
struct PhiloxSchedule {
    uint32_t ka[10], kb[10];
    __device__ __forceinline__ uint32_t a(int i) const { return ka[i]; }
    __device__ __forceinline__ uint32_t b(int i) const { return kb[i]; }
};

// RUN: rounds run (R, or R - 1 for the state before the last round).
template <int R, typename K, int RUN = R>
__device__ __forceinline__ uint4 philox4x32(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            const K &key)
{
    static_assert(R == 7 || R == 10, "draw specifications use 10 or 7 rounds");
    static_assert(RUN == R || RUN == R - 1, "all rounds, or all but the last");
#pragma unroll
    for (int round = 0; round < RUN; ++round) {
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, key.a(round));
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, key.b(round));
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return make_uint4(c0, c1, c2, c3);
}

template <int R>
__device__ __forceinline__ uint4 philox4x32(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1)
{
    return philox4x32<R>(c0, c1, c2, c3, PhiloxKey{k0, k1});
}

// The same block when only counter word 0 (the node) differs between lanes
// and t, r, b and the key are wave-uniform: the parts of the first two rounds
// that depend on uniform words only are written as plain arithmetic, which
// the compiler keeps on the scalar unit (the three-input xor builtin is a
// vector instruction; fed uniform operands it pulls the first round's word
// into vector registers and its product into quarter-rate vector
// multiplies).  Same function as philox4x32.
template <int R, typename K, int RUN = R>
__device__ __forceinline__ uint4 philox4x32_x(uint32_t x, uint32_t t, uint32_t r, uint32_t b,
                                              const K &key)
{
    static_assert(R == 7 || R == 10, "draw specifications use 10 or 7 rounds");
    static_assert(RUN == R || RUN == R - 1, "all rounds, or all but the last");
    // round 1 on (x, t, r, b)
    const uint64_t p0 = (uint64_t)kPhiloxM0 * x;
    const uint64_t q1 = (uint64_t)kPhiloxM1 * r;                    // uniform
    const uint32_t u0 = (uint32_t)(q1 >> 32) ^ t ^ key.a(0);        // uniform
    const uint32_t u1 = (uint32_t)q1;                               // uniform
    uint32_t c2 = (uint32_t)(p0 >> 32) ^ (b ^ key.b(0));
    uint32_t c3 = (uint32_t)p0;
    // round 2 on (u0, u1, c2, c3)
    const uint64_t q0 = (uint64_t)kPhiloxM0 * u0;                   // uniform
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
    uint32_t c0 = (uint32_t)(p1 >> 32) ^ (u1 ^ key.a(1));
    uint32_t c1 = (uint32_t)p1;
    c2 = c3 ^ ((uint32_t)(q0 >> 32) ^ key.b(1));
    const uint32_t u3 = (uint32_t)q0;                               // uniform
    // round 3 on (c0, c1, c2, u3)
    {
        const uint64_t a0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t a1 = (uint64_t)kPhiloxM1 * c2;
        c0 = xor3((uint32_t)(a1 >> 32), c1, key.a(2));
        c2 = (uint32_t)(a0 >> 32) ^ (u3 ^ key.b(2));
        c1 = (uint32_t)a1;
        c3 = (uint32_t)a0;
    }
#pragma unroll
    for (int round = 3; round < RUN; ++round) {
        const uint64_t a0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t a1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = xor3((uint32_t)(a1 >> 32), c1, key.a(round));
        const uint32_t n2 = xor3((uint32_t)(a0 >> 32), c3, key.b(round));
        c1 = (uint32_t)a1;
        c3 = (uint32_t)a0;
        c0 = n0;
        c2 = n2;
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
    return philox4x32<10>(c0, c1, c2, c3, k0, k1);
}

}  // namespace ilg
