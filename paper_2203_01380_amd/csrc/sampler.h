// Device-side sampler shared by the plain and batched lattice-gas kernels:
// Philox draws of one node-step, the chunked fixed-point binomial, and the
// node update (flip, removal binomials, multinomial redistribution).
//
// Per node x at step t (Eq. LGflip; D2Q5 nodes x + Lx y):
//   a_i   = n_{q-1-i}(x) if the flip is on, else n_i(x)          (Eq. flip)
//   k_i   = Bin(a_i, P)          removal: each particle collides w.p. P/2^32
//   M     = sum_i k_i
//   q = 2: m_0 = Bin(M, 2^31), m_1 = M - m_0
//   q = 3: m_1 = Bin(M, P_rest), R = M - m_1, m_0 = Bin(R, 2^31), m_2 = R - m_0
//   q = 5: m_2 = Bin(M, P_rest), R = M - m_2, m_x = Bin(R, 2^31), m_y = R - m_x,
//          m_0 = Bin(m_x, 2^31), m_4 = m_x - m_0, m_1 = Bin(m_y, 2^31), m_3 = m_y - m_1
//   c_i   = a_i - k_i + m_i   (streamed afterwards to x + v_i)
// Bin(n, p) takes ceil(n/64) 32-bit draws (full chunks of 64 first, then the
// remainder); a chunk of m trials with draw U yields #{j < m : T[m][j] <= U}.
// Draw j of a node-step is word j%4 of Philox4x32 block j/4 with counter
// (x, t, realization, j/4), the generator taking NR rounds (10: draw
// specification v1; 7: v2).
//
// gfx950 notes.  The work is integer VALU bound (Philox rounds and the
// inverse-CDF searches):
//  * the search starts at a guide entry (2^GB buckets per row) and makes two
//    table compares; longer scans run only for the lanes that need them;
//  * one wave-uniform test per node selects straight-line code with constant
//    draw-word indices when every lane shares the common chunk layout
//    (node_fast); for q = 3 a wave whose middle binomial needs 1, 2 or 3
//    chunks depending on the lane selects the later words per lane
//    (node_var3); the generic path picks words by a scalar switch when the
//    index is wave-uniform and by a select tree otherwise;
//  * the first NB Philox blocks are computed up front, later ones on demand.
#pragma once

#include <type_traits>

#include "ilg_internal.h"
#include "philox.h"

namespace ilg {
namespace sampler {

template <typename T, int N>
struct alignas(N * sizeof(T)) VecT {
    T v[N];
};

// Compile-time loop: f(std::integral_constant<int, K>) for K = B..E-1, so
// register arrays are only ever indexed by constants.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Element x of a velocity row.  For 16-bit counts the byte offset 2x fits in
// 32 bits (fewer than 2^31 nodes), so the address is a wave-uniform 64-bit
// row pointer plus a 32-bit lane offset, which the global load and store
// instructions take directly (no 64-bit add per lane).
template <typename P>
__device__ __forceinline__ P *row_elem(P *row, uint32_t x)
{
    if constexpr (sizeof(P) == 2) {
        using B = typename std::conditional<std::is_const<P>::value, const uint8_t, uint8_t>::type;
        return reinterpret_cast<P *>(reinterpret_cast<B *>(row) + (uint32_t)(x * 2u));
    } else {
        return row + x;
    }
}

__device__ __forceinline__ bool wave_any(bool p)
{
    return __builtin_amdgcn_ballot_w64(p) != 0ull;
}

// K: the key as two words (PhiloxKey) or with its round keys formed
// beforehand (PhiloxSchedule); both give the same draws.
template <int NB, int NR, typename K = PhiloxKey>
struct Draws {
    // Words of the eager blocks.  With two or more blocks the last block's
    // final round stops after its first product: its words 4 NB - 4 and
    // 4 NB - 3 are complete, while w[4 NB - 2] and w[4 NB - 1] hold the
    // inputs (counter words 0 and 3) of the second product, from which
    // word() forms words 4 NB - 2 and 4 NB - 1 where a path reads them (the
    // straight-line paths of most nodes read neither).
    uint32_t w[4 * NB];
    uint32_t x, t, r;
    K key;
    static constexpr bool kLazy = NB >= 2;

    __device__ __forceinline__ void init(uint32_t x_, uint32_t t_, uint32_t r_, const K &key_)
    {
        x = x_; t = t_; r = r_; key = key_;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            // with a precomputed schedule (serving slots) the uniform words
            // of the first rounds are per tile, so they are written for the
            // scalar unit; elsewhere the compiler hoists them anyway
            constexpr int kRun = NR;
            uint4 o;
            if (kLazy && b == NB - 1) {
                if constexpr (std::is_same<K, PhiloxSchedule>::value)
                    o = philox4x32_x<NR, K, NR - 1>(x, t, r, (uint32_t)b, key);
                else
                    o = philox4x32<NR, K, NR - 1>(x, t, r, (uint32_t)b, key);
                const uint64_t p1 = (uint64_t)kPhiloxM1 * o.z;
                w[4 * b + 0] = xor3((uint32_t)(p1 >> 32), o.y, key.a(NR - 1));
                w[4 * b + 1] = (uint32_t)p1;
                w[4 * b + 2] = o.x;
                w[4 * b + 3] = o.w;
                continue;
            }
            if constexpr (std::is_same<K, PhiloxSchedule>::value)
                o = philox4x32_x<kRun>(x, t, r, (uint32_t)b, key);
            else
                o = philox4x32<kRun>(x, t, r, (uint32_t)b, key);
            w[4 * b + 0] = o.x; w[4 * b + 1] = o.y; w[4 * b + 2] = o.z; w[4 * b + 3] = o.w;
        }
    }

    // Word k (a compile-time index below 4 NB) of the eager blocks.
    __device__ __forceinline__ uint32_t word(int k) const
    {
        if (!kLazy || k < 4 * NB - 2)
            return w[k];
        const uint64_t p0 = (uint64_t)kPhiloxM0 * w[4 * NB - 2];
        return k == 4 * NB - 2 ? xor3((uint32_t)(p0 >> 32), w[4 * NB - 1], key.b(NR - 1))
                               : (uint32_t)p0;
    }
};

__device__ __forceinline__ uint32_t pick4(uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                          uint32_t s)
{
    const uint32_t lo = (s & 1u) ? b : a;
    const uint32_t hi = (s & 1u) ? d : c;
    return (s & 2u) ? hi : lo;
}

// c3 ? c : (c2 ? b : a) on values (a conditional over array elements would
// be an lvalue select, i.e. a dynamically indexed array in scratch memory).
__device__ __forceinline__ uint32_t pick3(bool c2, bool c3, uint32_t a, uint32_t b, uint32_t c)
{
    const uint32_t lo = c2 ? b : a;
    return c3 ? c : lo;
}

// b ? y : x on values (see pick3).
__device__ __forceinline__ uint32_t pick2(bool b, uint32_t x, uint32_t y)
{
    return b ? y : x;
}

// f3 ? d : (f2 ? c : (f1 ? b : a)) on values, for f3 => f2 => f1.
__device__ __forceinline__ uint32_t pick_ge(bool f1, bool f2, bool f3, uint32_t a, uint32_t b,
                                            uint32_t c, uint32_t d)
{
    const uint32_t lo = f1 ? b : a;
    const uint32_t mid = f2 ? c : lo;
    return f3 ? d : mid;
}

// Word j of the lane's draw stream (lanes may ask for different j).
template <int NB, int NR, typename K>
__device__ __forceinline__ uint32_t draw_word(const Draws<NB, NR, K> &d, uint32_t j)
{
    constexpr uint32_t kEager = 4 * NB;
    const uint32_t j0 = __builtin_amdgcn_readfirstlane(j);
    uint32_t r;
    if (!wave_any(j != j0) && j0 < kEager) {
        // wave-uniform index: scalar branches pick the register
        static_assert(kEager <= 12, "at most three eager Philox blocks");
        switch (j0) {
        case 0: r = d.word(0); break;
        case 1: r = d.word(1); break;
        case 2: r = d.word(2); break;
        case 3: r = d.word(3); break;
        case 4: r = d.word(4 % kEager); break;
        case 5: r = d.word(5 % kEager); break;
        case 6: r = d.word(6 % kEager); break;
        case 7: r = d.word(7 % kEager); break;
        case 8: r = d.word(8 % kEager); break;
        case 9: r = d.word(9 % kEager); break;
        case 10: r = d.word(10 % kEager); break;
        default: r = d.word(kEager - 1); break;
        }
    } else {
        const uint32_t jc = j < kEager ? j : kEager - 1;
        if constexpr (NB == 1) {
            r = pick4(d.word(0), d.word(1), d.word(2), d.word(3), jc);
        } else if constexpr (NB == 2) {
            const uint32_t lo = pick4(d.word(0), d.word(1), d.word(2), d.word(3), jc & 3u);
            const uint32_t hi = pick4(d.word(4), d.word(5), d.word(6), d.word(7), jc & 3u);
            r = (jc & 4u) ? hi : lo;
        } else {
            const uint32_t b0 = pick4(d.word(0), d.word(1), d.word(2), d.word(3), jc & 3u);
            const uint32_t b1 = pick4(d.word(4), d.word(5), d.word(6), d.word(7), jc & 3u);
            const uint32_t b2 = pick4(d.word(8), d.word(9), d.word(10), d.word(11), jc & 3u);
            r = (jc >= 8u) ? b2 : ((jc >= 4u) ? b1 : b0);
        }
        if (wave_any(j >= kEager)) {
            if (j >= kEager) {
                const uint4 o = philox4x32<NR>(d.x, d.t, d.r, j >> 2, d.key);
                r = pick4(o.x, o.y, o.z, o.w, j & 3u);
            }
        }
    }
    return r;
}

// LDS addresses as 32-bit integers: ds instructions take them directly, so
// an address read from LDS needs no base added before the next read.
using lds_u32 = const __attribute__((address_space(3))) uint32_t;
__device__ __forceinline__ uint32_t lds_address(const void *p)
{
    return (uint32_t)(uintptr_t)((const __attribute__((address_space(3))) void *)p);
}
__device__ __forceinline__ uint32_t lds_load(uint32_t addr)
{
    return *(lds_u32 *)(uintptr_t)addr;
}

// Table ids of a kernel's table set: removal (P), half (2^31), rest (P_rest).
enum : int { kTidP = 0, kTidHalf = 1, kTidRest = 2 };

// LDS address of row m (m = 1..64, entry 0 unused) of each table of the
// kernel's set, in the padded device layout: one LDS word read in place of
// the multiply and shifts and of the table's base address, issued alongside
// the guide read.  Every kernel that runs the sampler fills it with
// stage_row_offsets() before its first barrier; the rows stay valid when a
// kernel restages a table at the same place.
static __shared__ uint32_t s_row_addr[3][kChunk + 1];

__device__ __forceinline__ void stage_row_offsets(const uint32_t *tab_p, const uint32_t *tab_half,
                                                  const uint32_t *tab_rest)
{
    for (uint32_t i = threadIdx.x; i < 3u * (kChunk + 1); i += blockDim.x) {
        const uint32_t t = i / (kChunk + 1), m = i % (kChunk + 1);
        const uint32_t *tab = t == 0 ? tab_p : (t == 1 ? tab_half : tab_rest);
        s_row_addr[t][m] = m == 0 ? 0u : lds_address(tab + dev_row_offset(m));
    }
}

// The table set of a kernel (LDS): the tables' guides, and the LDS address
// of the removal table's full-chunk row (m = 64), a constant of the kernel.
struct Tabs {
    const uint8_t *g_p, *g_half, *g_rest;
    uint32_t full_p;
};

// Table set of tables laid out at tab_p, tab_p + kDevTableEntries, tab_p +
// 2 kDevTableEntries with their guides at g, g + kG, g + 2 kG.
__device__ __forceinline__ Tabs make_tabs(const uint32_t *tab_p, const uint8_t *g, int kG)
{
    return Tabs{g, g + kG, g + 2 * kG, lds_address(tab_p + dev_row_offset(kChunk))};
}

// First phase of the inverse-CDF count of one chunk of m >= 1 trials,
// #{j < m : row[j] <= u}: the guide gives the count g <= m at the lower edge
// of u's bucket; rows are nondecreasing, so counting continues from there.
// Tables are in the padded device layout: entries g and g + 1 always exist
// (past the row they are all-ones sentinels), so the two probes need no
// bound test, and entry g + 1 <= u implies entry g <= u.  A sentinel
// compares <= u only for u = 2^32 - 1, where the count may exceed m; the
// callers' clamp to m then gives the count.  Lanes past both probes finish
// the count in a second phase (finish()), so that the probes of the
// independent chunks of a node can all be issued before any scan.
struct Probe {
    uint32_t c;     // g plus the probes at or below u
    uint32_t next;  // LDS address of the entry after the probes
    bool more;      // both probes were <= u: the count may go on
};

template <int GB>
__device__ __forceinline__ Probe probe_at(uint32_t row_addr, uint32_t g, uint32_t u)
{
    const uint32_t a = row_addr + (g << 2);
    const uint32_t t0 = lds_load(a), t1 = lds_load(a + 4u);
    Probe p;
    p.more = t1 <= u;
    p.c = g + (t0 <= u ? 1u : 0u) + (p.more ? 1u : 0u);
    p.next = a + 8u;
    return p;
}

// Probe of a row given at run time (m = 1..64) of table TID.
template <int TID, int GB>
__device__ __forceinline__ Probe probe_row(const uint8_t *guide, uint32_t m, uint32_t u)
{
    const uint32_t g = guide[((m - 1u) << GB) + (u >> (32 - GB))];
    return probe_at<GB>(s_row_addr[TID][m], g, u);
}

// Probe of the full chunk (m = 64) of the removal table, whose row address
// is a constant.
template <int GB>
__device__ __forceinline__ Probe probe_full(const Tabs &tb, uint32_t u)
{
    const uint32_t g = tb.g_p[((uint32_t)(kChunk - 1) << GB) + (u >> (32 - GB))];
    return probe_at<GB>(tb.full_p, g, u);
}

// Second phase: lanes whose probes were both <= u continue the count from
// the probed entry, under their own lane mask.
__device__ __forceinline__ uint32_t finish(const Probe &p, uint32_t m, uint32_t u)
{
    uint32_t c = p.c, next = p.next;
    bool go = p.more;
    while (go) {
        go = (c < m) && (lds_load(next) <= u);
        c += go ? 1u : 0u;
        next += 4u;
    }
    return c;
}

// #{j < m : row[j] <= u} for a chunk of m >= 1 trials of table TID.
template <int TID, int GB>
__device__ __forceinline__ uint32_t chunk_count(const uint8_t *guide, uint32_t m, uint32_t u)
{
    const uint32_t c = finish(probe_row<TID, GB>(guide, m, u), m, u);
    return c < m ? c : m;
}

__device__ __forceinline__ uint32_t clamp_to(uint32_t c, uint32_t m)
{
    return c < m ? c : m;
}

// Bin(n, table TID) with the chunked rule, consuming draws from index j on.
// p_zero: the probability is 0 (draws are still consumed).
template <int TID, typename W, int NB, int GB, int NR, typename K>
__device__ __forceinline__ W binomial(W n, uint32_t &j, const uint8_t *guide, bool p_zero,
                                      const Draws<NB, NR, K> &d)
{
    if (!wave_any(n > (W)kChunk)) {
        // at most one chunk per lane
        const bool has = n != 0;
        const uint32_t u = draw_word(d, j);
        j += has ? 1u : 0u;
        if (p_zero)
            return 0;
        const uint32_t m = has ? (uint32_t)n : 1u;
        const uint32_t c = chunk_count<TID, GB>(guide, m, u);
        return has ? (W)c : (W)0;
    }
    W total = 0;
    while (n > 0) {
        const uint32_t m = n >= (W)kChunk ? (uint32_t)kChunk : (uint32_t)n;
        const uint32_t u = draw_word(d, j);
        ++j;
        if (!p_zero)
            total += chunk_count<TID, GB>(guide, m, u);
        n -= m;
    }
    return total;
}

// One chunk whose draw word is known: m in [0, 64] trials.  m = 0 probes
// row 1 and the clamp to m = 0 gives 0.
template <int TID, int GB>
__device__ __forceinline__ Probe probe_or_zero(const uint8_t *guide, uint32_t m, uint32_t u)
{
    return probe_row<TID, GB>(guide, m != 0 ? m : 1u, u);
}

template <int TID, int GB>
__device__ __forceinline__ uint32_t chunk_or_zero(const uint8_t *guide, uint32_t m, uint32_t u)
{
    const uint32_t row = m != 0 ? m : 1u;
    return clamp_to(finish(probe_row<TID, GB>(guide, row, u), row, u), m);
}

// Second phase of K probes issued together: one wave-level test skips every
// scan when no lane needs one (the common case).  rows[k] is the probed row
// size, the bound of the scan.
template <int K>
__device__ __forceinline__ void finish_all(const Probe (&p)[K], const uint32_t (&rows)[K],
                                           const uint32_t (&u)[K], uint32_t (&c)[K])
{
    bool more = false;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        c[k] = p[k].c;
        more |= p[k].more;
    }
    if (wave_any(more)) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            c[k] = finish(p[k], rows[k], u[k]);
    }
}

// Bin(n, table TID) for 0 <= n <= 64 K with the chunked rule when the words
// of the chunks are known: chunk k (64 trials, the last one n - 64 k) uses
// u[k]; chunks past ceil(n / 64) add nothing, and chunks no lane of the wave
// needs are skipped.
template <int TID, int K, int GB>
__device__ __forceinline__ uint32_t chunks_upto(const uint8_t *guide, uint32_t n,
                                                const uint32_t (&u)[K])
{
    uint32_t total = chunk_or_zero<TID, GB>(guide, n < (uint32_t)kChunk ? n : kChunk, u[0]);
    static_for<1, K>([&](auto kc) {
        constexpr uint32_t k = decltype(kc)::value;
        const bool need = n > k * kChunk;
        if (wave_any(need)) {
            const uint32_t rest = n - k * kChunk;
            total += chunk_or_zero<TID, GB>(
                guide, need ? (rest < (uint32_t)kChunk ? rest : kChunk) : 0u, u[k]);
        }
    });
    return total;
}

// q = 3 redistribution for M <= 192 given the four draw words from the first
// redistribution draw on: m_1 = Bin(M, P_rest) over ceil(M / 64) chunks
// (words u[0..2]), then m_0 = Bin(R, 1/2), R = M - m_1, one chunk at the next
// word u[ceil(M / 64)] (for M = 0 neither consumes a word).  Returns false
// (nothing written) if some lane has R > 64.
template <typename W, int GB>
__device__ __forceinline__ bool redistribute3(W M, const uint32_t (&u)[4], W (&mv)[3],
                                              const Tabs &tb)
{
    const uint32_t m = (uint32_t)M;
    const uint32_t um1[3] = {u[0], u[1], u[2]};
    const W m1 = (W)chunks_upto<kTidRest, 3, GB>(tb.g_rest, m, um1);
    const W R = M - m1;
    if (wave_any(R > (W)kChunk))
        return false;
    const uint32_t um0 = pick3(m > (uint32_t)kChunk, m > 2u * kChunk, u[1], u[2], u[3]);
    mv[1] = m1;
    mv[0] = chunk_or_zero<kTidHalf, GB>(tb.g_half, (uint32_t)R, um0);
    mv[2] = R - mv[0];
    return true;
}

// Node update when the whole wave shares the common draw layout: every
// removal binomial has 1..64 trials except the middle one (q = 3), which has
// D1 chunks (1..64 or 65..128 trials).  Draw j then belongs to a fixed
// binomial, so every word index is a compile-time constant.  The probes of
// all removal chunks are issued together, before any scan.  The
// redistribution may take up to two (q = 2) or three (q = 3, m_1) chunks, the
// extra chunks masked per lane.  Returns false (nothing written) if the
// redistribution needs more, or m_0 of q = 3 more than one chunk; the caller
// then takes the generic path from scratch.
template <int Q, int D1, typename W, int NB, int GB, int NR, typename K>
__device__ __forceinline__ bool node_fast(const W (&av)[Q], W (&c)[Q], const Draws<NB, NR, K> &d,
                                          const Tabs &tb, bool p_zero)
{
    W kv[Q];
    if (p_zero) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
            kv[i] = 0;
    } else if constexpr (Q == 2) {
        const uint32_t rows[2] = {(uint32_t)av[0], (uint32_t)av[1]};
        const uint32_t u[2] = {d.word(0), d.word(1)};
        const Probe p[2] = {probe_row<kTidP, GB>(tb.g_p, rows[0], u[0]),
                            probe_row<kTidP, GB>(tb.g_p, rows[1], u[1])};
        uint32_t cc[2];
        finish_all<2>(p, rows, u, cc);
        kv[0] = clamp_to(cc[0], rows[0]);
        kv[1] = clamp_to(cc[1], rows[1]);
    } else if constexpr (D1 == 1) {
        const uint32_t rows[3] = {(uint32_t)av[0], (uint32_t)av[1], (uint32_t)av[2]};
        const uint32_t u[3] = {d.word(0), d.word(1), d.word(2)};
        const Probe p[3] = {probe_row<kTidP, GB>(tb.g_p, rows[0], u[0]),
                            probe_row<kTidP, GB>(tb.g_p, rows[1], u[1]),
                            probe_row<kTidP, GB>(tb.g_p, rows[2], u[2])};
        uint32_t cc[3];
        finish_all<3>(p, rows, u, cc);
#pragma unroll
        for (int i = 0; i < 3; ++i)
            kv[i] = clamp_to(cc[i], rows[i]);
    } else {
        // the middle binomial: a full chunk (word 1, constant row) and the
        // remainder (word 2); the outer ones take words 0 and 3
        const uint32_t rows[4] = {(uint32_t)av[0], (uint32_t)kChunk,
                                  (uint32_t)av[1] - (uint32_t)kChunk, (uint32_t)av[2]};
        const uint32_t u[4] = {d.word(0), d.word(1), d.word(2), d.word(3)};
        const Probe p[4] = {probe_row<kTidP, GB>(tb.g_p, rows[0], u[0]),
                            probe_full<GB>(tb, u[1]),
                            probe_row<kTidP, GB>(tb.g_p, rows[2], u[2]),
                            probe_row<kTidP, GB>(tb.g_p, rows[3], u[3])};
        uint32_t cc[4];
        finish_all<4>(p, rows, u, cc);
        kv[0] = clamp_to(cc[0], rows[0]);
        kv[1] = clamp_to(cc[1], rows[1]) + clamp_to(cc[2], rows[2]);
        kv[2] = clamp_to(cc[3], rows[3]);
    }
    W M = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        M += kv[i];
    constexpr int kFirst = (Q == 2) ? 2 : 2 + D1;  // first redistribution draw
    W mv[Q];
    if (!wave_any(M > (W)kChunk)) {
        // the common case: every redistribution binomial takes one chunk
        if constexpr (Q == 2) {
            mv[0] = chunk_or_zero<kTidHalf, GB>(tb.g_half, (uint32_t)M, d.word(kFirst));
            mv[1] = M - mv[0];
        } else {
            // m_0 uses the next word only if m_1 consumed one (M > 0); if M = 0
            // then R = 0 and m_0 consumes nothing, so the word is irrelevant.
            mv[1] = chunk_or_zero<kTidRest, GB>(tb.g_rest, (uint32_t)M, d.word(kFirst));
            const W R = M - mv[1];
            mv[0] = chunk_or_zero<kTidHalf, GB>(tb.g_half, (uint32_t)R, d.word(kFirst + 1));
            mv[2] = R - mv[0];
        }
    } else if constexpr (Q == 2) {
        // M <= 128: m_0 over one or two chunks, words 2 and 3
        if (wave_any(M > (W)(2 * kChunk)))
            return false;
        const uint32_t u[2] = {d.word(2), d.word(3)};
        mv[0] = (W)chunks_upto<kTidHalf, 2, GB>(tb.g_half, (uint32_t)M, u);
        mv[1] = M - mv[0];
    } else {
        // M <= 192: words kFirst .. kFirst + 3 (at most 7 for D1 <= 2)
        if (wave_any(M > (W)(3 * kChunk)))
            return false;
        const uint32_t u[4] = {d.word(kFirst), d.word(kFirst + 1), d.word(kFirst + 2), d.word(kFirst + 3)};
        if (!redistribute3<W, GB>(M, u, mv, tb))
            return false;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i)
        c[i] = av[i] - kv[i] + mv[i];
    return true;
}

// q = 3 node update when the outer removal binomials have 1..64 trials but
// the middle one's chunk count D1 = ceil(a_1 / 64) in {1, 2, 3} differs
// between lanes: chunks past the first are masked per lane, and the words of
// the later binomials (draws 1 + D1 on) are selected per lane.  The first two
// chunks of the middle binomial and the outer binomials are probed together.
// The redistribution is as in node_fast.  Returns false (nothing written)
// where node_fast would, or if a needed word lies beyond the eight computed.
template <typename W, int NB, int GB, int NR, typename K>
__device__ __forceinline__ bool node_var3(const W (&av)[3], W (&c)[3], const Draws<NB, NR, K> &d,
                                          const Tabs &tb, bool p_zero)
{
    static_assert(NB >= 2, "draws 0..6 must be computed up front");
    const uint32_t a1 = (uint32_t)av[1];
    const bool c2 = a1 > (uint32_t)kChunk, c3 = a1 > 2u * kChunk;
    W kv[3];
    if (p_zero) {
        kv[0] = kv[1] = kv[2] = 0;
    } else {
        // chunk sizes: a_0; the middle's first chunk; its second (0 where the
        // lane has one chunk; a zero-trial chunk probes row 1, clamped to 0);
        // a_2 at the word after the middle's chunks
        const uint32_t m1b = c3 ? (uint32_t)kChunk : (c2 ? a1 - kChunk : 0u);
        const uint32_t rows[4] = {(uint32_t)av[0], c2 ? (uint32_t)kChunk : a1,
                                  m1b != 0 ? m1b : 1u, (uint32_t)av[2]};
        const uint32_t u[4] = {d.word(0), d.word(1), d.word(2), pick3(c2, c3, d.word(2), d.word(3), d.word(4))};
        const Probe p[4] = {probe_row<kTidP, GB>(tb.g_p, rows[0], u[0]),
                            probe_row<kTidP, GB>(tb.g_p, rows[1], u[1]),
                            probe_row<kTidP, GB>(tb.g_p, rows[2], u[2]),
                            probe_row<kTidP, GB>(tb.g_p, rows[3], u[3])};
        uint32_t cc[4];
        finish_all<4>(p, rows, u, cc);
        kv[0] = clamp_to(cc[0], rows[0]);
        uint32_t k1 = clamp_to(cc[1], rows[1]) + clamp_to(cc[2], m1b);
        if (wave_any(c3))
            k1 += chunk_or_zero<kTidP, GB>(tb.g_p, c3 ? a1 - 2u * kChunk : 0u, d.word(3));
        kv[1] = (W)k1;
        kv[2] = clamp_to(cc[3], rows[3]);
    }
    const W M = kv[0] + kv[1] + kv[2];
    W mv[3];
    if (!wave_any(M > (W)kChunk)) {
        // the common case: m_1 and m_0 take one chunk each, at draws 2 + D1
        // and 3 + D1 (for M = 0 neither consumes a word)
        mv[1] = chunk_or_zero<kTidRest, GB>(tb.g_rest, (uint32_t)M,
                                            pick3(c2, c3, d.word(3), d.word(4), d.word(5)));
        const W R = M - mv[1];
        mv[0] = chunk_or_zero<kTidHalf, GB>(tb.g_half, (uint32_t)R,
                                            pick3(c2, c3, d.word(4), d.word(5), d.word(6)));
        mv[2] = R - mv[0];
    } else {
        // Redistribution words start at 2 + D1; the fourth of them would be
        // draw 8 (a third Philox block) when D1 = 3 and M > 128: left to the
        // generic path.
        if (wave_any(M > (W)(3 * kChunk) || (c3 && M > (W)(2 * kChunk))))
            return false;
        const uint32_t u[4] = {pick3(c2, c3, d.word(3), d.word(4), d.word(5)),
                               pick3(c2, c3, d.word(4), d.word(5), d.word(6)),
                               pick3(c2, c3, d.word(5), d.word(6), d.word(7)),
                               pick3(c2, c3, d.word(6), d.word(7), 0u)};
        if (!redistribute3<W, GB>(M, u, mv, tb))
            return false;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
        c[i] = av[i] - kv[i] + mv[i];
    return true;
}

// q = 3 node update when every lane has every count in 1..128, so each
// removal binomial takes one or two chunks (D_i = 1 + (a_i > 64), the first
// chunk 64 trials where there are two).  The draws are consumed in order:
// the chunks of a_0 from draw 0, of a_1 from D_0, of a_2 from D_0 + D_1, and
// the redistribution from D_0 + D_1 + D_2 (3..6) on; each lane selects its
// words among the eight computed.  The six removal chunks are probed
// together (a lane's absent second chunk probes row 1 and is clamped to 0).
// Where some lane has M > 64 the redistribution goes on chunk by chunk from
// the lane's first redistribution word, as the generic path takes it.
template <typename W, int NB, int GB, int NR, typename K>
__device__ __forceinline__ void node_wide3(const W (&av)[3], W (&c)[3], const Draws<NB, NR, K> &d,
                                           const Tabs &tb, bool p_zero)
{
    static_assert(NB >= 2, "draws 0..7 must be computed up front");
    uint32_t lo[3], hi[3];
    bool two[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const uint32_t a = (uint32_t)av[i];
        two[i] = a > (uint32_t)kChunk;
        lo[i] = two[i] ? (uint32_t)kChunk : a;
        hi[i] = two[i] ? a - (uint32_t)kChunk : 0u;
    }
    // e1, e2: D_0 + D_1 - 2 is at least 1, is 2; f1..f3: D_0 + D_1 + D_2 - 3
    // is at least 1, 2, is 3
    const bool e1 = two[0] || two[1], e2 = two[0] && two[1];
    const bool f1 = e1 || two[2], f2 = e2 || (e1 && two[2]), f3 = e2 && two[2];
    W kv[3];
    if (p_zero) {
        kv[0] = kv[1] = kv[2] = 0;
    } else {
        const uint32_t u[6] = {d.word(0),
                               d.word(1),
                               pick2(two[0], d.word(1), d.word(2)),
                               pick2(two[0], d.word(2), d.word(3)),
                               pick3(e1, e2, d.word(2), d.word(3), d.word(4)),
                               pick3(e1, e2, d.word(3), d.word(4), d.word(5))};
        // one binomial's two chunks probed together at a time (all six at
        // once hold too many registers)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const uint32_t rows[2] = {lo[i], hi[i] != 0 ? hi[i] : 1u};
            const uint32_t ui[2] = {u[2 * i], u[2 * i + 1]};
            const Probe p[2] = {probe_row<kTidP, GB>(tb.g_p, rows[0], ui[0]),
                                probe_row<kTidP, GB>(tb.g_p, rows[1], ui[1])};
            uint32_t cc[2];
            finish_all<2>(p, rows, ui, cc);
            kv[i] = (W)(clamp_to(cc[0], lo[i]) + clamp_to(cc[1], hi[i]));
        }
    }
    const W M = kv[0] + kv[1] + kv[2];
    W mv[3];
    if (wave_any(M > (W)kChunk)) {
        const uint32_t j = 3u + (two[0] ? 1u : 0u) + (two[1] ? 1u : 0u) + (two[2] ? 1u : 0u);
        redistribute_generic<3, W, NB, GB>(M, j, mv, d, tb);
    } else {
        // m_1 at the first redistribution word, m_0 at the next (for M = 0
        // neither consumes a word and both are 0)
        const uint32_t u1 = pick_ge(f1, f2, f3, d.word(3), d.word(4), d.word(5), d.word(6));
        const uint32_t u0 = pick_ge(f1, f2, f3, d.word(4), d.word(5), d.word(6), d.word(7));
        mv[1] = (W)chunk_or_zero<kTidRest, GB>(tb.g_rest, (uint32_t)M, u1);
        const W R = M - mv[1];
        mv[0] = (W)chunk_or_zero<kTidHalf, GB>(tb.g_half, (uint32_t)R, u0);
        mv[2] = R - mv[0];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
        c[i] = av[i] - kv[i] + mv[i];
}

// OR of the counts.  Kernels accumulate it over their nodes in an integer
// register: a count above kMax = 2^b - 1 exists exactly when the accumulated
// OR exceeds kMax (a loop-carried integer is far cheaper than a loop-carried
// per-lane flag, which the compiler keeps as a lane mask through every
// divergent branch of the sampler).
template <int Q, typename W>
__device__ __forceinline__ W or_all(const W (&c)[Q])
{
    W any = c[0];
#pragma unroll
    for (int i = 1; i < Q; ++i)
        any |= c[i];
    return any;
}

// The redistribution of M collided particles (the multinomial as
// conditional binomials), chunk by chunk in the draw order from draw j on:
// q = 2: Bin(M, 1/2) to -1; q = 3: the rest Bin(M, P_rest), then the movers'
// split Bin(R, 1/2) to -1; q = 5: the rest, then the x/y pair split
// Bin(R, 1/2), then -x within x and -y within y, Bin(., 1/2) each.
template <int Q, typename W, int NB, int GB, int NR, typename K>
__device__ __forceinline__ void redistribute_generic(W M, uint32_t j, W (&mv)[Q],
                                                     const Draws<NB, NR, K> &d, const Tabs &tb)
{
    if constexpr (Q == 2) {
        mv[0] = binomial<kTidHalf, W, NB, GB>(M, j, tb.g_half, false, d);
        mv[1] = M - mv[0];
    } else if constexpr (Q == 5) {
        mv[2] = binomial<kTidRest, W, NB, GB>(M, j, tb.g_rest, false, d);
        const W R = M - mv[2];
        const W mx = binomial<kTidHalf, W, NB, GB>(R, j, tb.g_half, false, d);
        const W my = R - mx;
        mv[0] = binomial<kTidHalf, W, NB, GB>(mx, j, tb.g_half, false, d);
        mv[4] = mx - mv[0];
        mv[1] = binomial<kTidHalf, W, NB, GB>(my, j, tb.g_half, false, d);
        mv[3] = my - mv[1];
    } else {
        mv[1] = binomial<kTidRest, W, NB, GB>(M, j, tb.g_rest, false, d);
        const W R = M - mv[1];
        mv[0] = binomial<kTidHalf, W, NB, GB>(R, j, tb.g_half, false, d);
        mv[2] = R - mv[0];
    }
}

// Word idx of the lane's stream for idx in [LO, LO + N) (lanes may differ),
// among the words computed up front: a select chain on values.
template <int LO, int N, int NB, int NR, typename K>
__device__ __forceinline__ uint32_t word_in(const Draws<NB, NR, K> &d, uint32_t idx)
{
    static_assert(LO + N <= 4 * NB, "only the words computed up front");
    uint32_t r = d.word(LO);
    static_for<1, N>([&](auto kc) {
        constexpr int k = LO + decltype(kc)::value;
        r = pick2(idx == (uint32_t)k, r, d.word(k));
    });
    return r;
}

// D2Q5 redistribution of M <= 192 collided particles from draw o = 5 + two
// on (two: the lane's rest removal took two chunks), in straight-line code:
// the rest Bin(M, P_rest) over up to three chunks at words o, o + 1, o + 2,
// the x/y split Bin(R, 1/2) over up to two chunks from word b1 = o + c1
// (c1 = ceil(M / 64) chunks before it), then Bin(m_x, 1/2) for -x from word
// b2 = b1 + ceil(R / 64) and Bin(m_y, 1/2) for -y after it; a binomial of
// no trials consumes no word.  Each lane selects its words among the twelve
// computed (the -y word may be the thirteenth, computed for the lanes that
// need it).  Where some lane has m_x or m_y above one chunk, the last two
// binomials go on chunk by chunk from word b2 as the generic path takes
// them.  Returns false (nothing written) where some lane has M > 192 or
// R > 128; the caller then takes the generic redistribution.
template <typename W, int NB, int GB, int NR, typename K>
__device__ __forceinline__ bool redistribute5(uint32_t M, bool two, W (&mv)[5],
                                              const Draws<NB, NR, K> &d, const Tabs &tb)
{
    static_assert(NB >= 3, "draws 0..11 must be computed up front");
    if (wave_any(M > 3u * kChunk))
        return false;
    const uint32_t ur[3] = {pick2(two, d.word(5), d.word(6)), pick2(two, d.word(6), d.word(7)),
                            pick2(two, d.word(7), d.word(8))};
    const uint32_t rest = chunks_upto<kTidRest, 3, GB>(tb.g_rest, M, ur);
    const uint32_t R = M - rest;
    if (wave_any(R > 2u * kChunk))
        return false;
    const uint32_t b1 = (two ? 6u : 5u) + (M + kChunk - 1) / kChunk;  // 5..9
    const uint32_t us[2] = {word_in<5, 5>(d, b1), word_in<6, 5>(d, b1 + 1u)};
    const uint32_t mx = chunks_upto<kTidHalf, 2, GB>(tb.g_half, R, us);
    const uint32_t my = R - mx;
    uint32_t j = b1 + (R + kChunk - 1) / kChunk;  // 5..11
    mv[2] = (W)rest;
    if (wave_any(mx > (uint32_t)kChunk || my > (uint32_t)kChunk)) {
        mv[0] = binomial<kTidHalf, W, NB, GB>((W)mx, j, tb.g_half, false, d);
        mv[1] = binomial<kTidHalf, W, NB, GB>((W)my, j, tb.g_half, false, d);
    } else {
        const uint32_t u0 = word_in<5, 7>(d, j);
        const uint32_t u1 = draw_word(d, j + (mx != 0 ? 1u : 0u));  // 5..12
        const uint32_t rows[2] = {mx != 0 ? mx : 1u, my != 0 ? my : 1u};
        const uint32_t u[2] = {u0, u1};
        const Probe p[2] = {probe_row<kTidHalf, GB>(tb.g_half, rows[0], u[0]),
                            probe_row<kTidHalf, GB>(tb.g_half, rows[1], u[1])};
        uint32_t cc[2];
        finish_all<2>(p, rows, u, cc);
        mv[0] = (W)clamp_to(cc[0], mx);
        mv[1] = (W)clamp_to(cc[1], my);
    }
    mv[4] = (W)mx - mv[0];
    mv[3] = (W)my - mv[1];
    return true;
}

// D2Q5 node update when every lane has the movers' counts in 1..64 and the
// rest count in 1..128 (one or two chunks: D = 1 or 2 by lane) and the
// redistribution fits one chunk per binomial (M <= 64).  Draws: movers -x
// and -y at 0 and 1, the rest at 2 (and 3 for a second chunk), then, shifted
// by D - 1 per lane, +y at 3, +x at 4, the rest redistribution Bin(M, 1 - 2
// theta) at 5, the x/y split Bin(R, 1/2) at 6, Bin(m_x, 1/2) for -x at 7 and
// Bin(m_y, 1/2) for -y at the next draw (8 if the -x split took one, else 7).
// Earlier zero counts make the later words irrelevant (M = 0 or R = 0 leaves
// nothing to split).  The removal chunks are probed together, and so are
// the two last splits.  Where some lane of the wave has M > 64 (most waves
// at high collision fractions: M is about omega* times the density), the
// redistribution goes on chunk by chunk from the word after the removal
// draws, as the generic path takes it; the removal is not repeated.
template <typename W, int NB, int GB, int NR, typename K>
__device__ __forceinline__ bool node_fast5(const W (&av)[5], W (&c)[5], const Draws<NB, NR, K> &d,
                                           const Tabs &tb, bool p_zero)
{
    static_assert(NB >= 3, "draws 0..9 must be computed up front");
    const uint32_t a2 = (uint32_t)av[2];
    const bool two = a2 > (uint32_t)kChunk;
    // word k of the layout after the rest binomial, shifted by one if it took two chunks
    auto wk = [&](auto kc) -> uint32_t {
        constexpr int k = decltype(kc)::value;
        return two ? d.word(k + 1) : d.word(k);
    };
    W kv[5];
    if (p_zero) {
#pragma unroll
        for (int i = 0; i < 5; ++i)
            kv[i] = 0;
    } else {
        const uint32_t m2b = two ? a2 - kChunk : 0u;
        const uint32_t rows[6] = {(uint32_t)av[0], (uint32_t)av[1],
                                  two ? (uint32_t)kChunk : a2, m2b != 0 ? m2b : 1u,
                                  (uint32_t)av[3], (uint32_t)av[4]};
        const uint32_t u[6] = {d.word(0), d.word(1), d.word(2), d.word(3),
                               wk(std::integral_constant<int, 3>{}),
                               wk(std::integral_constant<int, 4>{})};
        Probe p[6];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            p[k] = probe_row<kTidP, GB>(tb.g_p, rows[k], u[k]);
        uint32_t cc[6];
        finish_all<6>(p, rows, u, cc);
        kv[0] = (W)clamp_to(cc[0], rows[0]);
        kv[1] = (W)clamp_to(cc[1], rows[1]);
        kv[2] = (W)(clamp_to(cc[2], rows[2]) + clamp_to(cc[3], m2b));
        kv[3] = (W)clamp_to(cc[4], rows[4]);
        kv[4] = (W)clamp_to(cc[5], rows[5]);
    }
    const W M = kv[0] + kv[1] + kv[2] + kv[3] + kv[4];
    W mv[5];
    if (wave_any(M > (W)kChunk)) {
        // the removal took draws 0..4, and 5 with a two-chunk rest count
        if (!redistribute5<W, NB, GB>((uint32_t)M, two, mv, d, tb))
            redistribute_generic<5, W, NB, GB>(M, two ? 6u : 5u, mv, d, tb);
#pragma unroll
        for (int i = 0; i < 5; ++i)
            c[i] = av[i] - kv[i] + mv[i];
        return true;
    }
    mv[2] = (W)chunk_or_zero<kTidRest, GB>(tb.g_rest, (uint32_t)M,
                                           wk(std::integral_constant<int, 5>{}));
    const W R = M - mv[2];
    const W mx = (W)chunk_or_zero<kTidHalf, GB>(tb.g_half, (uint32_t)R,
                                                wk(std::integral_constant<int, 6>{}));
    const W my = R - mx;
    const uint32_t u7 = wk(std::integral_constant<int, 7>{});
    const uint32_t uy = mx > 0 ? wk(std::integral_constant<int, 8>{}) : u7;
    const uint32_t rows[2] = {mx != 0 ? (uint32_t)mx : 1u, my != 0 ? (uint32_t)my : 1u};
    const uint32_t u[2] = {u7, uy};
    const Probe p[2] = {probe_row<kTidHalf, GB>(tb.g_half, rows[0], u[0]),
                        probe_row<kTidHalf, GB>(tb.g_half, rows[1], u[1])};
    uint32_t cc[2];
    finish_all<2>(p, rows, u, cc);
    mv[0] = (W)clamp_to(cc[0], (uint32_t)mx);
    mv[4] = mx - mv[0];
    mv[1] = (W)clamp_to(cc[1], (uint32_t)my);
    mv[3] = my - mv[1];
#pragma unroll
    for (int i = 0; i < 5; ++i)
        c[i] = av[i] - kv[i] + mv[i];
    return true;
}

template <typename T> struct Wide;
template <> struct Wide<uint16_t> { using type = uint32_t; };
template <> struct Wide<uint32_t> { using type = uint64_t; };

// Full node update: av holds the (already flipped) occupations; cn receives
// the post-collision counts.  NR: Philox rounds of the draws (10 or 7).
// The generic path: every binomial chunk by chunk in the draw order, in
// the arithmetic type WW (wide enough for every count, sum and result).
template <int Q, typename WW, int NB, int GB, int NR, typename K>
__device__ __forceinline__ void node_generic(const WW (&av)[Q], WW (&cn)[Q],
                                             const Draws<NB, NR, K> &d,
                                             const Tabs &tb, bool p_zero)
{
    using W = WW;
    W kv[Q], mv[Q];
    uint32_t j = 0;
    W M = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        kv[i] = binomial<kTidP, W, NB, GB>(av[i], j, tb.g_p, p_zero, d);
        M += kv[i];
    }
    redistribute_generic<Q, W, NB, GB>(M, j, mv, d, tb);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        cn[i] = av[i] - kv[i] + mv[i];
}

template <int Q, typename W, int NB, int GB, int NR = 10, typename K = PhiloxKey>
__device__ __forceinline__ void node_update(const W (&av)[Q], W (&cn)[Q], uint32_t x, uint32_t t,
                                            uint32_t r, const K &key, const Tabs &tb, bool p_zero)
{
    Draws<NB, NR, K> d;
    d.init(x, t, r, key);
    // Common draw layout, decided once per wave for this node slot, from
    // lane masks of compares (no short-circuit branches): a count a lies in
    // 1..n exactly when a - 1 < n as an unsigned number, and several counts
    // lie in 1..64 exactly when the OR of their a - 1 is below 64.
    auto m1 = [](W a) { return (uint32_t)(a - (W)1); };
    auto ballot = [](bool p) { return __builtin_amdgcn_ballot_w64(p); };
    const uint64_t lanes = ballot(true);
    uint64_t ok_mask, two_mask = 0, three_mask = 0;
    if constexpr (Q == 2) {
        ok_mask = ballot((m1(av[0]) | m1(av[1])) < (uint32_t)kChunk);
    } else if constexpr (Q == 5) {
        ok_mask = ballot((m1(av[0]) | m1(av[1]) | m1(av[3]) | m1(av[4])) < (uint32_t)kChunk) &
                  ballot(m1(av[2]) < 2u * kChunk);
    } else {
        ok_mask = ballot((m1(av[0]) | m1(av[2])) < (uint32_t)kChunk) &
                  ballot(m1(av[1]) < 3u * kChunk);
        two_mask = ballot(av[1] > (W)kChunk);
        three_mask = ballot(av[1] > (W)(2 * kChunk));
    }
    bool done = false;
    if (ok_mask == lanes) {
        // Every count is at most three chunks here, so every intermediate and
        // result fits 32 bits: the straight-line paths run in 32-bit
        // arithmetic also for uint32 lattices (whose generic path is 64-bit).
        uint32_t a32[Q], c32[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i)
            a32[i] = (uint32_t)av[i];
        if constexpr (Q == 5)
            done = node_fast5<uint32_t, NB, GB>(a32, c32, d, tb, p_zero);
        else if (two_mask == 0ull)
            done = node_fast<Q, 1, uint32_t, NB, GB>(a32, c32, d, tb, p_zero);
        else if constexpr (Q == 3) {
            if (two_mask == lanes && three_mask == 0ull)
                done = node_fast<Q, 2, uint32_t, NB, GB>(a32, c32, d, tb, p_zero);
            else
                done = node_var3<uint32_t, NB, GB>(a32, c32, d, tb, p_zero);
        }
        if (done) {
#pragma unroll
            for (int i = 0; i < Q; ++i)
                cn[i] = (W)c32[i];
        }
    }
    if constexpr (Q == 3) {
        // every count in 1..128 (at a density of about 150 most waves have
        // some outer count above one chunk)
        if (!done && ballot((m1(av[0]) | m1(av[1]) | m1(av[2])) < 2u * kChunk) == lanes) {
            uint32_t a32[3], c32[3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
                a32[i] = (uint32_t)av[i];
            node_wide3<uint32_t, NB, GB>(a32, c32, d, tb, p_zero);
#pragma unroll
            for (int i = 0; i < 3; ++i)
                cn[i] = (W)c32[i];
            done = true;
        }
    }
    if (!done) {
        if constexpr (sizeof(W) > sizeof(uint32_t)) {
            // uint32 lattices: below 2^29 per count, every sum and result of
            // the node fits 32 bits (at most 5 x 2^29 + 2^29 < 2^32).
            bool small = true;
#pragma unroll
            for (int i = 0; i < Q; ++i)
                small &= av[i] < ((W)1 << 29);
            if (__builtin_amdgcn_ballot_w64(small) == lanes) {
                uint32_t a32[Q], c32[Q];
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    a32[i] = (uint32_t)av[i];
                node_generic<Q, uint32_t, NB, GB>(a32, c32, d, tb, p_zero);
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    cn[i] = (W)c32[i];
                return;
            }
        }
        node_generic<Q, W, NB, GB>(av, cn, d, tb, p_zero);
    }
}

// D1Q2 exchange form (draw specification v3): av holds the (flipped)
// occupations a_-, a_+; X = Bin(a_-, p_x) particles cross to +1, then
// Y = Bin(a_+, p_x) cross to -1 (the P table slot holds the crossing
// probability's table and guide).  When every lane has both counts in 1..64
// the two draws are words 0 and 1, probed together; otherwise the generic
// chunked binomials.
template <typename W, int NB, int GB, int NR = 10, typename K = PhiloxKey>
__device__ __forceinline__ void node_exchange(const W (&av)[2], W (&cn)[2], uint32_t x, uint32_t t,
                                              uint32_t r, const K &key, const Tabs &tb,
                                              bool p_zero)
{
    Draws<NB, NR, K> d;
    d.init(x, t, r, key);
    const bool ok = av[0] >= 1 && av[0] <= (W)kChunk && av[1] >= 1 && av[1] <= (W)kChunk;
    W X, Y;
    if (!wave_any(!ok)) {
        if (p_zero) {
            X = Y = 0;
        } else {
            const uint32_t rows[2] = {(uint32_t)av[0], (uint32_t)av[1]};
            const uint32_t u[2] = {d.word(0), d.word(1)};
            const Probe p[2] = {probe_row<kTidP, GB>(tb.g_p, rows[0], u[0]),
                                probe_row<kTidP, GB>(tb.g_p, rows[1], u[1])};
            uint32_t cc[2];
            finish_all<2>(p, rows, u, cc);
            X = (W)clamp_to(cc[0], rows[0]);
            Y = (W)clamp_to(cc[1], rows[1]);
        }
    } else {
        uint32_t j = 0;
        X = binomial<kTidP, W, NB, GB>(av[0], j, tb.g_p, p_zero, d);
        Y = binomial<kTidP, W, NB, GB>(av[1], j, tb.g_p, p_zero, d);
    }
    cn[0] = av[0] - X + Y;
    cn[1] = av[1] - Y + X;
}

// Destinations of a D2Q5 node's movers on the node index x + Lx y, periodic
// in both directions: -x, -y, +y, +x.  x0 (uniform) is the first node of the
// pass, x = x0 + lane index < x0 + BLOCK; the pass's row and column come from
// one scalar division, each lane's from a float quotient with one exact
// correction (its dividend is below Lx + BLOCK, and a quotient of such small
// integers is off by at most one below an exact multiple).
template <int BLOCK>
__device__ __forceinline__ void d2q5_neighbours(uint32_t x, uint32_t x0, uint32_t width,
                                                uint32_t nodes, uint32_t &dxm, uint32_t &dym,
                                                uint32_t &dyp, uint32_t &dxp)
{
    const uint32_t row0 = x0 / width;
    uint32_t cx = x0 - row0 * width + (x - x0), cy = row0;
    if (cx >= width) {
        uint32_t k;
        if (width >= (uint32_t)BLOCK) {
            k = 1u;
        } else {
            k = (uint32_t)((float)cx * (1.0f / (float)width));
            if (cx - k * width >= width)
                ++k;
        }
        cx -= k * width;
        cy += k;
    }
    dxm = cx == 0 ? x + width - 1 : x - 1;
    dxp = cx + 1 == width ? x + 1 - width : x + 1;
    dym = cy == 0 ? x + (nodes - width) : x - width;
    dyp = x + width >= nodes ? x + width - nodes : x + width;
}

}  // namespace sampler
}  // namespace ilg
