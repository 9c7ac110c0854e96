// Fused lattice-gas step for gfx950: load -> flip -> sampling collision ->
// push streaming, one pass over the structure-of-arrays occupation arrays.
//
// Per node x at step t (Eq. LGflip):
//   a_i   = n_{q-1-i}(x) if the flip is on, else n_i(x)          (Eq. flip)
//   k_i   = Bin(a_i, P)          removal: each particle collides w.p. P/2^32
//   M     = sum_i k_i
//   q = 2: m_0 = Bin(M, 2^31), m_1 = M - m_0
//   q = 3: m_1 = Bin(M, P_rest), R = M - m_1, m_0 = Bin(R, 2^31), m_2 = R - m_0
//   c_i   = a_i - k_i + m_i,   out_i[(x + v_i) mod L] = c_i         (Eq. ilgeq)
// Bin(n, p) takes ceil(n/64) 32-bit draws (full chunks of 64 first, then the
// remainder); a chunk of m trials with draw U yields #{j < m : T[m][j] <= U}.
// Draw j of a node-step is word j%4 of Philox4x32-10 block j/4 with counter
// (x, t, realization, j/4).
//
// gfx950 mapping.  The path is bound by integer VALU work (Philox rounds and
// the inverse-CDF searches), not by HBM, so the kernel is shaped to keep the
// VALU busy with useful work:
//  * the fixed-point tables and guide tables live in LDS (one copy per
//    workgroup, staged once for a persistent grid);
//  * the search starts at a guide entry (2^GB buckets per row) and needs one
//    table compare in the common case; longer scans run only for the lanes
//    that need them;
//  * binomials of at most 64 (one draw) or 128 trials (two draws) take
//    branch-free paths when the whole wave qualifies; the word index of each
//    draw is usually wave-uniform, so the word is picked by scalar branches
//    instead of a per-lane select tree;
//  * the first NB Philox blocks are computed up front, later ones on demand;
//  * every thread owns NPT consecutive nodes (vector loads, ILP across nodes);
//    tiles are dealt so that the workgroups of one XCD (dispatch is
//    round-robin over the 8 XCDs) cover one contiguous eighth of the lattice.
// Streaming stores are per element (the +-1 shift breaks vector alignment);
// the wave still writes contiguous bytes.
#include <cstdlib>
#include <type_traits>

#include "ilg_internal.h"
#include "philox.h"

namespace ilg {

namespace {

constexpr int kNumXcd = 8;

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

__device__ __forceinline__ bool wave_any(bool p)
{
    return __builtin_amdgcn_ballot_w64(p) != 0ull;
}

template <int NB>
struct Draws {
    uint32_t w[4 * NB];
    uint32_t x, t, r, k0, k1;

    __device__ __forceinline__ void init(uint32_t x_, uint32_t t_, uint32_t r_, uint32_t k0_,
                                         uint32_t k1_)
    {
        x = x_; t = t_; r = r_; k0 = k0_; k1 = k1_;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const uint4 o = philox4x32_10(x, t, r, (uint32_t)b, k0, k1);
            w[4 * b + 0] = o.x; w[4 * b + 1] = o.y; w[4 * b + 2] = o.z; w[4 * b + 3] = o.w;
        }
    }
};

__device__ __forceinline__ uint32_t pick4(uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                          uint32_t s)
{
    const uint32_t lo = (s & 1u) ? b : a;
    const uint32_t hi = (s & 1u) ? d : c;
    return (s & 2u) ? hi : lo;
}

// Word j of the lane's draw stream (lanes may ask for different j).
template <int NB>
__device__ __forceinline__ uint32_t draw_word(const Draws<NB> &d, uint32_t j)
{
    constexpr uint32_t kEager = 4 * NB;
    const uint32_t j0 = __builtin_amdgcn_readfirstlane(j);
    uint32_t r;
    if (!wave_any(j != j0) && j0 < kEager) {
        // wave-uniform index: scalar branches pick the register
        switch (j0) {
        case 0: r = d.w[0]; break;
        case 1: r = d.w[1]; break;
        case 2: r = d.w[2]; break;
        case 3: r = d.w[3]; break;
        case 4: r = d.w[4 % kEager]; break;
        case 5: r = d.w[5 % kEager]; break;
        case 6: r = d.w[6 % kEager]; break;
        default: r = d.w[kEager - 1]; break;
        }
    } else {
        const uint32_t jc = j < kEager ? j : kEager - 1;
        if constexpr (NB == 1) {
            r = pick4(d.w[0], d.w[1], d.w[2], d.w[3], jc);
        } else {
            const uint32_t lo = pick4(d.w[0], d.w[1], d.w[2], d.w[3], jc & 3u);
            const uint32_t hi = pick4(d.w[4], d.w[5], d.w[6], d.w[7], jc & 3u);
            r = (jc & 4u) ? hi : lo;
        }
        if (wave_any(j >= kEager)) {
            if (j >= kEager) {
                const uint4 o = philox4x32_10(d.x, d.t, d.r, j >> 2, d.k0, d.k1);
                r = pick4(o.x, o.y, o.z, o.w, j & 3u);
            }
        }
    }
    return r;
}

// Inverse-CDF count of one chunk of m >= 1 trials: #{j < m : row[j] <= u}.
// The guide gives the count at the lower edge of u's bucket; rows are
// nondecreasing, so counting continues from there to the first entry above u.
template <int GB>
__device__ __forceinline__ uint32_t chunk_count(const uint32_t *tab, const uint8_t *guide,
                                                uint32_t m, uint32_t u)
{
    const uint32_t *row = tab + (((m - 1u) * m) >> 1);
    const uint32_t g = guide[((m - 1u) << GB) + (u >> (32 - GB))];
    // Two compares cover almost every lane: entries g and g+1 (clamped to the
    // row; a clamped read is masked by the bound test).
    const uint32_t t0 = row[g < m ? g : m - 1u];
    const uint32_t t1 = row[g + 1u < m ? g + 1u : m - 1u];
    const bool s0 = (g < m) && (t0 <= u);
    const bool s1 = s0 && (g + 1u < m) && (t1 <= u);
    uint32_t c = g + (s0 ? 1u : 0u) + (s1 ? 1u : 0u);
    if (wave_any(s1)) {
        bool go = s1;
        while (go) {
            go = (c < m) && (row[c] <= u);
            c += go ? 1u : 0u;
        }
    }
    return c;
}

// Bin(n, table) with the chunked rule, consuming draws from index j on.
// p_zero: the probability is 0 (draws are still consumed).
template <typename W, int NB, int GB>
__device__ __forceinline__ W binomial(W n, uint32_t &j, const uint32_t *tab, const uint8_t *guide,
                                      bool p_zero, const Draws<NB> &d)
{
    if (!wave_any(n > (W)kChunk)) {
        // at most one chunk per lane
        const bool has = n != 0;
        const uint32_t u = draw_word<NB>(d, j);
        j += has ? 1u : 0u;
        if (p_zero)
            return 0;
        const uint32_t m = has ? (uint32_t)n : 1u;
        const uint32_t c = chunk_count<GB>(tab, guide, m, u);
        return has ? (W)c : (W)0;
    }
    W total = 0;
    while (n > 0) {
        const uint32_t m = n >= (W)kChunk ? (uint32_t)kChunk : (uint32_t)n;
        const uint32_t u = draw_word<NB>(d, j);
        ++j;
        if (!p_zero)
            total += chunk_count<GB>(tab, guide, m, u);
        n -= m;
    }
    return total;
}

// One chunk whose draw word is known: m in [0, 64] trials (m = 0 gives 0).
template <int GB>
__device__ __forceinline__ uint32_t chunk_or_zero(const uint32_t *tab, const uint8_t *guide,
                                                  uint32_t m, uint32_t u)
{
    const uint32_t c = chunk_count<GB>(tab, guide, m != 0 ? m : 1u, u);
    return m != 0 ? c : 0u;
}

// Node update when the whole wave shares the common draw layout: every
// removal binomial has 1..64 trials except the middle one (q = 3), which has
// D1 chunks (1..64 or 65..128 trials).  Draw j then belongs to a fixed
// binomial, so every word index is a compile-time constant.  Returns false
// (nothing written) if the redistribution does not fit one chunk per
// binomial; the caller then takes the generic path from scratch.
template <int Q, int D1, typename W, int NB, int GB>
__device__ __forceinline__ bool node_fast(const W (&av)[Q], W (&c)[Q], const Draws<NB> &d,
                                          const uint32_t *tab_p, const uint8_t *g_p,
                                          const uint32_t *tab_half, const uint8_t *g_half,
                                          const uint32_t *tab_rest, const uint8_t *g_rest,
                                          bool p_zero)
{
    W kv[Q];
    if (p_zero) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
            kv[i] = 0;
    } else if constexpr (Q == 2) {
        kv[0] = chunk_count<GB>(tab_p, g_p, (uint32_t)av[0], d.w[0]);
        kv[1] = chunk_count<GB>(tab_p, g_p, (uint32_t)av[1], d.w[1]);
    } else {
        kv[0] = chunk_count<GB>(tab_p, g_p, (uint32_t)av[0], d.w[0]);
        if constexpr (D1 == 1) {
            kv[1] = chunk_count<GB>(tab_p, g_p, (uint32_t)av[1], d.w[1]);
        } else {
            kv[1] = chunk_count<GB>(tab_p, g_p, (uint32_t)kChunk, d.w[1]) +
                    chunk_count<GB>(tab_p, g_p, (uint32_t)av[1] - (uint32_t)kChunk, d.w[2]);
        }
        kv[2] = chunk_count<GB>(tab_p, g_p, (uint32_t)av[2], d.w[1 + D1]);
    }
    W M = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        M += kv[i];
    if (wave_any(M > (W)kChunk))
        return false;
    constexpr int kFirst = (Q == 2) ? 2 : 2 + D1;  // first redistribution draw
    W mv[Q];
    if constexpr (Q == 2) {
        mv[0] = chunk_or_zero<GB>(tab_half, g_half, (uint32_t)M, d.w[kFirst]);
        mv[1] = M - mv[0];
    } else {
        // m_0 uses the next word only if m_1 consumed one (M > 0); if M = 0
        // then R = 0 and m_0 consumes nothing, so the word is irrelevant.
        mv[1] = chunk_or_zero<GB>(tab_rest, g_rest, (uint32_t)M, d.w[kFirst]);
        const W R = M - mv[1];
        mv[0] = chunk_or_zero<GB>(tab_half, g_half, (uint32_t)R, d.w[kFirst + 1]);
        mv[2] = R - mv[0];
    }
#pragma unroll
    for (int i = 0; i < Q; ++i)
        c[i] = av[i] - kv[i] + mv[i];
    return true;
}

template <typename T> struct Wide;
template <> struct Wide<uint16_t> { using type = uint32_t; };
template <> struct Wide<uint32_t> { using type = uint64_t; };

template <int Q, typename T, int NPT, int NB, int GB, int BLOCK>
__global__ __launch_bounds__(BLOCK) void step_kernel(StepArgs a)
{
    using W = typename Wide<T>::type;
    constexpr int kTabs = (Q == 3) ? 3 : 2;
    constexpr int kRowGuide = 1 << GB;
    __shared__ uint32_t s_tab[kTabs * kTableEntries];
    __shared__ uint8_t s_guide[kTabs * kChunk * kRowGuide];

    // Stage tables (16-byte copies) and the 2^GB-bucket view of the guides.
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.tables);
        uint4 *dst = reinterpret_cast<uint4 *>(s_tab);
        constexpr int n = kTabs * kTableEntries * 4 / 16;
        for (int i = threadIdx.x; i < n; i += BLOCK)
            dst[i] = src[i];
        const uint8_t *gsrc = guide_ptr(a.tables, 0);
        if constexpr (GB == kGuideBits) {
            const uint4 *g4 = reinterpret_cast<const uint4 *>(gsrc);
            uint4 *d4 = reinterpret_cast<uint4 *>(s_guide);
            constexpr int ng = kTabs * kGuideEntries / 16;
            for (int i = threadIdx.x; i < ng; i += BLOCK)
                d4[i] = g4[i];
        } else {
            constexpr int ng = kTabs * kChunk * kRowGuide;
            for (int i = threadIdx.x; i < ng; i += BLOCK)
                s_guide[i] = gsrc[i << (kGuideBits - GB)];
        }
    }
    __syncthreads();

    const uint32_t *tab_p = s_tab;
    const uint32_t *tab_half = s_tab + kTableEntries;
    const uint32_t *tab_rest = s_tab + 2 * kTableEntries;  // q = 3 only
    constexpr int kG = kChunk * kRowGuide;
    const uint8_t *g_p = s_guide;
    const uint8_t *g_half = s_guide + kG;
    const uint8_t *g_rest = s_guide + 2 * kG;
    const bool p_zero = a.p_zero != 0;
    const bool flip = a.flip != 0;
    const uint32_t L = a.length;
    const uint64_t pitch = a.pitch;
    const T *in = reinterpret_cast<const T *>(a.in);
    T *out = reinterpret_cast<T *>(a.out);
    constexpr W kMax = (W)(T)~(T)0;

    constexpr uint32_t kTile = (uint32_t)BLOCK * NPT;
    const uint32_t ntiles = (L + kTile - 1) / kTile;
    uint32_t first, stride, end;
    if (gridDim.x % kNumXcd == 0) {
        const uint32_t xcd = blockIdx.x % kNumXcd;
        first = (uint32_t)((uint64_t)ntiles * xcd / kNumXcd) + blockIdx.x / kNumXcd;
        end = (uint32_t)((uint64_t)ntiles * (xcd + 1) / kNumXcd);
        stride = gridDim.x / kNumXcd;
    } else {
        first = blockIdx.x;
        end = ntiles;
        stride = gridDim.x;
    }

    bool overflow = false;
    for (uint32_t tile = first; tile < end; tile += stride) {
        const uint32_t x0 = tile * kTile + threadIdx.x * NPT;
        if (x0 >= L)
            continue;
        W n[Q][NPT];
        if (x0 + NPT <= L) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const VecT<T, NPT> v =
                    *reinterpret_cast<const VecT<T, NPT> *>(in + i * pitch + x0);
#pragma unroll
                for (int k = 0; k < NPT; ++k)
                    n[i][k] = (W)v.v[k];
            }
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i)
#pragma unroll
                for (int k = 0; k < NPT; ++k)
                    n[i][k] = (x0 + k < L) ? (W)in[i * pitch + x0 + k] : (W)0;
        }

        W c[Q][NPT];
        static_for<0, NPT>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            W av[Q], kv[Q], mv[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i)
                av[i] = flip ? n[Q - 1 - i][k] : n[i][k];
            Draws<NB> d;
            d.init(x0 + k, a.t, a.realization, a.key0, a.key1);
            // Common draw layout, decided once per wave for this node slot.
            bool ok = true, two = false;
            if constexpr (Q == 2) {
                ok = av[0] >= 1 && av[0] <= (W)kChunk && av[1] >= 1 && av[1] <= (W)kChunk;
            } else {
                ok = av[0] >= 1 && av[0] <= (W)kChunk && av[2] >= 1 && av[2] <= (W)kChunk &&
                     av[1] >= 1 && av[1] <= (W)(2 * kChunk);
                two = av[1] > (W)kChunk;
            }
            W cn[Q];
            bool done = false;
            if (!wave_any(!ok)) {
                if (!wave_any(two))
                    done = node_fast<Q, 1, W, NB, GB>(av, cn, d, tab_p, g_p, tab_half, g_half,
                                                      tab_rest, g_rest, p_zero);
                else if (Q == 3 && !wave_any(!two))
                    done = node_fast<Q, 2, W, NB, GB>(av, cn, d, tab_p, g_p, tab_half, g_half,
                                                      tab_rest, g_rest, p_zero);
            }
            if (!done) {
                uint32_t j = 0;
                W M = 0;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    kv[i] = binomial<W, NB, GB>(av[i], j, tab_p, g_p, p_zero, d);
                    M += kv[i];
                }
                if constexpr (Q == 2) {
                    mv[0] = binomial<W, NB, GB>(M, j, tab_half, g_half, false, d);
                    mv[1] = M - mv[0];
                } else {
                    mv[1] = binomial<W, NB, GB>(M, j, tab_rest, g_rest, false, d);
                    const W R = M - mv[1];
                    mv[0] = binomial<W, NB, GB>(R, j, tab_half, g_half, false, d);
                    mv[2] = R - mv[0];
                }
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    cn[i] = av[i] - kv[i] + mv[i];
            }
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                c[i][k] = cn[i];
                overflow |= cn[i] > kMax;
            }
        });

        // Streaming: velocity -1 to x-1, 0 in place, +1 to x+1 (periodic).
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const uint32_t x = x0 + k;
            if (x < L) {
                const uint32_t xm = (x == 0) ? L - 1 : x - 1;
                const uint32_t xp = (x + 1 == L) ? 0 : x + 1;
                out[xm] = (T)c[0][k];
                out[(uint64_t)(Q - 1) * pitch + xp] = (T)c[Q - 1][k];
            }
        }
        if constexpr (Q == 3) {
            if (x0 + NPT <= L) {
                VecT<T, NPT> v;
#pragma unroll
                for (int k = 0; k < NPT; ++k)
                    v.v[k] = (T)c[1][k];
                *reinterpret_cast<VecT<T, NPT> *>(out + pitch + x0) = v;
            } else {
#pragma unroll
                for (int k = 0; k < NPT; ++k)
                    if (x0 + k < L)
                        out[pitch + x0 + k] = (T)c[1][k];
            }
        }
    }
    if (overflow)
        atomicOr(a.err, 1u);
}

template <int Q, typename T, int NPT, int NB, int GB, int BLOCK>
hipError_t launch_variant(const StepArgs &a, hipStream_t stream, int wg_per_cu)
{
    constexpr uint32_t kTile = (uint32_t)BLOCK * NPT;
    const uint32_t ntiles = (a.length + kTile - 1) / kTile;
    static int cus = 0;
    if (cus == 0)
        cus = device_cu_count();
    uint32_t grid = (uint32_t)cus * (uint32_t)wg_per_cu;
    if (ntiles < grid)
        grid = ntiles;
    if (grid >= (uint32_t)kNumXcd)
        grid -= grid % kNumXcd;
    if (grid == 0)
        grid = 1;
    hipLaunchKernelGGL((step_kernel<Q, T, NPT, NB, GB, BLOCK>), dim3(grid), dim3(BLOCK), 0, stream,
                       a);
    return hipGetLastError();
}

// Launch shapes (bit-identical results; only speed differs).  Variant 0 is
// the default; ILG_STEP_VARIANT selects another for tuning runs.
int step_variant()
{
    static int v = -1;
    if (v < 0) {
        const char *e = std::getenv("ILG_STEP_VARIANT");
        v = e ? std::atoi(e) : 0;
    }
    return v;
}

template <int Q, typename T, int NB>
hipError_t launch_q(const StepArgs &a, hipStream_t stream)
{
    switch (step_variant()) {
    case 1:
        return launch_variant<Q, T, 2, NB, 8, 1024>(a, stream, 2);
    case 2:
        return launch_variant<Q, T, 4, NB, 8, 1024>(a, stream, 2);
    case 3:
        return launch_variant<Q, T, 1, NB, 7, 1024>(a, stream, 2);
    case 4:
        return launch_variant<Q, T, 1, NB, 8, 512>(a, stream, 4);
    default:
        return launch_variant<Q, T, 1, NB, 8, 1024>(a, stream, 2);
    }
}

}  // namespace

hipError_t launch_step(int q, int count_bytes, const StepArgs &a, hipStream_t stream)
{
    if (q == 2 && count_bytes == 2)
        return launch_q<2, uint16_t, 1>(a, stream);
    if (q == 2 && count_bytes == 4)
        return launch_q<2, uint32_t, 1>(a, stream);
    if (q == 3 && count_bytes == 2)
        return launch_q<3, uint16_t, 2>(a, stream);
    if (q == 3 && count_bytes == 4)
        return launch_q<3, uint32_t, 2>(a, stream);
    return hipErrorInvalidValue;
}

}  // namespace ilg
