// Fused lattice-gas step for gfx950: load -> flip -> sampling collision ->
// push streaming, one pass over the structure-of-arrays occupation arrays
// (Eq. LGflip, then the streaming of Eq. ilgeq: out_i[(x + v_i) mod L] = c_i).
// The per-node sampler is in sampler.h.
//
// Mapping: a persistent grid of 1024-thread workgroups (two per CU), each
// holding the fixed-point tables and their guides in LDS, staged once.  A
// tile is BLOCK * NPT consecutive nodes; every thread owns NPT consecutive
// nodes and reads each velocity row with one vector load.  Tiles are dealt
// so that the workgroups of one XCD (dispatch is round-robin over the 8
// XCDs) cover one contiguous eighth of the lattice.  Streaming stores are per
// element (the +-1 shift breaks vector alignment); the wave still writes
// contiguous bytes.
#include <cstdlib>
#include <type_traits>

#include "ilg_internal.h"
#include "sampler.h"

namespace ilg {

namespace {

constexpr int kNumXcd = 8;
using sampler::VecT;
using sampler::static_for;
using sampler::Wide;

template <int Q, typename T, int NPT, int NB, int GB, int BLOCK>
__global__ __launch_bounds__(BLOCK) void step_kernel(StepArgs a)
{
    using W = typename Wide<T>::type;
    constexpr int kTabs = (Q == 3) ? 3 : 2;
    constexpr int kRowGuide = 1 << GB;
    __shared__ __align__(16) uint32_t s_tab[kTabs * kDevTableEntries];
    __shared__ uint8_t s_guide[kTabs * kChunk * kRowGuide];

    // Stage tables (16-byte copies) and the 2^GB-bucket view of the guides.
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.tables);
        uint4 *dst = reinterpret_cast<uint4 *>(s_tab);
        constexpr int n = kTabs * kDevTableEntries * 4 / 16;
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
    const uint32_t *tab_half = s_tab + kDevTableEntries;
    const uint32_t *tab_rest = s_tab + 2 * kDevTableEntries;  // q = 3 only
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
            W av[Q], cn[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i)
                av[i] = flip ? n[Q - 1 - i][k] : n[i][k];
            sampler::node_update<Q, W, NB, GB>(av, cn, x0 + k, a.t, a.realization, a.key0,
                                               a.key1, tab_p, g_p, tab_half, g_half, tab_rest,
                                               g_rest, p_zero);
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
