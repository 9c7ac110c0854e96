// Fused lattice-gas step for gfx950: load -> flip -> sampling collision ->
// push streaming, one pass over the structure-of-arrays occupation arrays
// (Eq. LGflip, then the streaming of Eq. ilgeq: out_i[(x + v_i) mod L] = c_i).
// The per-node sampler is in sampler.h.
//
// Mapping: a persistent grid of 1024-thread workgroups (two per CU), each
// holding the fixed-point tables and their guides in LDS, staged once.  A
// tile is BLOCK consecutive nodes, one per thread, so every wave reads and
// writes contiguous bytes of each velocity row.  Tiles are dealt so that the
// workgroups of one XCD (dispatch is round-robin over the 8 XCDs) cover one
// contiguous eighth of the lattice.  (Two or four nodes per thread, with
// vector loads, measured slower: the extra registers cost more than the
// wider accesses gain in this VALU-bound kernel.)
#include <type_traits>

#include "ilg_internal.h"
#include "sampler.h"

namespace ilg {

namespace {

constexpr int kNumXcd = 8;
// Launch shape: 1024-thread workgroups, two per CU (the LDS tables and guides
// of one workgroup take 74 KB).  512-thread workgroups and 128-bucket guides
// measured slower.
constexpr int kBlock = 1024;
constexpr int kWgPerCu = 2;
using sampler::Wide;

using sampler::row_elem;

// Waves per SIMD the kernel must fit.  The uint32 D1Q3 kernel is held to
// eight (two 1024-thread workgroups per CU, at most 64 registers): left free
// it takes 74 and runs one workgroup per CU, which measured slower than the
// capped kernel with its 12-byte spill.  The uint32 D2Q5 kernel spills far
// more under that cap and measured slower with it, so it and the rest keep
// the compiler's choice.
template <int Q, typename T>
constexpr int kMinWaves = (Q == 3 && sizeof(T) == 4) ? 8 : 1;

// EX: the D1Q2 exchange form (Q = 2 only).
template <int Q, typename T, int NB, int GB, int BLOCK, bool FLIP, bool PZ, int NR, bool EX>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kMinWaves<Q, T>))) void step_kernel(StepArgs a)
{
    using W = typename Wide<T>::type;
    constexpr int kTabs = (Q == 2) ? 2 : 3;
    constexpr int kRowGuide = 1 << GB;
    // Tables first, guides after them: every guide then sits at a nonzero
    // LDS address, which lets the row-and-bucket index fold into the
    // instruction's offset field.
    constexpr int kTabBytes = kTabs * kDevTableEntries * (int)sizeof(uint32_t);
    __shared__ __align__(16) uint8_t s_lds[kTabBytes + kTabs * kChunk * kRowGuide];
    uint32_t *s_tab = reinterpret_cast<uint32_t *>(s_lds);
    uint8_t *s_guide = s_lds + kTabBytes;

    const uint32_t *tab_p = s_tab;
    const uint32_t *tab_half = s_tab + kDevTableEntries;
    const uint32_t *tab_rest = s_tab + 2 * kDevTableEntries;  // q = 3, 5 only
    constexpr int kG = kChunk * kRowGuide;
    const sampler::Tabs tb = sampler::make_tabs(tab_p, s_guide, kG);
    // Stage tables (16-byte copies) and the 2^GB-bucket view of the guides.
    sampler::stage_row_offsets(tab_p, tab_half, tab_rest);
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

    const uint32_t L = a.length;
    const uint64_t pitch = a.pitch;
    const T *in = reinterpret_cast<const T *>(a.in);
    T *out = reinterpret_cast<T *>(a.out);
    constexpr W kMax = (W)(T)~(T)0;

    constexpr uint32_t kTile = (uint32_t)BLOCK;
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

    const T *in_row[Q];
    T *out_row[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        in_row[i] = in + (uint64_t)i * pitch;
        out_row[i] = out + (uint64_t)i * pitch;
    }

    W ovf = 0;
    for (uint32_t tile = first; tile < end; tile += stride) {
        const uint32_t x = tile * kTile + threadIdx.x;
        if (x >= L)
            continue;
        W n[Q], av[Q], cn[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i)
            n[i] = (W)*row_elem(in_row[i], x);
#pragma unroll
        for (int i = 0; i < Q; ++i)
            av[i] = FLIP ? n[Q - 1 - i] : n[i];
        if constexpr (EX) {
            static_assert(Q == 2, "the exchange form is defined for D1Q2");
            sampler::node_exchange<W, NB, GB, NR>(av, cn, x, a.t, a.realization,
                                                  PhiloxKey{a.key0, a.key1}, tb, PZ);
        } else {
            sampler::node_update<Q, W, NB, GB, NR>(av, cn, x, a.t, a.realization,
                                                   PhiloxKey{a.key0, a.key1}, tb, PZ);
        }
        ovf |= sampler::or_all<Q, W>(cn);
        if constexpr (Q == 5) {
            // D2Q5 streaming on the node index x + Lx y: -x, -y, rest, +y, +x
            uint32_t dxm, dym, dyp, dxp;
            sampler::d2q5_neighbours<BLOCK>(x, tile * kTile, a.width, L, dxm, dym, dyp, dxp);
            *row_elem(out_row[0], dxm) = (T)cn[0];
            *row_elem(out_row[1], dym) = (T)cn[1];
            *row_elem(out_row[2], x) = (T)cn[2];
            *row_elem(out_row[3], dyp) = (T)cn[3];
            *row_elem(out_row[4], dxp) = (T)cn[4];
            continue;
        }
        // Streaming: velocity -1 to x-1, 0 in place, +1 to x+1 (periodic).
        const uint32_t xm = (x == 0) ? L - 1 : x - 1;
        const uint32_t xp = (x + 1 == L) ? 0 : x + 1;
        *row_elem(out_row[0], xm) = (T)cn[0];
        *row_elem(out_row[Q - 1], xp) = (T)cn[Q - 1];
        if constexpr (Q == 3)
            *row_elem(out_row[1], x) = (T)cn[1];
    }
    if (ovf > kMax)
        atomicOr(a.err, 1u);
}

template <int Q, typename T, int NB, bool FLIP, bool PZ, int NR, bool EX = false>
hipError_t launch_mode(const StepArgs &a, hipStream_t stream)
{
    constexpr uint32_t kTile = (uint32_t)kBlock;
    const uint32_t ntiles = (a.length + kTile - 1) / kTile;
    static int cus = 0;
    if (cus == 0)
        cus = device_cu_count();
    uint32_t grid = (uint32_t)cus * (uint32_t)kWgPerCu;
    if (ntiles < grid)
        grid = ntiles;
    if (grid >= (uint32_t)kNumXcd)
        grid -= grid % kNumXcd;
    if (grid == 0)
        grid = 1;
    hipLaunchKernelGGL((step_kernel<Q, T, NB, kGuideBits, kBlock, FLIP, PZ, NR, EX>), dim3(grid),
                       dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

// The flip, a zero collision fraction, the Philox round count and the D1Q2
// exchange form are per-lattice constants, so each combination has its own
// kernel (no per-node tests for them).  With a zero collision fraction no
// particle moves whatever the draws are, so that kernel serves every round
// count and both D1Q2 forms.
template <int Q, typename T, int NB, bool FLIP, int NR>
hipError_t launch_ex(const StepArgs &a, hipStream_t stream)
{
    if constexpr (Q == 2) {
        if (a.exchange)
            return launch_mode<Q, T, NB, FLIP, false, NR, true>(a, stream);
    }
    return launch_mode<Q, T, NB, FLIP, false, NR>(a, stream);
}

template <int Q, typename T, int NB>
hipError_t launch_q(const StepArgs &a, hipStream_t stream)
{
    if (a.p_zero)
        return a.flip ? launch_mode<Q, T, NB, true, true, 10>(a, stream)
                      : launch_mode<Q, T, NB, false, true, 10>(a, stream);
    if (a.rounds == 7)
        return a.flip ? launch_ex<Q, T, NB, true, 7>(a, stream)
                      : launch_ex<Q, T, NB, false, 7>(a, stream);
    return a.flip ? launch_ex<Q, T, NB, true, 10>(a, stream)
                  : launch_ex<Q, T, NB, false, 10>(a, stream);
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
    if (q == 5 && count_bytes == 2)
        return launch_q<5, uint16_t, 3>(a, stream);
    if (q == 5 && count_bytes == 4)
        return launch_q<5, uint32_t, 3>(a, stream);
    return hipErrorInvalidValue;
}

}  // namespace ilg
