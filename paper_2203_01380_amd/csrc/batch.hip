// Batched ensembles in one persistent launch.
//
// Independent realizations (the ensemble of the Boltzmann average,
// f_i = <n_i>) each advance nsteps steps of the lattice gas with flip
// (Eq. LGflip).  Each workgroup repeatedly takes the next member from a device
// queue (members sorted longest first, so the long ones start early and the
// short ones fill the tail), stages that member's removal table in LDS, builds
// its guide, and runs all of the member's steps with one workgroup barrier
// per step.  The member's double-buffered state lives in its slice of the HBM
// arena; at these sizes (tens of KB per member) it stays resident in L2 and
// the MALL while the member runs, so LDS holds only tables and several
// workgroups fit on a CU.  The per-node update is the same code as the plain
// kernel (sampler.h), so every member is bit-identical to a plain run.
//
// Diagnostics on the member's own step clock: every sk_every steps the
// structure factor S(k) = |sum_x N(x) e^{-2 pi i k x/L}|^2 / sum_x N(x),
// k = 1..nk, is added to the member's sums (FP64; the phase e^{-2 pi i x/L}
// comes from sincospi and its powers by complex multiplication); every
// amp_every steps A^LG = sum_x sin(2 pi x/L) N(x) / sum_x sin^2(2 pi x/L)
// (Results section) is appended to the member's series.
#include "ilg_internal.h"
#include "sampler.h"

namespace ilg {

namespace {

using sampler::Wide;

template <int BLOCK>
__device__ __forceinline__ double block_sum_d(double v, double *scratch)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        scratch[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < BLOCK / 64; ++w)
            r += scratch[w];
    __syncthreads();
    return r;  // valid in thread 0
}

template <int BLOCK>
__device__ __forceinline__ unsigned long long block_sum_u(unsigned long long v,
                                                          unsigned long long *scratch)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        scratch[wid] = v;
    __syncthreads();
    unsigned long long r = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < BLOCK / 64; ++w)
            r += scratch[w];
    __syncthreads();
    return r;
}

// Guide of one LDS table: entry (m, b) = #{j < m : T[m][j] <= b << (32 - GB)},
// by binary search on the nondecreasing row.
template <int GB, int BLOCK>
__device__ __forceinline__ void build_guide_lds(const uint32_t *tab, uint8_t *guide)
{
    constexpr int kRow = 1 << GB;
    for (int e = threadIdx.x; e < kChunk * kRow; e += BLOCK) {
        const uint32_t m = (uint32_t)(e >> GB) + 1u;
        const uint32_t edge = (uint32_t)(e & (kRow - 1)) << (32 - GB);
        const uint32_t *row = tab + dev_row_offset(m);
        uint32_t lo = 0, hi = m;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (row[mid] <= edge)
                lo = mid + 1;
            else
                hi = mid;
        }
        guide[e] = (uint8_t)lo;
    }
}

// Adds S(k), k = 1..nk, of the state st to member r's sums.  Modes are
// accumulated kModesPerPass at a time (each pass re-reads N(x) from L2) to
// bound the number of live FP64 accumulators.
template <int Q, typename T, int BLOCK>
__device__ __forceinline__ void sk_sample(const BatchArgs &a, uint32_t r, const T *st, uint32_t L,
                                       uint64_t pitch, double *s_red, unsigned long long *s_redu)
{
    constexpr int kModesPerPass = 8;
    unsigned long long mass = 0;
    for (uint32_t x = threadIdx.x; x < L; x += BLOCK)
#pragma unroll
        for (int i = 0; i < Q; ++i)
            mass += st[(uint64_t)i * pitch + x];
    const unsigned long long tot = block_sum_u<BLOCK>(mass, s_redu);
    for (uint32_t k0 = 0; k0 < a.nk; k0 += kModesPerPass) {
        double re[kModesPerPass], im[kModesPerPass];
#pragma unroll
        for (int k = 0; k < kModesPerPass; ++k)
            re[k] = im[k] = 0.0;
        for (uint32_t x = threadIdx.x; x < L; x += BLOCK) {
            uint64_t N = 0;
#pragma unroll
            for (int i = 0; i < Q; ++i)
                N += st[(uint64_t)i * pitch + x];
            const double Nd = (double)N;
            double sv, cv;
            sincospi(2.0 * (double)x / (double)L, &sv, &cv);
            const double zr = cv, zi = -sv;  // e^{-2 pi i x / L}
            // p = z^(k0 + 1) by repeated multiplication, then successive powers
            double pr = zr, pim = zi;
            for (uint32_t e = 0; e < k0; ++e) {
                const double nr = pr * zr - pim * zi;
                pim = pr * zi + pim * zr;
                pr = nr;
            }
#pragma unroll
            for (int k = 0; k < kModesPerPass; ++k) {
                re[k] += Nd * pr;
                im[k] += Nd * pim;
                const double nr = pr * zr - pim * zi;
                pim = pr * zi + pim * zr;
                pr = nr;
            }
        }
        for (int k = 0; k < kModesPerPass; ++k) {
            if (k0 + k >= a.nk)
                break;
            const double fr = block_sum_d<BLOCK>(re[k], s_red);
            const double fi = block_sum_d<BLOCK>(im[k], s_red);
            if (threadIdx.x == 0 && tot > 0)
                a.sk_sum[(size_t)r * a.nk + k0 + k] += (fr * fr + fi * fi) / (double)tot;
        }
    }
    if (threadIdx.x == 0)
        a.sk_cnt[r] += 1ull;
}

// SK: the launch samples S(k).  Those FP64 accumulators need about twice
// the registers of the step loop, so the S(k) variant carries an occupancy
// attribute that caps the register count (the rare diagnostic code spills
// instead of the step loop losing waves); launches without S(k) use the
// variant without it.  kMinWaves(BLOCK) is the waves per SIMD needed for two
// workgroups of 1024 threads (8) or enough smaller ones (6).
// A member's descriptor read through the constant address space (scalar
// loads at a uniform index); it is rewritten only after the member's steps.
__device__ __forceinline__ BatchMeta read_meta(const BatchMeta *p)
{
    using ConstMeta = const __attribute__((address_space(4))) BatchMeta;
    ConstMeta *q = (ConstMeta *)p;
    BatchMeta m;
    m.off = q->off;
    m.length = q->length;
    m.pitch = q->pitch;
    m.t = q->t;
    m.realization = q->realization;
    m.key0 = q->key0;
    m.key1 = q->key1;
    m.flip = q->flip;
    m.p_zero = q->p_zero;
    m.cur = q->cur;
    m.pad = 0;
    return m;
}

template <int BLOCK>
constexpr int kMinWaves = BLOCK >= 1024 ? 8 : 6;

template <int Q, typename T, int BLOCK, int GB, bool SK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kMinWaves<BLOCK>, 8)))
void batch_kernel(BatchArgs a)
{
    using W = typename Wide<T>::type;
    constexpr int NB = (Q == 3) ? 2 : 1;
    constexpr int kTabs = (Q == 3) ? 3 : 2;
    constexpr int kRowGuide = 1 << GB;
    constexpr int kG = kChunk * kRowGuide;
    constexpr int kWaves = BLOCK / 64;
    // tables first, then guides (nonzero guide addresses fold into offsets)
    constexpr int kTabBytes = kTabs * kDevTableEntries * (int)sizeof(uint32_t);
    __shared__ __align__(16) uint8_t s_lds[kTabBytes + kTabs * kG];
    uint32_t *s_tab = reinterpret_cast<uint32_t *>(s_lds);
    uint8_t *s_guide = s_lds + kTabBytes;
    __shared__ uint32_t s_next;
    __shared__ double s_red[kWaves];
    __shared__ unsigned long long s_redu[kWaves];

    sampler::stage_row_offsets();
    // Shared tables (P = 2^31 and, for q = 3, P_rest) and their guides, once.
    for (int i = threadIdx.x; i < (kTabs - 1) * kDevTableEntries; i += BLOCK)
        s_tab[kDevTableEntries + i] = a.tabs_shared[i];
    __syncthreads();
    for (int s = 1; s < kTabs; ++s)
        build_guide_lds<GB, BLOCK>(s_tab + s * kDevTableEntries, s_guide + s * kG);

    const uint32_t *tab_p = s_tab, *tab_half = s_tab + kDevTableEntries;
    const uint32_t *tab_rest = s_tab + 2 * kDevTableEntries;
    const uint8_t *g_p = s_guide, *g_half = s_guide + kG, *g_rest = s_guide + 2 * kG;
    constexpr W kMax = (W)(T)~(T)0;
    W ovf = 0;

    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0)
            s_next = atomicAdd(a.queue, 1u);
        __syncthreads();
        // Uniform across the workgroup: reading it into a scalar register
        // makes the member's descriptor (key, step, rates) scalar loads, and
        // keeps the Philox key schedule out of vector registers.
        const uint32_t idx = __builtin_amdgcn_readfirstlane(s_next);
        if (idx >= a.nreal)
            break;
        // Member index and descriptor are uniform: scalar registers.  (The
        // descriptor is rewritten only after the member's steps, by thread 0.)
        const uint32_t r = __builtin_amdgcn_readfirstlane(a.order[idx]);
        const BatchMeta m = read_meta(a.meta + r);
        const bool p_zero = m.p_zero != 0;
        const bool flip = m.flip != 0;
        if (!p_zero) {
            const uint4 *src = reinterpret_cast<const uint4 *>(a.tabs_p + (size_t)r * kDevTableEntries);
            uint4 *dst = reinterpret_cast<uint4 *>(s_tab);
            for (int i = threadIdx.x; i < kDevTableEntries / 4; i += BLOCK)
                dst[i] = src[i];
            __syncthreads();
            build_guide_lds<GB, BLOCK>(s_tab, s_guide);
        }
        __syncthreads();

        const uint32_t L = m.length;
        const uint64_t pitch = m.pitch, qp = (uint64_t)Q * m.pitch;
        T *base = reinterpret_cast<T *>(a.arena) + m.off;
        uint32_t cur = m.cur;
        for (uint32_t s = 0; s < a.nsteps; ++s) {
            const T *in = base + cur * qp;
            T *out = base + (cur ^ 1u) * qp;
            const uint32_t t = m.t + s;
            // flipped loads by swapping the outer row pointers (uniform)
            const uint64_t outer = (uint64_t)(Q - 1) * pitch;
            const T *row_lo = in + (flip ? outer : 0), *row_hi = in + (flip ? 0 : outer);
            for (uint32_t x = threadIdx.x; x < L; x += BLOCK) {
                W av[Q], cn[Q];
                av[0] = (W)*sampler::row_elem(row_lo, x);
                av[Q - 1] = (W)*sampler::row_elem(row_hi, x);
                if constexpr (Q == 3)
                    av[1] = (W)*sampler::row_elem(in + pitch, x);
                sampler::node_update<Q, W, NB, GB>(av, cn, x, t, m.realization, m.key0, m.key1,
                                                   tab_p, g_p, tab_half, g_half, tab_rest, g_rest,
                                                   p_zero);
                ovf |= sampler::or_all<Q, W>(cn);
                const uint32_t xm = (x == 0) ? L - 1 : x - 1;
                const uint32_t xp = (x + 1 == L) ? 0 : x + 1;
                *sampler::row_elem(out, xm) = (T)cn[0];
                *sampler::row_elem(out + outer, xp) = (T)cn[Q - 1];
                if constexpr (Q == 3)
                    *sampler::row_elem(out + pitch, x) = (T)cn[1];
            }
            __syncthreads();
            cur ^= 1u;
            const uint32_t t_after = t + 1u;
            const T *st = base + cur * qp;
            if constexpr (SK) {
                if (a.sk_every != 0 && t_after % a.sk_every == 0)
                    sk_sample<Q, T, BLOCK>(a, r, st, L, pitch, s_red, s_redu);
            }
            if (a.amp_every != 0 && t_after % a.amp_every == 0) {
                double num = 0.0, den = 0.0;
                for (uint32_t x = threadIdx.x; x < L; x += BLOCK) {
                    uint64_t N = 0;
#pragma unroll
                    for (int i = 0; i < Q; ++i)
                        N += st[(uint64_t)i * pitch + x];
                    const double sv = sinpi(2.0 * (double)x / (double)L);
                    num += sv * (double)N;
                    den += sv * sv;
                }
                const double tn = block_sum_d<BLOCK>(num, s_red);
                const double td = block_sum_d<BLOCK>(den, s_red);
                if (threadIdx.x == 0) {
                    const uint32_t c = a.amp_cnt[r];
                    if (c < a.max_amp)
                        a.amp[(size_t)r * a.max_amp + c] = td > 0.0 ? tn / td : 0.0;
                    a.amp_cnt[r] = c + 1u;
                }
            }
        }
        if (threadIdx.x == 0) {
            a.meta[r].t = m.t + a.nsteps;
            a.meta[r].cur = cur;
        }
    }
    if (ovf > kMax)
        atomicOr(a.err, 1u);
}

__global__ void batch_reset_kernel(uint32_t *queue)
{
    if (threadIdx.x == 0)
        *queue = 0u;
}

struct Shape {
    int block;
    int guide_bits;
    int wg_per_cu_q2;
    int wg_per_cu_q3;
};
// LDS per workgroup: tables 8320 B each plus guides of 64 rows x 2^GB bytes;
// q = 2 holds two tables, q = 3 three.  Workgroups per CU follow from the
// 160 KB of LDS and 32 waves per CU.
constexpr Shape kShapes[] = {
    {256, 6, 6, 4},  {512, 6, 3, 2},  {1024, 6, 2, 2}, {128, 6, 8, 4},
    {256, 8, 3, 2},  {512, 8, 3, 2},  {1024, 8, 2, 2},
};

template <int Q, typename T, int BLOCK, int GB>
hipError_t launch_shape(const BatchArgs &a, hipStream_t stream, int wg_per_cu)
{
    const uint32_t cus = (uint32_t)device_cu_count();
    uint32_t grid = cus * (uint32_t)wg_per_cu;
    if (grid > a.nreal)
        grid = a.nreal;
    if (grid == 0)
        grid = 1;
    if (a.sk_every != 0)
        hipLaunchKernelGGL((batch_kernel<Q, T, BLOCK, GB, true>), dim3(grid), dim3(BLOCK), 0,
                           stream, a);
    else
        hipLaunchKernelGGL((batch_kernel<Q, T, BLOCK, GB, false>), dim3(grid), dim3(BLOCK), 0,
                           stream, a);
    return hipGetLastError();
}

template <int Q, typename T, int GB>
hipError_t launch_block(int block, const BatchArgs &a, hipStream_t stream, int wg)
{
    switch (block) {
    case 128:
        return launch_shape<Q, T, 128, GB>(a, stream, wg);
    case 512:
        return launch_shape<Q, T, 512, GB>(a, stream, wg);
    case 1024:
        return launch_shape<Q, T, 1024, GB>(a, stream, wg);
    default:
        return launch_shape<Q, T, 256, GB>(a, stream, wg);
    }
}

template <int Q, typename T>
hipError_t launch_qt(int shape, const BatchArgs &a, hipStream_t stream)
{
    const Shape &s = kShapes[shape];
    const int wg = (Q == 3) ? s.wg_per_cu_q3 : s.wg_per_cu_q2;
    if (s.guide_bits == 8)
        return launch_block<Q, T, 8>(s.block, a, stream, wg);
    return launch_block<Q, T, 6>(s.block, a, stream, wg);
}

}  // namespace

int batch_shape_count()
{
    return (int)(sizeof(kShapes) / sizeof(kShapes[0]));
}

void batch_shape(int shape, int q, int *block, int *wg_per_cu)
{
    *block = kShapes[shape].block;
    *wg_per_cu = q == 3 ? kShapes[shape].wg_per_cu_q3 : kShapes[shape].wg_per_cu_q2;
}

hipError_t launch_batch_reset(uint32_t *queue, hipStream_t stream)
{
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, stream, queue);
    return hipGetLastError();
}

hipError_t launch_batch(int q, int count_bytes, int shape, const BatchArgs &a, hipStream_t stream)
{
    if (shape < 0 || shape >= batch_shape_count())
        return hipErrorInvalidValue;
    if (q == 2 && count_bytes == 2)
        return launch_qt<2, uint16_t>(shape, a, stream);
    if (q == 2 && count_bytes == 4)
        return launch_qt<2, uint32_t>(shape, a, stream);
    if (q == 3 && count_bytes == 2)
        return launch_qt<3, uint16_t>(shape, a, stream);
    if (q == 3 && count_bytes == 4)
        return launch_qt<3, uint32_t>(shape, a, stream);
    return hipErrorInvalidValue;
}

}  // namespace ilg
