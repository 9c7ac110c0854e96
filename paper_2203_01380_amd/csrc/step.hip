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
// Mapping: a persistent grid of 512-thread workgroups, each holding the three
// fixed-point tables and their guides in LDS (37 KB).  A tile is 512 * NPT
// consecutive nodes; every thread owns NPT consecutive nodes and reads each
// velocity row with one vector load.  Streaming stores are per element (the
// +-1 shift breaks vector alignment); the wave still writes contiguous bytes.
// Tiles are dealt so that the workgroups of one XCD (dispatch is round-robin
// over the 8 XCDs) cover one contiguous eighth of the lattice.
#include "ilg_internal.h"
#include "philox.h"

namespace ilg {

namespace {

constexpr int kBlock = 512;
constexpr int kNumXcd = 8;

template <typename T, int N>
struct alignas(N * sizeof(T)) VecT {
    T v[N];
};

// Inverse-CDF count of one chunk: #{j < m : row[j] <= u}.  The guide gives
// the count at the bucket's lower edge; rows are nondecreasing, so the scan
// continues from there until the first entry above u.
__device__ __forceinline__ uint32_t chunk_count(const uint32_t *tab, const uint8_t *guide,
                                                uint32_t m, uint32_t u)
{
    const uint32_t *row = tab + (((m - 1u) * m) >> 1);
    uint32_t j = guide[((m - 1u) << kGuideBits) + (u >> (32 - kGuideBits))];
    while (j < m && row[j] <= u)
        ++j;
    return j;
}

// The draws of one node-step.  The first NB blocks are computed up front (all
// lanes need them at these occupation numbers); later blocks are computed on
// demand.
template <int NB>
struct Draws {
    uint32_t w[4 * NB];
    uint32_t cur[4];
    uint32_t cur_block;
    uint32_t j;
    uint32_t x, t, r, k0, k1;

    __device__ __forceinline__ void init(uint32_t x_, uint32_t t_, uint32_t r_, uint32_t k0_,
                                         uint32_t k1_)
    {
        x = x_; t = t_; r = r_; k0 = k0_; k1 = k1_;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            uint4 o = philox4x32_10(x, t, r, (uint32_t)b, k0, k1);
            w[4 * b + 0] = o.x; w[4 * b + 1] = o.y; w[4 * b + 2] = o.z; w[4 * b + 3] = o.w;
        }
        cur[0] = w[0]; cur[1] = w[1]; cur[2] = w[2]; cur[3] = w[3];
        cur_block = 0;
        j = 0;
    }

    __device__ __forceinline__ uint32_t next()
    {
        const uint32_t jj = j++;
        const uint32_t blk = jj >> 2;
        if (blk != cur_block) {
            bool have = false;
            if constexpr (NB >= 2) {
                if (blk == 1) {
                    cur[0] = w[4]; cur[1] = w[5]; cur[2] = w[6]; cur[3] = w[7];
                    have = true;
                }
            }
            if (!have) {
                uint4 o = philox4x32_10(x, t, r, blk, k0, k1);
                cur[0] = o.x; cur[1] = o.y; cur[2] = o.z; cur[3] = o.w;
            }
            cur_block = blk;
        }
        const uint32_t s = jj & 3u;
        const uint32_t lo = (s & 1u) ? cur[1] : cur[0];
        const uint32_t hi = (s & 1u) ? cur[3] : cur[2];
        return (s & 2u) ? hi : lo;
    }
};

// Bin(n, table) with the chunked rule; p_zero: the probability is 0 (draws
// are still consumed so that draw positions do not depend on p).
template <typename W, int NB>
__device__ __forceinline__ W binomial(W n, const uint32_t *tab, const uint8_t *guide,
                                      bool p_zero, Draws<NB> &d)
{
    W total = 0;
    while (n > 0) {
        const uint32_t m = n >= (W)kChunk ? (uint32_t)kChunk : (uint32_t)n;
        const uint32_t u = d.next();
        if (!p_zero)
            total += chunk_count(tab, guide, m, u);
        n -= m;
    }
    return total;
}

template <typename T> struct Wide;
template <> struct Wide<uint16_t> { using type = uint32_t; };
template <> struct Wide<uint32_t> { using type = uint64_t; };

template <int Q, typename T, int NPT, int NB>
__global__ __launch_bounds__(kBlock) void step_kernel(StepArgs a)
{
    using W = typename Wide<T>::type;
    constexpr int kTabs = (Q == 3) ? 3 : 2;
    __shared__ uint32_t s_tab[kTabs * kTableEntries];
    __shared__ uint8_t s_guide[kTabs * kGuideEntries];

    // Stage the table set in LDS (16-byte copies; both parts are multiples of 16).
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.tables);
        uint4 *dst = reinterpret_cast<uint4 *>(s_tab);
        const int n = kTabs * kTableEntries * 4 / 16;
        for (int i = threadIdx.x; i < n; i += kBlock)
            dst[i] = src[i];
        const uint4 *gsrc = reinterpret_cast<const uint4 *>(guide_ptr(a.tables, 0));
        uint4 *gdst = reinterpret_cast<uint4 *>(s_guide);
        const int ng = kTabs * kGuideEntries / 16;
        for (int i = threadIdx.x; i < ng; i += kBlock)
            gdst[i] = gsrc[i];
    }
    __syncthreads();

    const uint32_t *tab_p = s_tab;
    const uint32_t *tab_half = s_tab + kTableEntries;
    const uint32_t *tab_rest = s_tab + 2 * kTableEntries;  // q = 3 only
    const uint8_t *g_p = s_guide;
    const uint8_t *g_half = s_guide + kGuideEntries;
    const uint8_t *g_rest = s_guide + 2 * kGuideEntries;
    const bool p_zero = a.p_zero != 0;
    const bool flip = a.flip != 0;
    const uint32_t L = a.length;
    const uint64_t pitch = a.pitch;
    const T *in = reinterpret_cast<const T *>(a.in);
    T *out = reinterpret_cast<T *>(a.out);
    constexpr W kMax = (W)(T)~(T)0;

    constexpr uint32_t kTile = (uint32_t)kBlock * NPT;
    const uint32_t ntiles = (L + kTile - 1) / kTile;
    uint32_t first, stride, end;
    if (gridDim.x % kNumXcd == 0) {
        const uint32_t xcd = blockIdx.x % kNumXcd, per = gridDim.x / kNumXcd;
        first = (uint32_t)((uint64_t)ntiles * xcd / kNumXcd) + blockIdx.x / kNumXcd;
        end = (uint32_t)((uint64_t)ntiles * (xcd + 1) / kNumXcd);
        stride = per;
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
        T n[Q][NPT];
        if (x0 + NPT <= L) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                VecT<T, NPT> v = *reinterpret_cast<const VecT<T, NPT> *>(in + i * pitch + x0);
#pragma unroll
                for (int k = 0; k < NPT; ++k)
                    n[i][k] = v.v[k];
            }
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i)
#pragma unroll
                for (int k = 0; k < NPT; ++k)
                    n[i][k] = (x0 + k < L) ? in[i * pitch + x0 + k] : (T)0;
        }

        W c[Q][NPT];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const uint32_t x = x0 + k;
            W av[Q], kv[Q], mv[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i)
                av[i] = (W)(flip ? n[Q - 1 - i][k] : n[i][k]);
            Draws<NB> d;
            d.init(x, a.t, a.realization, a.key0, a.key1);
            W M = 0;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                kv[i] = binomial<W, NB>(av[i], tab_p, g_p, p_zero, d);
                M += kv[i];
            }
            if (Q == 2) {
                mv[0] = binomial<W, NB>(M, tab_half, g_half, false, d);
                mv[1] = M - mv[0];
            } else {
                mv[1] = binomial<W, NB>(M, tab_rest, g_rest, false, d);
                const W R = M - mv[1];
                mv[0] = binomial<W, NB>(R, tab_half, g_half, false, d);
                mv[Q - 1] = R - mv[0];
            }
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                c[i][k] = av[i] - kv[i] + mv[i];
                overflow |= c[i][k] > kMax;
            }
        }

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
        if (Q == 3) {
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

template <int Q, typename T, int NPT, int NB>
hipError_t launch_variant(const StepArgs &a, hipStream_t stream)
{
    constexpr uint32_t kTile = (uint32_t)kBlock * NPT;
    const uint32_t ntiles = (a.length + kTile - 1) / kTile;
    static int cus = 0;
    if (cus == 0)
        cus = device_cu_count();
    // Two 512-thread workgroups per CU (LDS 37 KB each); round to the XCD count.
    uint32_t grid = (uint32_t)cus * 2;
    if (ntiles < grid)
        grid = ntiles;
    if (grid >= (uint32_t)kNumXcd)
        grid -= grid % kNumXcd;
    if (grid == 0)
        grid = 1;
    hipLaunchKernelGGL((step_kernel<Q, T, NPT, NB>), dim3(grid), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step(int q, int count_bytes, const StepArgs &a, hipStream_t stream)
{
    if (q == 2 && count_bytes == 2)
        return launch_variant<2, uint16_t, 4, 1>(a, stream);
    if (q == 2 && count_bytes == 4)
        return launch_variant<2, uint32_t, 4, 1>(a, stream);
    if (q == 3 && count_bytes == 2)
        return launch_variant<3, uint16_t, 4, 2>(a, stream);
    if (q == 3 && count_bytes == 4)
        return launch_variant<3, uint32_t, 4, 2>(a, stream);
    return hipErrorInvalidValue;
}

}  // namespace ilg
