#pragma once
// Batched ensembles in one persistent launch: the kernel and its launch
// shapes, shared by the translation units that instantiate it (batch.hip:
// ten-round draws; batch_p7.hip: seven-round draws; batch_ex.hip: the D1Q2
// exchange form), which then compile in parallel.
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
// k = 1..nk, is added to the member's sums (FP64; the phases come from a
// per-member twiddle table and complex multiplication); every
// amp_every steps A^LG = sum_x sin(2 pi x/L) N(x) / sum_x sin^2(2 pi x/L)
// (Results section) is appended to the member's series.
#include "ilg_internal.h"
#include "sampler.h"

namespace ilg {

namespace {

using sampler::Wide;

// Workgroup sums of NV per-thread values with one barrier.  Within a wave
// the values are summed by halving exchanges: at the exchange over lane bit
// M a lane keeps half of its values (the upper half when the bit is set),
// adds its partner's copies of them and sends the other half, so NV values
// take NV - 1 shuffles before the last one is finished by butterflies;
// afterwards lane l holds value j(l) (lane bits 5, 4, ... give the binary
// digits of j).  One lane per value parks the wave's sum in LDS as
// s_red[wave][NV]; after the barrier wave_total() adds the parked sums in
// wave order.  The caller puts a barrier between the readers of one
// reduction and the next park into the same array.
template <int N, int M>
__device__ __forceinline__ void halve_exchange(double *v, int lane, int &j)
{
    if constexpr (N > 1) {
        const bool hi = (lane & M) != 0;
#pragma unroll
        for (int i = 0; i < N / 2; ++i) {
            const double keep = hi ? v[i + N / 2] : v[i];
            const double send = hi ? v[i] : v[i + N / 2];
            v[i] = keep + __shfl_xor(send, M, 64);
        }
        j += hi ? N / 2 : 0;
        halve_exchange<N / 2, M / 2>(v, lane, j);
    }
}

template <int NV>
__device__ __forceinline__ void park_wave_sums(double (&v)[NV], double *s_red)
{
    static_assert(NV >= 1 && NV <= 32 && (NV & (NV - 1)) == 0, "NV: a power of two <= 32");
    constexpr int kLog = NV >= 32 ? 5 : NV >= 16 ? 4 : NV >= 8 ? 3 : NV >= 4 ? 2 : NV >= 2 ? 1 : 0;
    constexpr int kGroup = 64 >> kLog;  // lanes that share one value after the exchanges
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int j = 0;
    halve_exchange<NV, 32>(v, lane, j);
    double t = v[0];
#pragma unroll
    for (int m = kGroup / 2; m > 0; m >>= 1)
        t += __shfl_xor(t, m, 64);
    if ((lane & (kGroup - 1)) == 0)
        s_red[wid * NV + j] = t;
}

template <int BLOCK, int NV>
__device__ __forceinline__ double wave_total(const double *s_red, int j)
{
    double r = 0.0;
    for (int w = 0; w < BLOCK / 64; ++w)
        r += s_red[w * NV + j];
    return r;
}

__device__ __forceinline__ unsigned long long wave_sum_u(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
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

// Modes of S(k) accumulated per pass over the member's nodes (each pass
// re-reads N(x) from L2); eight bounds the live FP64 accumulators.
constexpr int kModesPerPass = 8;
// Rows (BLOCK nodes apart) per twiddle run: inside a run the phase
// e^{-2 pi i x/L} advances row by row by complex multiplication, and the
// start of the next run by one multiplication with the run's stride, so the
// rounding accumulated in a twiddle stays at a few units in the last place
// per run plus one per run boundary.
constexpr uint32_t kTwiddleRun = 16;

// Per-member twiddle table in LDS, written once when a workgroup takes a
// member (sincospi never runs inside the step loop, where its polynomial
// constants would compete with the step's registers):
//   [0, 64)            e^{-2 pi i lane / L}
//   [64, 64 + waves)   e^{-2 pi i 64 w / L}
//   kRow               e^{-2 pi i BLOCK / L}       (one row)
//   kRun = kRow + 1    e^{-2 pi i kTwiddleRun BLOCK / L}   (one run)
template <int BLOCK>
struct Twiddles {
    static constexpr int kRow = 64 + BLOCK / 64;
    static constexpr int kRun = kRow + 1;
    static constexpr int kSize = kRow + 2;
};

__device__ __forceinline__ void cmul(double &ar, double &ai, double br, double bi)
{
    const double r = ar * br - ai * bi;
    ai = ar * bi + ai * br;
    ar = r;
}

// (br, bi)^e by square-and-multiply, e >= 1.
__device__ __forceinline__ void cpow(double br, double bi, uint32_t e, double &pr, double &pi)
{
    pr = 1.0;
    pi = 0.0;
    for (; e != 0; e >>= 1) {
        if (e & 1u)
            cmul(pr, pi, br, bi);
        if (e > 1u)
            cmul(br, bi, br, bi);
    }
}

template <int BLOCK>
__device__ __forceinline__ void build_twiddles(uint32_t L, double *twr, double *twi)
{
    using Tw = Twiddles<BLOCK>;
    for (int e = threadIdx.x; e < Tw::kSize; e += BLOCK) {
        uint64_t j;
        if (e < 64)
            j = (uint64_t)e;
        else if (e < Tw::kRow)
            j = 64ull * (uint64_t)(e - 64);
        else if (e == Tw::kRow)
            j = BLOCK;
        else
            j = (uint64_t)kTwiddleRun * BLOCK;
        double sv, cv;
        sincospi(2.0 * (double)(j % L) / (double)L, &sv, &cv);
        twr[e] = cv;
        twi[e] = -sv;
    }
}

// e^{-2 pi i tid / L} of this thread from the table (one multiplication).
template <int BLOCK>
__device__ __forceinline__ void thread_twiddle(const double *twr, const double *twi, double &zr,
                                               double &zi)
{
    const int lane = threadIdx.x & 63, w = 64 + (int)(threadIdx.x >> 6);
    zr = twr[lane];
    zi = twi[lane];
    cmul(zr, zi, twr[w], twi[w]);
}

// One pass of S(k): modes k0 + 1 .. k0 + kModesPerPass, k0 = 8 PASS.  Every
// thread accumulates Re and Im of sum_x N(x) z^k over its nodes
// x = tid + j BLOCK (z = e^{-2 pi i x/L}); the pass's first power z^(k0+1)
// is taken at the start of every run and advanced with the row twiddle's
// power.  Returns the thread's share of the mass sum_x N(x).
template <int Q, typename T, int BLOCK, int PASS>
__device__ __forceinline__ unsigned long long sk_pass(const T *st, uint32_t L, uint64_t pitch,
                                                      const double *twr, const double *twi,
                                                      double (&v)[2 * kModesPerPass])
{
    using Tw = Twiddles<BLOCK>;
    constexpr uint32_t e0 = kModesPerPass * PASS + 1;
    const double wr = twr[Tw::kRow], wi = twi[Tw::kRow];
    const double rr = twr[Tw::kRun], ri = twi[Tw::kRun];
    double ur = 0.0, ui = 0.0;
    if constexpr (PASS > 0)
        cpow(wr, wi, e0, ur, ui);
    double ar, ai;  // twiddle of the run's first node
    thread_twiddle<BLOCK>(twr, twi, ar, ai);
#pragma unroll
    for (int j = 0; j < 2 * kModesPerPass; ++j)
        v[j] = 0.0;
    unsigned long long mass = 0;
    for (uint64_t x0 = threadIdx.x; x0 < L; x0 += (uint64_t)kTwiddleRun * BLOCK) {
        double zr = ar, zi = ai, qr = 0.0, qi = 0.0;
        if constexpr (PASS > 0)
            cpow(zr, zi, e0, qr, qi);
        const uint64_t run_end = x0 + (uint64_t)kTwiddleRun * BLOCK;
        const uint32_t xend = run_end < L ? (uint32_t)run_end : L;
        for (uint32_t x = (uint32_t)x0; x < xend; x += BLOCK) {
            uint64_t N = 0;
#pragma unroll
            for (int i = 0; i < Q; ++i)
                N += st[(uint64_t)i * pitch + x];
            mass += N;
            const double Nd = (double)N;
            double pr = PASS > 0 ? qr : zr, pim = PASS > 0 ? qi : zi;
#pragma unroll
            for (int k = 0; k < kModesPerPass; ++k) {
                if (k > 0)
                    cmul(pr, pim, zr, zi);
                v[2 * k] += Nd * pr;
                v[2 * k + 1] += Nd * pim;
            }
            cmul(zr, zi, wr, wi);
            if constexpr (PASS > 0)
                cmul(qr, qi, ur, ui);
        }
        cmul(ar, ai, rr, ri);
    }
    return mass;
}

// Adds S(k), k = 1..nk, of the state st to member r's sums: one pass per
// eight modes, each closed by one barrier-separated reduction that gives
// thread j the sums of mode k0 + j + 1; the mass is reduced exactly
// (integers) with the first pass.
template <int Q, typename T, int BLOCK>
__device__ __forceinline__ void sk_sample(const BatchArgs &a, uint32_t r, const T *st, uint32_t L,
                                       uint64_t pitch, const double *twr, const double *twi,
                                       double *s_red, unsigned long long *s_redu)
{
    constexpr int kWaves = BLOCK / 64;
    constexpr int NV = 2 * kModesPerPass;
    static_assert(ILG_BATCH_MAX_K <= 2 * kModesPerPass, "two passes cover every mode");
    unsigned long long tot = 0;
    for (uint32_t k0 = 0; k0 < a.nk; k0 += kModesPerPass) {
        double v[NV];
        unsigned long long mass;
        if (k0 == 0)
            mass = sk_pass<Q, T, BLOCK, 0>(st, L, pitch, twr, twi, v);
        else
            mass = sk_pass<Q, T, BLOCK, 1>(st, L, pitch, twr, twi, v);
        __syncthreads();  // readers of the previous reduction are done
        park_wave_sums<NV>(v, s_red);
        if (k0 == 0) {
            mass = wave_sum_u(mass);
            if ((threadIdx.x & 63) == 0)
                s_redu[threadIdx.x >> 6] = mass;
        }
        __syncthreads();
        if (k0 == 0)
            for (int w = 0; w < kWaves; ++w)
                tot += s_redu[w];
        const uint32_t k = k0 + threadIdx.x;
        if (threadIdx.x < (uint32_t)kModesPerPass && k < a.nk && tot > 0) {
            const double fr = wave_total<BLOCK, NV>(s_red, 2 * threadIdx.x);
            const double fi = wave_total<BLOCK, NV>(s_red, 2 * threadIdx.x + 1);
            a.sk_sum[(size_t)r * a.nk + k] += (fr * fr + fi * fi) / (double)tot;
        }
    }
    if (threadIdx.x == 0)
        a.sk_cnt[r] += 1ull;
}

// A^LG of the state st: sum_x sin(2 pi x/L) N(x) / sum_x sin^2(2 pi x/L),
// with the twiddles of S(k) (sin = -Im z).  Valid in thread 0.
template <int Q, typename T, int BLOCK>
__device__ __forceinline__ double amp_sample(const T *st, uint32_t L, uint64_t pitch,
                                             const double *twr, const double *twi, double *s_red)
{
    using Tw = Twiddles<BLOCK>;
    const double wr = twr[Tw::kRow], wi = twi[Tw::kRow];
    const double rr = twr[Tw::kRun], ri = twi[Tw::kRun];
    double ar, ai;
    thread_twiddle<BLOCK>(twr, twi, ar, ai);
    double v[2] = {0.0, 0.0};  // sum sin N, sum sin^2
    for (uint64_t x0 = threadIdx.x; x0 < L; x0 += (uint64_t)kTwiddleRun * BLOCK) {
        double zr = ar, zi = ai;
        const uint64_t run_end = x0 + (uint64_t)kTwiddleRun * BLOCK;
        const uint32_t xend = run_end < L ? (uint32_t)run_end : L;
        for (uint32_t x = (uint32_t)x0; x < xend; x += BLOCK) {
            uint64_t N = 0;
#pragma unroll
            for (int i = 0; i < Q; ++i)
                N += st[(uint64_t)i * pitch + x];
            const double sv = -zi;
            v[0] += sv * (double)N;
            v[1] += sv * sv;
            cmul(zr, zi, wr, wi);
        }
        cmul(ar, ai, rr, ri);
    }
    __syncthreads();  // earlier readers of s_red are done
    park_wave_sums<2>(v, s_red);
    __syncthreads();
    if (threadIdx.x != 0)
        return 0.0;
    const double tn = wave_total<BLOCK, 2>(s_red, 0);
    const double td = wave_total<BLOCK, 2>(s_red, 1);
    return td > 0.0 ? tn / td : 0.0;
}

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
    m.width = q->width;
    return m;
}

template <int BLOCK>
constexpr int kMinWaves = BLOCK >= 1024 ? 8 : 6;

// SK: the launch samples S(k).  Every instantiation carries an occupancy
// attribute: kMinWaves(BLOCK) waves per SIMD, what two workgroups of 1024
// threads (8) or enough smaller ones (6) need, which caps the register
// count.  The S(k) variant's FP64 accumulators need about twice the
// registers of the step loop; under the cap that rare diagnostic code
// spills instead of the step loop losing waves.
// NR: Philox rounds of the draws (10, or 7 for draw specification v2); EX:
// the D1Q2 exchange form (specification v3).  Both are batch-wide.
template <int Q, typename T, int BLOCK, int GB, bool SK, int NR, bool EX>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kMinWaves<BLOCK>, 8)))
void batch_kernel(BatchArgs a)
{
    using W = typename Wide<T>::type;
    constexpr int NB = (Q == 5) ? 3 : (Q == 3) ? 2 : 1;  // Philox blocks drawn up front
    constexpr int kTabs = (Q == 2) ? 2 : 3;
    static_assert(Q != 5 || !SK, "S(k) is defined for 1D members");
    constexpr int kRowGuide = 1 << GB;
    constexpr int kG = kChunk * kRowGuide;
    constexpr int kWaves = BLOCK / 64;
    // tables first, then guides (nonzero guide addresses fold into offsets)
    constexpr int kTabBytes = kTabs * kDevTableEntries * (int)sizeof(uint32_t);
    __shared__ __align__(16) uint8_t s_lds[kTabBytes + kTabs * kG];
    uint32_t *s_tab = reinterpret_cast<uint32_t *>(s_lds);
    uint8_t *s_guide = s_lds + kTabBytes;
    __shared__ uint32_t s_next;
    // wave sums of the diagnostics' reductions (S(k): 2 x 8 modes per wave)
    __shared__ double s_red[kWaves * (SK ? 2 * kModesPerPass : 2)];
    __shared__ unsigned long long s_redu[kWaves];
    __shared__ double s_twr[Twiddles<BLOCK>::kSize], s_twi[Twiddles<BLOCK>::kSize];

    const uint32_t *tab_p = s_tab, *tab_half = s_tab + kDevTableEntries;
    const uint32_t *tab_rest = s_tab + 2 * kDevTableEntries;
    const sampler::Tabs tb = sampler::make_tabs(tab_p, s_guide, kG);
    sampler::stage_row_offsets(tab_p, tab_half, tab_rest);
    // Shared tables (P = 2^31 and, for q = 3, P_rest) and their guides, once.
    for (int i = threadIdx.x; i < (kTabs - 1) * kDevTableEntries; i += BLOCK)
        s_tab[kDevTableEntries + i] = a.tabs_shared[i];
    __syncthreads();
    for (int s = 1; s < kTabs; ++s)
        build_guide_lds<GB, BLOCK>(s_tab + s * kDevTableEntries, s_guide + s * kG);

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
        if (SK || a.amp_every != 0)
            build_twiddles<BLOCK>(m.length, s_twr, s_twi);
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
                if constexpr (Q == 5) {
                    // the flip also swaps the y pair (rows 1 and 3)
                    av[1] = (W)*sampler::row_elem(in + (flip ? 3 : 1) * pitch, x);
                    av[2] = (W)*sampler::row_elem(in + 2 * pitch, x);
                    av[3] = (W)*sampler::row_elem(in + (flip ? 1 : 3) * pitch, x);
                }
                if constexpr (EX) {
                    static_assert(Q == 2, "the exchange form is defined for D1Q2");
                    sampler::node_exchange<W, NB, GB, NR>(av, cn, x, t, m.realization,
                                                          PhiloxKey{m.key0, m.key1}, tb, p_zero);
                } else {
                    sampler::node_update<Q, W, NB, GB, NR>(av, cn, x, t, m.realization,
                                                           PhiloxKey{m.key0, m.key1}, tb, p_zero);
                }
                ovf |= sampler::or_all<Q, W>(cn);
                if constexpr (Q == 5) {
                    // D2Q5 on the node index x + Lx y: -x, -y, rest, +y, +x
                    uint32_t dxm, dym, dyp, dxp;
                    sampler::d2q5_neighbours<BLOCK>(
                        x, __builtin_amdgcn_readfirstlane(x - threadIdx.x), m.width, L, dxm, dym,
                        dyp, dxp);
                    *sampler::row_elem(out, dxm) = (T)cn[0];
                    *sampler::row_elem(out + pitch, dym) = (T)cn[1];
                    *sampler::row_elem(out + 2 * pitch, x) = (T)cn[2];
                    *sampler::row_elem(out + 3 * pitch, dyp) = (T)cn[3];
                    *sampler::row_elem(out + 4 * pitch, dxp) = (T)cn[4];
                } else {
                    const uint32_t xm = (x == 0) ? L - 1 : x - 1;
                    const uint32_t xp = (x + 1 == L) ? 0 : x + 1;
                    *sampler::row_elem(out, xm) = (T)cn[0];
                    *sampler::row_elem(out + outer, xp) = (T)cn[Q - 1];
                    if constexpr (Q == 3)
                        *sampler::row_elem(out + pitch, x) = (T)cn[1];
                }
            }
            __syncthreads();
            cur ^= 1u;
            const uint32_t t_after = t + 1u;
            const T *st = base + cur * qp;
            if constexpr (SK) {
                if (a.sk_every != 0 && t_after % a.sk_every == 0)
                    sk_sample<Q, T, BLOCK>(a, r, st, L, pitch, s_twr, s_twi, s_red, s_redu);
            }
            if (Q != 5 && a.amp_every != 0 && t_after % a.amp_every == 0) {
                const double amp = amp_sample<Q, T, BLOCK>(st, L, pitch, s_twr, s_twi, s_red);
                if (threadIdx.x == 0) {
                    const uint32_t c = a.amp_cnt[r];
                    if (c < a.max_amp)
                        a.amp[(size_t)r * a.max_amp + c] = amp;
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

template <int Q, typename T, int BLOCK, int GB, int NR, bool EX>
hipError_t launch_shape(const BatchArgs &a, hipStream_t stream, int wg_per_cu)
{
    const uint32_t cus = (uint32_t)device_cu_count();
    uint32_t grid = cus * (uint32_t)wg_per_cu;
    if (grid > a.nreal)
        grid = a.nreal;
    if (grid == 0)
        grid = 1;
    if constexpr (Q == 5) {
        if (a.sk_every != 0)
            return hipErrorInvalidValue;  // S(k) is defined for 1D members
        hipLaunchKernelGGL((batch_kernel<Q, T, BLOCK, GB, false, NR, EX>), dim3(grid), dim3(BLOCK),
                           0, stream, a);
    } else {
        if (a.sk_every != 0)
            hipLaunchKernelGGL((batch_kernel<Q, T, BLOCK, GB, true, NR, EX>), dim3(grid),
                               dim3(BLOCK), 0, stream, a);
        else
            hipLaunchKernelGGL((batch_kernel<Q, T, BLOCK, GB, false, NR, EX>), dim3(grid),
                               dim3(BLOCK), 0, stream, a);
    }
    return hipGetLastError();
}

template <int Q, typename T, int GB, int NR, bool EX>
hipError_t launch_block(int block, const BatchArgs &a, hipStream_t stream, int wg)
{
    switch (block) {
    case 128:
        return launch_shape<Q, T, 128, GB, NR, EX>(a, stream, wg);
    case 512:
        return launch_shape<Q, T, 512, GB, NR, EX>(a, stream, wg);
    case 1024:
        return launch_shape<Q, T, 1024, GB, NR, EX>(a, stream, wg);
    default:
        return launch_shape<Q, T, 256, GB, NR, EX>(a, stream, wg);
    }
}

template <int Q, typename T, int NR, bool EX>
hipError_t launch_qt(int shape, const BatchArgs &a, hipStream_t stream)
{
    const Shape &s = kShapes[shape];
    const int wg = (Q == 2) ? s.wg_per_cu_q2 : s.wg_per_cu_q3;  // q = 3, 5: three tables
    if (s.guide_bits == 8)
        return launch_block<Q, T, 8, NR, EX>(s.block, a, stream, wg);
    return launch_block<Q, T, 6, NR, EX>(s.block, a, stream, wg);
}

}  // namespace

}  // namespace ilg
