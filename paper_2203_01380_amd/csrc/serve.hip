// Multi-slot lattice-gas step for the continuous-batching server (D1Q2, D1Q3
// and D2Q5 requests).
//
// One launch advances every active request (slot) of one (q, count type) by
// one step: the host lists the slots' tiles of 1024 nodes, slot by slot (each
// slot's descriptor holds its tile range), and each workgroup of a persistent
// grid walks a contiguous range of that list.  Small requests (resident
// slots) instead each get a workgroup of their own beyond that grid, which
// advances the request by several steps per launch (as many as fit in the
// time of the tile walk), so their steps do not wait for the launches.  A count beyond the type sets
// the error word of its own slot only, so one overflowing request does not
// affect the others.
// When the walk enters a new slot the workgroup stages the slot's removal and
// rest tables with their guides in LDS (the half table is shared and staged
// once).  Slots whose quantum is shorter than the current step index are
// skipped.  The node update is the same code as the plain kernel (sampler.h),
// so every request's result equals the same configuration run alone.
#include "ilg_internal.h"
#include "sampler.h"

namespace ilg {

namespace {

using sampler::Wide;

// Element x of a velocity row given by its address in the descriptor, read
// and written as global memory (a bare 64-bit address would make flat
// accesses).  16-bit rows: 32-bit lane offset (fewer than 2^31 nodes).
template <typename T>
using GlobalT = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ GlobalT<T> *global_elem(uint64_t row, uint32_t x)
{
    using B = GlobalT<uint8_t>;
    B *base = (B *)(uintptr_t)row;
    if constexpr (sizeof(T) == 2)
        return reinterpret_cast<GlobalT<T> *>(base + (uint32_t)(x * 2u));
    else
        return reinterpret_cast<GlobalT<T> *>(base) + x;
}

constexpr int kBlock = kServeTile;  // one node per thread per tile

// The slot descriptors are read-only during a launch: read through the
// constant address space at a uniform index they are scalar loads.
using ConstSlot = const __attribute__((address_space(4))) ServeSlot;
__device__ __forceinline__ ConstSlot *const_space(const ServeSlot *p)
{
    return (ConstSlot *)p;
}

constexpr int kG = kChunk << kServeGuideBits;  // guide bytes per table

// LDS of a serving workgroup: tables first, then guides (nonzero guide
// addresses fold into offsets); table 0 removal, 1 half (shared by every
// request), 2 rest (q = 3, 5).
template <int Q>
struct ServeLds {
    static constexpr int kTabs = (Q == 2) ? 2 : 3;
    static constexpr int kTabBytes = kTabs * kDevTableEntries * (int)sizeof(uint32_t);
    static constexpr int kBytes = kTabBytes + kTabs * kG;
};

// Stages the shared half table and its guide (LDS table 1).
__device__ __forceinline__ void stage_half(const void *shared, uint32_t *s_tab, uint8_t *s_guide)
{
    const uint4 *src = reinterpret_cast<const uint4 *>(shared);
    uint4 *dst = reinterpret_cast<uint4 *>(s_tab + kDevTableEntries);
    for (int i = threadIdx.x; i < kDevTableEntries / 4; i += kBlock)
        dst[i] = src[i];
    const uint4 *gsrc =
        reinterpret_cast<const uint4 *>(reinterpret_cast<const uint8_t *>(shared) + kServeTableBytes);
    uint4 *gdst = reinterpret_cast<uint4 *>(s_guide + kG);
    for (int i = threadIdx.x; i < kG / 16; i += kBlock)
        gdst[i] = gsrc[i];
}

// Stages a slot's removal (+ rest) tables and their guides (LDS tables 0, 2).
template <int Q>
__device__ __forceinline__ void stage_slot(const void *arena, uint64_t table_off, uint32_t *s_tab,
                                           uint8_t *s_guide)
{
    const uint8_t *set = reinterpret_cast<const uint8_t *>(arena) + table_off;
    constexpr int nt = (Q == 2) ? 1 : 2;  // removal (+ rest) tables
    for (int t = 0; t < nt; ++t) {
        const uint4 *src = reinterpret_cast<const uint4 *>(set + t * kServeTableBytes);
        uint4 *dst = reinterpret_cast<uint4 *>(s_tab + (t == 0 ? 0 : 2) * kDevTableEntries);
        for (int i = threadIdx.x; i < kDevTableEntries / 4; i += kBlock)
            dst[i] = src[i];
        const uint4 *gsrc =
            reinterpret_cast<const uint4 *>(set + nt * kServeTableBytes + t * kServeGuideBytes);
        uint4 *gdst = reinterpret_cast<uint4 *>(s_guide + (t == 0 ? 0 : 2) * kG);
        for (int i = threadIdx.x; i < kG / 16; i += kBlock)
            gdst[i] = gsrc[i];
    }
}

// Counts of node x of one slot at step index j of its advance, with the
// flip applied (the descriptor's row addresses of this step's buffers).
template <int Q, typename T, typename W>
__device__ __forceinline__ void serve_load(ConstSlot *sl, uint32_t j, uint32_t x, W (&av)[Q])
{
    const uint32_t par = j & 1u;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        av[i] = (W)*global_elem<T>(sl->rows[par][i], x);
}

// Node x of one slot at step index j (absolute step sl->t0 + j), its counts
// av loaded: update, push to the neighbours.  x0: the first node of the
// thread's tile (uniform).  NB: Philox blocks drawn up front.
template <int Q, typename T, int NR, bool EX, int NB, typename W, typename K>
__device__ __forceinline__ void serve_update(ConstSlot *sl, uint32_t j, uint32_t x0, uint32_t x,
                                             const W (&av)[Q], const K &key,
                                             const sampler::Tabs &tb, W &ovf)
{
    constexpr int GB = kServeGuideBits;
    const uint32_t L = sl->length;
    const uint32_t par = j & 1u;
    uint64_t out_row[Q];
    W cn[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i)
        out_row[i] = sl->rows[par][5 + i];
    const uint32_t t = sl->t0 + j;
    if constexpr (EX) {
        static_assert(Q == 2, "the exchange form is defined for D1Q2");
        sampler::node_exchange<W, NB, GB, NR>(av, cn, x, t, sl->realization, key, tb,
                                              sl->p_zero != 0);
    } else {
        sampler::node_update<Q, W, NB, GB, NR>(av, cn, x, t, sl->realization, key, tb,
                                               sl->p_zero != 0);
    }
    ovf |= sampler::or_all<Q, W>(cn);
    if constexpr (Q == 5) {
        // D2Q5 on the node index x + Lx y: -x, -y, rest, +y, +x
        uint32_t dxm, dym, dyp, dxp;
        sampler::d2q5_neighbours<kBlock>(x, x0, sl->width, L, dxm, dym, dyp, dxp);
        *global_elem<T>(out_row[0], dxm) = (T)cn[0];
        *global_elem<T>(out_row[1], dym) = (T)cn[1];
        *global_elem<T>(out_row[2], x) = (T)cn[2];
        *global_elem<T>(out_row[3], dyp) = (T)cn[3];
        *global_elem<T>(out_row[4], dxp) = (T)cn[4];
    } else {
        const uint32_t xm = (x == 0) ? L - 1 : x - 1;
        const uint32_t xp = (x + 1 == L) ? 0 : x + 1;
        *global_elem<T>(out_row[0], xm) = (T)cn[0];
        *global_elem<T>(out_row[Q - 1], xp) = (T)cn[Q - 1];
        if constexpr (Q == 3)
            *global_elem<T>(out_row[1], x) = (T)cn[1];
    }
}

// Philox blocks drawn up front per node.
template <int Q>
constexpr int kNB = (Q == 5) ? 3 : (Q == 3) ? 2 : 1;

// NR: Philox rounds of the draws (10, or 7 for draw specification v2); EX:
// the D1Q2 exchange form (specification v3).  The server launches one group
// of requests per (q, count type, specification).  RES: the launch has
// resident slots.  A group without them runs the kernel without that path:
// compiled with it (more scalar registers, 82 against 70 for D1Q2) the tile
// walk ran a quarter slower (D1Q2, saturated).
using ConstArgs = const __attribute__((address_space(4))) ServeArgs;

// Waves per SIMD the kernel must fit: the uint32 D1Q3 kernel is held to
// eight (at most 64 registers), so that two of its 1024-thread workgroups
// share a CU as the launch grid assumes; left free it takes 70 registers and
// one workgroup per CU.
template <int Q, typename T>
constexpr int kServeMinWaves = (Q == 3 && sizeof(T) == 4) ? 8 : 1;

template <int Q, typename T, int NR, bool EX, bool RES>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kServeMinWaves<Q, T>))) void serve_kernel(const ServeArgs *argp, uint32_t j)
{
    using W = typename Wide<T>::type;
    // The launch's arguments from device memory (scalar loads): the grid is
    // the same for every launch, so that a quantum's launches can be
    // captured once and replayed; workgroups beyond this launch's return.
    ConstArgs *a = (ConstArgs *)argp;
    if (blockIdx.x >= a->grid + (RES ? a->nres : 0u))
        return;
    __shared__ __align__(16) uint8_t s_lds[ServeLds<Q>::kBytes];
    uint32_t *s_tab = reinterpret_cast<uint32_t *>(s_lds);
    uint8_t *s_guide = s_lds + ServeLds<Q>::kTabBytes;

    const uint32_t *tab_p = s_tab, *tab_half = s_tab + kDevTableEntries;
    const uint32_t *tab_rest = s_tab + 2 * kDevTableEntries;
    const sampler::Tabs tb = sampler::make_tabs(tab_p, s_guide, kG);
    sampler::stage_row_offsets(tab_p, tab_half, tab_rest);
    // The shared half table and the first slot's tables are staged together,
    // before one barrier.
    stage_half(a->shared, s_tab, s_guide);
    constexpr W kMax = (W)(T)~(T)0;
    W ovf = 0;

    if (RES && blockIdx.x >= a->grid) {
        // A resident slot: a small request advanced by this workgroup alone,
        // its steps of this launch back to back, a workgroup barrier after
        // each (it makes the step's stores visible to every wave, which read
        // them in the next step).
        const uint32_t slot = a->res_first + (blockIdx.x - a->grid);
        ConstSlot *sl = const_space(a->slots) + slot;
        const uint32_t first = j * sl->per_launch;
        if (first >= sl->steps)
            return;  // uniform: this slot's advance is complete
        const uint32_t last = min(first + sl->per_launch, sl->steps);
        const uint32_t L = sl->length;
        stage_slot<Q>(a->arena, sl->table_off, s_tab, s_guide);
        __syncthreads();  // every table is visible to every wave
        for (uint32_t js = first; js < last; ++js) {
            for (uint32_t x0 = 0; x0 < L; x0 += kBlock) {
                const uint32_t x = x0 + threadIdx.x;
                if (x >= L)
                    continue;
                W av[Q];
                serve_load<Q, T>(sl, js, x, av);
                PhiloxSchedule key;
#pragma unroll
                for (int i = 0; i < 10; ++i) {
                    key.ka[i] = sl->ka[i];
                    key.kb[i] = sl->kb[i];
                }
                serve_update<Q, T, NR, EX, kNB<Q>>(sl, js, x0, x, av, key, tb, ovf);
            }
            if (js + 1 < last)
                __syncthreads();
        }
        if (ovf > kMax)
            atomicOr(a->slot_err + slot, 1u);
        return;
    }

    // The host splits the tile list into contiguous ranges of equal
    // estimated work (the work per node grows with a slot's collision
    // fraction; the estimate is corrected from the measured times below), so
    // a launch does not wait on the workgroups of its most expensive
    // requests.
    const uint32_t lo = a->wg_tiles[blockIdx.x];
    const uint32_t hi = a->wg_tiles[blockIdx.x + 1];
    if (lo >= hi)
        return;
    const uint64_t t_begin = clock64();
    // The first tile's slot (from its own list, so that its read does not
    // wait for lo) gives the tables staged with the half table.
    // Only the slot index is carried from tile to tile: the descriptor is a
    // scalar-cache read with no dependence on a per-tile lookup.  (Carrying
    // the descriptor itself measured slower: the compiler keeps it in vector
    // registers.)  The descriptor holds the rows' addresses and the round
    // keys, so a tile reads them instead of forming them.
    uint32_t slot = __builtin_amdgcn_readfirstlane(a->wg_slot[blockIdx.x]);  // uniform
    stage_slot<Q>(a->arena, const_space(a->slots)[slot].table_off, s_tab, s_guide);
    uint32_t staged = slot;
    // D1Q3 carries the current slot's end in a scalar register, so that a
    // tile's first scalar read is not a wait of its own; D1Q2 reads it per
    // tile (carried, its walk measured a quarter slower).
    uint32_t s_end = const_space(a->slots)[slot].tile_end;
    __syncthreads();  // every table is visible to every wave
    for (uint32_t tile = lo; tile < hi; ++tile) {
        if (Q != 3)
            s_end = const_space(a->slots)[slot].tile_end;
        if (tile >= s_end) {
            // leaving a slot: its overflow is reported in its own error word
            if (ovf > kMax)
                atomicOr(a->slot_err + slot, 1u);
            ovf = 0;
            do
                ++slot;
            while (tile >= const_space(a->slots)[slot].tile_end);
            s_end = const_space(a->slots)[slot].tile_end;
        }
        ConstSlot *sl = const_space(a->slots) + slot;
        if (j >= sl->steps)
            continue;
        if (slot != staged) {
            // Barriers only where the walk enters a new slot: before the
            // restage (readers of the previous slot's tables are done) and
            // after it (the new tables are visible).
            __syncthreads();
            stage_slot<Q>(a->arena, sl->table_off, s_tab, s_guide);
            staged = slot;
            __syncthreads();
        }
        const uint32_t x0 = (tile - sl->tile_begin) * (uint32_t)kBlock;  // uniform
        const uint32_t x = x0 + threadIdx.x;
        if (x >= sl->length)
            continue;
        W av[Q];
        serve_load<Q, T>(sl, j, x, av);
        PhiloxSchedule key;
#pragma unroll
        for (int i = 0; i < 10; ++i) {
            key.ka[i] = sl->ka[i];
            key.kb[i] = sl->kb[i];
        }
        serve_update<Q, T, NR, EX, kNB<Q>>(sl, j, x0, x, av, key, tb, ovf);
    }
    if (ovf > kMax)
        atomicOr(a->slot_err + slot, 1u);
    // The first launch of a quantum (all of its slots take that step) times
    // each workgroup's range, from its start to its last wave's end; the host
    // corrects the slots' estimated cost per tile from these times.
    if (j == 0) {
        __syncthreads();
        if (threadIdx.x == 0)
            a->wg_time[blockIdx.x] = clock64() - t_begin;
    }
}

struct Launch {
    bool res;
    const ServeArgs *argp;
    uint32_t j;
};

template <int Q, typename T, int NR, bool EX>
hipError_t launch_qt(const Launch &l, hipStream_t stream)
{
    const dim3 grid(serve_launch_grid());
    if (l.res)
        hipLaunchKernelGGL((serve_kernel<Q, T, NR, EX, true>), grid, dim3(kBlock), 0, stream,
                           l.argp, l.j);
    else
        hipLaunchKernelGGL((serve_kernel<Q, T, NR, EX, false>), grid, dim3(kBlock), 0, stream,
                           l.argp, l.j);
    return hipGetLastError();
}

template <int NR, bool EX>
hipError_t launch_spec(int q, int count_bytes, const Launch &l, hipStream_t stream)
{
    if (q == 2 && count_bytes == 2)
        return launch_qt<2, uint16_t, NR, EX>(l, stream);
    if (q == 2 && count_bytes == 4)
        return launch_qt<2, uint32_t, NR, EX>(l, stream);
    if constexpr (!EX) {
        if (q == 3 && count_bytes == 2)
            return launch_qt<3, uint16_t, NR, EX>(l, stream);
        if (q == 3 && count_bytes == 4)
            return launch_qt<3, uint32_t, NR, EX>(l, stream);
        if (q == 5 && count_bytes == 2)
            return launch_qt<5, uint16_t, NR, EX>(l, stream);
        if (q == 5 && count_bytes == 4)
            return launch_qt<5, uint32_t, NR, EX>(l, stream);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_rounds(int q, int count_bytes, int rounds, bool exchange, const Launch &l,
                         hipStream_t stream)
{
    if (rounds == 10)
        return exchange ? launch_spec<10, true>(q, count_bytes, l, stream)
                        : launch_spec<10, false>(q, count_bytes, l, stream);
    if (rounds == 7)
        return exchange ? launch_spec<7, true>(q, count_bytes, l, stream)
                        : launch_spec<7, false>(q, count_bytes, l, stream);
    return hipErrorInvalidValue;
}

}  // namespace

uint32_t serve_grid(uint32_t ntiles, uint32_t reserved)
{
    // two 1024-thread workgroups per CU, less the launch's resident slots
    const uint32_t slots = (uint32_t)device_cu_count() * 2;
    const uint32_t floor = slots / 2;
    const uint32_t grid = reserved + floor < slots ? slots - reserved : floor;
    return grid < ntiles ? grid : ntiles;
}

uint32_t serve_launch_grid()
{
    return (uint32_t)device_cu_count() * 2;
}

hipError_t launch_serve(int q, int count_bytes, int rounds, bool exchange, bool res,
                        const ServeArgs *argp, uint32_t j, hipStream_t stream)
{
    return launch_rounds(q, count_bytes, rounds, exchange, Launch{res, argp, j}, stream);
}

}  // namespace ilg
