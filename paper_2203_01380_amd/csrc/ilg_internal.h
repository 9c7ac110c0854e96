// Internal declarations shared by the runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>

#include "ilg.h"

namespace ilg {

// Binomial draws work on chunks of at most 64 trials; a fixed-point CDF table
// holds rows m = 1..64 with m entries each, row m at offset (m-1)m/2.
constexpr int kChunk = 64;
constexpr int kTableEntries = kChunk * (kChunk + 1) / 2;  // 2080
// Device layout of a table: every row is followed by kRowPad all-ones
// sentinels, so row m starts at (m-1)(m+4)/2 and a two-entry probe at any
// count 0..m stays inside the row and its padding.
constexpr int kRowPad = 2;
constexpr int kDevTableEntries = kTableEntries + kRowPad * kChunk;  // 2208
__host__ __device__ constexpr uint32_t dev_row_offset(uint32_t m)
{
    return ((m - 1u) * (m + 4u)) >> 1;
}
// Guide tables for the inverse-CDF search: for row m and bucket b (the top
// kGuideBits bits of the draw), the number of row entries <= b << (32 - bits).
// Kernels may stage a coarser view (every 2^k-th bucket) in LDS.
constexpr int kGuideBits = 8;
constexpr int kGuideBuckets = 1 << kGuideBits;
constexpr int kGuideEntries = kChunk * kGuideBuckets;  // bytes per table
// A "table set" holds the removal table (P), the half table (P = 2^31) and the
// rest table (P = (1-theta) 2^32) with their guides, contiguous on the device.
constexpr int kTablesPerSet = 3;
constexpr size_t kTableSetBytes =
    kTablesPerSet * (kDevTableEntries * sizeof(uint32_t) + kGuideEntries);
enum TableId : int { kTabP = 0, kTabHalf = 1, kTabRest = 2 };

__host__ __device__ inline const uint32_t *table_ptr(const void *set, int id)
{
    return reinterpret_cast<const uint32_t *>(set) + id * kDevTableEntries;
}
__host__ __device__ inline const uint8_t *guide_ptr(const void *set, int id)
{
    return reinterpret_cast<const uint8_t *>(set) +
           kTablesPerSet * kDevTableEntries * sizeof(uint32_t) + id * kGuideEntries;
}

// Host: exact fixed-point tables (multiword integer arithmetic) and guides.
void build_binomial_table(uint64_t p, uint32_t *out);
void build_guide(const uint32_t *table, uint8_t *guide);
// Packed table (kTableEntries) -> device layout (kDevTableEntries).
void pad_table(const uint32_t *packed, uint32_t *dev);
// Fill a host table set (device layout) for (p, p_rest); p = 0 leaves the P
// table zeroed (the kernels never read it then).
void build_table_set(uint64_t p, uint64_t p_rest, void *host_set);

struct Fixed {
    int flip;
    int rounds;    // Philox rounds of the step draws: 10 (v1) or 7 (v2)
    int exchange;  // D1Q2 exchange form (v3): p is the crossing probability
    uint64_t p, p_half, p_rest;
    double omega_star;
};

// Arguments of one lattice step (one launch).
struct StepArgs {
    const void *in;        // [q][pitch] counts at step t
    void *out;             // [q][pitch] counts at step t+1
    uint64_t pitch;
    uint32_t length;       // nodes (L, or Lx Ly for D2Q5)
    uint32_t width;        // row length Lx (= length in 1D)
    uint32_t height;       // rows Ly (1 in 1D)
    uint32_t t;            // absolute step index being taken
    uint32_t realization;
    uint32_t key0, key1;   // Philox key
    uint32_t flip;
    uint32_t p_zero;       // collision fraction is exactly 0
    uint32_t rounds;       // Philox rounds of the draws: 10 or 7
    uint32_t exchange;     // D1Q2 exchange form: two crossing binomials
    const void *tables;    // device table set
    uint32_t *err;         // sticky error word (bit 0: overflow)
};

// Poisson sine initial state (init v1): counts into out, [q][pitch].
struct InitArgs {
    void *out;
    uint64_t pitch;
    uint32_t length, q;                // nodes, velocities
    uint32_t width;                    // row length: the profile is along x = node mod width
    uint32_t realization, key0, key1;  // Philox key = init seed
    double w[5];                       // velocity weights
    double nave, amp;
    uint32_t *err;                     // bit 0 set if a count exceeds the type
};
hipError_t launch_init(int count_bytes, const InitArgs &a, hipStream_t stream);

// Launch one step of a q-velocity, count_bytes lattice on stream.
hipError_t launch_step(int q, int count_bytes, const StepArgs &a, hipStream_t stream);

// Diagnostics of one state.
struct DiagArgs {
    const void *state;
    uint64_t pitch;
    uint32_t length;       // nodes
    uint32_t width;        // row length: sine and S(k) along x = node mod width
    uint32_t q;
    uint32_t count_bytes;
    uint32_t nk;
    int64_t *rho, *j, *e;  // device per-node moments or null
    void *partials;        // device scratch, diag_partials_bytes(nk) per block
    void *result;          // device DiagResult
};

struct DiagResult {
    uint64_t mass;
    uint64_t hash;
    double sin_num;        // sum_x sin(2 pi x/L) N(x)
    double sin_den;        // sum_x sin^2(2 pi x/L)
    double mass_f;
    double sk_re[64];
    double sk_im[64];
};

constexpr int kDiagBlocks = 512;
size_t diag_partials_bytes();
hipError_t launch_diag(const DiagArgs &a, hipStream_t stream);

// Compute units of the current device (cached after the first call).
int device_cu_count();
// Validation and fixed-point parameters of a configuration (runtime.cpp).
int check_config(const struct ilg_config *cfg, Fixed *fx);
// Message returned by ilg_last_error() on this thread.
void set_last_error(const std::string &msg);

// ---------------------------------------------------------------- batched
// One ensemble member: its buffer pair in the arena and its draw keys.
struct BatchMeta {
    uint64_t off;          // element offset of buffer 0; buffer 1 follows at q*pitch
    uint32_t length, pitch;
    uint32_t t;            // absolute index of the next step
    uint32_t realization, key0, key1;
    uint32_t flip, p_zero;
    uint32_t cur;          // which buffer holds the current state
    uint32_t width;        // nodes per row: Lx for D2Q5 (length = Lx Ly), L in 1D
};

constexpr int kBatchMaxK = 16;
constexpr int kBatchGuideBits = 6;

struct BatchArgs {
    void *arena;
    BatchMeta *meta;
    const uint32_t *tabs_p;       // [nreal][kDevTableEntries] removal tables
    const uint32_t *tabs_shared;  // [2][kDevTableEntries]: P = 2^31, P = P_rest (q = 3, 5)
    const uint32_t *order;        // members, longest first
    uint32_t *queue;              // next index into order
    uint32_t nreal;
    uint32_t nsteps;
    uint32_t sk_every, nk, amp_every, max_amp;
    double *sk_sum;               // [nreal][nk]
    unsigned long long *sk_cnt;   // [nreal]
    double *amp;                  // [nreal][max_amp]
    uint32_t *amp_cnt;            // [nreal]
    uint32_t *err;
    uint32_t rounds;              // Philox rounds of the draws, batch-wide: 10 or 7
    uint32_t exchange;            // D1Q2 exchange form, batch-wide
};

int batch_shape_count();
// Launch geometry of a shape: threads per workgroup and workgroups per CU.
void batch_shape(int shape, int q, int *block, int *wg_per_cu);
hipError_t launch_batch_reset(uint32_t *queue, hipStream_t stream);
hipError_t launch_batch(int q, int count_bytes, int shape, const BatchArgs &a, hipStream_t stream);
// The seven-round and exchange-form instantiations (their own translation units).
hipError_t launch_batch_p7(int q, int count_bytes, int shape, const BatchArgs &a,
                           hipStream_t stream);
hipError_t launch_batch_ex(int q, int count_bytes, int shape, const BatchArgs &a,
                           hipStream_t stream);

// ---------------------------------------------------------------- serving
// One active request of the server in one launch group's quantum: where its
// state and tables are and its draw keys, in the form the kernel uses them
// directly (row addresses and round keys formed on the host, so that a tile
// of the request costs only a few scalar loads).
struct ServeSlot {
    // Row addresses for the quantum's step j, by j & 1 (the buffers swap every
    // step): rows[j & 1][i], i < q, the rows read, with the flip applied
    // (the row of index i holds n_{q-1-i} when the flip is on, and for D2Q5
    // also the y pair swapped); rows[j & 1][5 + i] the rows written.
    uint64_t rows[2][10];
    uint32_t ka[10], kb[10];   // Philox round keys k0 + i W0, k1 + i W1
    uint64_t table_off;        // byte offset of the slot's table set
    uint32_t length;           // nodes (Lx Ly for D2Q5)
    uint32_t width;            // D2Q5: nodes per lattice row (Lx); 1D: L
    uint32_t t0;               // absolute index of the quantum's first step
    uint32_t steps;            // steps in this quantum
    uint32_t realization;
    uint32_t p_zero;
    uint32_t tile_begin, tile_end;  // the slot's tiles in the launch's tile list
    // Resident slot (a small request advanced by its own workgroup): steps
    // per launch; launch j takes steps [j per_launch, (j + 1) per_launch)
    // of the `steps`.  0 for a slot of the tile walk.
    uint32_t per_launch;
};
constexpr int kServeGuideBits = 8;
constexpr int kServeTile = 1024;  // nodes per tile (one workgroup pass)
// Slot table set: removal table, rest table (q = 3, 5), then their guides.
constexpr size_t kServeTableBytes = kDevTableEntries * sizeof(uint32_t);
constexpr size_t kServeGuideBytes = (size_t)kChunk << kServeGuideBits;
inline size_t serve_table_set_bytes(int q)
{
    return (q == 2 ? 1 : 2) * (kServeTableBytes + kServeGuideBytes);
}

struct ServeArgs {
    void *arena;
    const ServeSlot *slots;      // in tile order: slot s owns tiles [tile_begin, tile_end)
    const uint32_t *tile_slot;   // slot of each tile
    const uint32_t *wg_tiles;    // workgroup w walks tiles [wg_tiles[w], wg_tiles[w + 1])
    const uint32_t *wg_slot;     // slot of tile wg_tiles[w]
    uint32_t ntiles;
    uint32_t grid;               // workgroups of the launch
    uint32_t j;             // step index within the quantum
    const void *shared;     // half table then its guide
    uint32_t *slot_err;     // one sticky error word per slot (bit 0: overflow)
    // Workgroups grid .. grid + nres - 1 each advance one resident slot,
    // slots res_first .. res_first + nres - 1.
    uint32_t nres;
    uint32_t res_first;
    // Clock ticks of each tile-walk workgroup's range in the launch with
    // j = 0 (written by workgroups with a nonempty range only).
    uint64_t *wg_time;
};
// Most resident slots in one launch.
constexpr uint32_t kResidentMaxWg = 128;
// Workgroups of the tile walk of a serving launch over ntiles tiles: two per
// CU at most, less `reserved` for the launch's resident slots (at least one
// per CU).
uint32_t serve_grid(uint32_t ntiles, uint32_t reserved);

// One step launch of a group: the kernel reads its arguments from argp
// (device memory the host writes before the launches; its field j is
// ignored) and takes the step index j of the quantum; res: the arguments
// have resident slots.  Every launch has serve_launch_grid() workgroups
// (those beyond the arguments' grid + nres return at once), so a quantum's
// launches can be captured in a graph once and replayed.
uint32_t serve_launch_grid();
hipError_t launch_serve(int q, int count_bytes, int rounds, bool exchange, bool res,
                        const ServeArgs *argp, uint32_t j, hipStream_t stream);


}  // namespace ilg
