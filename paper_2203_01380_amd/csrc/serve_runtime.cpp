// Continuous-batching server behind ilg_server_* (include/ilg.h): the
// device executor of the scheduler (scheduler.h).  One device arena of the
// budget's size holds every active request's double-buffered state and its
// table set; each poll admits what fits, advances all active requests by a
// quantum with the multi-slot step kernel (one launch per step and per
// (q, count type, draw specification) group, groups on their own streams so
// their work overlaps), and copies finished states back to host memory.
// Small requests are resident slots of those launches: each has a workgroup
// of its own that advances it by as many steps per launch as fit in the time
// of the launch's tile walk.
// Every slot of a launch has its own error word, so a request whose counts
// overflow is retired alone (ILG_REQ_FAILED) and the others go on.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ilg.h"
#include "ilg_internal.h"
#include "philox.h"
#include "scheduler.h"

namespace {

using ilg::serve::Req;
using ilg::serve::ReqState;

int sfail(int code, const std::string &msg)
{
    ilg::set_last_error(msg);
    return code;
}

int shfail(hipError_t e, const char *what)
{
    return sfail(ILG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define SHIP(call)                                     \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess)                          \
            return shfail(e_, #call);                  \
    } while (0)

double steady_now()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

uint64_t pitch_of(uint64_t length)
{
    return (length + 63) / 64 * 64;
}

uint64_t align256(uint64_t x)
{
    return (x + 255) / 256 * 256;
}

// Per-request data kept by the executor.
struct Payload {
    ilg_config cfg;
    ilg::Fixed fx;
    std::vector<unsigned char> host;  // initial state, later the final state ([q][L])
    uint64_t t = 0;                   // absolute index of the next step
    uint32_t cur = 0;                 // buffer holding the current state
    // initial state drawn on the device at admission instead of copied in
    bool device_init = false;
    double nave = 0.0, amp = 0.0;
    uint64_t init_seed = 0;
    // Measured cost per tile relative to the model 1 + omega*, learned from
    // the tile walk's workgroup times (density and the sampler's chunking
    // make the true cost depart from the model).
    double cost = 1.0;
};

Payload *payload_of(Req &r)
{
    return static_cast<Payload *>(r.payload.get());
}

// Nodes of a request: L in 1D, Lx Ly for D2Q5 (node x + Lx y).
uint64_t nodes_of(const ilg_config &c)
{
    return c.length * (c.q == 5 ? (uint64_t)c.height : 1u);
}

uint64_t state_bytes(const ilg_config &c)
{
    return align256(2ull * c.q * pitch_of(nodes_of(c)) * c.count_bytes);
}

class DeviceExecutor : public ilg::serve::Executor {
public:
    void *arena = nullptr;
    void *shared = nullptr;  // half table + guide
    uint32_t *init_err = nullptr;  // error word of a device-drawn initial state
    // Launch groups: (q, count type, Philox rounds, exchange form); a group's
    // stream is created when the group first has work.
    static constexpr int kGroups = 24;
    hipStream_t streams[kGroups] = {};
    ilg::ServeSlot *d_slots[kGroups] = {};
    uint32_t *d_err[kGroups] = {};    // error word of each slot of the last launch
    uint32_t *d_tiles[kGroups] = {};  // as h_tiles
    uint64_t *d_time[kGroups] = {};   // clock of each workgroup's range (launch j = 0)
    size_t cap_slots[kGroups] = {}, cap_tiles[kGroups] = {};
    hipStream_t io = nullptr;  // copies in and out
    // Small requests (at most resident_nodes nodes, 0: none) are advanced
    // as resident slots, several steps per launch; quantum: the scheduler's.
    uint64_t resident_nodes = 0;
    uint32_t quantum = 1;
    // Each group's launch arguments in device memory, and for a full
    // quantum of launches a graph of them (with and without resident
    // slots), captured once on the stream `cap` and replayed every poll
    // (the kernels read the arguments at run time, and a graph launch costs
    // a fraction of the separate launches).
    ilg::ServeArgs *d_args[kGroups] = {};
    ilg::ServeArgs h_args[kGroups] = {};
    hipGraphExec_t quanta[kGroups][2] = {};
    hipStream_t cap = nullptr;

    static int group(uint32_t q, uint32_t cb, const ilg::Fixed &fx)
    {
        return (q == 5 ? 16 : q == 3 ? 8 : 0) + (cb == 4 ? 4 : 0) + (fx.rounds == 7 ? 2 : 0) +
               (fx.exchange ? 1 : 0);
    }

    uint64_t footprint(const Req &r) override
    {
        const Payload *p = static_cast<const Payload *>(r.payload.get());
        return state_bytes(p->cfg) + align256(ilg::serve_table_set_bytes((int)p->cfg.q));
    }

    int load(Req &r) override
    {
        Payload *p = payload_of(r);
        const ilg_config &c = p->cfg;
        const size_t cb = c.count_bytes, n = nodes_of(c), pitch = pitch_of(n);
        unsigned char *base = static_cast<unsigned char *>(arena) + r.mem_off;
        if (p->device_init) {
            // Poisson sine state drawn in place; a count above the type sets
            // init_err, read back below: the request then fails at admission.
            const double theta = c.theta == 0.0 ? 1.0 / 3.0 : c.theta;
            ilg::InitArgs a;
            a.out = base;
            a.pitch = pitch;
            a.length = (uint32_t)n;
            a.width = (uint32_t)c.length;
            a.q = c.q;
            a.realization = c.realization;
            a.key0 = (uint32_t)(p->init_seed & 0xFFFFFFFFu);
            a.key1 = (uint32_t)(p->init_seed >> 32);
            for (int i = 0; i < 5; ++i)
                a.w[i] = 0.0;
            if (c.q == 2) {
                a.w[0] = a.w[1] = 0.5;
            } else if (c.q == 3) {
                a.w[0] = a.w[2] = theta * 0.5;
                a.w[1] = 1.0 - theta;
            } else {
                a.w[0] = a.w[1] = a.w[3] = a.w[4] = theta * 0.5;
                a.w[2] = 1.0 - 2.0 * theta;
            }
            a.nave = p->nave;
            a.amp = p->amp;
            a.err = init_err;
            SHIP(hipMemsetAsync(init_err, 0, sizeof(uint32_t), io));
            hipError_t e = ilg::launch_init((int)cb, a, io);
            if (e != hipSuccess)
                return shfail(e, "init launch");
        } else {
            SHIP(hipMemcpy2DAsync(base, pitch * cb, p->host.data(), n * cb, n * cb, c.q,
                                  hipMemcpyHostToDevice, io));
        }
        // table set: removal table (+ rest table for q = 3, 5) then their guides
        const int nt = c.q == 2 ? 1 : 2;
        std::vector<unsigned char> set(ilg::serve_table_set_bytes((int)c.q), 0);
        const uint64_t ps[2] = {p->fx.p, p->fx.p_rest};
        std::vector<uint32_t> packed(ilg::kTableEntries);
        for (int t = 0; t < nt; ++t) {
            uint32_t *tab = reinterpret_cast<uint32_t *>(set.data() + t * ilg::kServeTableBytes);
            if (ps[t] == 0)
                continue;
            ilg::build_binomial_table(ps[t], packed.data());
            guide(packed.data(), set.data() + nt * ilg::kServeTableBytes + t * ilg::kServeGuideBytes);
            ilg::pad_table(packed.data(), tab);
        }
        SHIP(hipMemcpyAsync(base + state_bytes(c), set.data(), set.size(), hipMemcpyHostToDevice,
                            io));
        uint32_t ierr = 0;
        if (p->device_init)
            SHIP(hipMemcpyAsync(&ierr, init_err, sizeof(ierr), hipMemcpyDeviceToHost, io));
        SHIP(hipStreamSynchronize(io));
        if (ierr & 1u)
            r.failed = true;  // a drawn count does not fit the count type
        p->t = c.t0;
        p->cur = 0;
        return ILG_OK;
    }

    // Guide of a removal/rest table: #{j < m : T[m][j] <= b << (32 - bits)}
    // per row m and bucket b, by binary search on the nondecreasing row.
    static void guide(const uint32_t *tab, unsigned char *g)
    {
        constexpr int kRow = 1 << ilg::kServeGuideBits;
        for (int m = 1; m <= ilg::kChunk; ++m) {
            const uint32_t *row = tab + (m - 1) * m / 2;
            for (int b = 0; b < kRow; ++b) {
                const uint64_t edge = uint64_t(b) << (32 - ilg::kServeGuideBits);
                int lo = 0, hi = m;
                while (lo < hi) {
                    const int mid = (lo + hi) / 2;
                    if (row[mid] <= edge)
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                g[(m - 1) * kRow + b] = (unsigned char)lo;
            }
        }
    }

    // Host copies of the last launch's slot and tile lists (kept alive until
    // the copies from them have completed).
    std::vector<ilg::ServeSlot> h_slots[kGroups];
    // slot of each tile, then the workgroups' tile ranges, then the slot of
    // each workgroup's first tile
    std::vector<uint32_t> h_tiles[kGroups];
    std::vector<double> h_weight[kGroups];     // estimated work of each tile
    std::vector<Payload *> h_walk[kGroups];    // request of each tile-walk slot
    std::vector<uint64_t> h_time;
    std::vector<double> h_corr;
    std::vector<uint32_t> h_err[kGroups];
    std::vector<Req *> launched;
    std::vector<uint32_t> launched_steps;  // planned by the scheduler
    std::vector<uint32_t> taken_steps;     // what the launches take (resident: may be fewer)
    std::vector<std::pair<int, uint32_t>> launched_slot;  // (group, slot) of launched[i]

    // Descriptor of request r for an advance of `steps` steps from its
    // current state.
    ilg::ServeSlot make_slot(const Req &r, const Payload *p, uint32_t steps) const
    {
        const ilg_config &c = p->cfg;
        ilg::ServeSlot s;
        std::memset(&s, 0, sizeof(s));
        // rows of both buffers: buffer b starts at the request's block plus
        // b q pitch counts; step j reads buffer cur ^ (j & 1)
        const uint64_t pitch = pitch_of(nodes_of(c)), cb = c.count_bytes;
        const uint64_t base = reinterpret_cast<uint64_t>(arena) + r.mem_off;
        for (uint32_t par = 0; par < 2; ++par) {
            const uint64_t in = base + (uint64_t)(p->cur ^ par) * c.q * pitch * cb;
            const uint64_t out = base + (uint64_t)(p->cur ^ par ^ 1u) * c.q * pitch * cb;
            for (uint32_t i = 0; i < c.q; ++i) {
                // a_i = n_{q-1-i} under the flip (Eq. flip)
                const uint32_t src = p->fx.flip ? c.q - 1 - i : i;
                s.rows[par][i] = in + (uint64_t)src * pitch * cb;
                s.rows[par][5 + i] = out + (uint64_t)i * pitch * cb;
            }
        }
        const uint32_t k0 = (uint32_t)(c.seed & 0xFFFFFFFFu), k1 = (uint32_t)(c.seed >> 32);
        for (uint32_t k = 0; k < 10; ++k) {
            s.ka[k] = k0 + k * ilg::kPhiloxW0;
            s.kb[k] = k1 + k * ilg::kPhiloxW1;
        }
        s.table_off = r.mem_off + state_bytes(c);
        s.length = (uint32_t)nodes_of(c);
        s.width = (uint32_t)c.length;
        s.t0 = (uint32_t)p->t;
        s.steps = steps;
        s.realization = c.realization;
        s.p_zero = p->fx.p == 0 ? 1u : 0u;
        return s;
    }

    static void spec_of(int g, int *q, int *cb, int *rounds, bool *exchange)
    {
        *q = g >= 16 ? 5 : (g & 8) ? 3 : 2;
        *cb = (g & 4) ? 4 : 2;
        *rounds = (g & 2) ? 7 : 10;
        *exchange = (g & 1) != 0;
    }

    // Cost model of a launch, in units of one full tile of the tile walk at
    // omega* = 0 (about 2 us): a tile costs (1 + omega*) times the request's
    // measured factor (more collided particles, larger redistribution
    // binomials; a partial tile about as much as a full one, its waves being
    // latency bound; see calibrate()), and a workgroup
    // entering a slot pays about half a tile to stage the slot's tables.  A
    // resident step of a request of n tiles costs n (1 + omega*) plus half a
    // tile (the step's barrier and latency-bound waves).  A launch also
    // spends about 4 units beyond its busiest workgroup's tiles (the gap
    // between launches, the shared table's staging, the tail), which a
    // resident workgroup can use.
    static constexpr double kStage = 0.5, kResidentStep = 0.5, kLaunch = 4.0;

    int launch(const std::vector<Req *> &active, const std::vector<uint32_t> &steps) override
    {
        std::vector<ilg::ServeSlot> *slots = h_slots;
        std::vector<uint32_t> *tiles = h_tiles;
        struct Res {
            size_t i;
            ilg::ServeSlot s;
            double w;  // cost of one step
        };
        std::vector<Res> res[kGroups];
        for (int g = 0; g < kGroups; ++g) {
            slots[g].clear();
            tiles[g].clear();
            h_weight[g].clear();
            h_walk[g].clear();
        }
        launched = active;
        launched_steps = steps;
        taken_steps = steps;
        launched_slot.assign(active.size(), {0, 0});
        uint32_t maxsteps[kGroups] = {};
        // Resident slots of a group: at most half the launch grid, so that
        // the tile walk (at least the other half) and they fit the grid.
        const uint32_t max_res = std::min<uint32_t>(ilg::kResidentMaxWg,
                                                    ilg::serve_launch_grid() / 2);
        for (size_t i = 0; i < active.size(); ++i) {
            Req &r = *active[i];
            Payload *p = payload_of(r);
            const ilg_config &c = p->cfg;
            const int g = group(c.q, c.count_bytes, p->fx);
            const uint32_t nt = (uint32_t)((nodes_of(c) + ilg::kServeTile - 1) / ilg::kServeTile);
            const double w = (1.0 + p->fx.omega_star) * p->cost;
            if (resident_nodes != 0 && nodes_of(c) <= resident_nodes &&
                res[g].size() < max_res) {
                res[g].push_back({i, make_slot(r, p, steps[i]), nt * w + kResidentStep});
                continue;
            }
            // the tile walk advances a request by at most the quantum (a
            // small request beyond the launch's resident slots included)
            taken_steps[i] = std::min(steps[i], quantum);
            const uint32_t idx = (uint32_t)slots[g].size();
            launched_slot[i] = {g, idx};
            slots[g].push_back(make_slot(r, p, taken_steps[i]));
            h_walk[g].push_back(p);
            slots[g].back().tile_begin = (uint32_t)tiles[g].size();
            slots[g].back().tile_end = (uint32_t)tiles[g].size() + nt;
            tiles[g].insert(tiles[g].end(), nt, idx);
            for (uint32_t k = 0; k < nt; ++k)
                h_weight[g].push_back(w + (k == 0 ? kStage : 0.0));
            maxsteps[g] = std::max(maxsteps[g], taken_steps[i]);
        }
        // Tile walk of each group: contiguous tile ranges of equal estimated
        // work, one per workgroup, beside the group's resident workgroups.
        uint32_t grid[kGroups] = {};
        double per_wg[kGroups] = {}, longest = 0.0;
        for (int g = 0; g < kGroups; ++g) {
            const uint32_t ntiles = (uint32_t)tiles[g].size();
            if (ntiles == 0)
                continue;
            grid[g] = ilg::serve_grid(ntiles, (uint32_t)res[g].size());
            double total = 0.0;
            for (double w : h_weight[g])
                total += w;
            per_wg[g] = total / grid[g];
            longest = std::max(longest, per_wg[g] * maxsteps[g]);
            tiles[g].push_back(0);
            double acc = 0.0;
            uint32_t t = 0;
            for (uint32_t b = 1; b < grid[g]; ++b) {
                const double target = total * b / grid[g];
                while (t < ntiles && acc + 0.5 * h_weight[g][t] < target)
                    acc += h_weight[g][t++];
                tiles[g].push_back(t);
            }
            tiles[g].push_back(ntiles);
            // then the slot of each workgroup's first tile
            for (uint32_t b = 0; b < grid[g]; ++b) {
                const uint32_t first = tiles[g][ntiles + b];
                tiles[g].push_back(first < ntiles ? tiles[g][first] : 0u);
            }
        }
        // Resident slots: as many steps per launch as fit in the time of the
        // group's tile walk (at least one); a group without a tile walk takes
        // one launch about as long as the longest quantum of the other
        // groups (at least the quantum's steps), or all the planned steps
        // when no group has a tile walk.
        for (int g = 0; g < kGroups; ++g) {
            const uint32_t walk_steps = maxsteps[g];  // launches of the group's tile walk
            for (Res &x : res[g]) {
                const uint32_t planned = x.s.steps;
                uint64_t per;
                uint32_t take;
                if (walk_steps > 0) {
                    per = (uint64_t)std::max(1.0,
                                             std::floor((per_wg[g] + kLaunch - kStage) / x.w));
                    take = (uint32_t)std::min<uint64_t>(planned, per * walk_steps);
                } else if (longest > 0.0) {
                    // one launch, at least the quantum (what the tile walk
                    // would have given it)
                    per = std::max<uint64_t>((uint64_t)std::floor(longest / x.w), quantum);
                    take = (uint32_t)std::min<uint64_t>(planned, per);
                } else {
                    per = planned;
                    take = planned;
                }
                x.s.steps = take;
                x.s.per_launch = (uint32_t)std::min<uint64_t>(per, take);
                taken_steps[x.i] = take;
                const uint32_t launches = (take + x.s.per_launch - 1) / x.s.per_launch;
                maxsteps[g] = std::max(maxsteps[g], launches);
            }
        }
        for (int g = 0; g < kGroups; ++g) {
            if (slots[g].empty() && res[g].empty())
                continue;
            if (!streams[g])
                SHIP(hipStreamCreateWithFlags(&streams[g], hipStreamNonBlocking));
            const uint32_t ntiles = (uint32_t)h_weight[g].size();
            const uint32_t res_first = (uint32_t)slots[g].size();
            for (const Res &x : res[g]) {
                launched_slot[x.i] = {g, (uint32_t)slots[g].size()};
                slots[g].push_back(x.s);
            }
            if (tiles[g].empty())
                tiles[g].push_back(0);  // no tile walk: nothing reads the list
            int rc = ensure(g, slots[g].size(), tiles[g].size());
            if (rc != ILG_OK)
                return rc;
            SHIP(hipMemcpyAsync(d_slots[g], slots[g].data(), slots[g].size() * sizeof(ilg::ServeSlot),
                                hipMemcpyHostToDevice, streams[g]));
            SHIP(hipMemcpyAsync(d_tiles[g], tiles[g].data(), tiles[g].size() * sizeof(uint32_t),
                                hipMemcpyHostToDevice, streams[g]));
            SHIP(hipMemsetAsync(d_err[g], 0, slots[g].size() * sizeof(uint32_t), streams[g]));
            if (grid[g] + (uint32_t)res[g].size() > ilg::serve_launch_grid())
                return sfail(ILG_E_DEVICE, "serving launch needs more workgroups than its grid");
            ilg::ServeArgs &a = h_args[g];
            std::memset(&a, 0, sizeof(a));
            a.arena = arena;
            a.slots = d_slots[g];
            a.tile_slot = d_tiles[g];
            a.wg_tiles = d_tiles[g] + ntiles;
            a.wg_slot = d_tiles[g] + ntiles + grid[g] + 1;
            a.ntiles = ntiles;
            a.grid = grid[g];
            a.shared = shared;
            a.slot_err = d_err[g];
            a.nres = (uint32_t)res[g].size();
            a.res_first = res_first;
            a.wg_time = d_time[g];
            SHIP(hipMemcpyAsync(d_args[g], &a, sizeof(a), hipMemcpyHostToDevice, streams[g]));
            const bool with_res = a.nres != 0;
            if (maxsteps[g] == quantum) {
                rc = capture_quantum(g, with_res);
                if (rc != ILG_OK)
                    return rc;
                SHIP(hipGraphLaunch(quanta[g][with_res ? 1 : 0], streams[g]));
                continue;
            }
            int q, cb, rounds;
            bool exchange;
            spec_of(g, &q, &cb, &rounds, &exchange);
            for (uint32_t j = 0; j < maxsteps[g]; ++j) {
                hipError_t e = ilg::launch_serve(q, cb, rounds, exchange, with_res, d_args[g], j,
                                                 streams[g]);
                if (e != hipSuccess)
                    return shfail(e, "serve launch");
            }
        }
        return ILG_OK;
    }

    // The graph of a full quantum of group g's launches (j = 0 .. quantum - 1
    // on the arguments in d_args[g]), captured at its first use.
    int capture_quantum(int g, bool with_res)
    {
        hipGraphExec_t &exec = quanta[g][with_res ? 1 : 0];
        if (exec)
            return ILG_OK;
        if (!cap)
            SHIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        int q, cb, rounds;
        bool exchange;
        spec_of(g, &q, &cb, &rounds, &exchange);
        SHIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (uint32_t j = 0; j < quantum && e == hipSuccess; ++j)
            e = ilg::launch_serve(q, cb, rounds, exchange, with_res, d_args[g], j, cap);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cap, &graph);
        if (e == hipSuccess)
            e = e2;
        if (e == hipSuccess)
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph)
            (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            exec = nullptr;
            return shfail(e, "quantum graph");
        }
        return ILG_OK;
    }

    int wait(std::vector<uint32_t> *steps) override
    {
        int rc = ILG_OK;
        for (int g = 0; g < kGroups && rc == ILG_OK; ++g) {
            if (h_slots[g].empty())
                continue;
            hipError_t e = hipStreamSynchronize(streams[g]);
            h_err[g].assign(h_slots[g].size(), 0u);
            if (e == hipSuccess)
                e = hipMemcpy(h_err[g].data(), d_err[g], h_err[g].size() * sizeof(uint32_t),
                              hipMemcpyDeviceToHost);
            if (e == hipSuccess)
                e = calibrate(g);
            if (e != hipSuccess)
                rc = shfail(e, "serve quantum");
        }
        // Every launched request's step count and buffer parity advance with
        // the steps its launches took (a resident request's may be fewer
        // than planned), also when its own work overflowed (it is then
        // retired).
        for (size_t i = 0; i < launched.size(); ++i) {
            const uint32_t k = taken_steps[i];
            (*steps)[i] = k;
            Payload *p = payload_of(*launched[i]);
            p->t += k;
            p->cur ^= (k & 1u);
            if (rc == ILG_OK) {
                const auto gs = launched_slot[i];
                if (h_err[gs.first][gs.second] & 1u)
                    launched[i]->failed = true;
            }
        }
        launched.clear();
        launched_steps.clear();
        taken_steps.clear();
        launched_slot.clear();
        return rc;
    }

    // Corrects the cost factor of each request of group g's last tile walk
    // from the times its workgroups took (at most a third up or a quarter
    // down per quantum, so that one noisy time cannot swing the split).
    hipError_t calibrate(int g)
    {
        const uint32_t ntiles = h_args[g].ntiles, grid = h_args[g].grid;
        if (ntiles == 0 || grid == 0 || h_walk[g].empty())
            return hipSuccess;
        h_time.resize(grid);
        hipError_t e = hipMemcpy(h_time.data(), d_time[g], grid * sizeof(uint64_t),
                                 hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            return e;
        h_corr.resize(h_walk[g].size());
        ilg::serve::tile_cost_correction(h_tiles[g].data() + ntiles, grid, h_weight[g].data(),
                                         h_tiles[g].data(), h_time.data(),
                                         (uint32_t)h_walk[g].size(), 0.75, 4.0 / 3.0,
                                         h_corr.data());
        for (size_t s = 0; s < h_walk[g].size(); ++s)
            h_walk[g][s]->cost = std::min(4.0, std::max(0.25, h_walk[g][s]->cost * h_corr[s]));
        return hipSuccess;
    }

    int unload(Req &r) override
    {
        Payload *p = payload_of(r);
        const ilg_config &c = p->cfg;
        const size_t cb = c.count_bytes, n = nodes_of(c), pitch = pitch_of(n);
        const unsigned char *src = static_cast<const unsigned char *>(arena) + r.mem_off +
                                   (size_t)p->cur * c.q * pitch * cb;
        // a request drawn on the device has no host copy of its state yet
        p->host.resize((size_t)c.q * n * cb);
        SHIP(hipMemcpy2DAsync(p->host.data(), n * cb, src, pitch * cb, n * cb, c.q,
                              hipMemcpyDeviceToHost, io));
        SHIP(hipStreamSynchronize(io));
        return ILG_OK;
    }

    int ensure(int g, size_t nslots, size_t ntiles)
    {
        if (!d_args[g])
            SHIP(hipMalloc((void **)&d_args[g], sizeof(ilg::ServeArgs)));
        if (!d_time[g])
            SHIP(hipMalloc((void **)&d_time[g], ilg::serve_launch_grid() * sizeof(uint64_t)));
        if (nslots > cap_slots[g]) {
            (void)hipFree(d_slots[g]);
            (void)hipFree(d_err[g]);
            d_slots[g] = nullptr;
            d_err[g] = nullptr;
            cap_slots[g] = std::max(nslots, 2 * cap_slots[g]);
            SHIP(hipMalloc((void **)&d_slots[g], cap_slots[g] * sizeof(ilg::ServeSlot)));
            SHIP(hipMalloc((void **)&d_err[g], cap_slots[g] * sizeof(uint32_t)));
        }
        if (ntiles > cap_tiles[g]) {
            (void)hipFree(d_tiles[g]);
            cap_tiles[g] = std::max(ntiles, 2 * cap_tiles[g]);
            SHIP(hipMalloc((void **)&d_tiles[g], cap_tiles[g] * sizeof(uint32_t)));
        }
        return ILG_OK;
    }

    ~DeviceExecutor() override
    {
        for (int g = 0; g < kGroups; ++g) {
            (void)hipFree(d_slots[g]);
            (void)hipFree(d_err[g]);
            (void)hipFree(d_tiles[g]);
            (void)hipFree(d_time[g]);
            (void)hipFree(d_args[g]);
            for (int k = 0; k < 2; ++k)
                if (quanta[g][k])
                    (void)hipGraphExecDestroy(quanta[g][k]);
            if (streams[g])
                (void)hipStreamDestroy(streams[g]);
        }
        if (io)
            (void)hipStreamDestroy(io);
        if (cap)
            (void)hipStreamDestroy(cap);
        (void)hipFree(arena);
        (void)hipFree(shared);
        (void)hipFree(init_err);
    }
};

}  // namespace

struct ilg_server {
    std::unique_ptr<ilg::serve::Scheduler> sched;
    DeviceExecutor ex;
};

extern "C" {

double ilg_server_clock(void)
{
    return steady_now();
}

int ilg_server_create(uint64_t budget_bytes, uint32_t quantum_steps, ilg_server **out)
{
    if (!out || budget_bytes < 4096 || quantum_steps == 0)
        return sfail(ILG_E_INVALID, "need an output, a budget of at least 4 KiB and a quantum > 0");
    *out = nullptr;
    (void)ilg::device_cu_count();
    ilg_server *s = new (std::nothrow) ilg_server;
    if (!s)
        return sfail(ILG_E_NOMEM, "host allocation failed");
    s->sched.reset(new ilg::serve::Scheduler(budget_bytes, quantum_steps));
    DeviceExecutor &ex = s->ex;
    hipError_t e = hipMalloc(&ex.arena, budget_bytes);
    if (e == hipSuccess)
        e = hipMalloc(&ex.shared, ilg::kServeTableBytes + ilg::kServeGuideBytes);
    if (e == hipSuccess)
        e = hipMalloc((void **)&ex.init_err, sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&ex.io, hipStreamNonBlocking);
    if (e == hipSuccess) {
        std::vector<unsigned char> sh(ilg::kServeTableBytes + ilg::kServeGuideBytes, 0);
        std::vector<uint32_t> packed(ilg::kTableEntries);
        ilg::build_binomial_table(uint64_t(1) << 31, packed.data());
        DeviceExecutor::guide(packed.data(), sh.data() + ilg::kServeTableBytes);
        ilg::pad_table(packed.data(), reinterpret_cast<uint32_t *>(sh.data()));
        e = hipMemcpy(ex.shared, sh.data(), sh.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        const int code = e == hipErrorOutOfMemory ? ILG_E_NOMEM : ILG_E_DEVICE;
        std::string msg = std::string("server setup: ") + hipGetErrorString(e);
        delete s;
        return sfail(code, msg);
    }
    // Small requests advance as resident slots, by up to 16 quanta per poll.
    const uint64_t rsteps = std::min<uint64_t>(16ull * quantum_steps, 1u << 30);
    s->sched->set_resident(ILG_RESIDENT_DEFAULT_NODES, (uint32_t)rsteps);
    ex.resident_nodes = ILG_RESIDENT_DEFAULT_NODES;
    ex.quantum = quantum_steps;
    *out = s;
    return ILG_OK;
}

int ilg_server_set_resident(ilg_server *s, uint64_t max_nodes, uint32_t max_steps)
{
    if (!s)
        return sfail(ILG_E_INVALID, "null server");
    if (max_nodes > ILG_RESIDENT_MAX_NODES)
        return sfail(ILG_E_INVALID, "resident requests hold at most " +
                                        std::to_string(ILG_RESIDENT_MAX_NODES) + " nodes");
    s->sched->set_resident(max_nodes, max_steps);
    s->ex.resident_nodes = max_nodes;
    return ILG_OK;
}

int ilg_server_set_step_nodes(ilg_server *s, uint64_t max_nodes)
{
    if (!s)
        return sfail(ILG_E_INVALID, "null server");
    s->sched->set_step_nodes(max_nodes);
    return ILG_OK;
}

int ilg_server_submit(ilg_server *s, const ilg_config *cfg, const void *init_host, uint64_t nsteps,
                      uint64_t *id)
{
    if (!s || !init_host || !id)
        return sfail(ILG_E_INVALID, "null argument");
    ilg::Fixed fx;
    int rc = ilg::check_config(cfg, &fx);
    if (rc != ILG_OK)
        return rc;
    if (nsteps == 0)
        return sfail(ILG_E_INVALID, "nsteps must be positive");
    if (cfg->t0 + nsteps > (uint64_t(1) << 32))
        return sfail(ILG_E_RANGE, "step index would pass 2^32 - 1");
    auto p = std::make_shared<Payload>();
    p->cfg = *cfg;
    p->fx = fx;
    const size_t bytes = (size_t)cfg->q * nodes_of(*cfg) * cfg->count_bytes;
    p->host.assign(static_cast<const unsigned char *>(init_host),
                   static_cast<const unsigned char *>(init_host) + bytes);
    std::unique_ptr<Req> r(new Req);
    r->q = cfg->q;
    r->nodes = nodes_of(*cfg);
    r->total = nsteps;
    r->payload = p;
    if (!s->sched->submit(std::move(r), s->ex, id, steady_now()))
        return sfail(ILG_E_BUSY, "request does not fit the server's memory budget");
    return ILG_OK;
}

int ilg_server_submit_poisson_sine(ilg_server *s, const ilg_config *cfg, double nave, double amp,
                                   uint64_t init_seed, uint64_t nsteps, uint64_t *id)
{
    if (!s || !id)
        return sfail(ILG_E_INVALID, "null argument");
    if (!std::isfinite(nave) || !std::isfinite(amp) || nave < 0.0 || nave > 1.0e6 ||
        std::fabs(amp) > nave)
        return sfail(ILG_E_INVALID, "need 0 <= nave <= 1e6 and |amp| <= nave");
    ilg::Fixed fx;
    int rc = ilg::check_config(cfg, &fx);
    if (rc != ILG_OK)
        return rc;
    if (nsteps == 0)
        return sfail(ILG_E_INVALID, "nsteps must be positive");
    if (cfg->t0 + nsteps > (uint64_t(1) << 32))
        return sfail(ILG_E_RANGE, "step index would pass 2^32 - 1");
    auto p = std::make_shared<Payload>();
    p->cfg = *cfg;
    p->fx = fx;
    p->device_init = true;
    p->nave = nave;
    p->amp = amp;
    p->init_seed = init_seed;
    std::unique_ptr<Req> r(new Req);
    r->q = cfg->q;
    r->nodes = nodes_of(*cfg);
    r->total = nsteps;
    r->payload = p;
    if (!s->sched->submit(std::move(r), s->ex, id, steady_now()))
        return sfail(ILG_E_BUSY, "request does not fit the server's memory budget");
    return ILG_OK;
}

int ilg_server_poll(ilg_server *s, ilg_poll_info *info)
{
    if (!s)
        return sfail(ILG_E_INVALID, "null server");
    ilg::serve::PollStats st;
    int rc = s->sched->poll(s->ex, &st, &steady_now);
    if (rc != 0)
        return rc;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->admitted = st.admitted;
        info->active = st.active;
        info->queued = st.queued;
        info->finished = st.finished;
        info->quantum_steps = st.quantum_steps;
        info->failed = st.failed;
        info->bytes_in_use = s->sched->used_bytes();
        info->bytes_peak = s->sched->peak_bytes();
    }
    return ILG_OK;
}

int ilg_server_info(ilg_server *s, uint64_t id, ilg_request_info *out)
{
    if (!s || !out)
        return sfail(ILG_E_INVALID, "null argument");
    Req *r = s->sched->find(id);
    if (!r)
        return sfail(ILG_E_INVALID, "unknown request id");
    const Payload *p = static_cast<const Payload *>(r->payload.get());
    std::memset(out, 0, sizeof(*out));
    out->id = r->id;
    out->state = (uint32_t)r->state;
    out->q = r->q;
    out->length = p ? p->cfg.length : 0;
    out->steps_total = r->total;
    out->steps_done = r->done;
    out->t_submit = r->t_submit;
    out->t_admit = r->t_admit;
    out->t_done = r->t_done;
    return ILG_OK;
}

int ilg_server_result(ilg_server *s, uint64_t id, void *host_out)
{
    if (!s || !host_out)
        return sfail(ILG_E_INVALID, "null argument");
    Req *r = s->sched->find(id);
    if (r && r->state == ReqState::Failed) {
        s->sched->release(id);
        return sfail(ILG_E_OVERFLOW, "request " + std::to_string(id) +
                                         ": a count exceeded the count type (its state is lost)");
    }
    if (!r || r->state != ReqState::Done)
        return sfail(ILG_E_INVALID, "request is not finished");
    const Payload *p = static_cast<const Payload *>(r->payload.get());
    std::memcpy(host_out, p->host.data(), p->host.size());
    s->sched->release(id);
    return ILG_OK;
}

int ilg_server_cancel(ilg_server *s, uint64_t id)
{
    if (!s)
        return sfail(ILG_E_INVALID, "null server");
    if (!s->sched->cancel(id, s->ex, &steady_now))
        return sfail(ILG_E_INVALID, "request is not queued or active");
    s->sched->release(id);
    return ILG_OK;
}

int ilg_server_destroy(ilg_server *s)
{
    if (!s)
        return ILG_OK;
    (void)s->sched->settle(s->ex, &steady_now, nullptr);
    for (int g = 0; g < DeviceExecutor::kGroups; ++g) {
        if (s->ex.streams[g])
            (void)hipStreamSynchronize(s->ex.streams[g]);
    }
    delete s;
    return ILG_OK;
}

}  // extern "C"
