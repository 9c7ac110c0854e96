// Continuous-batching scheduler for lattice-gas requests (host only, no HIP).
//
// Requests wait in a FIFO queue until their device memory (state buffers and
// tables) fits the budget; admitted requests become active slots.  Each poll
// admits what fits memory that is already free (its copies overlap the quantum
// in flight), waits for the quantum launched by the previous poll, retires the
// requests it finished (freeing their memory), admits again, and launches the
// next quantum for every active slot (fewer steps for a slot that finishes
// earlier).  With a node cap (set_step_nodes) a quantum advances only the
// active requests with the least remaining work (nodes x steps left) that
// fit the cap together, at least one: shortest-remaining-work first, which
// shortens the typical latency while the device is near saturation, since
// every launch advances its requests by one step and costs time in
// proportion to the nodes it holds.  Small requests (set_resident) are
// planned up to a longer step count per poll: the executor advances each of
// them inside one workgroup, several steps per launch, and may take fewer
// steps than planned (at least one), reporting the steps it took.  It
// returns while the device
// works, so the caller's host work overlaps the quantum.  The executor does
// the device work; the scheduler only does bookkeeping, so it is tested on
// the CPU with a counting executor.
#pragma once

#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <vector>

namespace ilg {
namespace serve {

enum class ReqState : uint32_t { Queued = 0, Active = 1, Done = 2, Cancelled = 3, Failed = 4 };

struct Req {
    uint64_t id = 0;
    uint32_t q = 0;
    uint64_t nodes = 0;     // lattice nodes (for the step node cap)
    uint64_t bytes = 0;     // device bytes while active (from the executor's layout)
    uint64_t total = 0;     // steps requested
    uint64_t done = 0;      // steps taken so far
    double t_submit = 0.0, t_admit = -1.0, t_done = -1.0;  // steady-clock seconds
    ReqState state = ReqState::Queued;
    uint64_t mem_off = 0;   // arena offset while active
    // Set by the executor when this request's own device work reported an
    // error (a count beyond its type, at admission or in a quantum): the
    // scheduler then retires the request as Failed and frees its memory;
    // the other requests are unaffected.
    bool failed = false;
    std::shared_ptr<void> payload;  // executor data (initial / final state, tables)
};

// First-fit allocator over [0, size) with coalescing free list.
class Arena {
public:
    explicit Arena(uint64_t size);
    bool alloc(uint64_t bytes, uint64_t *off);  // 256-byte aligned blocks
    void free(uint64_t off, uint64_t bytes);
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }

private:
    uint64_t size_, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;  // offset -> length
};

class Executor {
public:
    virtual ~Executor() = default;
    // Bytes of device memory a request needs while active.
    virtual uint64_t footprint(const Req &r) = 0;
    // Place the request's initial state and tables at r.mem_off.  Sets
    // r.failed if the request itself cannot start (its initial state does not
    // fit the count type); a nonzero return is a failure of the device.
    virtual int load(Req &r) = 0;
    // Start advancing active[i] by steps[i] >= 1 steps (may return before the
    // work is done).
    virtual int launch(const std::vector<Req *> &active, const std::vector<uint32_t> &steps) = 0;
    // Wait for the work of the last launch and account for it; sets failed on
    // each launched request whose own work reported an error.  `steps` holds
    // the steps launched per request (the order of the launch); the executor
    // lowers an entry, to no less than 1, where that request's advance ended
    // early.  A nonzero return is a failure of the device (every launched
    // request is then lost).
    virtual int wait(std::vector<uint32_t> *steps) = 0;
    // Copy a finished request's final state out of the device.
    virtual int unload(Req &r) = 0;
};

struct PollStats {
    uint32_t admitted = 0, active = 0, queued = 0, finished = 0;
    uint32_t failed = 0;         // requests retired as Failed by this poll
    uint32_t quantum_steps = 0;  // steps of the longest slot advance launched by this poll
};

class Scheduler {
public:
    Scheduler(uint64_t budget_bytes, uint32_t quantum_steps);
    // Queue a request; ILG_E_BUSY-style failure (returns false) if it could
    // never fit the budget.
    bool submit(std::unique_ptr<Req> r, Executor &ex, uint64_t *id, double now);
    // Wait for the previous quantum and retire what it finished, admit what
    // fits (FIFO), launch the next quantum.  After a poll that reports no
    // active and no queued request, nothing is in flight.
    int poll(Executor &ex, PollStats *st, double (*clock)());
    // Wait for the quantum in flight, if any (and retire what it finished or
    // what failed).
    int settle(Executor &ex, double (*clock)(), uint32_t *finished, uint32_t *failed = nullptr);
    Req *find(uint64_t id);
    // Cancel a queued or active request (its memory is released; an active
    // one only after the quantum in flight has completed).
    bool cancel(uint64_t id, Executor &ex, double (*clock)());
    // Forget a finished, failed or cancelled request.
    bool release(uint64_t id);
    uint64_t peak_bytes() const { return arena_.peak(); }
    uint64_t used_bytes() const { return arena_.used(); }
    size_t queued() const { return queue_.size(); }
    size_t active() const { return active_.size(); }
    // At most this many nodes advanced per quantum (0: every active request).
    void set_step_nodes(uint64_t nodes) { step_nodes_ = nodes; }
    // Requests of at most max_nodes nodes are advanced by up to max_steps
    // steps per poll (at least the quantum) instead of the quantum; 0 nodes:
    // none.
    void set_resident(uint64_t max_nodes, uint32_t max_steps)
    {
        resident_nodes_ = max_nodes;
        resident_steps_ = max_steps > quantum_ ? max_steps : quantum_;
    }
    bool resident(const Req &r) const { return r.nodes != 0 && r.nodes <= resident_nodes_; }
    uint64_t resident_nodes() const { return resident_nodes_; }

private:
    int admit(Executor &ex, double (*clock)(), uint32_t *admitted, uint32_t *failed);
    void retire_failed(Req *r, double now);
    void pick(std::vector<Req *> *out) const;

    uint64_t budget_;
    uint32_t quantum_;
    uint64_t step_nodes_ = 0;
    uint64_t resident_nodes_ = 0;
    uint32_t resident_steps_ = 0;
    Arena arena_;
    uint64_t next_id_ = 1;
    std::deque<Req *> queue_;
    std::vector<Req *> active_;
    std::vector<Req *> inflight_;       // slots of the quantum in flight
    std::vector<uint32_t> inflight_steps_;
    std::map<uint64_t, std::unique_ptr<Req>> all_;
};

// Measured correction of the estimated cost of the slots of one launch's
// tile walk.  Workgroup b walked tiles [range[b], range[b + 1]) in time[b]
// (any clock; workgroups with an empty range are ignored); tile t belongs to
// slot tile_slot[t] < nslots and was estimated at w[t] > 0.  The times are
// first scaled so that their total equals the estimated total (only relative
// cost matters), then each workgroup's ratio of measured to estimated work
// is shared among the slots of its range in proportion to their estimated
// work there.  corr[s] is that weighted ratio, clamped to [lo, hi]; a slot no
// measured workgroup walked gets 1.
void tile_cost_correction(const uint32_t *range, uint32_t grid, const double *w,
                          const uint32_t *tile_slot, const uint64_t *time, uint32_t nslots,
                          double lo, double hi, double *corr);

}  // namespace serve
}  // namespace ilg
