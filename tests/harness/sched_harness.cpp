// Test harness: the serving scheduler (paper_2203_01380_amd/csrc/scheduler.cpp)
// driven by a counting executor on the CPU, behind a small C API for ctypes.
// The executor checks the scheduler's contract: a request is loaded once,
// advanced only while active, never by more than the quantum (the resident
// step count for a small request) or past its step count, unloaded once when
// done; and the arena never exceeds the budget while the sum of active
// footprints matches the arena's use.  It can end a small request's advance
// early, as the device executor does, and counts the steps it reports.
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <set>
#include <vector>

#include "scheduler.h"

using namespace ilg::serve;

namespace {

struct Counting : Executor {
    uint32_t quantum = 0;
    uint64_t budget = 0;
    std::map<uint64_t, uint64_t> steps_seen, loads, unloads;
    std::vector<uint64_t> load_order;
    std::vector<uint64_t> last_launch;  // ids of the last launch, in order
    uint64_t step_nodes = 0;            // node cap the scheduler was given
    uint64_t resident_nodes = 0;        // small requests: up to resident_steps a poll
    uint32_t resident_steps = 0;
    uint32_t resident_stop = 0;         // end a small request's advance after this many (0: never)
    std::vector<uint32_t> planned;      // steps of the last launch
    uint64_t active_bytes = 0;
    int violations = 0;
    // failure injection: requests whose admission fails, and requests whose
    // next quantum reports an overflow
    std::set<uint64_t> fail_load, fail_wait;
    std::vector<Req *> launched;
    uint64_t footprint(const Req &r) override
    {
        return *static_cast<const uint64_t *>(r.payload.get());
    }
    int load(Req &r) override
    {
        loads[r.id] += 1;
        load_order.push_back(r.id);
        if (r.mem_off + r.bytes > budget)
            ++violations;
        if (fail_load.count(r.id)) {
            r.failed = true;
            return 0;
        }
        active_bytes += r.bytes;
        return 0;
    }
    bool in_flight = false;
    int launch(const std::vector<Req *> &active, const std::vector<uint32_t> &steps) override
    {
        if (in_flight)
            ++violations;  // a launch before the previous one was waited for
        in_flight = true;
        last_launch.clear();
        launched = active;
        uint64_t nodes = 0;
        for (const Req *r : active) {
            last_launch.push_back(r->id);
            nodes += r->nodes;
        }
        if (step_nodes != 0 && active.size() > 1 && nodes > step_nodes)
            ++violations;  // more nodes than the cap in a multi-request quantum
        for (size_t i = 0; i < active.size(); ++i) {
            Req *r = active[i];
            const bool small = r->nodes != 0 && r->nodes <= resident_nodes;
            const uint32_t cap = small ? resident_steps : quantum;
            if (r->state != ReqState::Active || steps[i] == 0 || steps[i] > cap ||
                r->done + steps[i] > r->total)
                ++violations;
        }
        planned = steps;
        return 0;
    }
    int wait(std::vector<uint32_t> *steps) override
    {
        in_flight = false;
        if (steps->size() != launched.size() || *steps != planned)
            ++violations;  // not the steps of the launch being waited for
        for (size_t i = 0; i < launched.size() && i < steps->size(); ++i) {
            const Req *r = launched[i];
            uint32_t k = (*steps)[i];
            if (resident_stop != 0 && r->nodes != 0 && r->nodes <= resident_nodes &&
                k > resident_stop)
                k = resident_stop;
            (*steps)[i] = k;
            steps_seen[r->id] += k;
        }
        for (Req *r : launched) {
            if (fail_wait.count(r->id)) {
                if (r->failed)
                    ++violations;  // a failed request was launched again
                r->failed = true;
                active_bytes -= r->bytes;
            }
        }
        launched.clear();
        return 0;
    }
    int unload(Req &r) override
    {
        if (in_flight)
            ++violations;  // results read while their quantum may still run
        unloads[r.id] += 1;
        active_bytes -= r.bytes;
        if (steps_seen[r.id] != r.total)
            ++violations;
        return 0;
    }
};

double fake_now = 0.0;
double fake_clock()
{
    fake_now += 1.0;
    return fake_now;
}

struct Harness {
    Scheduler sched;
    Counting ex;
    Harness(uint64_t budget, uint32_t quantum) : sched(budget, quantum)
    {
        ex.quantum = quantum;
        ex.budget = budget;
    }
};

}  // namespace

extern "C" {

void *h_new(uint64_t budget, uint32_t quantum)
{
    return new Harness(budget, quantum);
}

void h_free(void *h)
{
    delete static_cast<Harness *>(h);
}

int h_submit_nodes(void *hv, uint32_t q, uint64_t bytes, uint64_t steps, uint64_t nodes,
                   uint64_t *id)
{
    Harness *h = static_cast<Harness *>(hv);
    std::unique_ptr<Req> r(new Req);
    r->q = q;
    r->nodes = nodes;
    r->total = steps;
    r->payload = std::make_shared<uint64_t>(bytes);
    return h->sched.submit(std::move(r), h->ex, id, fake_now) ? 0 : -6;
}

void h_set_step_nodes(void *hv, uint64_t nodes)
{
    Harness *h = static_cast<Harness *>(hv);
    h->sched.set_step_nodes(nodes);
    h->ex.step_nodes = nodes;
}

void h_set_resident(void *hv, uint64_t nodes, uint32_t steps, uint32_t stop_after)
{
    Harness *h = static_cast<Harness *>(hv);
    h->sched.set_resident(nodes, steps);
    h->ex.resident_nodes = nodes;
    h->ex.resident_steps = steps > h->ex.quantum ? steps : h->ex.quantum;
    h->ex.resident_stop = stop_after;
}

int h_last_steps(void *hv, uint32_t *out, int cap)
{
    Harness *h = static_cast<Harness *>(hv);
    int n = (int)h->ex.planned.size();
    for (int i = 0; i < n && i < cap; ++i)
        out[i] = h->ex.planned[i];
    return n;
}

int h_last_launch(void *hv, uint64_t *out, int cap)
{
    Harness *h = static_cast<Harness *>(hv);
    int n = (int)h->ex.last_launch.size();
    for (int i = 0; i < n && i < cap; ++i)
        out[i] = h->ex.last_launch[i];
    return n;
}

int h_submit(void *hv, uint32_t q, uint64_t bytes, uint64_t steps, uint64_t *id)
{
    Harness *h = static_cast<Harness *>(hv);
    std::unique_ptr<Req> r(new Req);
    r->q = q;
    r->total = steps;
    r->payload = std::make_shared<uint64_t>(bytes);
    return h->sched.submit(std::move(r), h->ex, id, fake_now) ? 0 : -6;
}

void h_fail_load(void *hv, uint64_t id)
{
    static_cast<Harness *>(hv)->ex.fail_load.insert(id);
}

void h_fail_wait(void *hv, uint64_t id)
{
    static_cast<Harness *>(hv)->ex.fail_wait.insert(id);
}

int h_poll5(void *hv, uint32_t *out5)
{
    Harness *h = static_cast<Harness *>(hv);
    PollStats st;
    int rc = h->sched.poll(h->ex, &st, &fake_clock);
    out5[0] = st.admitted;
    out5[1] = st.active;
    out5[2] = st.queued;
    out5[3] = st.finished;
    out5[4] = st.failed;
    if (h->sched.used_bytes() > h->ex.budget)
        ++h->ex.violations;
    return rc;
}

int h_poll(void *hv, uint32_t *out4)
{
    Harness *h = static_cast<Harness *>(hv);
    PollStats st;
    int rc = h->sched.poll(h->ex, &st, &fake_clock);
    out4[0] = st.admitted;
    out4[1] = st.active;
    out4[2] = st.queued;
    out4[3] = st.finished;
    if (h->sched.used_bytes() > h->ex.budget)
        ++h->ex.violations;
    return rc;
}

int h_state(void *hv, uint64_t id, uint64_t *done, double *t_admit, double *t_done)
{
    Req *r = static_cast<Harness *>(hv)->sched.find(id);
    if (!r)
        return -1;
    *done = r->done;
    *t_admit = r->t_admit;
    *t_done = r->t_done;
    return (int)r->state;
}

int h_cancel(void *hv, uint64_t id)
{
    Harness *h = static_cast<Harness *>(hv);
    Req *r = h->sched.find(id);
    const bool was_active = r && r->state == ReqState::Active;
    const bool ok = h->sched.cancel(id, h->ex, &fake_clock);
    if (ok && was_active) {
        if (h->ex.in_flight)
            ++h->ex.violations;  // memory freed under a running quantum
        h->ex.active_bytes -= r->bytes;
    }
    return ok ? 0 : -1;
}

int h_release(void *hv, uint64_t id)
{
    return static_cast<Harness *>(hv)->sched.release(id) ? 0 : -1;
}

uint64_t h_peak(void *hv)
{
    return static_cast<Harness *>(hv)->sched.peak_bytes();
}

uint64_t h_used(void *hv)
{
    return static_cast<Harness *>(hv)->sched.used_bytes();
}

int h_violations(void *hv)
{
    Harness *h = static_cast<Harness *>(hv);
    int v = h->ex.violations;
    if (h->ex.active_bytes != 0 && h->sched.active() == 0)
        ++v;
    return v;
}

int h_load_order(void *hv, uint64_t *out, int cap)
{
    Harness *h = static_cast<Harness *>(hv);
    int n = (int)h->ex.load_order.size();
    for (int i = 0; i < n && i < cap; ++i)
        out[i] = h->ex.load_order[i];
    return n;
}

void h_tile_cost_correction(const uint32_t *range, uint32_t grid, const double *w,
                            const uint32_t *tile_slot, const uint64_t *time, uint32_t nslots,
                            double lo, double hi, double *corr)
{
    ilg::serve::tile_cost_correction(range, grid, w, tile_slot, time, nslots, lo, hi, corr);
}

}  // extern "C"
