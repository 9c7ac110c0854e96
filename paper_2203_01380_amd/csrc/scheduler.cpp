// Continuous-batching scheduler: FIFO admission under a device-memory
// budget, quantum advances of all active slots, retirement.
#include "scheduler.h"

#include <algorithm>

namespace ilg {
namespace serve {

namespace {
constexpr uint64_t kAlign = 256;
uint64_t round_up(uint64_t x)
{
    return (x + kAlign - 1) / kAlign * kAlign;
}
}  // namespace

Arena::Arena(uint64_t size) : size_(size / kAlign * kAlign)
{
    if (size_ > 0)
        free_[0] = size_;
}

bool Arena::alloc(uint64_t bytes, uint64_t *off)
{
    const uint64_t need = round_up(std::max<uint64_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second >= need) {
            *off = it->first;
            const uint64_t rest = it->second - need, start = it->first + need;
            free_.erase(it);
            if (rest)
                free_[start] = rest;
            used_ += need;
            peak_ = std::max(peak_, used_);
            return true;
        }
    }
    return false;
}

void Arena::free(uint64_t off, uint64_t bytes)
{
    const uint64_t len = round_up(std::max<uint64_t>(bytes, 1));
    used_ -= len;
    auto it = free_.emplace(off, len).first;
    // merge with the following block
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        free_.erase(nx);
    }
    // merge with the preceding block
    if (it != free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            free_.erase(it);
        }
    }
}

Scheduler::Scheduler(uint64_t budget_bytes, uint32_t quantum_steps)
    : budget_(budget_bytes), quantum_(quantum_steps ? quantum_steps : 1), arena_(budget_bytes)
{
}

bool Scheduler::submit(std::unique_ptr<Req> r, Executor &ex, uint64_t *id, double now)
{
    r->bytes = ex.footprint(*r);
    if (round_up(r->bytes) > arena_.size() || r->total == 0)
        return false;
    r->id = next_id_++;
    r->t_submit = now;
    r->state = ReqState::Queued;
    Req *raw = r.get();
    all_[raw->id] = std::move(r);
    queue_.push_back(raw);
    *id = raw->id;
    return true;
}

void Scheduler::retire_failed(Req *r, double now)
{
    arena_.free(r->mem_off, r->bytes);
    r->state = ReqState::Failed;
    r->t_done = now;
    r->payload.reset();
}

int Scheduler::settle(Executor &ex, double (*clock)(), uint32_t *finished, uint32_t *failed)
{
    uint32_t nfin = 0, nfail = 0;
    if (!inflight_.empty()) {
        int rc = ex.wait(&inflight_steps_);
        const double now = clock();
        for (size_t i = 0; i < inflight_.size() && rc == 0; ++i) {
            Req *r = inflight_[i];
            if (r->failed) {
                retire_failed(r, now);
                ++nfail;
                continue;
            }
            r->done += inflight_steps_[i];
            if (r->done >= r->total) {
                rc = ex.unload(*r);
                if (rc != 0)
                    break;
                arena_.free(r->mem_off, r->bytes);
                r->state = ReqState::Done;
                r->t_done = now;
                ++nfin;
            }
        }
        if (rc != 0) {
            // The device failed: the state of every request of the quantum is
            // lost.  Retire them so that the others (queued) can still run.
            for (Req *r : inflight_)
                if (r->state == ReqState::Active) {
                    retire_failed(r, now);
                    ++nfail;
                }
        }
        std::vector<Req *> still;
        for (Req *r : active_)
            if (r->state == ReqState::Active)
                still.push_back(r);
        active_.swap(still);
        inflight_.clear();
        inflight_steps_.clear();
        if (finished)
            *finished = nfin;
        if (failed)
            *failed += nfail;
        return rc;
    }
    if (finished)
        *finished = nfin;
    return 0;
}

int Scheduler::admit(Executor &ex, double (*clock)(), uint32_t *admitted, uint32_t *failed)
{
    // Strict FIFO, so a large request is never starved by later small ones.
    while (!queue_.empty()) {
        Req *r = queue_.front();
        uint64_t off = 0;
        if (!arena_.alloc(r->bytes, &off))
            break;
        r->mem_off = off;
        int rc = ex.load(*r);
        if (rc != 0) {
            arena_.free(off, r->bytes);
            return rc;
        }
        queue_.pop_front();
        r->t_admit = clock();
        if (r->failed) {
            retire_failed(r, r->t_admit);
            ++*failed;
            continue;
        }
        r->state = ReqState::Active;
        active_.push_back(r);
        ++*admitted;
    }
    return 0;
}

void Scheduler::pick(std::vector<Req *> *out) const
{
    if (step_nodes_ == 0) {
        *out = active_;
        return;
    }
    // Least remaining work first (ties by id), greedily within the cap; a
    // request that does not fit is passed over for smaller ones after it.
    std::vector<Req *> order(active_);
    std::stable_sort(order.begin(), order.end(), [](const Req *a, const Req *b) {
        const uint64_t wa = a->nodes * (a->total - a->done);
        const uint64_t wb = b->nodes * (b->total - b->done);
        return wa != wb ? wa < wb : a->id < b->id;
    });
    out->clear();
    uint64_t used = 0;
    for (Req *r : order) {
        if (!out->empty() && used + r->nodes > step_nodes_)
            continue;
        out->push_back(r);
        used += r->nodes;
    }
}

int Scheduler::poll(Executor &ex, PollStats *st, double (*clock)())
{
    PollStats s;
    // Admissions into memory that is already free overlap the quantum in
    // flight (they touch only their own, unused, memory); a second pass after
    // the quantum has completed uses the memory its finished requests freed.
    int rc = admit(ex, clock, &s.admitted, &s.failed);
    if (rc == 0)
        rc = settle(ex, clock, &s.finished, &s.failed);
    if (rc == 0)
        rc = admit(ex, clock, &s.admitted, &s.failed);
    if (rc != 0)
        return rc;
    if (!active_.empty()) {
        pick(&inflight_);
        inflight_steps_.resize(inflight_.size());
        for (size_t i = 0; i < inflight_.size(); ++i) {
            const uint64_t left = inflight_[i]->total - inflight_[i]->done;
            const uint32_t cap = resident(*inflight_[i]) ? resident_steps_ : quantum_;
            inflight_steps_[i] = (uint32_t)std::min<uint64_t>(left, cap);
            s.quantum_steps = std::max(s.quantum_steps, inflight_steps_[i]);
        }
        rc = ex.launch(inflight_, inflight_steps_);
        if (rc != 0) {
            inflight_.clear();
            inflight_steps_.clear();
            return rc;
        }
    }
    s.active = (uint32_t)active_.size();
    s.queued = (uint32_t)queue_.size();
    if (st)
        *st = s;
    return 0;
}

Req *Scheduler::find(uint64_t id)
{
    auto it = all_.find(id);
    return it == all_.end() ? nullptr : it->second.get();
}

bool Scheduler::cancel(uint64_t id, Executor &ex, double (*clock)())
{
    Req *r = find(id);
    if (!r)
        return false;
    if (r->state == ReqState::Queued) {
        queue_.erase(std::find(queue_.begin(), queue_.end(), r));
    } else if (r->state == ReqState::Active) {
        // the device may still be writing its memory: finish the quantum first
        if (settle(ex, clock, nullptr) != 0 || r->state != ReqState::Active)
            return false;
        active_.erase(std::find(active_.begin(), active_.end(), r));
        arena_.free(r->mem_off, r->bytes);
    } else {
        return false;
    }
    r->state = ReqState::Cancelled;
    r->payload.reset();
    return true;
}

bool Scheduler::release(uint64_t id)
{
    Req *r = find(id);
    if (!r || (r->state != ReqState::Done && r->state != ReqState::Cancelled &&
               r->state != ReqState::Failed))
        return false;
    all_.erase(id);
    return true;
}

void tile_cost_correction(const uint32_t *range, uint32_t grid, const double *w,
                          const uint32_t *tile_slot, const uint64_t *time, uint32_t nslots,
                          double lo, double hi, double *corr)
{
    std::vector<double> est(grid, 0.0), num(nslots, 0.0), den(nslots, 0.0);
    double total_t = 0.0, total_e = 0.0;
    for (uint32_t b = 0; b < grid; ++b) {
        for (uint32_t t = range[b]; t < range[b + 1]; ++t)
            est[b] += w[t];
        if (est[b] > 0.0) {
            total_t += (double)time[b];
            total_e += est[b];
        }
    }
    for (uint32_t s = 0; s < nslots; ++s)
        corr[s] = 1.0;
    if (total_t <= 0.0 || total_e <= 0.0)
        return;
    const double scale = total_e / total_t;  // estimated units per clock tick
    for (uint32_t b = 0; b < grid; ++b) {
        if (est[b] <= 0.0)
            continue;
        const double r = (double)time[b] * scale / est[b];
        for (uint32_t t = range[b]; t < range[b + 1]; ++t) {
            num[tile_slot[t]] += w[t] * r;
            den[tile_slot[t]] += w[t];
        }
    }
    for (uint32_t s = 0; s < nslots; ++s)
        if (den[s] > 0.0)
            corr[s] = std::min(hi, std::max(lo, num[s] / den[s]));
}

}  // namespace serve
}  // namespace ilg
