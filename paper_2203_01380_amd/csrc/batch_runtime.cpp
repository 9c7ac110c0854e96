// Host runtime of batched ensembles (ilg_batch_* in include/ilg.h): member
// layout in one device arena, per-member fixed-point tables, the
// longest-first member order, HIP-graph capture of the persistent launch and
// the launch-shape autotuner.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "ilg.h"
#include "ilg_internal.h"

namespace {

int bfail(int code, const std::string &msg)
{
    ilg::set_last_error(msg);
    return code;
}

int bhip(hipError_t e, const char *what)
{
    return bfail(ILG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define BHIP(call)                                     \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess)                          \
            return bhip(e_, #call);                    \
    } while (0)

uint64_t pitch_of(uint64_t length)
{
    return (length + 63) / 64 * 64;
}

}  // namespace

struct ilg_batch {
    uint32_t q = 0, cb = 0, nreal = 0;
    uint32_t rounds = 10, exchange = 0;  // draw specification, batch-wide
    hipStream_t stream = nullptr;      // caller's stream
    hipStream_t cap = nullptr;         // private stream used for graph capture
    std::vector<uint32_t> lengths;
    std::vector<uint64_t> t_next;      // host mirror of each member's next step
    std::vector<uint64_t> off;         // element offsets
    uint64_t arena_elems = 0;
    void *arena = nullptr;
    ilg::BatchMeta *meta = nullptr;
    uint32_t *tabs_p = nullptr, *tabs_shared = nullptr, *order = nullptr, *queue = nullptr;
    uint32_t *err = nullptr;
    ilg_batch_diag diag{0, 0, 0, 0};
    double *sk_sum = nullptr, *amp = nullptr;
    unsigned long long *sk_cnt = nullptr;
    uint32_t *amp_cnt = nullptr;
    int shape = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t graph_nsteps = 0;
    int graph_shape = -1;
};

namespace {

void release(ilg_batch *b)
{
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    (void)hipFree(b->arena);
    (void)hipFree(b->meta);
    (void)hipFree(b->tabs_p);
    (void)hipFree(b->tabs_shared);
    (void)hipFree(b->order);
    (void)hipFree(b->queue);
    (void)hipFree(b->err);
    (void)hipFree(b->sk_sum);
    (void)hipFree(b->sk_cnt);
    (void)hipFree(b->amp);
    (void)hipFree(b->amp_cnt);
    if (b->cap)
        (void)hipStreamDestroy(b->cap);
    delete b;
}

ilg::BatchArgs make_args(const ilg_batch *b, uint32_t nsteps)
{
    ilg::BatchArgs a;
    a.arena = b->arena;
    a.meta = b->meta;
    a.tabs_p = b->tabs_p;
    a.tabs_shared = b->tabs_shared;
    a.order = b->order;
    a.queue = b->queue;
    a.nreal = b->nreal;
    a.nsteps = nsteps;
    a.sk_every = b->diag.sk_every;
    a.nk = b->diag.nk;
    a.amp_every = b->diag.amp_every;
    a.max_amp = b->diag.max_amp;
    a.sk_sum = b->sk_sum;
    a.sk_cnt = b->sk_cnt;
    a.amp = b->amp;
    a.amp_cnt = b->amp_cnt;
    a.err = b->err;
    a.rounds = b->rounds;
    a.exchange = b->exchange;
    return a;
}

int sticky(ilg_batch *b)
{
    uint32_t e = 0;
    BHIP(hipMemcpyAsync(&e, b->err, sizeof(e), hipMemcpyDeviceToHost, b->stream));
    BHIP(hipStreamSynchronize(b->stream));
    if (e & 1u)
        return bfail(ILG_E_OVERFLOW, "a post-collision count exceeded the count type");
    return ILG_OK;
}

}  // namespace

extern "C" {

int ilg_batch_create(const ilg_config *cfgs, uint32_t nreal, const void *const *inits,
                     const ilg_batch_diag *diag, void *stream, ilg_batch **out)
{
    if (!out || !cfgs || !inits || nreal == 0)
        return bfail(ILG_E_INVALID, "need nreal > 0 configurations, initial states and an output");
    *out = nullptr;
    std::vector<ilg::Fixed> fx(nreal);
    for (uint32_t r = 0; r < nreal; ++r) {
        int rc = ilg::check_config(&cfgs[r], &fx[r]);
        if (rc != ILG_OK)
            return rc;
        if (fx[r].rounds != fx[0].rounds || fx[r].exchange != fx[0].exchange)
            return bfail(ILG_E_INVALID,
                         "batch members must share the draw specification (flags "
                         "ILG_DRAWS_PHILOX7 and ILG_DRAWS_EXCHANGE)");
        if (!inits[r])
            return bfail(ILG_E_INVALID, "null initial state");
        if (cfgs[r].q != cfgs[0].q || cfgs[r].count_bytes != cfgs[0].count_bytes ||
            (cfgs[0].q != 2 && fx[r].p_rest != fx[0].p_rest))
            return bfail(ILG_E_INVALID, "batch members must share q, count_bytes and theta");
    }
    ilg_batch_diag d{0, 0, 0, 0};
    if (diag) {
        d = *diag;
        if (d.sk_every && (d.nk == 0 || d.nk > ILG_BATCH_MAX_K))
            return bfail(ILG_E_INVALID, "nk must lie in 1..ILG_BATCH_MAX_K");
        if (!d.sk_every)
            d.nk = 0;
        if (cfgs[0].q == 5 && (d.sk_every || d.amp_every))
            return bfail(ILG_E_INVALID, "S(k) and A^LG are defined for 1D members");
        if (!d.amp_every)
            d.max_amp = 0;
    }
    (void)ilg::device_cu_count();  // cached now, never queried during graph capture
    ilg_batch *b = new (std::nothrow) ilg_batch;
    if (!b)
        return bfail(ILG_E_NOMEM, "host allocation failed");
    b->q = cfgs[0].q;
    b->cb = cfgs[0].count_bytes;
    b->rounds = (uint32_t)fx[0].rounds;
    b->exchange = (uint32_t)fx[0].exchange;
    b->nreal = nreal;
    b->stream = reinterpret_cast<hipStream_t>(stream);
    b->diag = d;
    const uint32_t q = b->q, cb = b->cb;

    // Layout: member r owns two [q][pitch_r] buffers starting at off[r].
    std::vector<ilg::BatchMeta> meta(nreal);
    b->lengths.resize(nreal);
    b->t_next.resize(nreal);
    b->off.resize(nreal);
    uint64_t off = 0;
    for (uint32_t r = 0; r < nreal; ++r) {
        // nodes: L in 1D, Lx Ly for D2Q5 (node x + Lx y)
        const uint64_t L = cfgs[r].length * (q == 5 ? (uint64_t)cfgs[r].height : 1u);
        const uint64_t pitch = pitch_of(L);
        b->lengths[r] = (uint32_t)L;
        b->t_next[r] = cfgs[r].t0;
        b->off[r] = off;
        ilg::BatchMeta &m = meta[r];
        std::memset(&m, 0, sizeof(m));
        m.off = off;
        m.length = (uint32_t)L;
        m.width = (uint32_t)cfgs[r].length;
        m.pitch = (uint32_t)pitch;
        m.t = (uint32_t)cfgs[r].t0;
        m.realization = cfgs[r].realization;
        m.key0 = (uint32_t)(cfgs[r].seed & 0xFFFFFFFFu);
        m.key1 = (uint32_t)(cfgs[r].seed >> 32);
        m.flip = (uint32_t)fx[r].flip;
        m.p_zero = fx[r].p == 0 ? 1u : 0u;
        m.cur = 0;
        off += 2 * q * pitch;
    }
    b->arena_elems = off;

    // Initial states into buffer 0 of each member (one host staging copy).
    std::vector<unsigned char> stage(off * cb, 0);
    for (uint32_t r = 0; r < nreal; ++r) {
        const uint64_t L = b->lengths[r], pitch = meta[r].pitch;
        const unsigned char *src = reinterpret_cast<const unsigned char *>(inits[r]);
        for (uint32_t i = 0; i < q; ++i)
            std::memcpy(stage.data() + (b->off[r] + i * pitch) * cb, src + i * L * cb, L * cb);
    }

    // Removal tables per member (host threads), shared half/rest tables, all
    // in the padded device layout.
    std::vector<uint32_t> tabs((size_t)nreal * ilg::kDevTableEntries, 0);
    {
        const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> pool;
        for (unsigned k = 0; k < nth; ++k)
            pool.emplace_back([&, k]() {
                std::vector<uint32_t> packed(ilg::kTableEntries);
                for (uint32_t r = k; r < nreal; r += nth)
                    if (fx[r].p != 0) {
                        ilg::build_binomial_table(fx[r].p, packed.data());
                        ilg::pad_table(packed.data(),
                                       tabs.data() + (size_t)r * ilg::kDevTableEntries);
                    }
            });
        for (auto &th : pool)
            th.join();
    }
    std::vector<uint32_t> shared(2 * ilg::kDevTableEntries, 0);
    {
        std::vector<uint32_t> packed(ilg::kTableEntries);
        ilg::build_binomial_table(uint64_t(1) << 31, packed.data());
        ilg::pad_table(packed.data(), shared.data());
        if (q != 2) {
            ilg::build_binomial_table(fx[0].p_rest, packed.data());
            ilg::pad_table(packed.data(), shared.data() + ilg::kDevTableEntries);
        }
    }

    // Longest first (ties by index), so long members start early.
    std::vector<uint32_t> order(nreal);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        return b->lengths[x] > b->lengths[y];
    });

    auto fail_release = [&](int code) {
        std::string msg = ilg_last_error();
        release(b);
        return bfail(code, msg);
    };
#define BTRY(call)                                                          \
    do {                                                                    \
        hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) {                                             \
            bhip(e_, #call);                                                \
            return fail_release(e_ == hipErrorOutOfMemory ? ILG_E_NOMEM     \
                                                          : ILG_E_DEVICE);  \
        }                                                                   \
    } while (0)
    BTRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    BTRY(hipMalloc(&b->arena, off * cb));
    BTRY(hipMalloc((void **)&b->meta, sizeof(ilg::BatchMeta) * nreal));
    BTRY(hipMalloc((void **)&b->tabs_p, tabs.size() * sizeof(uint32_t)));
    BTRY(hipMalloc((void **)&b->tabs_shared, shared.size() * sizeof(uint32_t)));
    BTRY(hipMalloc((void **)&b->order, sizeof(uint32_t) * nreal));
    BTRY(hipMalloc((void **)&b->queue, sizeof(uint32_t)));
    BTRY(hipMalloc((void **)&b->err, sizeof(uint32_t)));
    const size_t nsk = (size_t)nreal * std::max(1u, d.nk);
    const size_t namp = (size_t)nreal * std::max(1u, d.max_amp);
    BTRY(hipMalloc((void **)&b->sk_sum, nsk * sizeof(double)));
    BTRY(hipMalloc((void **)&b->sk_cnt, nreal * sizeof(unsigned long long)));
    BTRY(hipMalloc((void **)&b->amp, namp * sizeof(double)));
    BTRY(hipMalloc((void **)&b->amp_cnt, nreal * sizeof(uint32_t)));
    BTRY(hipMemcpyAsync(b->arena, stage.data(), stage.size(), hipMemcpyHostToDevice, b->stream));
    BTRY(hipMemcpyAsync(b->meta, meta.data(), sizeof(ilg::BatchMeta) * nreal, hipMemcpyHostToDevice,
                        b->stream));
    BTRY(hipMemcpyAsync(b->tabs_p, tabs.data(), tabs.size() * sizeof(uint32_t),
                        hipMemcpyHostToDevice, b->stream));
    BTRY(hipMemcpyAsync(b->tabs_shared, shared.data(), shared.size() * sizeof(uint32_t),
                        hipMemcpyHostToDevice, b->stream));
    BTRY(hipMemcpyAsync(b->order, order.data(), sizeof(uint32_t) * nreal, hipMemcpyHostToDevice,
                        b->stream));
    BTRY(hipMemsetAsync(b->err, 0, sizeof(uint32_t), b->stream));
    BTRY(hipMemsetAsync(b->sk_sum, 0, nsk * sizeof(double), b->stream));
    BTRY(hipMemsetAsync(b->sk_cnt, 0, nreal * sizeof(unsigned long long), b->stream));
    BTRY(hipMemsetAsync(b->amp, 0, namp * sizeof(double), b->stream));
    BTRY(hipMemsetAsync(b->amp_cnt, 0, nreal * sizeof(uint32_t), b->stream));
    BTRY(hipStreamSynchronize(b->stream));
#undef BTRY
    *out = b;
    return ILG_OK;
}

static int capture(ilg_batch *b, uint64_t nsteps)
{
    if (b->exec && b->graph_nsteps == nsteps && b->graph_shape == b->shape)
        return ILG_OK;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    // The queue is cleared by a kernel node (not a memset node) so that every
    // replay starts from an empty queue.
    BHIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e1 = ilg::launch_batch_reset(b->queue, b->cap);
    hipError_t e2 = ilg::launch_batch((int)b->q, (int)b->cb, b->shape,
                                      make_args(b, (uint32_t)nsteps), b->cap);
    hipGraph_t g = nullptr;
    hipError_t e3 = hipStreamEndCapture(b->cap, &g);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        if (g)
            (void)hipGraphDestroy(g);
        return bhip(e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3), "graph capture");
    }
    b->graph = g;
    BHIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_nsteps = nsteps;
    b->graph_shape = b->shape;
    return ILG_OK;
}

int ilg_batch_run(ilg_batch *b, uint64_t nsteps)
{
    if (!b)
        return bfail(ILG_E_INVALID, "null batch");
    if (nsteps == 0)
        return ILG_OK;
    for (uint32_t r = 0; r < b->nreal; ++r)
        if (b->t_next[r] + nsteps > (uint64_t(1) << 32))
            return bfail(ILG_E_RANGE, "step index would pass 2^32 - 1");
    int rc = capture(b, nsteps);
    if (rc != ILG_OK)
        return rc;
    BHIP(hipGraphLaunch(b->exec, b->stream));
    for (uint32_t r = 0; r < b->nreal; ++r)
        b->t_next[r] += nsteps;
    return ILG_OK;
}

int ilg_batch_tune(ilg_batch *b, uint32_t tune_steps, uint32_t *chosen)
{
    if (!b || tune_steps == 0)
        return bfail(ILG_E_INVALID, "need a batch and tune_steps > 0");
    for (uint32_t r = 0; r < b->nreal; ++r)
        if (b->t_next[r] + tune_steps > (uint64_t(1) << 32))
            return bfail(ILG_E_RANGE, "step index would pass 2^32 - 1");
    BHIP(hipStreamSynchronize(b->stream));
    // Scratch copies of everything a launch writes (state, descriptors,
    // error word, diagnostics), so the timed launches run the kernel variant
    // of the batch's own diagnostic settings and leave the batch untouched.
    const size_t arena_bytes = b->arena_elems * b->cb;
    const size_t nsk = (size_t)b->nreal * std::max(1u, b->diag.nk);
    const size_t namp = (size_t)b->nreal * std::max(1u, b->diag.max_amp);
    void *arena = nullptr;
    ilg::BatchMeta *meta = nullptr;
    uint32_t *err = nullptr, *amp_cnt = nullptr;
    double *sk_sum = nullptr, *amp = nullptr;
    unsigned long long *sk_cnt = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int best = b->shape;
    float best_ms = 0.0f;
    int rc = ILG_OK;
    hipError_t he = hipMalloc(&arena, arena_bytes);
    if (he == hipSuccess)
        he = hipMalloc((void **)&meta, sizeof(ilg::BatchMeta) * b->nreal);
    if (he == hipSuccess)
        he = hipMalloc((void **)&err, sizeof(uint32_t));
    if (he == hipSuccess)
        he = hipMalloc((void **)&sk_sum, nsk * sizeof(double));
    if (he == hipSuccess)
        he = hipMalloc((void **)&sk_cnt, b->nreal * sizeof(unsigned long long));
    if (he == hipSuccess)
        he = hipMalloc((void **)&amp, namp * sizeof(double));
    if (he == hipSuccess)
        he = hipMalloc((void **)&amp_cnt, b->nreal * sizeof(uint32_t));
    if (he == hipSuccess)
        he = hipEventCreate(&e0);
    if (he == hipSuccess)
        he = hipEventCreate(&e1);
    // Per shape: one warm-up launch, then the best of three timed launches,
    // each from the same copy of the ensemble.
    constexpr int kTimed = 3;
    for (int s = 0; he == hipSuccess && s < ilg::batch_shape_count(); ++s) {
        float shape_ms = 0.0f;
        for (int k = 0; he == hipSuccess && k <= kTimed; ++k) {
            he = hipMemcpyAsync(arena, b->arena, arena_bytes, hipMemcpyDeviceToDevice, b->stream);
            if (he == hipSuccess)
                he = hipMemcpyAsync(meta, b->meta, sizeof(ilg::BatchMeta) * b->nreal,
                                    hipMemcpyDeviceToDevice, b->stream);
            if (he == hipSuccess)
                he = hipMemsetAsync(err, 0, sizeof(uint32_t), b->stream);
            if (he == hipSuccess)
                he = hipMemsetAsync(sk_cnt, 0, b->nreal * sizeof(unsigned long long), b->stream);
            if (he == hipSuccess)
                he = hipMemsetAsync(amp_cnt, 0, b->nreal * sizeof(uint32_t), b->stream);
            ilg::BatchArgs a = make_args(b, tune_steps);
            a.arena = arena;
            a.meta = meta;
            a.err = err;
            a.sk_sum = sk_sum;
            a.sk_cnt = sk_cnt;
            a.amp = amp;
            a.amp_cnt = amp_cnt;
            if (he == hipSuccess)
                he = ilg::launch_batch_reset(b->queue, b->stream);
            if (he == hipSuccess)
                he = hipEventRecord(e0, b->stream);
            if (he == hipSuccess)
                he = ilg::launch_batch((int)b->q, (int)b->cb, s, a, b->stream);
            if (he == hipSuccess)
                he = hipEventRecord(e1, b->stream);
            if (he == hipSuccess)
                he = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (he == hipSuccess)
                he = hipEventElapsedTime(&ms, e0, e1);
            if (k == 1 || (k > 1 && ms < shape_ms))
                shape_ms = ms;
        }
        if (he == hipSuccess && (s == 0 || shape_ms < best_ms)) {
            best_ms = shape_ms;
            best = s;
        }
    }
    if (he != hipSuccess)
        rc = bhip(he, "autotune");
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipFree(arena);
    (void)hipFree(meta);
    (void)hipFree(err);
    (void)hipFree(sk_sum);
    (void)hipFree(sk_cnt);
    (void)hipFree(amp);
    (void)hipFree(amp_cnt);
    if (rc != ILG_OK)
        return rc;
    b->shape = best;
    if (chosen)
        *chosen = (uint32_t)best;
    return ILG_OK;
}

int ilg_batch_set_shape(ilg_batch *b, uint32_t shape)
{
    if (!b || shape >= (uint32_t)ilg::batch_shape_count())
        return bfail(ILG_E_INVALID, "bad batch or shape index");
    b->shape = (int)shape;
    return ILG_OK;
}

uint32_t ilg_batch_shape_count(void)
{
    return (uint32_t)ilg::batch_shape_count();
}

int ilg_batch_get_state(ilg_batch *b, uint32_t r, void *host_out)
{
    if (!b || !host_out || r >= b->nreal)
        return bfail(ILG_E_INVALID, "bad batch member or output");
    ilg::BatchMeta m;
    BHIP(hipMemcpyAsync(&m, b->meta + r, sizeof(m), hipMemcpyDeviceToHost, b->stream));
    BHIP(hipStreamSynchronize(b->stream));
    const size_t cb = b->cb;
    const unsigned char *src = reinterpret_cast<const unsigned char *>(b->arena) +
                               (m.off + (uint64_t)m.cur * b->q * m.pitch) * cb;
    BHIP(hipMemcpy2DAsync(host_out, (size_t)m.length * cb, src, (size_t)m.pitch * cb,
                          (size_t)m.length * cb, b->q, hipMemcpyDeviceToHost, b->stream));
    return sticky(b);
}

int ilg_batch_structure_factor(ilg_batch *b, double *sk_sum, uint64_t *count)
{
    if (!b || !sk_sum || !count)
        return bfail(ILG_E_INVALID, "null argument");
    if (b->diag.nk)
        BHIP(hipMemcpyAsync(sk_sum, b->sk_sum, (size_t)b->nreal * b->diag.nk * sizeof(double),
                            hipMemcpyDeviceToHost, b->stream));
    BHIP(hipMemcpyAsync(count, b->sk_cnt, (size_t)b->nreal * sizeof(uint64_t),
                        hipMemcpyDeviceToHost, b->stream));
    return sticky(b);
}

int ilg_batch_amplitudes(ilg_batch *b, double *amp, uint32_t *count)
{
    if (!b || !amp || !count)
        return bfail(ILG_E_INVALID, "null argument");
    if (b->diag.max_amp)
        BHIP(hipMemcpyAsync(amp, b->amp, (size_t)b->nreal * b->diag.max_amp * sizeof(double),
                            hipMemcpyDeviceToHost, b->stream));
    BHIP(hipMemcpyAsync(count, b->amp_cnt, (size_t)b->nreal * sizeof(uint32_t),
                        hipMemcpyDeviceToHost, b->stream));
    return sticky(b);
}

int ilg_batch_destroy(ilg_batch *b)
{
    if (!b)
        return ILG_OK;
    int rc = ILG_OK;
    if (hipStreamSynchronize(b->stream) == hipSuccess)
        rc = sticky(b);
    release(b);
    return rc;
}

}  // extern "C"
