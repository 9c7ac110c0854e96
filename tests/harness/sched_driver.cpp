// Sanitizer driver for the serving scheduler: a random workload through the
// counting executor of sched_harness.cpp; exits non-zero on any violation.
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
void *h_new(uint64_t budget, uint32_t quantum);
void h_free(void *h);
int h_submit(void *h, uint32_t q, uint64_t bytes, uint64_t steps, uint64_t *id);
int h_poll(void *h, uint32_t *out4);
int h_cancel(void *h, uint64_t id);
int h_release(void *h, uint64_t id);
uint64_t h_used(void *h);
int h_violations(void *h);
}

int main()
{
    std::mt19937_64 rng(11);
    void *h = h_new(300000, 9);
    uint32_t st[4];
    std::vector<uint64_t> ids;
    for (int it = 0; it < 3000; ++it) {
        uint64_t id;
        if (rng() % 3 != 0 && h_submit(h, 2 + rng() % 2, 1 + rng() % 80000, 1 + rng() % 100, &id) == 0)
            ids.push_back(id);
        if (!ids.empty() && rng() % 17 == 0)
            h_cancel(h, ids[rng() % ids.size()]);
        h_poll(h, st);
        if (rng() % 5 == 0 && !ids.empty())
            h_release(h, ids[rng() % ids.size()]);
    }
    do {
        h_poll(h, st);
    } while (st[1] || st[2]);
    const int v = h_violations(h);
    const uint64_t used = h_used(h);
    h_free(h);
    std::printf("violations=%d used=%llu\n", v, (unsigned long long)used);
    return (v == 0 && used == 0) ? 0 : 1;
}
