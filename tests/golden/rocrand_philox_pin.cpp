// Test helper: prints rocRAND's Philox4x32-10 output for (counter, key) pairs
// read from stdin, one "c0 c1 c2 c3 k0 k1" line each (decimal).  rocRAND's
// engine starts at counter (0, 0, subsequence_lo, subsequence_hi), and an
// offset of 4*n numbers adds n to the 64-bit low half of the counter, so
// rocrand_init(key, c2 + 2^32 c3, 4 (c0 + 2^32 c1)) lands exactly on the
// counter (c0, c1, c2, c3); the next four rocrand() calls return its block.
#include <cstdio>
#include <rocrand/rocrand_kernel.h>

int main()
{
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        rocrand_state_philox4x32_10 st;
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long subseq = c2 | (c3 << 32);
        rocrand_init(seed, subseq, 4ull * c0, &st);
        for (int k = 0; k < 4; ++k)
            skipahead(c1 << 32, &st);
        unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
