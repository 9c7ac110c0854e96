/* Test driver for sanitizer builds of the oracle (ASan/UBSan, TSan): reads
 * fixed-point tables written by the test, runs periodic and window steps with
 * several threads and prints the state hash.  Usage:
 *   oracle_driver TABLES_FILE Q LENGTH STEPS FLIP NTHREADS SEED */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_run(int q, int count_bytes, uint64_t length, int flip, const uint32_t *tab_p,
               const uint32_t *tab_half, const uint32_t *tab_rest, uint64_t seed,
               uint32_t realization, uint64_t t0, uint64_t nsteps, void *state, uint64_t *hashes,
               int nthreads);
int oracle_run_window(int q, int count_bytes, uint64_t length, uint64_t x0, uint64_t width,
                      int flip, const uint32_t *tab_p, const uint32_t *tab_half,
                      const uint32_t *tab_rest, uint64_t seed, uint32_t realization, uint64_t t0,
                      uint64_t nsteps, void *state, int nthreads);

int main(int argc, char **argv)
{
    if (argc != 8)
        return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f)
        return 2;
    static uint32_t tabs[3 * 2080];
    if (fread(tabs, sizeof(uint32_t), 3 * 2080, f) != 3 * 2080)
        return 2;
    fclose(f);
    const int q = atoi(argv[2]);
    const uint64_t L = strtoull(argv[3], NULL, 10), T = strtoull(argv[4], NULL, 10);
    const int flip = atoi(argv[5]), nth = atoi(argv[6]);
    const uint64_t seed = strtoull(argv[7], NULL, 10);
    uint16_t *st = malloc(sizeof(uint16_t) * q * L);
    for (uint64_t i = 0; i < (uint64_t)q * L; ++i)
        st[i] = (uint16_t)(20 + (i * 2654435761u >> 27) % 40);
    uint64_t *hashes = malloc(sizeof(uint64_t) * T);
    int ov = oracle_run(q, 2, L, flip, tabs, tabs + 2080, tabs + 4160, seed, 3, 0, T, st, hashes,
                        nth);
    const uint64_t W = L / 2 + 7;
    uint16_t *win = malloc(sizeof(uint16_t) * q * W);
    for (uint64_t i = 0; i < (uint64_t)q * W; ++i)
        win[i] = st[i % ((uint64_t)q * L)];
    ov |= oracle_run_window(q, 2, L, 5, W, flip, tabs, tabs + 2080, tabs + 4160, seed, 3, T,
                            T / 2, win, nth);
    printf("%llu %d\n", (unsigned long long)hashes[T - 1], ov);
    free(st);
    free(hashes);
    free(win);
    return 0;
}
