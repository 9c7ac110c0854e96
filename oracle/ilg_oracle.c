/*
 * Plain CPU oracle for the diffusive integer lattice gas step with the flip
 * (over-relaxation) operator.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  The product
 * library never links it, and it shares no code, header, table or constant
 * generator with the product's HIP sources.
 *
 * What it computes (paper: Strand & Wagner, "Over-Relaxation in Diffusive
 * Integer Lattice Gas"):
 *   - lattice-gas evolution with flip, Eq. LGflip: each node first flips its
 *     occupations, F_i(n) = n_{-i} (Eq. flip, v_{-i} = -v_i), then a sampling
 *     collision redistributes a random fraction omega* of the particles to
 *     velocity i with probability w_i (Integer Lattice Gas section, the
 *     Seekins sampling collision; Over-relaxation section for omega*),
 *     then every count streams to x + v_i (Eq. ilgeq);
 *   - mass is the only conserved quantity (sum_i Xi_i = 0).
 *
 * Reading of the collision (the paper defers the algorithm to Seekins et al.):
 * every particle collides independently with probability p = P / 2^32; the
 * collided particles are redistributed multinomially with the weights w_i.
 * Sampling is in exact 32-bit fixed point:
 *   Bin(n, p): n is cut into chunks of 64 (full chunks first, remainder last);
 *   for a chunk of size m one 32-bit draw U is taken and the chunk's result is
 *   #{ j < m : T_p[m][j] <= U }, where T_p[m][j] = floor(2^32 * CDF_{m,p}(j)),
 *   supplied by the caller (built with exact big integers in exact.py).
 *   p = 0 is passed as a NULL table: the result is 0 but the draws are still
 *   consumed, so draw alignment does not depend on p.
 * D2Q5 (reading; the paper works the flip out in 1D and states that odd
 * moments change sign and even moments do not): velocities (-1,0), (0,-1),
 * (0,0), (0,+1), (+1,0), weights theta/2 for each mover and 1 - 2 theta at
 * rest; the collided particles go to rest with probability 1 - 2 theta, the
 * others to the x or the y pair with probability 1/2 and then to either
 * direction of the pair with probability 1/2 (conditional binomials, drawn
 * in that order).  Nodes are numbered x + Lx y.
 * D1Q2 exchange form (draw specification v3, a reformulation of the same
 * collision): a particle of either velocity is removed with probability p
 * and then sent to each velocity with probability 1/2, so it ends on the
 * opposite velocity with probability p/2, independently of the others.  The
 * exchange form draws that directly: X = Bin(a_-, p_x) particles cross from
 * -1 to +1, then Y = Bin(a_+, p_x) from +1 to -1, with p_x the fixed-point
 * crossing probability round(omega* 2^31) / 2^32 (two binomials per node
 * instead of three); c_- = a_- - X + Y, c_+ = a_+ - Y + X.
 * Draws (specification v1): Philox4x32-10 (Salmon, Moraes, Dror & Shaw,
 * SC'11); v2 uses the same generator with 7 rounds.  Key = the 64-bit
 * seed split into two 32-bit words (low word first), counter =
 * (node x, step t, realization r, block b).  Draw number j of a node-step is
 * word (j mod 4) of block j / 4.  Draw order within a node-step: removal
 * Bin(a_i, P) for i = 0..Q-1, then the redistribution binomials.
 *
 * This code is written to be checked by eye, not to be fast.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORACLE_CHUNK 64
#define ORACLE_TABLE_ENTRIES 2080 /* rows m = 1..64, m entries each */

/* ------------------------------------------------------------------ Philox */

/* Philox4x32 with 10 rounds.  Round: multiply words 0 and 2 by the two Philox
 * multipliers (full 64-bit products), then
 *   out0 = hi(M1*c2) ^ c1 ^ k0,  out1 = lo(M1*c2),
 *   out2 = hi(M0*c0) ^ c3 ^ k1,  out3 = lo(M0*c0);
 * the key is advanced by the two Weyl constants between rounds. */
void oracle_philox4x32(const uint32_t ctr_in[4], const uint32_t key_in[2], int rounds,
                       uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < rounds; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    oracle_philox4x32(ctr_in, key_in, 10, out);
}

/* The stream of 32-bit draws of one node-step. */
typedef struct {
    uint32_t key[2];
    uint32_t ctr[4];   /* x, t, r, block */
    uint32_t block[4];
    uint64_t used;     /* number of draws consumed so far */
    int rounds;        /* Philox rounds: 10 (specification v1) or 7 (v2) */
} draw_stream;

static void stream_init(draw_stream *s, uint64_t seed, uint32_t x, uint32_t t, uint32_t r,
                        int rounds)
{
    s->rounds = rounds;
    s->key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    s->key[1] = (uint32_t)(seed >> 32);
    s->ctr[0] = x;
    s->ctr[1] = t;
    s->ctr[2] = r;
    s->ctr[3] = 0;
    s->used = 0;
}

static uint32_t next_draw(draw_stream *s)
{
    uint64_t j = s->used;
    if (j % 4 == 0) {
        s->ctr[3] = (uint32_t)(j / 4);
        oracle_philox4x32(s->ctr, s->key, s->rounds, s->block);
    }
    s->used = j + 1;
    return s->block[j % 4];
}

/* ---------------------------------------------------------------- binomial */

static const uint32_t *table_row(const uint32_t *table, uint32_t m)
{
    return table + (size_t)(m - 1) * m / 2;
}

/* Bin(n, p) by chunked inverse CDF; table == NULL means p = 0. */
static uint64_t binomial(uint64_t n, const uint32_t *table, draw_stream *s)
{
    uint64_t total = 0;
    while (n > 0) {
        uint32_t m = n >= ORACLE_CHUNK ? ORACLE_CHUNK : (uint32_t)n;
        uint32_t U = next_draw(s);
        if (table != NULL) {
            const uint32_t *row = table_row(table, m);
            for (uint32_t j = 0; j < m; ++j)
                if (row[j] <= U)
                    total += 1;
        }
        n -= m;
    }
    return total;
}

/* ------------------------------------------------------------ node update */

typedef struct {
    int q;                     /* 2: v = (-1,+1); 3: v = (-1,0,+1);
                                  5 (D2Q5): v = (-1,0), (0,-1), (0,0), (0,+1), (+1,0) */
    int flip;                  /* apply F before the collision */
    const uint32_t *tab_p;     /* removal fraction P (NULL: P = 0) */
    const uint32_t *tab_half;  /* P = 2^31 */
    const uint32_t *tab_rest;  /* rest weight: P = (1 - theta) 2^32 for q = 3,
                                  (1 - 2 theta) 2^32 for q = 5 */
    uint64_t seed;
    uint32_t realization;
    int rounds;                /* Philox rounds of the step draws */
    int exchange;              /* D1Q2 exchange form; tab_p is then the table
                                  of the crossing probability p_x */
} oracle_params;

/* The `flip` word of the entry points: bit 0 applies the flip; bit 1 selects
 * the D1Q2 exchange form; bits 8..15 give the Philox round count of the step
 * draws (0 means 10, the draw specification v1; 7 selects v2). */
static oracle_params make_params(int q, int flipword, const uint32_t *tab_p,
                                 const uint32_t *tab_half, const uint32_t *tab_rest,
                                 uint64_t seed, uint32_t realization)
{
    const int rounds = (flipword >> 8) & 0xFF;
    oracle_params pp = {q, flipword & 1, tab_p, tab_half, tab_rest, seed, realization,
                        rounds ? rounds : 10, q == 2 && ((flipword >> 1) & 1)};
    return pp;
}

/* One node: flip, then removal binomials, then multinomial redistribution.
 * Returns the post-collision counts c_i = a_i - k_i + m_i (before streaming). */
static void collide_node(const oracle_params *pp, const uint64_t n_in[5], uint32_t x, uint32_t t,
                         uint64_t c_out[5])
{
    const int q = pp->q;
    uint64_t a[5] = {0, 0, 0, 0, 0}, k[5] = {0, 0, 0, 0, 0}, m[5] = {0, 0, 0, 0, 0};
    draw_stream s;
    stream_init(&s, pp->seed, x, t, pp->realization, pp->rounds);

    /* Flip, Eq. flip: a_i = n_{-i}; with the index orders above the mirror
     * of index i is q-1-i (in 2D: -x <-> +x, -y <-> +y, rest fixed). */
    for (int i = 0; i < q; ++i)
        a[i] = pp->flip ? n_in[q - 1 - i] : n_in[i];

    if (pp->exchange) {
        /* D1Q2 exchange form: X particles cross from -1 to +1, Y from +1 to
         * -1, each particle independently with probability p_x. */
        const uint64_t X = binomial(a[0], pp->tab_p, &s);
        const uint64_t Y = binomial(a[1], pp->tab_p, &s);
        c_out[0] = a[0] - X + Y;
        c_out[1] = a[1] - Y + X;
        return;
    }

    /* Each particle of velocity i collides with probability p. */
    uint64_t M = 0;
    for (int i = 0; i < q; ++i) {
        k[i] = binomial(a[i], pp->tab_p, &s);
        M += k[i];
    }

    /* The M collided particles go to velocity i with probability w_i. */
    if (q == 2) {
        m[0] = binomial(M, pp->tab_half, &s);   /* w_- = 1/2 */
        m[1] = M - m[0];
    } else if (q == 3) {
        m[1] = binomial(M, pp->tab_rest, &s);   /* w_0 = 1 - theta */
        uint64_t R = M - m[1];
        m[0] = binomial(R, pp->tab_half, &s);   /* w_- / (w_- + w_+) = 1/2 */
        m[2] = R - m[0];
    } else {
        /* D2Q5 weights: rest 1 - 2 theta, each mover theta / 2.  The movers
         * split into the x pair and the y pair (1/2 each), each pair into its
         * negative and positive direction (1/2 each). */
        m[2] = binomial(M, pp->tab_rest, &s);   /* w_0 = 1 - 2 theta */
        uint64_t R = M - m[2];
        uint64_t mx = binomial(R, pp->tab_half, &s);
        uint64_t my = R - mx;
        m[0] = binomial(mx, pp->tab_half, &s);  /* -x */
        m[4] = mx - m[0];                       /* +x */
        m[1] = binomial(my, pp->tab_half, &s);  /* -y */
        m[3] = my - m[1];                       /* +y */
    }
    for (int i = 0; i < q; ++i)
        c_out[i] = a[i] - k[i] + m[i];
}

static uint64_t load_count(const void *buf, int count_bytes, size_t idx)
{
    if (count_bytes == 2)
        return ((const uint16_t *)buf)[idx];
    return ((const uint32_t *)buf)[idx];
}

static void store_count(void *buf, int count_bytes, size_t idx, uint64_t v)
{
    if (count_bytes == 2)
        ((uint16_t *)buf)[idx] = (uint16_t)v;
    else
        ((uint32_t *)buf)[idx] = (uint32_t)v;
}

/* ----------------------------------------------------------- lattice step */

typedef struct {
    const oracle_params *pp;
    int count_bytes;
    uint64_t length;   /* global lattice length L (periodic) */
    uint64_t x0;       /* global index of window position 0 */
    uint64_t width;    /* window width W (== L for a whole periodic lattice) */
    int periodic;      /* 1: whole lattice, wrap; 0: window, drop what leaves */
    const void *in;    /* [q][W] */
    void *out;         /* [q][W] */
    uint32_t t;
    uint64_t w_begin, w_end;
    int overflow;
} step_job;

static void *step_worker(void *arg)
{
    step_job *job = (step_job *)arg;
    const int q = job->pp->q;
    const uint64_t maxval = job->count_bytes == 2 ? 0xFFFFu : 0xFFFFFFFFu;
    for (uint64_t w = job->w_begin; w < job->w_end; ++w) {
        uint64_t n[5] = {0, 0, 0, 0, 0}, c[5];
        for (int i = 0; i < q; ++i)
            n[i] = load_count(job->in, job->count_bytes, (size_t)i * job->width + w);
        uint32_t xg = (uint32_t)((job->x0 + w) % job->length);
        collide_node(job->pp, n, xg, job->t, c);
        for (int i = 0; i < q; ++i) {
            /* velocity of index i: -1, (0,) +1 */
            int64_t v = (q == 2) ? (i == 0 ? -1 : 1) : (int64_t)i - 1;
            int64_t dst = (int64_t)w + v;
            if (job->periodic) {
                dst = (dst + (int64_t)job->width) % (int64_t)job->width;
            } else if (dst < 0 || dst >= (int64_t)job->width) {
                continue;
            }
            if (c[i] > maxval)
                job->overflow = 1;
            store_count(job->out, job->count_bytes, (size_t)i * job->width + (size_t)dst, c[i]);
        }
    }
    return NULL;
}

/* One time step t -> t+1 over a window (or the whole periodic lattice).
 * In window mode the first and last node of `out` receive nothing from outside
 * and are set to 0; after s steps only nodes [s, W-s) are valid.
 * Returns 1 if any post-collision count exceeded the count type, else 0. */
int oracle_step(int q, int count_bytes, uint64_t length, uint64_t x0, uint64_t width, int periodic,
                int flip, const uint32_t *tab_p, const uint32_t *tab_half, const uint32_t *tab_rest,
                uint64_t seed, uint32_t realization, uint32_t t, const void *in, void *out,
                int nthreads)
{
    oracle_params pp = make_params(q, flip, tab_p, tab_half, tab_rest, seed, realization);
    if (!periodic)
        memset(out, 0, (size_t)q * width * (size_t)count_bytes);
    if (nthreads < 1)
        nthreads = 1;
    if ((uint64_t)nthreads > width)
        nthreads = (int)(width > 0 ? width : 1);
    step_job *jobs = (step_job *)calloc((size_t)nthreads, sizeof(step_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int k = 0; k < nthreads; ++k) {
        step_job j = {&pp, count_bytes, length, x0, width, periodic, in, out, t,
                      width * (uint64_t)k / (uint64_t)nthreads,
                      width * (uint64_t)(k + 1) / (uint64_t)nthreads, 0};
        jobs[k] = j;
    }
    for (int k = 1; k < nthreads; ++k)
        pthread_create(&th[k], NULL, step_worker, &jobs[k]);
    step_worker(&jobs[0]);
    for (int k = 1; k < nthreads; ++k)
        pthread_join(th[k], NULL);
    int overflow = 0;
    for (int k = 0; k < nthreads; ++k)
        overflow |= jobs[k].overflow;
    free(jobs);
    free(th);
    return overflow;
}

/* ------------------------------------------------------- D2Q5 lattice step */

/* One whole-lattice D2Q5 step on an Lx x Ly periodic lattice; state layout
 * [5][Ly][Lx] (node index x + Lx y, which is also the Philox counter word 0).
 * Velocity i moves to (x + vx_i mod Lx, y + vy_i mod Ly). */
typedef struct {
    const oracle_params *pp;
    int count_bytes;
    uint64_t lx, ly;
    const void *in;
    void *out;
    uint32_t t;
    uint64_t n_begin, n_end;
    int overflow;
} step2d_job;

static void *step2d_worker(void *arg)
{
    step2d_job *job = (step2d_job *)arg;
    static const int vx[5] = {-1, 0, 0, 0, 1}, vy[5] = {0, -1, 0, 1, 0};
    const uint64_t nodes = job->lx * job->ly;
    const uint64_t maxval = job->count_bytes == 2 ? 0xFFFFu : 0xFFFFFFFFu;
    for (uint64_t id = job->n_begin; id < job->n_end; ++id) {
        const uint64_t x = id % job->lx, y = id / job->lx;
        uint64_t n[5], c[5];
        for (int i = 0; i < 5; ++i)
            n[i] = load_count(job->in, job->count_bytes, (size_t)i * nodes + id);
        collide_node(job->pp, n, (uint32_t)id, job->t, c);
        for (int i = 0; i < 5; ++i) {
            const uint64_t xd = (x + job->lx + (uint64_t)(int64_t)vx[i]) % job->lx;
            const uint64_t yd = (y + job->ly + (uint64_t)(int64_t)vy[i]) % job->ly;
            if (c[i] > maxval)
                job->overflow = 1;
            store_count(job->out, job->count_bytes, (size_t)i * nodes + xd + job->lx * yd, c[i]);
        }
    }
    return NULL;
}

int oracle_step2d(int count_bytes, uint64_t lx, uint64_t ly, int flip, const uint32_t *tab_p,
                  const uint32_t *tab_half, const uint32_t *tab_rest, uint64_t seed,
                  uint32_t realization, uint32_t t, const void *in, void *out, int nthreads)
{
    oracle_params pp = make_params(5, flip, tab_p, tab_half, tab_rest, seed, realization);
    const uint64_t nodes = lx * ly;
    if (nthreads < 1)
        nthreads = 1;
    if ((uint64_t)nthreads > nodes)
        nthreads = (int)nodes;
    step2d_job *jobs = (step2d_job *)calloc((size_t)nthreads, sizeof(step2d_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int k = 0; k < nthreads; ++k) {
        step2d_job j = {&pp, count_bytes, lx, ly, in, out, t,
                        nodes * (uint64_t)k / (uint64_t)nthreads,
                        nodes * (uint64_t)(k + 1) / (uint64_t)nthreads, 0};
        jobs[k] = j;
    }
    for (int k = 1; k < nthreads; ++k)
        pthread_create(&th[k], NULL, step2d_worker, &jobs[k]);
    step2d_worker(&jobs[0]);
    for (int k = 1; k < nthreads; ++k)
        pthread_join(th[k], NULL);
    int overflow = 0;
    for (int k = 0; k < nthreads; ++k)
        overflow |= jobs[k].overflow;
    free(jobs);
    free(th);
    return overflow;
}

/* ------------------------------------------------------------------ hash */

static uint64_t splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Order-independent state fingerprint: sum over (x, i) of
 * splitmix64(((x*q + i) << 32) ^ n_i(x)) modulo 2^64. */
uint64_t oracle_hash(int q, int count_bytes, uint64_t length, const void *state)
{
    uint64_t h = 0;
    for (uint64_t x = 0; x < length; ++x)
        for (int i = 0; i < q; ++i) {
            uint64_t n = load_count(state, count_bytes, (size_t)i * length + x);
            h += splitmix64(((x * (uint64_t)q + (uint64_t)i) << 32) ^ n);
        }
    return h;
}

/* nsteps whole-lattice steps starting at absolute step t0; `state` is updated
 * in place.  If hashes != NULL, hashes[s] is the hash after step s+1.
 * Returns 1 on count overflow (state then undefined), else 0. */
int oracle_run(int q, int count_bytes, uint64_t length, int flip, const uint32_t *tab_p,
               const uint32_t *tab_half, const uint32_t *tab_rest, uint64_t seed,
               uint32_t realization, uint64_t t0, uint64_t nsteps, void *state, uint64_t *hashes,
               int nthreads)
{
    size_t bytes = (size_t)q * length * (size_t)count_bytes;
    void *tmp = malloc(bytes);
    int overflow = 0;
    for (uint64_t s = 0; s < nsteps; ++s) {
        overflow |= oracle_step(q, count_bytes, length, 0, length, 1, flip, tab_p, tab_half,
                                tab_rest, seed, realization, (uint32_t)(t0 + s), state, tmp,
                                nthreads);
        memcpy(state, tmp, bytes);
        if (hashes)
            hashes[s] = oracle_hash(q, count_bytes, length, state);
    }
    free(tmp);
    return overflow;
}

/* nsteps whole-lattice D2Q5 steps from absolute step t0, `state` [5][Ly][Lx]
 * updated in place; hashes[s] (if not NULL) is the hash after step s+1 (node
 * index x + Lx y).  Returns 1 on count overflow. */
int oracle_run2d(int count_bytes, uint64_t lx, uint64_t ly, int flip, const uint32_t *tab_p,
                 const uint32_t *tab_half, const uint32_t *tab_rest, uint64_t seed,
                 uint32_t realization, uint64_t t0, uint64_t nsteps, void *state,
                 uint64_t *hashes, int nthreads)
{
    const size_t bytes = (size_t)5 * lx * ly * (size_t)count_bytes;
    void *tmp = malloc(bytes);
    int overflow = 0;
    for (uint64_t s = 0; s < nsteps; ++s) {
        overflow |= oracle_step2d(count_bytes, lx, ly, flip, tab_p, tab_half, tab_rest, seed,
                                  realization, (uint32_t)(t0 + s), state, tmp, nthreads);
        memcpy(state, tmp, bytes);
        if (hashes)
            hashes[s] = oracle_hash(5, count_bytes, lx * ly, state);
    }
    free(tmp);
    return overflow;
}

/* Window run for light-cone sampling: `state` holds [q][width] counts of the
 * global nodes x0 .. x0+width-1 (mod length) at step t0; after nsteps steps the
 * nodes [nsteps, width-nsteps) hold the exact state of those global nodes. */
int oracle_run_window(int q, int count_bytes, uint64_t length, uint64_t x0, uint64_t width,
                      int flip, const uint32_t *tab_p, const uint32_t *tab_half,
                      const uint32_t *tab_rest, uint64_t seed, uint32_t realization, uint64_t t0,
                      uint64_t nsteps, void *state, int nthreads)
{
    size_t bytes = (size_t)q * width * (size_t)count_bytes;
    void *tmp = malloc(bytes);
    int overflow = 0;
    for (uint64_t s = 0; s < nsteps; ++s) {
        overflow |= oracle_step(q, count_bytes, length, x0, width, 0, flip, tab_p, tab_half,
                                tab_rest, seed, realization, (uint32_t)(t0 + s), state, tmp,
                                nthreads);
        memcpy(state, tmp, bytes);
    }
    free(tmp);
    return overflow;
}

/* ---------------------------------------------- sampler-level entry points */

/* One node-step collision (no streaming): c_out[i] for input counts n_in. */
void oracle_collide_node(int q, int flip, const uint32_t *tab_p, const uint32_t *tab_half,
                         const uint32_t *tab_rest, uint64_t seed, uint32_t realization,
                         uint32_t x, uint32_t t, const uint64_t *n_in, uint64_t *c_out)
{
    oracle_params pp = make_params(q, flip, tab_p, tab_half, tab_rest, seed, realization);
    uint64_t n[5] = {0, 0, 0, 0, 0}, c[5] = {0, 0, 0, 0, 0};
    for (int i = 0; i < q; ++i)
        n[i] = n_in[i];
    collide_node(&pp, n, x, t, c);
    for (int i = 0; i < q; ++i)
        c_out[i] = c[i];
}

/* nsamples collisions of the same input, sample s keyed at node x = s. */
void oracle_collide_samples(int q, int flip, const uint32_t *tab_p, const uint32_t *tab_half,
                            const uint32_t *tab_rest, uint64_t seed, uint32_t realization,
                            uint32_t t, const uint64_t *n_in, uint64_t nsamples, uint64_t *c_out)
{
    oracle_params pp = make_params(q, flip, tab_p, tab_half, tab_rest, seed, realization);
    uint64_t n[5] = {0, 0, 0, 0, 0};
    for (int i = 0; i < q; ++i)
        n[i] = n_in[i];
    for (uint64_t s = 0; s < nsamples; ++s) {
        uint64_t c[5] = {0, 0, 0, 0, 0};
        collide_node(&pp, n, (uint32_t)s, t, c);
        for (int i = 0; i < q; ++i)
            c_out[s * (uint64_t)q + (uint64_t)i] = c[i];
    }
}

/* nsamples draws of Bin(n, p), sample s keyed at counter (s, 0, 0, b). */
void oracle_binomial_samples(uint64_t n, const uint32_t *table, uint64_t seed, uint64_t nsamples,
                             uint64_t *out)
{
    for (uint64_t s = 0; s < nsamples; ++s) {
        draw_stream st;
        stream_init(&st, seed, (uint32_t)s, 0, 0, 10);
        out[s] = binomial(n, table, &st);
    }
}

/* ------------------------------------------------ Poisson sine initialisation
 *
 * The paper's initial state (Results, the sine density profile): occupation
 * n_i(x) is a Poisson variate with expectation w_i times the density profile
 * N [1 + sin(2 pi x / L)]; here with a general amplitude A,
 *   mean_i(x) = w_i (N + A sin(2 pi x / L)).
 * Reading (a specification fixed here and in the library, "init v1"): so
 * that two IEEE-754 machines draw the same counts, every floating-point step
 * below is one correctly rounded double operation (no fused multiply-add, no
 * library transcendental):
 *   sin(2 pi x / L): 8x = k L + rem with integers (octant k); for even k
 *     t = rem / L, for odd k t = (L - rem) / L (the distance to the octant's
 *     end, again from integers); a = t * (pi/4), a2 = a * a,
 *     S = a * (1 + a2 (s1 + a2 (s2 + ... + a2 s8))),  s_j = (-1)^j / (2j+1)!
 *     C = 1 + a2 (c1 + a2 (c2 + ... + a2 c9)),         c_j = (-1)^j / (2j)!
 *     (Horner from the innermost coefficient); the value for k = 0..7 is
 *     S, C, C, S, -S, -C, -C, -S;
 *   e^-m for 0 <= m <= 256 (Cody-Waite reduction): n = (int)(m log2(e) + 0.5),
 *     r = (m - n ln2_hi) - n ln2_lo, e^-r = sum_{j=0..17} (-r)^j / j! (Horner),
 *     times 2^-n;
 *   mean = w_i * (N + A * value); mean <= 0 gives 0;
 *   parts P = max(1, ceil(mean / 256)), m = mean / P, and per part p a Philox
 *   block with key = init seed, counter = (x, p, realization, 2^31 + i / 4);
 *   word i mod 4 is the part's draw u, U = (u + 1/2) 2^-32, and the part's
 *   count is the
 *   least k with U <= F(k), F(0) = f(0) = e^-m, f(k) = (f(k-1) m) / k,
 *   F(k) = F(k-1) + f(k) (the Poisson CDF by its recurrence), capped at 10^5;
 *   n_i(x) = the sum over the parts (a sum of independent Poisson(m) is
 *   Poisson(mean)).
 * D2Q5: nodes x + Lx y; the profile runs along the column x = node mod Lx
 * (sine of the column), the counter's word 0 is the node.
 * Coefficients 1/j! are 1.0 / j! with j! exact in double (j <= 18).  The
 * counter's last word 2^31 keeps these blocks apart from the step's draw
 * blocks (whose last word is a small block index). */

static const double ORACLE_PI_4 = 0x1.921fb54442d18p-1;  /* pi / 4 */
static const double ORACLE_LOG2E = 0x1.71547652b82fep+0; /* log2(e) */
static const double ORACLE_LN2_HI = 0x1.62e42feep-1;     /* ln 2, upper bits */
static const double ORACLE_LN2_LO = 0x1.a39ef35793c76p-33; /* ln 2 - ln2_hi */

static double inv_factorial(int j)
{
    double f = 1.0;
    for (int i = 2; i <= j; ++i)
        f = f * (double)i;
    return 1.0 / f;
}

/* sin(2 pi x / L) for integers 0 <= x < L */
double oracle_sin2pi_frac(uint64_t x, uint64_t L)
{
    const uint64_t eight_x = 8 * x;
    const uint64_t k = eight_x / L, rem = eight_x % L;
    const double t = (double)(k % 2 == 0 ? rem : L - rem) / (double)L;
    const double a = t * ORACLE_PI_4;
    const double a2 = a * a;
    double hs = (8 % 2 ? -1.0 : 1.0) * inv_factorial(17);   /* s8 = +1/17! */
    for (int j = 7; j >= 1; --j)
        hs = (j % 2 ? -1.0 : 1.0) * inv_factorial(2 * j + 1) + a2 * hs;
    hs = 1.0 + a2 * hs;
    const double S = a * hs;
    double hc = (9 % 2 ? -1.0 : 1.0) * inv_factorial(18);   /* c9 = -1/18! */
    for (int j = 8; j >= 1; --j)
        hc = (j % 2 ? -1.0 : 1.0) * inv_factorial(2 * j) + a2 * hc;
    const double C = 1.0 + a2 * hc;
    switch (k) {
    case 0: return S;
    case 1: return C;
    case 2: return C;
    case 3: return S;
    case 4: return -S;
    case 5: return -C;
    case 6: return -C;
    default: return -S;
    }
}

/* e^-m for 0 <= m <= 256 */
double oracle_exp_neg(double m)
{
    const int n = (int)(m * ORACLE_LOG2E + 0.5);
    const double r = (m - (double)n * ORACLE_LN2_HI) - (double)n * ORACLE_LN2_LO;
    const double y = -r;
    double h = inv_factorial(17);
    for (int j = 16; j >= 0; --j)
        h = inv_factorial(j) + y * h;
    return ldexp(h, -n);
}

/* Poisson(m) by the inverse CDF, 0 < m <= 256, from one 32-bit draw */
static uint64_t poisson_part(double m, uint32_t u)
{
    const double U = ((double)u + 0.5) * 0x1p-32;
    double f = oracle_exp_neg(m);
    double F = f;
    uint64_t k = 0;
    while (U > F && k < 100000) {
        k += 1;
        f = (f * m) / (double)k;
        F = F + f;
    }
    return k;
}

/* Counts of nodes x0 .. x0+width-1 (taken mod the node count `length`) into
 * out[q][width] (count type count_bytes); weights w[0..q-1]; row length
 * `row` (the profile's period: L in 1D, Lx for D2Q5).  Returns 1 if a count
 * exceeds the count type (the stored value is then truncated), else 0. */
int oracle_init_poisson_sine(int q, int count_bytes, uint64_t length, uint64_t row, uint64_t x0,
                             uint64_t width, const double *w, double nave, double amp,
                             uint64_t seed, uint32_t realization, void *out)
{
    const uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    const uint64_t maxv = count_bytes == 2 ? 0xFFFFu : 0xFFFFFFFFu;
    int overflow = 0;
    for (uint64_t k = 0; k < width; ++k) {
        const uint64_t x = (x0 + k) % length;
        const double s = oracle_sin2pi_frac(x % row, row);
        const double rho = nave + amp * s;
        for (int i = 0; i < q; ++i) {
            const double mean = w[i] * rho;
            uint64_t n = 0;
            if (mean > 0.0) {
                const double parts_d = ceil(mean / 256.0);
                const uint32_t parts = parts_d < 1.0 ? 1u : (uint32_t)parts_d;
                const double m = mean / (double)parts;
                for (uint32_t p = 0; p < parts; ++p) {
                    const uint32_t ctr[4] = {(uint32_t)x, p, realization,
                                             0x80000000u + (uint32_t)(i / 4)};
                    uint32_t blk[4];
                    oracle_philox4x32_10(ctr, key, blk);
                    n += poisson_part(m, blk[i % 4]);
                }
            }
            if (n > maxv)
                overflow = 1;
            store_count(out, count_bytes, (size_t)i * width + k, n);
        }
    }
    return overflow;
}
