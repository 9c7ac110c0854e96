/*
 * ilg.h -- C ABI of the MI355X (gfx950) diffusive integer lattice gas library.
 *
 * The library advances integer occupation numbers n_i(x, t) of a periodic 1D
 * lattice (D1Q2, D1Q3) or 2D lattice (D2Q5, an extension by the paper's
 * general rule that the flip changes the sign of odd velocity moments only)
 * by the lattice-gas evolution with the flip operator of Strand &
 * Wagner, "Over-Relaxation in Diffusive Integer Lattice Gas":
 *   n_i(x + v_i, t + 1) = F_i(n) + Xi_i({F(n)})            (Eq. LGflip)
 * where F_i(n) = n_{-i} (Eq. flip) and Xi is the sampling collision of the
 * Integer Lattice Gas section: a fraction omega* of the particles, each picked
 * independently, is redistributed to velocity i with probability w_i.  Mass is
 * the only conserved quantity (sum_i Xi_i = 0).  The relaxation rate of the
 * current is omega^j = 2 - omega* with the flip (Eq. omegaj), omega* without,
 * and the density obeys diffusion with D = theta (1/omega^j - 1/2).
 *
 * Sampling is exact 32-bit fixed point with Philox4x32-10 draws keyed by
 * (seed; node x, step t, realization r, block b), so every run is
 * bit-reproducible and independent of launch shapes, batching or placement.
 *
 * Conventions for every function:
 *   - Return value: ILG_OK (0) or a negative ilg_status.  No exception or abort
 *     crosses the ABI; ilg_last_error() gives a thread-local message.
 *   - Host pointers are read or written before the call returns unless stated;
 *     device pointers are HIP device addresses on the handle's device.
 *   - "stream" arguments are hipStream_t values (NULL: the legacy default
 *     stream).  Work is enqueued on that stream; functions marked "syncs"
 *     wait for it.
 *   - A handle must not be used from two threads at once; distinct handles may.
 *   - Device-side errors (a count exceeding its type) are sticky: they are
 *     reported as ILG_E_OVERFLOW by the next syncing call, and the state is
 *     undefined afterwards.
 */
#ifndef ILG_H
#define ILG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ILG_ABI_VERSION 1u
#define ILG_MAX_K 64u          /* largest structure-factor mode count */
#define ILG_TABLE_ENTRIES 2080u /* fixed-point CDF table: rows m = 1..64 */

typedef enum ilg_status {
    ILG_OK = 0,
    ILG_E_INVALID = -1,  /* bad argument or configuration */
    ILG_E_NOMEM = -2,    /* device or host allocation failed */
    ILG_E_DEVICE = -3,   /* a HIP call failed */
    ILG_E_OVERFLOW = -4, /* a post-collision count exceeded the count type */
    ILG_E_RANGE = -5,    /* step index would pass 2^32 - 1 */
    ILG_E_BUSY = -6      /* resource budget exhausted (serving) */
} ilg_status;

/* ilg_config.flags */
#define ILG_FLIP_AUTO 0u  /* flip iff omega > 1 (over-relaxation) */
#define ILG_FLIP_OFF 1u   /* never flip; needs omega <= 1 */
#define ILG_FLIP_ON 2u    /* always flip; needs omega >= 1 */
#define ILG_FLIP_MASK 3u
/* Draw specification v2: the step draws come from Philox4x32 with 7 rounds
 * instead of 10 (same counters, key and word order); the generator's authors
 * report that seven rounds pass their statistical test batteries.  A
 * different but equally valid random stream (the collision law of the
 * Integer Lattice Gas section is unchanged), with 30% fewer Philox rounds
 * per node.  Every form:
 * plain, batched (all members of a batch share the flag) and served.
 * Device-drawn initial states keep the 10-round generator. */
#define ILG_DRAWS_PHILOX7 4u
/* Draw specification v3, D1Q2 only: the exchange form of the same collision.
 * A particle removed with probability omega* and sent to either velocity with
 * probability 1/2 ends on the opposite velocity with probability omega* / 2;
 * the step draws the crossing counts directly, X = Bin(a_-, p_x) from -1 to
 * +1 and then Y = Bin(a_+, p_x) from +1 to -1 (chunked as every binomial),
 * with p_x = round-half-even(omega* 2^31) / 2^32, and sets c_- = a_- - X + Y,
 * c_+ = a_+ - Y + X: two binomials per node instead of three.  Combines with
 * ILG_DRAWS_PHILOX7.  Plain, batched (all members of a batch share the flag)
 * and served forms; other q reject it (ILG_E_INVALID). */
#define ILG_DRAWS_EXCHANGE 8u

/* One lattice run.  Velocity index order is fixed: q = 2 -> v = (-1, +1),
 * q = 3 -> v = (-1, 0, +1), q = 5 -> v = (-1,0), (0,-1), (0,0), (0,+1),
 * (+1,0); the mirror -v_i of index i is always index q-1-i.  Weights:
 * (1/2, 1/2), (theta/2, 1-theta, theta/2) and (theta/2, theta/2, 1-2 theta,
 * theta/2, theta/2); theta is the second velocity moment of the weights
 * (Eq. Thetadef, per axis in 2D) and D1Q3 uses the transformation matrix of
 * Eq. transform.  A D2Q5 lattice has length x height nodes numbered
 * x + length y; the collided particles go to rest with probability
 * 1 - 2 theta, else to the x or y pair (1/2 each), then to either direction
 * (1/2 each). */
typedef struct ilg_config {
    uint32_t abi_version; /* ILG_ABI_VERSION */
    uint32_t q;           /* 2, 3 or 5 */
    uint32_t count_bytes; /* 2 (uint16 counts) or 4 (uint32 counts) */
    uint32_t flags;       /* one ILG_FLIP_* mode, optionally | ILG_DRAWS_PHILOX7
                             | ILG_DRAWS_EXCHANGE */
    uint64_t length;      /* L (1D) or Lx (D2Q5), periodic; nodes < 2^31 */
    double omega;         /* target rate omega^j in (0, 2]; with the flip the
                             collision fraction is omega* = 2 - omega, else
                             omega* = omega (Over-relaxation section) */
    double theta;         /* q = 3: in (0, 1); q = 5: in (0, 1/2); 0 selects
                             1/3; ignored for q = 2 */
    uint64_t seed;        /* Philox key (low word, high word) */
    uint32_t realization; /* Philox counter word 2 */
    uint32_t height;      /* D2Q5: Ly >= 1 (periodic); must be 0 for q = 2, 3 */
    uint64_t t0;          /* absolute index of the first step to take */
} ilg_config;

/* Fixed-point form of a configuration. */
typedef struct ilg_fixed {
    uint32_t flip;     /* 1 if the flip is applied */
    uint32_t q;
    uint64_t p;        /* round-half-even(omega* 2^32), in [0, 2^32]; with
                          ILG_DRAWS_EXCHANGE the crossing probability
                          round-half-even(omega* 2^31) */
    uint64_t p_half;   /* 2^31 */
    uint64_t p_rest;   /* round-half-even(w_rest 2^32): 1 - theta (q = 3),
                          1 - 2 theta (q = 5) */
    double omega_star;
} ilg_fixed;

/* Reductions of the current state. */
typedef struct ilg_summary {
    uint64_t mass;      /* sum over x, i of n_i(x) (exact) */
    uint64_t step;      /* absolute step index of the state */
    uint64_t hash;      /* sum of splitmix64(((x q + i) << 32) ^ n_i(x)) mod 2^64 */
    double amplitude;   /* A^LG = sum_x sin(2 pi x/L) N(x) / sum_x sin^2(2 pi x/L);
                           D2Q5: sums over all nodes with x the column */
    uint32_t nk;        /* number of S(k) values filled */
    uint32_t reserved;
    double sk[ILG_MAX_K]; /* S(k) = |sum_x N(x) e^{-2 pi i k x/L}|^2 / sum_x N(x), k = 1..nk
                             (D2Q5: modes along x, sums over all nodes) */
} ilg_summary;

typedef struct ilg_handle ilg_handle; /* opaque; owned by the library */

/* Message of the last failing call on this thread ("" if none). */
const char *ilg_last_error(void);

/* Fixed-point parameters for cfg (host only, no device work). */
int ilg_fixed_point(const ilg_config *cfg, ilg_fixed *out);

/* Exact table T_p[m][j] = floor(2^32 CDF_{m, p/2^32}(j)), m = 1..64,
 * j = 0..m-1, row m at offset (m-1)m/2, written to out[ILG_TABLE_ENTRIES]
 * (host).  p in (0, 2^32]; p = 0 has no table (ILG_E_INVALID). */
int ilg_binomial_table(uint64_t p, uint32_t *out);

/* Device layout of a lattice state: velocity-major [q][pitch] counts of
 * count_bytes each over the nodes (L, or Lx Ly for D2Q5, node x + Lx y),
 * pitch = the node count rounded up to a multiple of 64; entries beyond the
 * last node are padding and never read.  Returns the byte size. */
uint64_t ilg_state_bytes(const ilg_config *cfg);
uint64_t ilg_state_pitch(const ilg_config *cfg);

/* Create a lattice: the integer occupation numbers n_i(x, t0) of the
 * Integer Lattice Gas section (one count per node and velocity) and the
 * configuration's collision fraction and flip (Over-relaxation section).
 * init_host is [q][nodes] counts (compact, count_bytes each; D2Q5
 * [5][Ly][Lx]), copied before return, or NULL for an all-zero state (to be
 * replaced by ilg_init_poisson_sine).  Device buffers, tables and the error
 * word are owned by the handle.  *out is NULL on failure.  ILG_E_INVALID for
 * a bad configuration, ILG_E_NOMEM / ILG_E_DEVICE if device memory or a copy
 * fails. */
int ilg_create(const ilg_config *cfg, const void *init_host, void *stream, ilg_handle **out);

/* Create a lattice on caller-owned device buffers of ilg_state_bytes(cfg)
 * each.  buf0 must already hold the initial state in the device layout; buf1
 * is scratch.  The buffers are borrowed: they must outlive the handle and are
 * never freed by the library. */
int ilg_create_on(const ilg_config *cfg, void *buf0, void *buf1, void *stream, ilg_handle **out);

/* Device address of the buffer holding the current state (device layout). */
void *ilg_state_device(const ilg_handle *h);

/* Enqueue nsteps time steps on the handle's stream (asynchronous): each is
 * Eq. LGflip at every node (the flip of Eq. flip, then the sampling collision
 * of the Integer Lattice Gas section with fraction omega*), followed by the
 * streaming of Eq. ilgeq, n_i(x + v_i, t + 1) <- c_i(x).  Draws use the
 * absolute step index, so the split of steps over calls does not matter.
 * ILG_E_RANGE (nothing enqueued) if the step index would pass 2^32 - 1;
 * ILG_E_DEVICE if a launch fails; a count overflow is reported later by a
 * syncing call. */
int ilg_step(ilg_handle *h, uint64_t nsteps);

/* Copy the current occupations n_i(x, t) (Integer Lattice Gas section) to
 * host_out, [q][nodes] compact counts of count_bytes each (D2Q5
 * [5][Ly][Lx]); caller-owned.  Syncs; ILG_E_OVERFLOW if an earlier step
 * overflowed (the copied state is then undefined). */
int ilg_get_state(ilg_handle *h, void *host_out);

/* Replace the state by host [q][nodes] counts and set the absolute step index of
 * the next step to t (checkpoint restore).  Syncs. */
int ilg_set_state(ilg_handle *h, const void *host_in, uint64_t t);

/* Replace the state by the paper's Poisson sine initial condition drawn on
 * the device (Results section, the sinusoidal initial density with integer
 * occupations): n_i(x) ~ Poisson(w_i (nave + amp sin(2 pi x / L))) with the
 * configuration's weights (D2Q5: the profile along x, x the column), drawn
 * with Philox4x32-10 keyed by init_seed (independent of the step seed) and
 * the configuration's realization.  The arithmetic is fixed ("init v1":
 * correctly rounded double operations only, no library transcendental), so
 * the counts are reproducible bit for bit on any IEEE-754 machine.
 * Requires 0 <= nave <= 1e6 and |amp| <= nave (ILG_E_INVALID otherwise);
 * ILG_E_OVERFLOW if a count exceeds the count type, the state then being
 * left unchanged.  The step index is not changed; the sticky error word is
 * cleared.  Syncs. */
int ilg_init_poisson_sine(ilg_handle *h, double nave, double amp, uint64_t init_seed);

/* Reductions of the current state (device kernels, then a small copy).
 * rho, j, e: optional host arrays of one int64 per node receiving the raw
 * moments sum_i n_i, sum_i v_i n_i, sum_i v_i^2 n_i (D2Q5: the x component
 * v_ix in j, |v_i|^2 in e) (NULL to skip).
 * nk <= ILG_MAX_K structure-factor modes are computed.  Syncs. */
int ilg_moments(ilg_handle *h, int64_t *rho, int64_t *j, int64_t *e, uint32_t nk,
                ilg_summary *out);

/* Order-independent 64-bit fingerprint of the current occupations (the
 * state of Eq. ilgeq): the sum over nodes x and velocities i of
 * splitmix64(((x q + i) << 32) ^ n_i(x)) modulo 2^64, with the SplitMix64
 * finaliser of Steele, Lea & Flood.  Equal states give equal hashes, so runs
 * can be compared step by step without copying states.  Syncs; sticky errors
 * as ilg_get_state. */
int ilg_state_hash(ilg_handle *h, uint64_t *out);

/* Absolute index of the next step. */
uint64_t ilg_current_step(const ilg_handle *h);

/* End a lattice run (the evolution of Eq. LGflip stops): wait for the
 * handle's work, report a sticky overflow (ILG_E_OVERFLOW) of the steps not
 * yet checked, and free what the handle owns (borrowed buffers of
 * ilg_create_on are left to the caller).  h is invalid afterwards, whatever
 * the return value; NULL is accepted. */
int ilg_destroy(ilg_handle *h);


/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the steps
 * of ilg_step on caller-owned state buffers, with no handle.  The fixed-point
 * table set the step kernel stages into LDS and the sticky error word live
 * in a fixed device array of the library, ILG_NOALLOC_SCRATCH_BYTES on each
 * device the library runs on, held until the process ends; its use does not
 * grow with the lattice (nodes < 2^31, as ilg_create).
 *   cfg: as ilg_create; cfg->t0 is the absolute index of the first step.
 *   buf0, buf1: distinct device buffers of ilg_state_bytes(cfg) each in the
 *     device layout; buf0 holds the state at t0 and both are rewritten; after
 *     nsteps steps the state is in buf0 if nsteps is even, else in buf1.
 *   stream: hipStream_t (NULL: the legacy default stream); the copy of the
 *     call's tables and the steps are enqueued on it.
 *   sync = 0: return after enqueueing (a count overflow stays recorded in the
 *     error word); sync != 0: wait, then return ILG_E_OVERFLOW if a count
 *     exceeded its type in this or an earlier call since the last report,
 *     which clears the word.
 * Calls no allocating routine.  Every call on one device shares its array
 * and rewrites its tables: calls that overlap on one device (concurrent
 * streams or threads) race.  Results equal ilg_create_on + ilg_step.
 * ILG_E_INVALID / ILG_E_RANGE as ilg_create and ilg_step. */
#define ILG_NOALLOC_SCRATCH_BYTES 76032u
int ilg_step_noalloc(const ilg_config *cfg, void *buf0, void *buf1, uint64_t nsteps, void *stream,
                     uint32_t sync);


/* ------------------------------------------------------------------------
 * Batched ensembles: many independent realizations (the ensemble average of
 * the Integer Lattice Gas section), each with its own length, relaxation
 * rate, seed, realization id and start step, advanced by one persistent
 * launch captured in a HIP graph.  All members share q, count_bytes, theta
 * and the draw specification flags (ILG_DRAWS_*).  Every member's result is bit-identical to the same configuration
 * run alone through ilg_create/ilg_step (draws depend only on the member's
 * own seed, realization, step and node).
 * ---------------------------------------------------------------------- */
#define ILG_BATCH_MAX_K 16u

typedef struct ilg_batch ilg_batch; /* opaque; owned by the library */

typedef struct ilg_batch_diag {
    uint32_t sk_every;  /* add S(k), k = 1..nk, to each member's sum every
                           sk_every steps of its own step count (0: off) */
    uint32_t nk;        /* 1..ILG_BATCH_MAX_K when sk_every > 0 */
    uint32_t amp_every; /* record A^LG every amp_every steps (0: off) */
    uint32_t max_amp;   /* capacity of each member's amplitude series */
} ilg_batch_diag;

/* cfgs[nreal] and inits[nreal] (host [q][L_r] compact counts, copied before
 * return; [5][height][length] for D2Q5).  diag may be NULL (no
 * diagnostics).  q = 2, 3 or 5; S(k) and A^LG are defined along a 1D
 * lattice, so a D2Q5 batch with sk_every or amp_every set is refused
 * (ILG_E_INVALID). */
int ilg_batch_create(const ilg_config *cfgs, uint32_t nreal, const void *const *inits,
                     const ilg_batch_diag *diag, void *stream, ilg_batch **out);

/* Advance every member by nsteps: one persistent launch (members taken
 * longest first from a device queue), replayed from a HIP graph. */
int ilg_batch_run(ilg_batch *b, uint64_t nsteps);

/* Autotuner: time each launch shape for tune_steps steps on a scratch copy of
 * the ensemble (the ensemble itself is not advanced) and keep the fastest for
 * later ilg_batch_run calls.  *chosen (nullable) receives the shape index.
 * Shapes differ only in speed, never in results.  Syncs. */
int ilg_batch_tune(ilg_batch *b, uint32_t tune_steps, uint32_t *chosen);

/* Launch shape used by later ilg_batch_run calls (an index below
 * ilg_batch_shape_count(); shapes differ only in speed, never in results). */
int ilg_batch_set_shape(ilg_batch *b, uint32_t shape);
uint32_t ilg_batch_shape_count(void);

/* Member r's state as host [q][L_r] counts.  Syncs. */
int ilg_batch_get_state(ilg_batch *b, uint32_t r, void *host_out);

/* Sum over samples of S(k) (sk_sum[nreal][nk]) and the sample counts
 * (count[nreal]); host arrays.  Syncs. */
int ilg_batch_structure_factor(ilg_batch *b, double *sk_sum, uint64_t *count);

/* Recorded A^LG series (amp[nreal][max_amp]) and their lengths
 * (count[nreal]); host arrays.  Syncs. */
int ilg_batch_amplitudes(ilg_batch *b, double *amp, uint32_t *count);

/* Wait for the batch's work, report sticky errors, free what it owns. */
int ilg_batch_destroy(ilg_batch *b);

/* ------------------------------------------------------------------------
 * Serving: a continuous-batching request server.  Requests (a configuration,
 * its initial state and a step count) queue in FIFO order until their device
 * memory (double-buffered state and fixed-point tables) fits the budget;
 * admitted requests become active slots whose state stays on the device.
 * Each ilg_server_poll admits what fits, advances every active request (or,
 * under a step node cap, those with the least remaining work that fit it) by
 * up to quantum_steps steps in shared launches (one per step and per
 * (q, count type, draw specification) group, groups on separate streams),
 * and retires finished requests to host memory.  A request's result is bit-identical to the same
 * configuration run alone through ilg_create/ilg_step.
 * ---------------------------------------------------------------------- */
typedef struct ilg_server ilg_server; /* opaque; owned by the library */

#define ILG_REQ_QUEUED 0u
#define ILG_REQ_ACTIVE 1u
#define ILG_REQ_DONE 2u
#define ILG_REQ_CANCELLED 3u
#define ILG_REQ_FAILED 4u   /* a count of this request exceeded its count type
                               (at admission or in a quantum); its memory is
                               freed and its state lost; the other requests are
                               unaffected */

typedef struct ilg_request_info {
    uint64_t id;
    uint32_t state;       /* ILG_REQ_* */
    uint32_t q;
    uint64_t length;
    uint64_t steps_total, steps_done;
    double t_submit, t_admit, t_done; /* ilg_server_clock() seconds; -1 if not yet */
} ilg_request_info;

typedef struct ilg_poll_info {
    uint32_t admitted, active, queued, finished; /* in this poll / after it */
    uint32_t quantum_steps;                      /* longest advance in this poll */
    uint32_t failed;                             /* requests that failed in this poll
                                                    (ILG_REQ_FAILED) */
    uint64_t bytes_in_use, bytes_peak;           /* device budget accounting */
} ilg_poll_info;

/* Steady clock (seconds) used for the request timestamps. */
double ilg_server_clock(void);

/* Server owning a device arena of budget_bytes; every poll advances active
 * requests by up to quantum_steps steps (small requests by up to 16 quanta,
 * see ilg_server_set_resident). */
int ilg_server_create(uint64_t budget_bytes, uint32_t quantum_steps, ilg_server **out);

#define ILG_RESIDENT_DEFAULT_NODES 4096u
#define ILG_RESIDENT_MAX_NODES 65536u
/* Small requests: those of at most max_nodes nodes (default
 * ILG_RESIDENT_DEFAULT_NODES; 0: none; ILG_E_INVALID above
 * ILG_RESIDENT_MAX_NODES) are advanced by a workgroup of their own in each
 * step launch, with a workgroup barrier per step, by as many steps per
 * launch as fit in the time of the launch's work on the other requests, and
 * by up to max_steps steps per poll (at least the quantum; default 16
 * quanta).  A small request's steps then do not each wait for a launch, so
 * its latency falls; the request is accounted with the steps it took.  At
 * most 128 small requests per launch group are resident; the others are
 * advanced like large ones.  Results do not depend on this setting (every
 * step is the same map with the same draws).  Takes effect from the next
 * poll. */
int ilg_server_set_resident(ilg_server *s, uint64_t max_nodes, uint32_t max_steps);

/* Scheduling policy of the polls that follow.  max_nodes = 0 (the default):
 * every poll advances every active request.  max_nodes > 0: a poll advances
 * the active requests in increasing order of remaining work (nodes x steps
 * left, ties by id), skipping any that would bring the quantum's total past
 * max_nodes nodes, and always at least one.  Every launch advances its
 * requests by one step in time proportional to the nodes it holds, so near
 * saturation this shortens the typical latency; a request can wait while
 * smaller ones keep arriving.  Results do not depend on the policy. */
int ilg_server_set_step_nodes(ilg_server *s, uint64_t max_nodes);

/* Queue a request: cfg (q = 2, 3 or 5), host initial counts (copied):
 * [q][L], or [5][height][length] for D2Q5; nsteps > 0.  ILG_E_BUSY if it can
 * never fit the budget. */
int ilg_server_submit(ilg_server *s, const ilg_config *cfg, const void *init_host,
                      uint64_t nsteps, uint64_t *id);

/* Queue a request whose initial state is the paper's Poisson sine condition
 * drawn on the device at admission (no host state is copied): as
 * ilg_init_poisson_sine with nave, amp and init_seed, the configuration's
 * realization and theta.  Same argument rules as ilg_init_poisson_sine; a
 * drawn count above the count type is reported as ILG_E_OVERFLOW by a later
 * poll, like an overflow during the steps. */
int ilg_server_submit_poisson_sine(ilg_server *s, const ilg_config *cfg, double nave, double amp,
                                   uint64_t init_seed, uint64_t nsteps, uint64_t *id);

/* One scheduling round: admit what fits free memory, wait for the quantum
 * launched by the previous poll and retire the requests it finished (or
 * that failed), admit again, then launch the next quantum and return while
 * it runs on the device (the caller's host work overlaps it).  After a poll
 * that reports no active and no queued request nothing is in flight. */
int ilg_server_poll(ilg_server *s, ilg_poll_info *info);

/* State and timestamps of a request that has not been collected. */
int ilg_server_info(ilg_server *s, uint64_t id, ilg_request_info *out);

/* Copy a finished request's final [q][L] counts to host_out and forget it.
 * For a failed request (ILG_REQ_FAILED) nothing is copied: it is forgotten
 * and ILG_E_OVERFLOW is returned, with the request id in ilg_last_error(). */
int ilg_server_result(ilg_server *s, uint64_t id, void *host_out);

/* Drop a queued or active request and release its memory. */
int ilg_server_cancel(ilg_server *s, uint64_t id);

/* Wait for the server's work and free everything it owns. */
int ilg_server_destroy(ilg_server *s);

/* ------------------------------------------------------------------------
 * Measurement probes (not part of the method): each runs one of the two
 * costs the fused step combines, with the step kernel's launch shape, so
 * that a benchmark can place the step between them.  Both are asynchronous
 * on `stream` and write only their output buffer.
 * ---------------------------------------------------------------------- */

/* Streaming only: the memory pattern of one uint16 step of a q = 2 or 3
 * lattice of `length` nodes (the streaming of Eq. ilgeq without the flip or
 * the collision): out_i[(x + v_i) mod L] = in_i[x].  in_dev and out_dev are
 * distinct device buffers of ilg_state_bytes() for that lattice ([q][pitch]
 * uint16).  ILG_E_INVALID for other q or lengths outside [1, 2^31). */
int ilg_probe_stream(uint32_t q, uint64_t length, const void *in_dev, void *out_dev,
                     void *stream);

/* Draws only: for every node x < length the Philox4x32 blocks with counter
 * (x, t, 0, b), b < blocks, key = seed, with `rounds` rounds (10 or 7), as
 * the step draws them; out_dev[x] (device, length uint32) receives the xor of
 * all their words.  blocks in [1, 64]. */
int ilg_probe_philox(uint64_t length, uint32_t blocks, uint32_t rounds, uint32_t t, uint64_t seed,
                     void *out_dev, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ILG_H */
