/*
 * mcrng.h - C ABI of the MI355X (gfx950) library for hash- and
 * stride-seeded LCG random-number streams driving a fixed-source 1-D slab
 * Monte Carlo transport loop.
 *
 * Method: Cuneo & Variansyah, "An Alternative to Stride-Based RNG for Monte
 * Carlo Transport" (arXiv 2403.06362).
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device pointers (HIP device memory on the
 *     current device); every other pointer is a host pointer.  The caller
 *     owns all of them.  Host arrays are read during the call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is enqueued on it asynchronously; the call returns once
 *     the work is enqueued, not when it has finished.
 *   - Return value: MCRNG_OK (0) or a positive warning on success, a
 *     negative MCRNG_E* code on failure.  On failure nothing is enqueued
 *     and mcrng_last_error() (thread-local) describes the cause.  No C++
 *     exception crosses this interface.
 *   - Unless stated otherwise, calls that use one device are not safe to run
 *     concurrently from several threads on the same mcrng_ctx.
 */
#ifndef MCRNG_H
#define MCRNG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCRNG_ABI_VERSION 2

enum {
    MCRNG_OK = 0,
    MCRNG_WSTRIDE_WRAP = 1,   /* success; a stride allocation wraps the cycle (N Q > 2^m) */
    MCRNG_EINVAL = -1,        /* bad argument (null pointer, size, malformed geometry) */
    MCRNG_ENOMEM = -2,        /* device or host allocation failed */
    MCRNG_EDEVICE = -3,       /* HIP runtime error (no device, launch failure) */
    MCRNG_ERANGE = -4,        /* a track length could reach 2^7, the fixed-point tally range */
    MCRNG_ESTATE = -5         /* call order: reduce_tallies before any run_histories */
};

/* ------------------------------------------------------------------ */
/* Generator and stream seeding                                        */
/* ------------------------------------------------------------------ */

/* LCG of Sec. "Linear Congruential Generator", eq. (1):
 *   X_{n+1} = (g X_n + c) mod 2^m,  the new state is also the output.
 * Requires 1 <= m <= 64 (the transport needs m >= 53: a uniform takes the
 * top 53 state bits).  The workloads use g = 2806196910506780709, c = 1,
 * m = 63. */
typedef struct {
    uint64_t g;
    uint64_t c;
    uint32_t m;
    uint32_t reserved;   /* must be 0 */
} mcrng_lcg;

enum { MCRNG_SEED_STRIDE = 0, MCRNG_SEED_HASH = 1 };

/* Where stream i (0-based, global index first_index + i) starts.
 *   MCRNG_SEED_STRIDE: X_{Q (first_index + i)} with X_0 = base and Q = stride
 *     (Sec. "Parallel LCG with Seed Striding": unit u_k is assigned X_{Qk};
 *     the skip-ahead is eq. (2)).
 *   MCRNG_SEED_HASH: hash(first_index + i + 1, parent) mod 2^m, with
 *     parent = base, or parent = hash(group_key, base) when hier = 1
 *     (Listing 1 for hash(k, s); eq. (3) seed splitting with 1-based keys;
 *     eq. (4) hierarchical splitting, the group id hashed first). */
typedef struct {
    uint32_t kind;         /* MCRNG_SEED_STRIDE or MCRNG_SEED_HASH */
    uint32_t hier;         /* hash only: 1 = hash the group key first */
    uint64_t base;         /* stride: X_0; hash: the seed s */
    uint64_t stride;       /* stride only: Q >= 1 */
    uint64_t first_index;  /* global index of this set's stream 0 */
    uint64_t group_key;    /* hash with hier = 1: the group (problem/batch) id */
} mcrng_seeding;

/* Writes the start state of streams 0..n-1 to d_state[0..n-1] (uint64,
 * state in the low m bits).  n = 0 is a no-op.  Returns MCRNG_WSTRIDE_WRAP
 * when a stride allocation passes 2^m states (allocations wrap around the
 * cycle, Sec. "Parallel LCG with Seed Striding"); the states are written
 * all the same. */
int mcrng_init_streams(const mcrng_lcg *lcg, const mcrng_seeding *seeding, uint64_t n,
                       uint64_t *d_state, void *stream);

/* Draw microbenchmark and stream advance.  Stream i takes d_count[i] LCG
 * steps (eq. (1)) from its start state and d_checksum[i] receives the sum
 * of its outputs X_1 .. X_count modulo 2^64 (0 for count 0).
 *   seeding != NULL: start states come from the seeding (fused seed + draw);
 *                    d_state may be NULL, else it receives the final states.
 *   seeding == NULL: start states are read from d_state, which receives the
 *                    final states (in place).
 * d_count: n uint32; d_checksum: n uint64.  n = 0 is a no-op.
 * Launch-shape overrides read from the environment (results never change):
 * MCRNG_DRAW_ROUND (8, 16, 20, 24 or 32 steps per round; default 20),
 * MCRNG_DRAW_BLOCKS_PER_CU (default 32), MCRNG_DRAW_GENERIC=1 (the masked
 * kernel instead of the round-aligned one). */
int mcrng_draw(const mcrng_lcg *lcg, const mcrng_seeding *seeding, uint64_t n,
               const uint32_t *d_count, uint64_t *d_state, uint64_t *d_checksum, void *stream);

/* Uniform random numbers.  Stream i takes k LCG steps (eq. (1)) and its
 * j-th output X (j = 1..k) gives
 *   d_u[(j - 1) n + i] = ((X >> (m - 53)) + 1) 2^-53,
 * an exact double in (0, 1] (the mapping every transport draw uses).  The
 * layout is draw-major: row j - 1 holds the j-th number of every stream.
 * Start states as in mcrng_draw: from the seeding (d_state may be NULL,
 * else it receives the final states) or, with seeding == NULL, from d_state
 * (updated in place).  Requires m >= 53.  d_u: k x n doubles.  n = 0 or
 * k = 0 is a no-op. */
int mcrng_uniforms(const mcrng_lcg *lcg, const mcrng_seeding *seeding, uint64_t n, uint32_t k,
                   uint64_t *d_state, double *d_u, void *stream);

/* ------------------------------------------------------------------ */
/* Slab transport                                                      */
/* ------------------------------------------------------------------ */

/* One fixed-source slab problem.  The source is mono-directional (mu = +1)
 * at the left face x = region_edges[0], at t = time_edges[0] (or t = 0);
 * both faces are vacuum.  Cells are the intervals between the merged
 * region and bin edges.  History j (0-based) uses stream j of `seeding`
 * and belongs to batch floor(j / ceil(n_histories / n_batches)).
 * Host arrays:
 *   region_edges  n_regions + 1, strictly increasing, within [-2^40, 2^40]
 *   sigma_t       n_regions, in [2^-64, 2^64] (total cross section)
 *   scatter       n_regions, in [0, 1] (scattering ratio c)
 *   bin_edges     n_space_bins + 1, strictly increasing, same first and
 *                 last value as region_edges
 *   time_edges    n_time_bins + 1, strictly increasing (the last is the
 *                 census time), or NULL with n_time_bins = 0 (steady state) */
typedef struct {
    uint32_t n_regions;
    uint32_t n_space_bins;
    uint32_t n_time_bins;
    uint32_t n_batches;          /* >= 1 */
    const double *region_edges;
    const double *sigma_t;
    const double *scatter;
    const double *bin_edges;
    const double *time_edges;
    uint64_t n_histories;
    mcrng_seeding seeding;
} mcrng_problem;

enum { MCRNG_FP64 = 0, MCRNG_FP32 = 1 };
enum { MCRNG_SCHED_HISTORY = 0, MCRNG_SCHED_EVENT = 1 };

/* Launch options.  Zero means "default" for every field.  No option changes
 * any result bit: tallies are exact integers, so every schedule, block
 * size, histories-per-lane and tally tiling gives the same output.
 *   precision       MCRNG_FP64, or MCRNG_FP32 (flight, direction, position
 *                   and time in single precision; -ln(u) and tallies stay
 *                   exact / double; a different, also deterministic result)
 *   schedule        history-based persistent kernel, or event-sorted
 *                   particle bank (one event per particle per launch)
 *   block           threads per block: 64, 128, 256, 512 or 1024
 *   hist_per_lane   histories each lane carries at once: 1, 2 or 4
 *   unit_histories  histories per work unit (the scheduling grain), at most
 *                   2^18 (0 = automatic, at most 2^16: total / 4096, or
 *                   total / 10240 when that takes the chained kernel
 *                   below).  A unit's partial
 *                   tally is exact while fewer than 2^32 of its scores fall
 *                   in one bin (2^14 per history on average at 2^18
 *                   histories); the event schedule's slots that collect a
 *                   whole slice carry and have no such limit.
 *   grid            persistent blocks (0 = fill the device)
 *   tally_copies    LDS tally copies per block: 1, or one per wave (= 2)
 *                   A set of one problem with one history per lane, one
 *                   tally copy and units of at least 20 x block histories
 *                   runs on the chained kernel, where a block holds two
 *                   units (two LDS tally slices) and starts its next unit
 *                   while the last histories of the current one finish, if
 *                   the second slice costs no blocks per CU.  Environment
 *                   override MCRNG_TRANSPORT_CHAIN: 0 = never, 2 = for
 *                   every run of one problem with one history per lane and
 *                   one tally copy, whatever its units and even where it
 *                   costs blocks per CU (any other history-schedule run
 *                   fails with MCRNG_EINVAL); read at every run.
 *   use_graph       1 = capture the launches of a run in a hipGraph once
 *                   per (problem set, options) and replay it
 *   bank_size       event schedule: particles per bank slice
 *   coll_batch      history schedule: a wave runs its collision pass
 *                   (absorption draw, new direction, next flight; empty
 *                   lanes take new histories) once this many of its lanes
 *                   wait at a collision site or stand empty (1..64 per
 *                   history slot; default 36) */
typedef struct {
    uint32_t precision;
    uint32_t schedule;
    uint32_t block;
    uint32_t hist_per_lane;
    uint32_t unit_histories;
    uint32_t grid;
    uint32_t tally_copies;
    uint32_t use_graph;
    uint32_t bank_size;
    uint32_t coll_batch;
    uint32_t reserved[6];        /* must be 0 */
} mcrng_run_opts;

/* Diagnostics per problem, MCRNG_NDIAG uint64 words in this order.  All are
 * sums except MCRNG_D_MAX_DRAWS (a maximum).  OVER_STRIDE counts histories
 * that drew more than Q numbers under stride seeding (they ran into the next
 * unit's stream, Sec. "Repetition and State Space Exhaustion"). */
enum {
    MCRNG_D_HISTORIES = 0, MCRNG_D_LEAK_LEFT, MCRNG_D_LEAK_RIGHT, MCRNG_D_ABSORBED,
    MCRNG_D_CENSUS, MCRNG_D_EVENTS, MCRNG_D_COLLISIONS, MCRNG_D_DRAWS,
    MCRNG_D_MAX_DRAWS, MCRNG_D_OVER_STRIDE, MCRNG_NDIAG
};

typedef struct mcrng_ctx mcrng_ctx;

/* Creates a context bound to HIP device `device`.  The context owns the
 * device tables, work-unit partial tallies and cached graphs of its runs;
 * they are allocated on demand and grow, never shrink, until destroy. */
int mcrng_ctx_create(int device, mcrng_ctx **out);
int mcrng_ctx_destroy(mcrng_ctx *ctx);

/* Number of tally bins of a problem set: sum over problems of
 * n_batches * max(n_time_bins, 1) * n_space_bins.  Host-only. */
uint64_t mcrng_tally_bins(const mcrng_problem *problems, uint32_t n_problems);

/* Runs every history of every problem (the hot path: stream seeding, LCG
 * draws, flight sampling, cell and time marching, collisions, track-length
 * scoring).  Per-work-unit exact partial tallies stay in the context until
 * the next run.  Validation errors: MCRNG_EINVAL (geometry, sizes,
 * options), MCRNG_ERANGE (a flight could exceed 2^7 length units:
 * -ln(2^-53)/min sigma_t >= 128 and no time bin bounds it).  Returns
 * MCRNG_WSTRIDE_WRAP when a stride allocation passes 2^m states. */
int mcrng_run_histories(mcrng_ctx *ctx, const mcrng_lcg *lcg, const mcrng_problem *problems,
                        uint32_t n_problems, const mcrng_run_opts *opts, void *stream);

/* Reduces the partial tallies of the last run in a fixed order.
 *   d_raw   2 uint64 per bin (low, high word): the exact 128-bit sum of the
 *           quantised track lengths q = round-half-even(s 2^56) of the bin
 *   d_flux  1 double per bin: RN(sum) 2^-56 / (N_b dx [dt]), N_b the
 *           histories of the bin's batch, dx its width, dt its duration
 *   d_diag  n_problems x MCRNG_NDIAG uint64 (may be NULL)
 * Bins are ordered problem, batch, time bin, space bin. */
int mcrng_reduce_tallies(mcrng_ctx *ctx, uint64_t *d_raw, double *d_flux, uint64_t *d_diag,
                         void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): runs every
 * history of the problem set and reduces its tallies in one call, like
 * mcrng_run_histories followed by mcrng_reduce_tallies with the same
 * options, with the same outputs bit for bit (d_raw, d_flux, d_diag as for
 * mcrng_reduce_tallies), without a context and without allocating any
 * device memory: no hipMalloc, hipFree or allocating library call.
 * Limits:
 *   - every device buffer of the run (tables, stride skip tables, work
 *     units, one partial tally slot per work unit, unit diagnostics, the
 *     scheduling counter) comes from one static device array of 64 MiB per
 *     device, which the library allocates with its code object the first
 *     time this call runs on a device and keeps until the process ends;
 *     a run that needs more (about units x slice_bins x 16 bytes, e.g. the
 *     2e8-history multi-region slab takes 49 MB) returns MCRNG_EINVAL and
 *     enqueues nothing;
 *   - history schedule only; opts.schedule = MCRNG_SCHED_EVENT or
 *     opts.use_graph = 1 return MCRNG_EINVAL;
 *   - every call on a device shares that device's array and leaves its
 *     contents to the next call (the scheduling counter is cleared by a
 *     kernel at the start of each run, the partial slots are overwritten):
 *     calls whose work overlaps on one device (other streams, other
 *     threads' streams) race and give undefined results.  Calls from several
 *     host threads are serialised while they enqueue, not on the device.
 * Uses the current device.  Returns MCRNG_WSTRIDE_WRAP as
 * mcrng_run_histories does. */
int mcrng_run_histories_noalloc(const mcrng_lcg *lcg, const mcrng_problem *problems, uint32_t n_problems,
                                const mcrng_run_opts *opts, uint64_t *d_raw, double *d_flux, uint64_t *d_diag,
                                void *stream);

/* Times candidate launch options for the problem set (each candidate run
 * once after a warm-up, timed with HIP events on `stream`; the call
 * synchronises the stream) and writes the fastest to *best.  `base` (NULL =
 * all defaults) fixes precision, schedule, grid, bank size and use_graph;
 * the search covers block size, histories per lane, work-unit size, tally
 * copies and (history schedule) the collision batch, by coordinate
 * descent.  The generator, problems and options are validated as by
 * mcrng_run_histories before anything is timed.  The choice is cached in
 * the context per (problem set, normalised base options): a repeated call
 * returns it without timing and sets *best_ms to -1.  *best_ms receives the
 * chosen options' time otherwise (may be NULL).  The runs leave the
 * context's partial tallies in the state of the last candidate's run. */
int mcrng_autotune(mcrng_ctx *ctx, const mcrng_lcg *lcg, const mcrng_problem *problems,
                   uint32_t n_problems, const mcrng_run_opts *base, mcrng_run_opts *best,
                   float *best_ms, void *stream);

/* Kernel time of the last run_histories (HIP events around its launches on
 * its stream), in milliseconds, once that stream has reached the end of the
 * run; negative if unavailable. */
float mcrng_last_run_ms(mcrng_ctx *ctx);

/* Name of the transport kernel the last run_histories of `ctx` launched:
 * "k_transport_chain" (one problem, two units in flight per block),
 * "k_transport" (per-unit) or "k_event_step" (event schedule); "" before
 * any run or for a NULL ctx.  A static string; host-only. */
const char *mcrng_last_run_kernel(const mcrng_ctx *ctx);

/* ------------------------------------------------------------------ */
/* Pulse in an infinite multiplying medium, with secondary particles   */
/* ------------------------------------------------------------------ */

/* The paper's test problem (Sec. "Implementation and Results"): a pulse of
 * source particles at x = 0, t = 0 in an infinite homogeneous medium with
 * total cross section sigma_t, isotropic scattering ratio
 * scatter = Sigma_s / Sigma_t and scattering multiplicity nu, run to the
 * census time (the last time edge), with the collision estimator of the
 * flux averaged over [x_lo, x_hi] in time bins.  Particle speed 1.
 * One particle: its first draw u gives mu = 2u - 1; its flight is
 * s = -ln(u) / sigma_t; if t + s is not below the census time it ends at
 * census, else it moves to (x + mu s, t + s) and collides there; a
 * collision with x_lo <= x <= x_hi and t >= time_edges[0] adds 1 to its
 * (batch, time bin); the next draw decides absorption (absorbed unless
 * u < scatter); on a scattering the next draw gives the number of emerging
 * particles n = floor(nu) + (u < nu - floor(nu)), which start at the
 * collision site, and the parent ends.
 * Seeds (Secs. "Hierarchical Seed Splitting" and "On-Demand Seed
 * Splitting", eqs. 4 and 5).  Source i (0-based) of batch b has the global
 * batch id B = first_batch + b:
 *   MCRNG_SEED_HASH:   the source starts at hash(i + 1, hash(B + 1, base));
 *                      the k-th particle emerging from a scattering
 *                      (k = 1..n) starts its own stream at hash(k, X_p),
 *                      X_p the parent's state after its draws (all states
 *                      reduced modulo 2^m);
 *   MCRNG_SEED_STRIDE: the source starts at X_{Q (B per_batch + i)}; the
 *                      particles it gives rise to draw from its stream,
 *                      depth first (the first emerging particle at once,
 *                      its siblings afterwards in order).
 * Host array: time_edges, n_time_bins + 1 values, finite, >= 0, strictly
 * increasing. */
typedef struct {
    double sigma_t;              /* in [2^-64, 2^64] */
    double scatter;              /* in [0, 1] */
    double multiplicity;         /* nu in [0, 14] */
    double x_lo, x_hi;           /* finite, x_lo < x_hi */
    uint32_t n_time_bins;        /* 1 .. 4096 */
    uint32_t n_batches;          /* >= 1 */
    const double *time_edges;
    uint64_t per_batch;          /* sources per batch, >= 1; n_batches x per_batch < 2^40 */
    uint64_t first_batch;        /* global id of batch 0 (shards, repetitions) */
    mcrng_seeding seeding;       /* kind, base, stride; hier, first_index, group_key must be 0 */
} mcrng_pulse_problem;

enum { MCRNG_PULSE_AUTO = 0, MCRNG_PULSE_BANK = 1, MCRNG_PULSE_FAMILY = 2, MCRNG_PULSE_EVENT = 3 };

/* Options (zero = default).  No option changes a result bit: counts are
 * integers.
 *   schedule     MCRNG_PULSE_BANK (hash seeding only): generations; a
 *                launch runs the lines of descent of its input particles
 *                (the first particle emerging from a scattering at once) in
 *                any order and banks the siblings for the next launch;
 *                MCRNG_PULSE_FAMILY: one source family per lane, depth
 *                first (history based); MCRNG_PULSE_EVENT (hash seeding
 *                only): event based, every launch advances each live
 *                particle by one flight and its collision and banks all
 *                emerging particles for the next launch (the tail is
 *                finished as for the bank schedule, unless finish_div says
 *                never); AUTO: for hash seeding the bank below 16 sources per
 *                resident lane (2048 lanes per CU) and families from there
 *                on (the bank with population control), family for stride
 *   block        threads per block: 64, 128, 256, 512 or 1024
 *   stack_depth  family schedule: stack entries per lane (default 128; an
 *                entry holds the siblings of one scattering on the current
 *                line of descent)
 *   finish_div   bank schedule: once a generation is smaller than the one
 *                before it, at most 1/finish_div of the largest of its chain
 *                and at most 65536 particles, one launch runs the rest depth
 *                first per lane, up to 64 particles per banked particle
 *                (default 1: the first shrinking generation of that size;
 *                0xffffffff: never)
 *   chunk        bank and event schedules: particles a wave takes from a
 *                launch's input per atomic, 64 .. 2^20 (default 0: chosen
 *                per launch from its input count) */
typedef struct {
    uint32_t schedule;
    uint32_t block;
    uint32_t stack_depth;
    uint32_t finish_div;
    uint32_t chunk;
    uint32_t reserved[3];        /* must be 0 */
} mcrng_pulse_opts;

/* Diagnostics of a pulse run, MCRNG_NDIAG uint64 words in this order; sums
 * except MCRNG_PD_MAX_DRAWS (the most numbers one stream drew: a particle's
 * under hash seeding, a family's under stride seeding).  OVER_STRIDE counts
 * stride families that drew more than Q numbers. */
enum {
    MCRNG_PD_SOURCES = 0, MCRNG_PD_COLLISIONS, MCRNG_PD_TALLIED, MCRNG_PD_SCATTERS,
    MCRNG_PD_ABSORBED, MCRNG_PD_CENSUS, MCRNG_PD_SECONDARIES, MCRNG_PD_DRAWS,
    MCRNG_PD_MAX_DRAWS, MCRNG_PD_OVER_STRIDE
};

/* Runs every source of every batch and everything they give rise to.
 *   d_counts  n_batches x n_time_bins uint64 (required): collisions scored
 *             per (batch, time bin)
 *   d_flux    same shape, double (may be NULL):
 *             count / (((sigma_t per_batch) (x_hi - x_lo)) dt)
 *   d_diag    MCRNG_NDIAG uint64 (may be NULL)
 * Unlike the other calls this one returns after the run has finished on
 * `stream` (the bank schedule reads each generation's size).  Errors:
 * MCRNG_EINVAL (arguments), MCRNG_ERANGE (a family outgrew
 * opts.stack_depth; the outputs are then incomplete), MCRNG_ENOMEM.
 * Returns MCRNG_WSTRIDE_WRAP when the stride allocation passes 2^m states.
 * The run's time (first to last launch of the run) is mcrng_last_run_ms.
 * Family-kernel overrides read from the environment (counts never change):
 * MCRNG_PULSE_DEEP = 0 or 1 (the lane-major stack, or the register-held top
 * over depth-major planes; by default the latter from 16 families per lane),
 * MCRNG_PULSE_SLOTS = 0..16 (per-wave LDS tally slots when the counters do
 * not fit one LDS copy per block; default 16, 0 counts into HBM). */
int mcrng_run_pulse(mcrng_ctx *ctx, const mcrng_lcg *lcg, const mcrng_pulse_problem *problem,
                    const mcrng_pulse_opts *opts, uint64_t *d_counts, double *d_flux,
                    uint64_t *d_diag, void *stream);

/* Population control of the pulse problem at census times, with one-off
 * hashed values (Sec. "Hierarchical Seed Splitting": where a full stream
 * is not needed, as for population control, hashing a per-phase seed gives
 * one-off values, one per key).  Hash seeding only.
 * With K = census_every, census c (0-based) is at time_edges[(c+1) K], for
 * every (c+1) K < n_time_bins; n_census is the number of such points.  A
 * particle whose flight reaches a census time C stops at x + mu (C - t),
 * keeping its direction and stream state (exponential flights are
 * memoryless, so the rest of its flight is not kept).  Per batch, N
 * particles reach census c; with M = target, q = floor(M / N),
 * r = M mod N, the particle with state X leaves q + [u < r / N] copies,
 *   u = U(hash(X, hash(c + 1, hash(B + 1, seed))) mod 2^m),
 * U(S) = ((S >> (m - 53)) + 1) 2^-53 and the comparison exact in integers:
 * the phase seed of (batch, census) is the parent and the particle's own
 * state the key, so no ordering of the particles is needed.  Copy k
 * (k = 1..) starts at the census point with the particle's direction (no
 * direction draw) and the stream hash(k, X) mod 2^m (eq. 5).  All particles
 * of a batch carry one weight per epoch, 1 before the first census and
 * w_{c+1} = (w_c N_c) / M after census c, so the counts stay integers;
 * the flux of a time bin of epoch e is ((double)count w_e) / den, den as
 * for mcrng_run_pulse.  A batch that no particle reaches a census with
 * scores nothing afterwards. */
typedef struct {
    uint32_t census_every;       /* K >= 1 */
    uint32_t reserved0;          /* must be 0 */
    uint64_t target;             /* M, 1 .. 2^40 */
    uint64_t seed;               /* the population-control seed */
    uint64_t reserved[2];        /* must be 0 */
} mcrng_pulse_pc;

/* Runs a pulse problem with population control: as mcrng_run_pulse (the
 * bank or event schedule; opts.schedule AUTO, BANK or EVENT), plus
 *   d_pop  n_batches x n_census x 2 uint64 (may be NULL): the particles of
 *          each batch reaching each census, and the copies leaving it.
 * Diagnostics: CENSUS counts every census arrival; copies are neither
 * sources nor secondaries (their number is the sum of the copies in
 * d_pop).  Returns after the run.  Errors: MCRNG_EINVAL (arguments, stride
 * seeding, the family schedule), MCRNG_ENOMEM. */
int mcrng_run_pulse_pc(mcrng_ctx *ctx, const mcrng_lcg *lcg, const mcrng_pulse_problem *problem,
                       const mcrng_pulse_pc *pc, const mcrng_pulse_opts *opts, uint64_t *d_counts,
                       double *d_flux, uint64_t *d_diag, uint64_t *d_pop, void *stream);

/* Thread-local text of the last failure (never NULL). */
const char *mcrng_last_error(void);

/* MCRNG_ABI_VERSION of the built library. */
int mcrng_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MCRNG_H */
