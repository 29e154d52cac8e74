/*
 * CPU oracle for hash- vs stride-seeded LCG streams driving a 1-D slab
 * Monte Carlo transport loop (Cuneo & Variansyah, "An Alternative to
 * Stride-Based RNG for Monte Carlo Transport", arXiv 2403.06362).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU library computes.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it.  It shares no code,
 * header, table or constant with the HIP library, and the library never
 * calls it.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared
 * (no FMA contraction, IEEE double and single arithmetic, round-to-nearest).
 *
 * Sections of the paper each function follows:
 *   lcg step ............ Sec. "Linear Congruential Generator", eq. (1)
 *   skip-ahead .......... Sec. "Parallel LCG with Seed Striding", eq. (2)
 *   stride allocation ... same section: unit u_k starts at X_{Qk}
 *   hash(k, s) .......... Sec. "Parallel LCG with Seed Hashing", Listing 1
 *   seed splitting ...... Sec. "Seed Splitting", eq. (3): S_k = hash(k, s)
 *   hierarchical seeds .. Sec. "Hierarchical Seed Splitting", eq. (4)
 *   secondary seeds ..... Sec. "On-Demand Seed Splitting", eq. (5)
 *   pulse problem ....... Sec. "Implementation and Results" (the test problem)
 *   population control .. Sec. "Hierarchical Seed Splitting": one-off hashed
 *                          values from a per-phase seed
 * The transport loop, the uniform mapping, the logarithm and the fixed-point
 * tally are readings of points the paper leaves open; each is stated where
 * it is implemented.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <stdlib.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* LCG, eq. (1): X_{n+1} = (g X_n + c) mod 2^m; the new state is also the
 * generator's output. */
/* ------------------------------------------------------------------ */

static uint64_t mask_of(uint32_t m)
{
    return (m >= 64) ? ~(uint64_t)0 : (((uint64_t)1 << m) - 1);
}

uint64_t orc_lcg_next(uint64_t x, uint64_t g, uint64_t c, uint32_t m)
{
    /* exact product in 128 bits, then reduce modulo 2^m */
    u128 full = (u128)g * (u128)x + (u128)c;
    return (uint64_t)full & mask_of(m);
}

/* ------------------------------------------------------------------ */
/* Skip-ahead, eq. (2).  X_k = G_k X_0 + C_k (mod 2^m) with
 *   G_k = prod_j (g^{2^j})^{k_(j)},   C_k = c (1 + g + ... + g^{k-1}),
 * where k_(j) is bit j of k.  Both factors are built in O(m) steps by
 * walking the bits of k with the 2^j-step map (g^{2^j}, c(1+...+g^{2^j-1})),
 * which doubles as  g_{2h} = g_h^2,  c_{2h} = c_h (1 + g_h).
 * (As printed, eq. (2) omits X_0 from the first term; it is the X_0 = 1
 * case of the affine form used here.) */
/* ------------------------------------------------------------------ */

void orc_skip_coeffs(uint64_t k, uint64_t g, uint64_t c, uint32_t m,
                     uint64_t *G_out, uint64_t *C_out)
{
    const uint64_t msk = mask_of(m);
    uint64_t G = 1 & msk, C = 0;     /* map for the bits of k consumed so far */
    uint64_t gj = g & msk, cj = c & msk;  /* map for 2^j steps */
    for (int j = 0; j < 64; ++j) {
        if ((k >> j) & 1) {
            /* X -> gj (G X + C) + cj */
            G = (uint64_t)((u128)gj * G) & msk;
            C = (uint64_t)((u128)gj * C + cj) & msk;
        }
        cj = (uint64_t)((u128)cj * (u128)(gj + 1)) & msk;
        gj = (uint64_t)((u128)gj * gj) & msk;
    }
    *G_out = G;
    *C_out = C;
}

uint64_t orc_skip(uint64_t x0, uint64_t k, uint64_t g, uint64_t c, uint32_t m)
{
    uint64_t G, C;
    orc_skip_coeffs(k, g, c, m, &G, &C);
    return (uint64_t)((u128)G * x0 + C) & mask_of(m);
}

/* ------------------------------------------------------------------ */
/* hash(k, s) of Listing 1 (a modified 64-bit MurmurHash, one 64-bit key
 * and one 64-bit seed), written as a composition of two bijections of the
 * 64-bit words (all arithmetic modulo 2^64):
 *   mul_m(x)  = M x          (M is odd, so this is invertible)
 *   fold47(y) = y ^ (y >> 47) (its own inverse, since 2 x 47 > 64)
 *   mix       = fold47 after mul_m
 * The seed enters as the word mix(s ^ 8M), the key as mul_m(mix(k)), and the
 * hash is mix of their exclusive or. */
/* ------------------------------------------------------------------ */

static const uint64_t MURMUR_M = 0xC6A4A7935BD1E995ull;

static uint64_t mul_m(uint64_t x) { return x * MURMUR_M; }

static uint64_t fold47(uint64_t y) { return y ^ (y >> 47); }

uint64_t orc_subhash(uint64_t x) { return fold47(mul_m(x)); }

uint64_t orc_hash(uint64_t k, uint64_t s)
{
    const uint64_t seed_word = orc_subhash(s ^ mul_m(8));
    const uint64_t key_word = mul_m(orc_subhash(k));
    return orc_subhash(seed_word ^ key_word);
}

/* ------------------------------------------------------------------ */
/* Stream start states.
 *  stride: unit with global 0-based index i starts at X_{Q i}
 *          (Sec. "Parallel LCG with Seed Striding"; X_0 is the base seed).
 *  hash:   S_k = hash(k, s) with the 1-based key k = i + 1 (eq. 3); with a
 *          group key p, the parent is hash(p, s) first (eq. 4, the group id
 *          is hashed first).  The 64-bit hash is reduced modulo 2^m to give
 *          an LCG state (the paper seeds an m-bit generator with a 64-bit
 *          hash without saying how; reduction modulo 2^m is the reading). */
/* ------------------------------------------------------------------ */

typedef struct {
    uint64_t g, c;
    uint32_t m;
    uint32_t pad_;
} orc_lcg;

enum { ORC_SEED_STRIDE = 0, ORC_SEED_HASH = 1 };

typedef struct {
    uint32_t kind;       /* ORC_SEED_STRIDE or ORC_SEED_HASH */
    uint32_t hier;       /* hash only: 1 => parent = hash(group_key, base) */
    uint64_t base;       /* stride: X_0; hash: global seed s */
    uint64_t stride;     /* stride only: Q */
    uint64_t first_index;/* global 0-based index of this set's stream 0 */
    uint64_t group_key;  /* hash with hier = 1: the group (problem/batch) id */
} orc_seeding;

uint64_t orc_stream_start(const orc_lcg *L, const orc_seeding *S, uint64_t i)
{
    const uint64_t idx = S->first_index + i;
    if (S->kind == ORC_SEED_STRIDE) {
        /* k = Q * idx; the cycle length 2^m divides 2^64, so the product
         * may wrap modulo 2^64 without changing X_k */
        return orc_skip(S->base & mask_of(L->m), S->stride * idx, L->g, L->c, L->m);
    }
    uint64_t parent = S->hier ? orc_hash(S->group_key, S->base) : S->base;
    return orc_hash(idx + 1, parent) & mask_of(L->m);
}

void orc_init_streams(const orc_lcg *L, const orc_seeding *S, uint64_t n, uint64_t *out)
{
    for (uint64_t i = 0; i < n; ++i)
        out[i] = orc_stream_start(L, S, i);
}

/* Draw microbenchmark: stream i takes count[i] LCG steps from its start
 * state; its checksum is the sum of the outputs X_1..X_count modulo 2^64.
 * With S == NULL the start states are read from state_inout instead.  The
 * final states go back to state_inout when it is not NULL. */
void orc_seed_and_draw(const orc_lcg *L, const orc_seeding *S, uint64_t n,
                       const uint32_t *count, uint64_t *state_inout,
                       uint64_t *checksum)
{
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t x = S ? orc_stream_start(L, S, i) : state_inout[i];
        uint64_t sum = 0;
        for (uint32_t d = 0; d < count[i]; ++d) {
            x = orc_lcg_next(x, L->g, L->c, L->m);
            sum += x;
        }
        checksum[i] = sum;
        if (state_inout)
            state_inout[i] = x;
    }
}

/* ------------------------------------------------------------------ */
/* Uniform from a state (reading; the paper does not give the mapping):
 * the top 53 of the m state bits, plus one, times 2^-53.  The result is an
 * exact double in (0, 1], so -ln(u) is always finite.  Requires m >= 53. */
/* ------------------------------------------------------------------ */

double orc_uniform(uint64_t x, uint32_t m)
{
    uint64_t top = x >> (m - 53);
    return (double)(top + 1) * 0x1p-53;
}

/* Uniforms of n streams: stream i takes k LCG steps from its start state
 * and its j-th output X (j = 1..k) gives out[(j-1) n + i] = orc_uniform(X)
 * (draw-major).  With S == NULL the start states are read from state_inout;
 * the final states go back to state_inout when it is not NULL. */
void orc_uniforms(const orc_lcg *L, const orc_seeding *S, uint64_t n, uint32_t k,
                  uint64_t *state_inout, double *out)
{
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t x = S ? orc_stream_start(L, S, i) : state_inout[i];
        for (uint32_t j = 0; j < k; ++j) {
            x = orc_lcg_next(x, L->g, L->c, L->m);
            out[(uint64_t)j * n + i] = orc_uniform(x, L->m);
        }
        if (state_inout)
            state_inout[i] = x;
    }
}

/* ------------------------------------------------------------------ */
/* Natural logarithm with a fixed operation sequence (reading; the paper
 * does not fix the flight-sampling arithmetic, and bit-exact tallies need
 * the same rounded result on every device).  Textbook route:
 *   u = f 2^e with f in [1,2); if f >= 3/2 then f <- f/2, e <- e+1, so that
 *   f = 1 + a with a in [-1/4, 1/2);  s = a/(2+a);  ln(1+a) = 2 atanh(s)
 *   = 2s + sum_{k>=1} 2 s^{2k+1}/(2k+1)   (Taylor series of atanh),
 *   and 2s = a - a s, so  ln(1+a) = a - s (a - h),  h = sum_{k>=1} 2 s^{2k}/(2k+1);
 *   ln u = e ln2 + ln(1+a), with ln 2 split as LN2_HI + LN2_LO where
 *   LN2_HI holds ln 2 truncated to 40 fraction bits (so e LN2_HI is exact)
 *   and LN2_LO is the double nearest to ln 2 - LN2_HI.
 * Every step is one IEEE double operation rounded to nearest, in this order,
 * with no fused multiply-add:
 *   a = f - 1;  b = 2 + a;  s = a / b;  w = s * s;
 *   p = 2/(2K+1);  for k = K-1 .. 1:  p = p * w;  p = p + 2/(2k+1);
 *   h = w * p;  t = a - h;  c = s * t;  l = a - c;
 *   r = l + (double)e * LN2_LO;   result = (double)e * LN2_HI + r
 * with K = 11; the series coefficients are the correctly rounded quotients
 * 2/(2k+1). */
/* ------------------------------------------------------------------ */

#define ORC_LN_K 11

double orc_ln(double u)
{
    const double LN2_HI = 0x1.62e42fefa2000p-1;
    const double LN2_LO = 0x1.9ef35793c7673p-41;
    int ex;
    double fr = frexp(u, &ex);      /* u = fr 2^ex, fr in [1/2, 1) */
    double f = fr * 2.0;            /* exact */
    int e = ex - 1;
    if (f >= 1.5) {
        f = f * 0.5;                /* exact */
        e = e + 1;
    }
    double a = f - 1.0;             /* exact */
    double b = 2.0 + a;
    double s = a / b;
    double w = s * s;
    double p = 2.0 / (double)(2 * ORC_LN_K + 1);
    for (int k = ORC_LN_K - 1; k >= 1; --k) {
        p = p * w;
        p = p + 2.0 / (double)(2 * k + 1);
    }
    double h = w * p;
    double t = a - h;
    double c = s * t;
    double l = a - c;
    double r = l + (double)e * LN2_LO;
    return (double)e * LN2_HI + r;
}

/* ------------------------------------------------------------------ */
/* Fixed-source 1-D slab transport.
 *
 * Geometry: cells are the intervals between the merged, increasing edges
 * of material regions and tally bins; each cell has one total cross
 * section sigma_t, one scattering ratio c and one space tally bin.  With
 * n_time_bins > 0 the problem is time dependent at particle speed 1; the
 * last time edge is the census time.
 *
 * One history (readings of points the paper leaves open):
 *   start at the left face, x = E[0], mu = +1, t = T[0], cell 0;
 *   tau = -ln(u) remaining optical depth to the next collision.
 *   step:  s_col  = tau / sigma_t[cell]
 *          s_edge = (E[cell+1]-x)/mu (mu>0), (E[cell]-x)/mu (mu<0), inf (mu=0)
 *          s_time = T[tb+1] - t                     (time dependent only)
 *          the smallest wins; on equal distances collision beats edge and
 *          edge beats time (strict-less updates in that order);
 *   score  track length s into (batch, time bin, space bin);
 *   t += s (clamped to T[tb+1]);  tau -= sigma_t s (clamped at 0);
 *   edge:  move onto the crossed edge; leaving E[0] or E[last] leaks;
 *   time:  x += mu s (clamped into the cell); t = T[tb+1]; next time bin;
 *          passing the last time edge ends the history at census;
 *   collision: x += mu s (clamped into the cell); draw u1: scatter if
 *          u1 < c[cell], else absorbed; on scatter draw u2 -> mu = 2 u2 - 1
 *          (isotropic in the slab), draw u3 -> tau = -ln(u3).
 *
 * Tally (reading: bit-reproducible track-length sums).  Each track length
 * s is quantised once to q = round-half-even(s 2^56) (an integer, exact
 * because s < 2^7 is enforced by the caller) and summed exactly as a
 * 128-bit integer.  The flux of a bin is (sum q) 2^-56 / (N dx [dt]).
 *
 * FP32 flight mode: the remaining optical depth tau (the -ln(u) sample the
 * flight consumes) stays in double: it is orc_ln's result, each event
 * subtracts the product (double)sigma_t x (double)s of two floats (exact)
 * and clamps at 0, and the collision distance is (float)tau / sigma_t in
 * single precision (a float tau would lose absolute precision over the
 * many subtractions of a flight through thin cells, and the last segment,
 * the small remainder, would carry that error relative to its own length);
 * mu = 2 u2 - 1 is computed in double (exact) and rounded once
 * to float; the position is kept relative to the current cell's left edge
 * (xl in [0, W[cell]]) and the time relative to the current time bin's
 * start (tl in [0, DT[tb]]), so FP32 keeps its relative precision deep in a
 * thick slab and late in a long run; s, xl, mu, tl, sigma_t, the cell widths
 * W and the time-bin durations DT are floats (W, DT and sigma_t rounded once
 * from doubles); every distance, position and time operation is one IEEE
 * single operation:  se = (W - xl)/mu (mu > 0), (0 - xl)/mu (mu < 0);
 * st = DT[tb] - tl; tl = tl + s clamped to DT[tb]; an edge crossing sets
 * xl = 0 (moving right) or xl = W[new cell] (moving left); a time step sets
 * tl = 0.  The absorption test u1 < c stays in double; q is computed from
 * (double)s.
 */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t n_cells;
    int32_t n_space_bins;
    int32_t n_time_bins;      /* 0 => steady state */
    uint32_t n_batches;       /* >= 1 */
    const double *edges;      /* n_cells + 1 */
    const double *sigma_t;    /* n_cells */
    const double *scatter;    /* n_cells */
    const int32_t *bin;       /* n_cells: space bin of each cell */
    const double *t_edges;    /* n_time_bins + 1, or NULL */
    uint64_t n_histories;     /* N of the whole problem (sets batch size) */
    orc_lcg lcg;
    orc_seeding seeding;
} orc_problem;

enum {
    ORC_D_HISTORIES = 0, ORC_D_LEAK_LEFT, ORC_D_LEAK_RIGHT, ORC_D_ABSORBED,
    ORC_D_CENSUS, ORC_D_EVENTS, ORC_D_COLLISIONS, ORC_D_DRAWS,
    ORC_D_MAX_DRAWS, ORC_D_OVER_STRIDE, ORC_NDIAG
};

enum { EV_COLL = 0, EV_EDGE = 1, EV_TIME = 2 };

typedef struct {
    int32_t type;    /* EV_COLL, EV_EDGE or EV_TIME */
    int32_t cell;    /* cell the step was taken in */
    int32_t tbin;
    int32_t pad_;
    double s;        /* track length of the step */
} orc_event;

typedef struct {
    uint64_t x;              /* LCG state */
    const orc_lcg *lcg;
    const double *script;    /* when not NULL: uniforms are read from here */
    uint64_t n_script, pos;
    uint64_t draws;
    int exhausted;
} orc_rng;

static double rng_draw(orc_rng *R)
{
    R->draws++;
    if (R->script) {
        if (R->pos >= R->n_script) {
            R->exhausted = 1;
            return 0.5;
        }
        return R->script[R->pos++];
    }
    R->x = orc_lcg_next(R->x, R->lcg->g, R->lcg->c, R->lcg->m);
    return orc_uniform(R->x, R->lcg->m);
}

static u128 quantise(double s)
{
    double v = rint(s * 0x1p56);   /* s * 2^56 is exact; rint rounds half-even */
    return (u128)(uint64_t)v;
}

typedef struct {
    orc_event *log;
    uint64_t cap, n;
} orc_log;

static void log_event(orc_log *lg, int type, int cell, int tb, double s)
{
    if (!lg || !lg->log) return;
    if (lg->n < lg->cap) {
        orc_event *e = &lg->log[lg->n];
        e->type = type; e->cell = cell; e->tbin = tb; e->pad_ = 0; e->s = s;
    }
    lg->n++;
}

static void history_f64(const orc_problem *P, orc_rng *R, u128 *T, uint64_t *d, orc_log *lg)
{
    const int nc = P->n_cells, nt = P->n_time_bins, nsb = P->n_space_bins;
    const int timed = nt > 0;
    double x = P->edges[0], mu = 1.0, t = timed ? P->t_edges[0] : 0.0;
    int cell = 0, tb = 0;
    double tau = -orc_ln(rng_draw(R));
    for (;;) {
        const double sig = P->sigma_t[cell];
        double s = tau / sig;
        int ev = EV_COLL;
        double se;
        if (mu > 0.0)
            se = (P->edges[cell + 1] - x) / mu;
        else if (mu < 0.0)
            se = (P->edges[cell] - x) / mu;
        else
            se = INFINITY;
        if (se < s) { s = se; ev = EV_EDGE; }
        if (timed) {
            double st = P->t_edges[tb + 1] - t;
            if (st < s) { s = st; ev = EV_TIME; }
        }
        T[(size_t)tb * nsb + P->bin[cell]] += quantise(s);
        d[ORC_D_EVENTS]++;
        log_event(lg, ev, cell, tb, s);
        if (timed) {
            t = t + s;
            if (t > P->t_edges[tb + 1]) t = P->t_edges[tb + 1];
        }
        double dtau = sig * s;
        tau = tau - dtau;
        if (tau < 0.0) tau = 0.0;
        if (ev == EV_EDGE) {
            if (mu > 0.0) {
                cell = cell + 1;
                if (cell == nc) { d[ORC_D_LEAK_RIGHT]++; break; }
                x = P->edges[cell];
            } else {
                x = P->edges[cell];
                cell = cell - 1;
                if (cell < 0) { d[ORC_D_LEAK_LEFT]++; break; }
            }
            continue;
        }
        double step = mu * s;
        double nx = x + step;
        if (nx < P->edges[cell]) nx = P->edges[cell];
        if (nx > P->edges[cell + 1]) nx = P->edges[cell + 1];
        x = nx;
        if (ev == EV_TIME) {
            tb = tb + 1;
            t = P->t_edges[tb];
            if (tb == nt) { d[ORC_D_CENSUS]++; break; }
            continue;
        }
        d[ORC_D_COLLISIONS]++;
        double u1 = rng_draw(R);
        if (!(u1 < P->scatter[cell])) { d[ORC_D_ABSORBED]++; break; }
        double u2 = rng_draw(R);
        mu = 2.0 * u2 - 1.0;
        double u3 = rng_draw(R);
        tau = -orc_ln(u3);
    }
}

static void history_f32(const orc_problem *P, const float *W, const float *SG, const float *DT,
                        orc_rng *R, u128 *T, uint64_t *d, orc_log *lg)
{
    const int nc = P->n_cells, nt = P->n_time_bins, nsb = P->n_space_bins;
    const int timed = nt > 0;
    float xl = 0.0f, mu = 1.0f, tl = 0.0f;   /* position in the cell, time in the time bin */
    int cell = 0, tb = 0;
    double tau = -orc_ln(rng_draw(R));   /* the remaining optical depth stays double */
    for (;;) {
        const float sig = SG[cell], w = W[cell];
        float s = (float)tau / sig;
        int ev = EV_COLL;
        float se;
        if (mu > 0.0f)
            se = (w - xl) / mu;
        else if (mu < 0.0f)
            se = (0.0f - xl) / mu;
        else
            se = INFINITY;
        if (se < s) { s = se; ev = EV_EDGE; }
        if (timed) {
            float st = DT[tb] - tl;
            if (st < s) { s = st; ev = EV_TIME; }
        }
        T[(size_t)tb * nsb + P->bin[cell]] += quantise((double)s);
        d[ORC_D_EVENTS]++;
        log_event(lg, ev, cell, tb, (double)s);
        if (timed) {
            tl = tl + s;
            if (tl > DT[tb]) tl = DT[tb];
        }
        double dtau = (double)sig * (double)s;   /* exact: a product of two floats */
        tau = tau - dtau;
        if (tau < 0.0) tau = 0.0;
        if (ev == EV_EDGE) {
            if (mu > 0.0f) {
                cell = cell + 1;
                if (cell == nc) { d[ORC_D_LEAK_RIGHT]++; break; }
                xl = 0.0f;
            } else {
                cell = cell - 1;
                if (cell < 0) { d[ORC_D_LEAK_LEFT]++; break; }
                xl = W[cell];
            }
            continue;
        }
        float step = mu * s;
        float nx = xl + step;
        if (nx < 0.0f) nx = 0.0f;
        if (nx > w) nx = w;
        xl = nx;
        if (ev == EV_TIME) {
            tb = tb + 1;
            tl = 0.0f;
            if (tb == nt) { d[ORC_D_CENSUS]++; break; }
            continue;
        }
        d[ORC_D_COLLISIONS]++;
        double u1 = rng_draw(R);
        if (!(u1 < P->scatter[cell])) { d[ORC_D_ABSORBED]++; break; }
        double u2 = rng_draw(R);
        mu = (float)(2.0 * u2 - 1.0);
        double u3 = rng_draw(R);
        tau = -orc_ln(u3);
    }
}

/* FP32 copies, each rounded once from a double: cell widths
 * W[c] = (float)(E[c+1] - E[c]), total cross sections, time-bin durations
 * DT[t] = (float)(T[t+1] - T[t]). */
static float *f32_tables(const orc_problem *P, float **W, float **SG, float **DT)
{
    const int nc = P->n_cells, nt = P->n_time_bins;
    float *f = (float *)calloc((size_t)(2 * nc + nt + 1), sizeof(float));
    if (!f) return NULL;
    *W = f;
    *SG = f + nc;
    *DT = f + 2 * nc;
    for (int i = 0; i < nc; ++i) {
        (*W)[i] = (float)(P->edges[i + 1] - P->edges[i]);
        (*SG)[i] = (float)P->sigma_t[i];
    }
    for (int i = 0; i < nt; ++i) (*DT)[i] = (float)(P->t_edges[i + 1] - P->t_edges[i]);
    return f;
}

/* Tally slice sizes: per batch, n_time_bins' x n_space_bins, with
 * n_time_bins' = max(n_time_bins, 1). */
static size_t slice_bins(const orc_problem *P)
{
    size_t ntb = P->n_time_bins > 0 ? (size_t)P->n_time_bins : 1;
    return ntb * (size_t)P->n_space_bins;
}

/* History j (0-based within the problem) belongs to batch
 * floor(j / ceil(N / n_batches)). */
static uint64_t batch_of(const orc_problem *P, uint64_t j)
{
    uint64_t nb = P->n_batches ? P->n_batches : 1;
    uint64_t bs = (P->n_histories + nb - 1) / nb;
    if (bs == 0) bs = 1;
    return j / bs;
}

static void update_diag_history(const orc_problem *P, uint64_t *d, uint64_t draws)
{
    d[ORC_D_HISTORIES]++;
    d[ORC_D_DRAWS] += draws;
    if (draws > d[ORC_D_MAX_DRAWS]) d[ORC_D_MAX_DRAWS] = draws;
    if (P->seeding.kind == ORC_SEED_STRIDE && draws > P->seeding.stride)
        d[ORC_D_OVER_STRIDE]++;
}

/* Runs histories j0 .. j1-1 of the problem and ADDS their tallies into
 * tally_lo/tally_hi (each 128-bit bin sum split in two 64-bit words; the
 * arrays hold n_batches x slice_bins entries) and their counts into diag
 * (ORC_NDIAG words; ORC_D_MAX_DRAWS is a maximum).  float_mode selects the
 * FP32 flight arithmetic.  Returns 0, or -1 on a bad argument. */
int orc_transport(const orc_problem *P, int float_mode, uint64_t j0, uint64_t j1,
                  uint64_t *tally_lo, uint64_t *tally_hi, uint64_t *diag)
{
    if (!P || !tally_lo || !tally_hi || !diag) return -1;
    if (P->n_cells < 1 || P->n_space_bins < 1 || P->n_time_bins < 0) return -1;
    if (P->lcg.m < 53 || P->lcg.m > 64) return -1;
    const size_t sb = slice_bins(P);
    const size_t nb = P->n_batches ? P->n_batches : 1;
    const size_t need = sb * nb;
    /* 128-bit accumulators for this call, added into the caller's words at the end */
    u128 *acc = (u128 *)calloc(need, sizeof(u128));
    float *W32 = NULL, *SG32 = NULL, *DT32 = NULL;
    float *f32 = f32_tables(P, &W32, &SG32, &DT32);
    if (!acc || !f32) { free(acc); free(f32); return -1; }
    for (uint64_t j = j0; j < j1; ++j) {
        orc_rng R;
        memset(&R, 0, sizeof R);
        R.lcg = &P->lcg;
        R.x = orc_stream_start(&P->lcg, &P->seeding, j);
        u128 *T = acc + (size_t)batch_of(P, j) * sb;
        if (float_mode)
            history_f32(P, W32, SG32, DT32, &R, T, diag, NULL);
        else
            history_f64(P, &R, T, diag, NULL);
        update_diag_history(P, diag, R.draws);
    }
    for (size_t i = 0; i < need; ++i) {
        u128 cur = ((u128)tally_hi[i] << 64) | tally_lo[i];
        cur += acc[i];
        tally_lo[i] = (uint64_t)cur;
        tally_hi[i] = (uint64_t)(cur >> 64);
    }
    free(acc);
    free(f32);
    return 0;
}

/* One history driven by a given list of uniforms instead of an LCG (for
 * unit tests of the transport steps).  Tallies of that one history go to
 * tally_lo/tally_hi (one slice, overwritten), its events to log (up to
 * log_cap entries; *log_n receives the full count).  Returns the number of
 * uniforms consumed, or -1 if the script ran out or an argument is bad. */
int64_t orc_transport_scripted(const orc_problem *P, int float_mode,
                               const double *u, uint64_t n_u,
                               uint64_t *tally_lo, uint64_t *tally_hi, uint64_t *diag,
                               orc_event *log, uint64_t log_cap, uint64_t *log_n)
{
    if (!P || !u || !tally_lo || !tally_hi || !diag) return -1;
    const size_t sb = slice_bins(P);
    u128 T[4096];
    if (sb > 4096) return -1;
    memset(T, 0, sizeof T);
    orc_rng R;
    memset(&R, 0, sizeof R);
    R.lcg = &P->lcg;
    R.script = u;
    R.n_script = n_u;
    orc_log lg = { log, log_cap, 0 };
    if (float_mode) {
        float *W32 = NULL, *SG32 = NULL, *DT32 = NULL;
        float *f32 = f32_tables(P, &W32, &SG32, &DT32);
        if (!f32) return -1;
        history_f32(P, W32, SG32, DT32, &R, T, diag, &lg);
        free(f32);
    } else {
        history_f64(P, &R, T, diag, &lg);
    }
    update_diag_history(P, diag, R.draws);
    for (size_t i = 0; i < sb; ++i) {
        tally_lo[i] = (uint64_t)T[i];
        tally_hi[i] = (uint64_t)(T[i] >> 64);
    }
    if (log_n) *log_n = lg.n;
    if (R.exhausted) return -1;
    return (int64_t)R.pos;
}

/* ------------------------------------------------------------------ */
/* Supercritical pulse in an infinite homogeneous medium: the paper's test
 * problem (Sec. "Implementation and Results"): a pulse of particles at
 * x = 0, t = 0 in an infinite medium with total cross section sigma_t,
 * isotropic scattering ratio c = Sigma_s / Sigma_t and scattering
 * multiplicity nu (c nu is the multiplication factor), run to a census
 * time; the flux averaged over a central interval [x_lo, x_hi] is tallied
 * with the collision estimator in time bins.
 *
 * Secondary particles (Sec. "On-Demand Seed Splitting", eq. 5):
 *   hash seeding:   the k-th particle emerging from a scattering (k = 1..n)
 *                   starts its own stream at hash(k, X_p) mod 2^m, where X_p
 *                   is the parent's state after the scattering's draws;
 *   stride seeding: only source particles receive streams (X_{Q i}); the
 *                   particles a source gives rise to draw from the source's
 *                   stream one after another, depth first: the first
 *                   emerging particle continues at once, its siblings wait
 *                   on a last-in-first-out stack (siblings are identical
 *                   until they draw, so their order among themselves does
 *                   not matter).
 * Source i (0-based) of batch b has the global batch id B = first_batch + b:
 *   hash:   S = hash(i + 1, hash(B + 1, base))   (eq. 4, batch id first)
 *   stride: S = X_{Q (B per_batch + i)}           (X_0 = base)
 *
 * Readings (the paper gives the problem, not these details):
 *   start:     a particle's first draw u gives its direction mu = 2u - 1
 *              (isotropic); sources start at x = 0, t = 0, secondaries at
 *              their parent's collision site and time;
 *   flight:    draw u, tau = -ln(u) (orc_ln), s = tau / sigma_t; with
 *              tn = t + s: if tn < T_end the particle moves to x + mu s
 *              (x = x + (mu * s)) and t = tn and collides there, else it
 *              reaches the census and ends (no score);
 *   score:     a collision with x_lo <= x <= x_hi and t >= T[0] adds 1 to
 *              its batch and time bin b with T[b] <= t < T[b+1];
 *   collision: draw u1; absorbed unless u1 < c; else draw u2 and
 *              n = floor(nu) + (u2 < nu - floor(nu)) particles emerge (the
 *              parent ends; n may be 0);
 *   flux:      count / (((sigma_t N_b) (x_hi - x_lo)) (T[b+1] - T[b])),
 *              N_b = per_batch, one IEEE operation per step.
 * T_end is the last time edge.  Every floating-point step is one IEEE
 * double operation, rounded to nearest, without contraction.
 */
/* ------------------------------------------------------------------ */

typedef struct {
    double sigma_t, scatter, nu;
    double x_lo, x_hi;
    int32_t n_time_bins;        /* >= 1 */
    uint32_t n_batches;         /* >= 1 */
    const double *t_edges;      /* n_time_bins + 1 */
    uint64_t per_batch;         /* sources per batch */
    uint64_t first_batch;       /* global id of batch 0 */
    orc_lcg lcg;
    orc_seeding seeding;        /* kind, base, stride used */
    /* population control (orc_pulse_pc_run only): census every census_every
     * time bins, pc_target particles per batch after each census, one-off
     * values from the global seed pc_seed */
    uint32_t census_every;
    uint64_t pc_target;
    uint64_t pc_seed;
} orc_pulse;

enum {
    ORC_P_SOURCES = 0, ORC_P_COLLISIONS, ORC_P_TALLIED, ORC_P_SCATTERS,
    ORC_P_ABSORBED, ORC_P_CENSUS, ORC_P_SECONDARIES, ORC_P_DRAWS,
    ORC_P_MAX_DRAWS, ORC_P_OVER_STRIDE, ORC_P_NDIAG
};

/* a particle waiting to start: position, time, time bin, and (hash
 * seeding) its stream's start state; `count` identical stride siblings */
typedef struct {
    double x, t;
    int32_t tb;
    uint32_t count;
    uint64_t seed;
} orc_pending;

typedef struct {
    orc_pending *a;
    size_t n, cap;
} orc_stack;

static int stack_push(orc_stack *S, orc_pending e)
{
    if (S->n == S->cap) {
        size_t nc = S->cap ? 2 * S->cap : 64;
        orc_pending *na = (orc_pending *)realloc(S->a, nc * sizeof *na);
        if (!na) return -1;
        S->a = na;
        S->cap = nc;
    }
    S->a[S->n++] = e;
    return 0;
}

/* time bin of t: the largest b < n_time_bins with T[b] <= t, starting the
 * search from the bin of an earlier time; -1 before T[0] */
static int32_t advance_tbin(const orc_pulse *P, int32_t tb, double t)
{
    while (tb + 1 < P->n_time_bins && P->t_edges[tb + 1] <= t) ++tb;
    return tb;
}

/* a particle at its start: position, time, time bin; a census copy keeps
 * its direction (has_mu), every other particle draws one first */
typedef struct {
    double x, t;
    int32_t tb;
    int has_mu;
    double mu;
} orc_start;

enum { ORC_END_CENSUS = 0, ORC_END_ABSORBED = 1, ORC_END_SCATTERED = 2 };

/* Runs one particle from its start s0 to its end with random numbers from
 * R; t_cen is the census time (the last time edge, or the next census of a
 * population-controlled run).  Adds its scores to cnt (the batch's
 * n_time_bins counters) and its counts to d.  Returns the outcome;
 * *n_out receives the number of emerging particles (0 unless it scattered)
 * and *at the end point: the collision site (scattered), or the census
 * point x + mu (t_cen - t), t_cen with the particle's direction (census). */
static int pulse_particle(const orc_pulse *P, orc_rng *R, const orc_start *s0, double t_cen,
                          uint64_t *cnt, uint64_t *d, uint32_t *n_out, orc_start *at)
{
    const double nu_floor = floor(P->nu);
    const double nu_frac = P->nu - nu_floor;
    double x = s0->x, t = s0->t;
    int32_t tb = s0->tb;
    *n_out = 0;
    double mu = s0->has_mu ? s0->mu : 2.0 * rng_draw(R) - 1.0;
    double tau = -orc_ln(rng_draw(R));
    double s = tau / P->sigma_t;
    double tn = t + s;
    if (!(tn < t_cen)) {
        double rest = t_cen - t;
        double step = mu * rest;
        at->x = x + step;
        at->t = t_cen;
        at->tb = tb;
        at->has_mu = 1;
        at->mu = mu;
        d[ORC_P_CENSUS]++;
        return ORC_END_CENSUS;
    }
    double step = mu * s;
    x = x + step;
    t = tn;
    tb = advance_tbin(P, tb, t);
    d[ORC_P_COLLISIONS]++;
    if (tb >= 0 && P->x_lo <= x && x <= P->x_hi) {
        cnt[tb]++;
        d[ORC_P_TALLIED]++;
    }
    double u1 = rng_draw(R);
    if (!(u1 < P->scatter)) { d[ORC_P_ABSORBED]++; return ORC_END_ABSORBED; }
    double u2 = rng_draw(R);
    uint32_t n = (uint32_t)nu_floor + (u2 < nu_frac ? 1u : 0u);
    d[ORC_P_SCATTERS]++;
    d[ORC_P_SECONDARIES] += n;
    *n_out = n;
    at->x = x;
    at->t = t;
    at->tb = tb;
    at->has_mu = 0;
    at->mu = 0.0;
    return ORC_END_SCATTERED;
}

static void note_stream(const orc_pulse *P, uint64_t *d, uint64_t draws)
{
    d[ORC_P_DRAWS] += draws;
    if (draws > d[ORC_P_MAX_DRAWS]) d[ORC_P_MAX_DRAWS] = draws;
    if (P->seeding.kind == ORC_SEED_STRIDE && draws > P->seeding.stride) d[ORC_P_OVER_STRIDE]++;
}

/* per-particle record of a traced family (tests) */
typedef struct {
    uint64_t start, end;     /* stream state when the particle starts / ends */
    double x0, t0;           /* start position and time */
    uint32_t n_out;          /* particles emerging from its end (0 unless it scattered) */
    uint32_t draws;          /* numbers drawn by the particle */
} orc_ptrace;

typedef struct {
    orc_ptrace *a;
    uint64_t cap, n;
} orc_plog;

/* a census arrival of a population-controlled run: position at the census
 * time, direction, and the stream state after the particle's draws */
typedef struct {
    double x, mu;
    uint64_t X;
} orc_cpoint;

typedef struct {
    orc_cpoint *a;
    size_t n, cap;
} orc_clist;

static int clist_push(orc_clist *L, orc_cpoint e)
{
    if (L->n == L->cap) {
        size_t nc = L->cap ? 2 * L->cap : 256;
        orc_cpoint *na = (orc_cpoint *)realloc(L->a, nc * sizeof *na);
        if (!na) return -1;
        L->a = na;
        L->cap = nc;
    }
    L->a[L->n++] = e;
    return 0;
}

/* One starting particle (a source, or a census copy) and everything it
 * gives rise to, up to the census time t_cen.  Stride seeding: one stream
 * for the whole family (R), depth first.  Hash seeding: each particle its
 * own stream; the family is walked depth first too, which for hash seeding
 * is only one of many orders that give the same counts.  With `census`
 * given, particles reaching t_cen are appended to it (population control);
 * otherwise they end there. */
static int pulse_family(const orc_pulse *P, orc_rng *R, const orc_start *first, double t_cen,
                        uint64_t *cnt, uint64_t *d, orc_stack *S, orc_plog *lg, orc_clist *census)
{
    const int hash = P->seeding.kind == ORC_SEED_HASH;
    const uint64_t msk = mask_of(P->lcg.m);
    orc_start cur = *first;
    S->n = 0;
    for (;;) {
        uint32_t n = 0;
        orc_start at;
        memset(&at, 0, sizeof at);
        const uint64_t start = R->x, draws0 = R->draws;
        const int end = pulse_particle(P, R, &cur, t_cen, cnt, d, &n, &at);
        if (lg && lg->a) {
            if (lg->n < lg->cap) {
                orc_ptrace *e = &lg->a[lg->n];
                e->start = start; e->end = R->x; e->x0 = cur.x; e->t0 = cur.t;
                e->n_out = n; e->draws = (uint32_t)(R->draws - draws0);
            }
            lg->n++;
        }
        if (end == ORC_END_CENSUS && census) {
            orc_cpoint cp = { at.x, at.mu, R->x };
            if (clist_push(census, cp)) return -1;
        }
        if (hash) {
            /* this particle's stream ends here */
            note_stream(P, d, R->draws);
            for (uint32_t k = n; k >= 1; --k) {   /* k = 1 ends on top */
                orc_pending e = { at.x, at.t, at.tb, 1, orc_hash(k, R->x) & msk };
                if (stack_push(S, e)) return -1;
            }
        } else if (n > 0) {
            orc_pending e = { at.x, at.t, at.tb, n, 0 };
            if (stack_push(S, e)) return -1;
        }
        if (S->n == 0) break;
        orc_pending *top = &S->a[S->n - 1];
        cur.x = top->x;
        cur.t = top->t;
        cur.tb = top->tb;
        cur.has_mu = 0;
        cur.mu = 0.0;
        if (hash) {
            R->x = top->seed;
            R->draws = 0;
            S->n--;
        } else if (--top->count == 0) {
            S->n--;
        }
    }
    if (!hash) note_stream(P, d, R->draws);
    return 0;
}

static orc_start source_start(const orc_pulse *P)
{
    orc_start s = { 0.0, 0.0, advance_tbin(P, -1, 0.0), 0, 0.0 };
    return s;
}

static int pulse_check(const orc_pulse *P)
{
    if (!P || P->n_time_bins < 1 || !P->t_edges || P->n_batches < 1) return -1;
    if (P->lcg.m < 53 || P->lcg.m > 64) return -1;
    if (!(P->sigma_t > 0) || !(P->scatter >= 0 && P->scatter <= 1) || !(P->nu >= 0 && P->nu <= 64)) return -1;
    return 0;
}

/* Runs batches b0 .. b1-1 (every source of each) and ADDS their scores into
 * counts (n_batches x n_time_bins) and their counts into diag
 * (ORC_P_NDIAG words; ORC_P_MAX_DRAWS is a maximum).  Returns 0 or -1. */
int orc_pulse_run(const orc_pulse *P, uint64_t b0, uint64_t b1, uint64_t *counts, uint64_t *diag)
{
    if (pulse_check(P) || !counts || !diag || b1 > P->n_batches) return -1;
    orc_stack S = { NULL, 0, 0 };
    int rc = 0;
    for (uint64_t b = b0; b < b1 && rc == 0; ++b) {
        const uint64_t B = P->first_batch + b;
        const uint64_t parent = orc_hash(B + 1, P->seeding.base);
        for (uint64_t i = 0; i < P->per_batch && rc == 0; ++i) {
            orc_rng R;
            memset(&R, 0, sizeof R);
            R.lcg = &P->lcg;
            if (P->seeding.kind == ORC_SEED_HASH)
                R.x = orc_hash(i + 1, parent) & mask_of(P->lcg.m);
            else
                R.x = orc_skip(P->seeding.base & mask_of(P->lcg.m), P->seeding.stride * (B * P->per_batch + i),
                               P->lcg.g, P->lcg.c, P->lcg.m);
            const orc_start s0 = source_start(P);
            diag[ORC_P_SOURCES]++;
            rc = pulse_family(P, &R, &s0, P->t_edges[P->n_time_bins], counts + b * (uint64_t)P->n_time_bins,
                              diag, &S, NULL, NULL);
        }
    }
    free(S.a);
    return rc;
}

/* One source family driven by a given list of uniforms (stride-seeding
 * semantics: the whole family draws from the list in order).  Scores go to
 * counts (n_time_bins, overwritten).  Returns the number of uniforms used,
 * or -1 if the list ran out or an argument is bad. */
int64_t orc_pulse_scripted(const orc_pulse *P, const double *u, uint64_t n_u, uint64_t *counts,
                           uint64_t *diag)
{
    if (pulse_check(P) || !u || !counts || !diag || P->seeding.kind != ORC_SEED_STRIDE) return -1;
    memset(counts, 0, (size_t)P->n_time_bins * sizeof *counts);
    orc_stack S = { NULL, 0, 0 };
    orc_rng R;
    memset(&R, 0, sizeof R);
    R.lcg = &P->lcg;
    R.script = u;
    R.n_script = n_u;
    const orc_start s0 = source_start(P);
    diag[ORC_P_SOURCES]++;
    int rc = pulse_family(P, &R, &s0, P->t_edges[P->n_time_bins], counts, diag, &S, NULL, NULL);
    free(S.a);
    if (rc || R.exhausted) return -1;
    return (int64_t)R.pos;
}

/* Source i of batch b alone, with every particle of its family recorded in
 * processing order (up to cap records; *n receives the full number).
 * Scores go to counts (n_time_bins, overwritten).  Returns 0 or -1. */
int orc_pulse_trace(const orc_pulse *P, uint64_t b, uint64_t i, uint64_t *counts, uint64_t *diag,
                    orc_ptrace *log, uint64_t cap, uint64_t *n)
{
    if (pulse_check(P) || !counts || !diag || b >= P->n_batches) return -1;
    memset(counts, 0, (size_t)P->n_time_bins * sizeof *counts);
    const uint64_t B = P->first_batch + b;
    orc_rng R;
    memset(&R, 0, sizeof R);
    R.lcg = &P->lcg;
    if (P->seeding.kind == ORC_SEED_HASH)
        R.x = orc_hash(i + 1, orc_hash(B + 1, P->seeding.base)) & mask_of(P->lcg.m);
    else
        R.x = orc_skip(P->seeding.base & mask_of(P->lcg.m), P->seeding.stride * (B * P->per_batch + i),
                       P->lcg.g, P->lcg.c, P->lcg.m);
    orc_stack S = { NULL, 0, 0 };
    orc_plog lg = { log, cap, 0 };
    const orc_start s0 = source_start(P);
    diag[ORC_P_SOURCES]++;
    int rc = pulse_family(P, &R, &s0, P->t_edges[P->n_time_bins], counts, diag, &S, &lg, NULL);
    free(S.a);
    if (n) *n = lg.n;
    return rc;
}

/* Flux of each (batch, time bin) from the integer counts. */
void orc_pulse_flux(const orc_pulse *P, const uint64_t *counts, double *flux)
{
    const double dx = P->x_hi - P->x_lo;
    for (uint32_t b = 0; b < P->n_batches; ++b)
        for (int32_t k = 0; k < P->n_time_bins; ++k) {
            const double dt = P->t_edges[k + 1] - P->t_edges[k];
            const double den = ((P->sigma_t * (double)P->per_batch) * dx) * dt;
            flux[(size_t)b * P->n_time_bins + k] = (double)counts[(size_t)b * P->n_time_bins + k] / den;
        }
}

/* ------------------------------------------------------------------ */
/* Population control at census times with one-off hashed values (Sec.
 * "Hierarchical Seed Splitting": where a full stream is not needed, as for
 * population control, a hash of a per-phase seed gives one-off values, each
 * under its own key).  Hash seeding only.
 *
 * Readings (the paper names the use, not the scheme):
 *   census:    with K = census_every, census c (0-based) is at the time edge
 *              T[(c+1) K], for every (c+1) K < n_time_bins; epoch e runs from
 *              the previous census (or t = 0) to the next census (or the
 *              last edge).  A particle whose flight reaches the census time
 *              C stops there at x + mu (C - t) (x = x + (mu * (C - t))) with
 *              its direction and stream state; its remaining flight is not
 *              kept (exponential flights are memoryless);
 *   control:   per batch, N particles reach census c; M = pc_target.  With
 *              q = floor(M / N), r = M mod N, particle i (state X_i) leaves
 *              n_i = q + [u_i < r / N] copies, so E[sum n_i] = M, where
 *                u_i = U(hash(X_i, Phi) mod 2^m),
 *                Phi = hash(c + 1, hash(B + 1, pc_seed))   (B the batch id)
 *              is the one-off value: the per-phase seed Phi is the parent,
 *              the particle's own state its key.  U is the uniform mapping
 *              ((S >> (m-53)) + 1) 2^-53, and the test is the exact integer
 *              comparison ((S >> (m-53)) + 1) N < r 2^53;
 *   copies:    copy k (k = 1..n_i) starts at the census point with the
 *              particle's direction (no direction draw) and the stream
 *              hash(k, X_i) mod 2^m (eq. 5: the copies are the particle's
 *              children at the census);
 *   weights:   every particle of a batch carries the same weight in an
 *              epoch: 1 in epoch 0 and w_{c+1} = (w_c N_c) / M after census
 *              c, so the counts stay integers and the flux of a time bin
 *              of epoch e is ((double)count w_e) / den, den as in the plain
 *              problem.
 * The batches are independent, so a batch is run whole, epoch by epoch. */
/* ------------------------------------------------------------------ */

static uint32_t pc_n_census(const orc_pulse *P)
{
    if (P->census_every == 0) return 0;
    return (uint32_t)((uint32_t)(P->n_time_bins - 1) / P->census_every);
}

/* a census copy waiting to start: census point, direction, stream start */
typedef struct {
    double x, mu;
    uint64_t seed;
} orc_copy;

/* number of copies particle X leaves at a census of N particles */
static uint64_t pc_copies(const orc_pulse *P, uint64_t phi, uint64_t X, uint64_t N)
{
    const uint64_t M = P->pc_target;
    const uint64_t q = M / N, r = M % N;
    const uint64_t S = orc_hash(X, phi) & mask_of(P->lcg.m);
    const u128 j1 = (u128)((S >> (P->lcg.m - 53)) + 1);
    const int extra = j1 * (u128)N < ((u128)r << 53);
    return q + (uint64_t)extra;
}

/* Runs batches b0 .. b1-1 of a population-controlled problem and ADDS their
 * scores into counts, their counts into diag (as orc_pulse_run) and writes
 * pop[b][c][0] = particles of batch b reaching census c, pop[b][c][1] =
 * copies leaving it (pop: n_batches x n_census x 2, may be NULL).  Returns
 * 0, or -1 for a bad argument or an allocation failure. */
int orc_pulse_pc_run(const orc_pulse *P, uint64_t b0, uint64_t b1, uint64_t *counts, uint64_t *diag,
                     uint64_t *pop)
{
    if (pulse_check(P) || !counts || !diag || b1 > P->n_batches) return -1;
    if (P->seeding.kind != ORC_SEED_HASH || P->census_every == 0 || P->pc_target == 0) return -1;
    const uint32_t nc = pc_n_census(P);
    const uint64_t msk = mask_of(P->lcg.m);
    orc_stack S = { NULL, 0, 0 };
    orc_clist cl = { NULL, 0, 0 };
    orc_copy *items = NULL, *next = NULL;
    size_t cap_items = 0, cap_next = 0;
    int rc = 0;
    for (uint64_t b = b0; b < b1 && rc == 0; ++b) {
        const uint64_t B = P->first_batch + b;
        uint64_t *cnt = counts + b * (uint64_t)P->n_time_bins;
        const uint64_t parent = orc_hash(B + 1, P->seeding.base);
        size_t n_items = 0;
        for (uint32_t e = 0; e <= nc && rc == 0; ++e) {
            const double t_cen = (e < nc) ? P->t_edges[(size_t)(e + 1) * P->census_every]
                                          : P->t_edges[P->n_time_bins];
            cl.n = 0;
            const uint64_t n_start = (e == 0) ? P->per_batch : n_items;
            for (uint64_t i = 0; i < n_start && rc == 0; ++i) {
                orc_rng R;
                memset(&R, 0, sizeof R);
                R.lcg = &P->lcg;
                orc_start s0;
                if (e == 0) {
                    s0 = source_start(P);
                    R.x = orc_hash(i + 1, parent) & msk;
                    diag[ORC_P_SOURCES]++;
                } else {
                    s0.x = items[i].x;
                    s0.t = P->t_edges[(size_t)e * P->census_every];
                    s0.tb = (int32_t)(e * P->census_every);
                    s0.has_mu = 1;
                    s0.mu = items[i].mu;
                    R.x = items[i].seed;
                }
                rc = pulse_family(P, &R, &s0, t_cen, cnt, diag, &S, NULL, (e < nc) ? &cl : NULL);
            }
            if (rc || e == nc) break;
            /* population control at census e */
            const uint64_t N = cl.n;
            const uint64_t phi = orc_hash((uint64_t)e + 1, orc_hash(B + 1, P->pc_seed));
            size_t n_next = 0;
            for (size_t i = 0; i < cl.n && rc == 0; ++i) {
                const uint64_t n = pc_copies(P, phi, cl.a[i].X, N);
                for (uint64_t k = 1; k <= n; ++k) {
                    if (n_next == cap_next) {
                        size_t ncap = cap_next ? 2 * cap_next : 1024;
                        orc_copy *na = (orc_copy *)realloc(next, ncap * sizeof *na);
                        if (!na) { rc = -1; break; }
                        next = na;
                        cap_next = ncap;
                    }
                    orc_copy cp = { cl.a[i].x, cl.a[i].mu, orc_hash(k, cl.a[i].X) & msk };
                    next[n_next++] = cp;
                }
            }
            if (pop) {
                pop[(b * nc + e) * 2] = N;
                pop[(b * nc + e) * 2 + 1] = n_next;
            }
            orc_copy *tmp = items; items = next; next = tmp;
            size_t tc = cap_items; cap_items = cap_next; cap_next = tc;
            n_items = n_next;
        }
    }
    free(S.a);
    free(cl.a);
    free(items);
    free(next);
    return rc;
}

/* Flux of a population-controlled run: epoch weights from the census
 * populations (pop as written by orc_pulse_pc_run). */
void orc_pulse_pc_flux(const orc_pulse *P, const uint64_t *counts, const uint64_t *pop, double *flux)
{
    const uint32_t nc = pc_n_census(P);
    const double dx = P->x_hi - P->x_lo;
    for (uint32_t b = 0; b < P->n_batches; ++b) {
        double w = 1.0;
        uint32_t e = 0;
        for (int32_t k = 0; k < P->n_time_bins; ++k) {
            while (e < nc && (uint32_t)k >= (e + 1) * P->census_every) {
                w = (w * (double)pop[((size_t)b * nc + e) * 2]) / (double)P->pc_target;
                ++e;
            }
            const double dt = P->t_edges[k + 1] - P->t_edges[k];
            const double den = ((P->sigma_t * (double)P->per_batch) * dx) * dt;
            flux[(size_t)b * P->n_time_bins + k] = ((double)counts[(size_t)b * P->n_time_bins + k] * w) / den;
        }
    }
}

/* One source family driven by a list of uniforms (stride semantics) up to
 * the first census T[census_every]: scores into counts (n_time_bins,
 * overwritten) and the census arrivals (x, mu) into cx, cmu (up to cap;
 * *n_census receives their number).  Returns the uniforms used, or -1. */
int64_t orc_pulse_pc_scripted(const orc_pulse *P, const double *u, uint64_t n_u, uint64_t *counts,
                              uint64_t *diag, double *cx, double *cmu, uint64_t cap, uint64_t *n_census)
{
    if (pulse_check(P) || !u || !counts || !diag || P->seeding.kind != ORC_SEED_STRIDE) return -1;
    if (P->census_every == 0 || (int32_t)P->census_every >= P->n_time_bins) return -1;
    memset(counts, 0, (size_t)P->n_time_bins * sizeof *counts);
    orc_stack S = { NULL, 0, 0 };
    orc_clist cl = { NULL, 0, 0 };
    orc_rng R;
    memset(&R, 0, sizeof R);
    R.lcg = &P->lcg;
    R.script = u;
    R.n_script = n_u;
    const orc_start s0 = source_start(P);
    diag[ORC_P_SOURCES]++;
    int rc = pulse_family(P, &R, &s0, P->t_edges[P->census_every], counts, diag, &S, NULL, &cl);
    for (size_t i = 0; i < cl.n && i < cap; ++i) {
        cx[i] = cl.a[i].x;
        cmu[i] = cl.a[i].mu;
    }
    if (n_census) *n_census = cl.n;
    free(S.a);
    free(cl.a);
    if (rc || R.exhausted) return -1;
    return (int64_t)R.pos;
}

/* The census arrivals of batch b at census c of a population-controlled
 * run, and the copies leaving it (tests): states X (up to cap) and the
 * copies' start states in arrival order, copy k of arrival i at
 * position sum_{i' < i} n_i' + k - 1 (up to cap); *n_arr and *n_cop receive
 * the full numbers.  Returns 0 or -1. */
int orc_pulse_pc_census(const orc_pulse *P, uint64_t b, uint32_t c, uint64_t *arr, uint64_t *cop, uint64_t cap,
                        uint64_t *n_arr, uint64_t *n_cop)
{
    if (pulse_check(P) || b >= P->n_batches || P->seeding.kind != ORC_SEED_HASH || P->pc_target == 0) return -1;
    const uint32_t nc = pc_n_census(P);
    if (c >= nc) return -1;
    const uint64_t msk = mask_of(P->lcg.m);
    const uint64_t B = P->first_batch + b;
    const uint64_t parent = orc_hash(B + 1, P->seeding.base);
    uint64_t *cnt = (uint64_t *)calloc((size_t)P->n_time_bins, sizeof *cnt);
    uint64_t d[ORC_P_NDIAG];
    memset(d, 0, sizeof d);
    orc_stack S = { NULL, 0, 0 };
    orc_clist cl = { NULL, 0, 0 };
    orc_copy *items = NULL;
    size_t n_items = 0, cap_items = 0;
    int rc = cnt ? 0 : -1;
    for (uint32_t e = 0; e <= c && rc == 0; ++e) {
        const double t_cen = P->t_edges[(size_t)(e + 1) * P->census_every];
        cl.n = 0;
        const uint64_t n_start = (e == 0) ? P->per_batch : n_items;
        for (uint64_t i = 0; i < n_start && rc == 0; ++i) {
            orc_rng R;
            memset(&R, 0, sizeof R);
            R.lcg = &P->lcg;
            orc_start s0;
            if (e == 0) {
                s0 = source_start(P);
                R.x = orc_hash(i + 1, parent) & msk;
            } else {
                s0.x = items[i].x;
                s0.t = P->t_edges[(size_t)e * P->census_every];
                s0.tb = (int32_t)(e * P->census_every);
                s0.has_mu = 1;
                s0.mu = items[i].mu;
                R.x = items[i].seed;
            }
            rc = pulse_family(P, &R, &s0, t_cen, cnt, d, &S, NULL, &cl);
        }
        if (rc) break;
        const uint64_t N = cl.n;
        const uint64_t phi = orc_hash((uint64_t)e + 1, orc_hash(B + 1, P->pc_seed));
        size_t n_new = 0;
        orc_copy *nw = NULL;
        size_t cap_new = 0;
        for (size_t i = 0; i < cl.n && rc == 0; ++i) {
            const uint64_t n = pc_copies(P, phi, cl.a[i].X, N);
            for (uint64_t k = 1; k <= n; ++k) {
                if (n_new == cap_new) {
                    size_t ncap = cap_new ? 2 * cap_new : 1024;
                    orc_copy *na = (orc_copy *)realloc(nw, ncap * sizeof *na);
                    if (!na) { rc = -1; break; }
                    nw = na;
                    cap_new = ncap;
                }
                orc_copy cp = { cl.a[i].x, cl.a[i].mu, orc_hash(k, cl.a[i].X) & msk };
                nw[n_new++] = cp;
            }
        }
        if (e == c) {
            for (size_t i = 0; i < cl.n && i < cap; ++i) arr[i] = cl.a[i].X;
            for (size_t i = 0; i < n_new && i < cap; ++i) cop[i] = nw[i].seed;
            *n_arr = cl.n;
            *n_cop = n_new;
        }
        free(items);
        items = nw;
        n_items = n_new;
        cap_items = cap_new;
    }
    (void)cap_items;
    free(cnt);
    free(S.a);
    free(cl.a);
    free(items);
    return rc;
}

/* 128-bit unsigned integer to double, rounded to nearest, ties to even:
 * the plain definition is "the double nearest to the integer"; long double
 * is not used so that the rounding is explicit. */
double orc_u128_to_f64(uint64_t lo, uint64_t hi)
{
    u128 v = ((u128)hi << 64) | lo;
    if (v == 0) return 0.0;
    int nbits = 128;
    while (!((v >> (nbits - 1)) & 1)) --nbits;   /* bit length */
    if (nbits <= 53) return (double)(uint64_t)v;
    int sh = nbits - 53;
    u128 mant = v >> sh;
    u128 rem = v - (mant << sh);
    u128 half = (u128)1 << (sh - 1);
    if (rem > half || (rem == half && (mant & 1))) mant += 1;
    /* mant may have become 2^53: ldexp handles it exactly */
    return ldexp((double)(uint64_t)mant, sh);
}
