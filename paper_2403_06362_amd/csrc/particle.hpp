// One particle event: the per-history arithmetic shared by the history-based
// and the event-sorted schedules, so that both run the identical operation
// sequence for every particle.
//
// An event is split in three parts that a schedule may run at different
// times for one particle (never reordered, never skipped):
//   sample_tau   X = lcg(X); tau = -ln(uniform(X))                 (the flight)
//   geom_*       distances to collision / edge / time, choice, score,
//                move; returns END_*, END_NONE (edge or time step) or
//                STEP_COLLIDE (the particle stands at its collision site)
//   collide      X = lcg(X), absorbed unless uniform < c; X = lcg(X),
//                mu = R(2 u - 1); the next part is sample_tau
// Every floating-point result is the IEEE operation's, rounded to nearest,
// with no fused multiply-add where the operation is a separate multiply and
// add (the library is built with -ffp-contract=off).  Divisions by a
// cell's sigma_t and by the flight's mu go through the divisor's refined
// reciprocal (quot, device_rng.hpp), which gives the correctly rounded
// quotient; minima and maxima are the compare-and-replace clamps of the
// operation sequence (their operands are never NaN, and a zero's sign never
// reaches a tally, a decision or a stored state).
#pragma once

#include <type_traits>

#include "internal.hpp"

namespace mcrng {

template <bool F32>
struct Particle {
    using R = typename std::conditional<F32, float, double>::type;
    R x, mu, t;         // FP64: global x, t; FP32: x from the cell's left edge, t from the time bin start
    double tau;         // remaining optical depth of the flight (double in both modes)
    R rmu;              // refined reciprocal of mu (set_direction)
    R far;              // +inf when mu == 0 (the flight meets no edge), else 0
    uint64_t X;         // LCG state
    int32_t cell, tb;
    uint32_t hdraws;    // numbers drawn by this history
    bool need_tau;      // the next event starts by sampling a flight
};

// Derived direction values, after every change of mu.
template <bool F32>
__device__ __forceinline__ void set_direction(Particle<F32>& p) {
    using R = typename Particle<F32>::R;
    p.rmu = recip_refined(p.mu);
    p.far = (p.mu == R(0)) ? static_cast<R>(__builtin_huge_val()) : R(0);
}

// Cell data of the current problem (LDS-staged or global).  FP64: edge[c]
// is the position of edge c (n_cells + 1), tedge[t] the time edges.  FP32:
// edge[c] is the width of cell c, tedge[t] the duration of time bin t.
// rsig[c] is recip_refined(sig[c]) (staged with the cells), or null: then
// it is computed per event.
template <bool F32>
struct CellsLds {
    using R = typename std::conditional<F32, float, double>::type;
    const R* edge;
    const R* sig;       // n_cells
    const R* rsig;      // n_cells, or null
    const double* scat; // n_cells (the absorption test stays in double)
    const int32_t* bin; // n_cells
    const R* tedge;
    int32_t n_cells;
    int32_t n_time_bins;
    int32_t n_space_bins;
};

template <bool F32>
__device__ __forceinline__ typename CellsLds<F32>::R cell_recip(const CellsLds<F32>& C, int c,
                                                               typename CellsLds<F32>::R sig) {
    return C.rsig ? C.rsig[c] : recip_refined(sig);
}

enum : int { STEP_COLLIDE = -1, END_NONE = 0, END_LEAK_LEFT, END_LEAK_RIGHT, END_ABSORBED, END_CENSUS };

struct LaneCounters {
    uint64_t events = 0, draws = 0, collisions = 0;
    uint32_t histories = 0, leak_left = 0, leak_right = 0, absorbed = 0, census = 0;
    uint32_t max_draws = 0, over_stride = 0;
};

// Adds q to a tally word pair: the low and the high 32-bit halves of q are
// summed into separate 64-bit words (LDS or global memory); the pair holds
// low + 2^32 high.
__device__ __forceinline__ void lds_score(uint64_t* slot, uint64_t q) {
    atomicAdd(reinterpret_cast<unsigned long long*>(slot), static_cast<unsigned long long>(q & 0xffffffffull));
    atomicAdd(reinterpret_cast<unsigned long long*>(slot + 1), static_cast<unsigned long long>(q >> 32));
}

// Adds lo + 2^32 hi to a global word pair that may collect more than 2^32
// additions: when the low word wraps (it lost 2^64 = 2^32 x 2^32), 2^32 more
// goes to the high word, so the pair's value stays exact below 2^96.
__device__ __forceinline__ void carry_add(uint64_t* slot, uint64_t lo, uint64_t hi) {
    const unsigned long long old = atomicAdd(reinterpret_cast<unsigned long long*>(slot), static_cast<unsigned long long>(lo));
    if (old + lo < old) hi += 1ull << 32;
    if (hi != 0) atomicAdd(reinterpret_cast<unsigned long long*>(slot + 1), static_cast<unsigned long long>(hi));
}

// A score: lds_score, or (CARRY) carry_add into a global pair.
template <bool CARRY>
__device__ __forceinline__ void add_score(uint64_t* slot, uint64_t q) {
    if constexpr (CARRY)
        carry_add(slot, q & 0xffffffffull, q >> 32);
    else
        lds_score(slot, q);
}

template <bool F32>
__device__ __forceinline__ void sample_tau(Particle<F32>& p, const LcgDev& L) {
    p.X = lcg_next_wide(L, p.X);
    p.hdraws++;
    p.tau = -fixed_log(to_uniform(L, p.X));
    p.need_tau = false;
}

// FP64 geometry in global coordinates:
//   s = tau / sig[c]                                          -> collision
//   se = (E[c+1] - x) / mu if mu > 0, (E[c] - x) / mu if mu < 0, +inf if
//   mu == 0;  if se < s: s = se                               -> edge
//   timed: st = T[tb+1] - t;  if st < s: s = st               -> time
//   score q(s) into (tb, bin[c]);  timed: t = t + s, clamped to T[tb+1]
//   tau = tau - sig * s, clamped at 0
//   edge:  mu > 0: c + 1 (leak right past the last), x = E[c+1]
//          mu < 0: x = E[c], c - 1 (leak left past the first)
//   other: x = x + mu * s, clamped to [E[c], E[c+1]]
//   time:  tb + 1, t = T[tb+1]; census past the last time edge
// (far turns the mu == 0 edge distance into +inf or NaN, which loses the
// strict comparison as +inf does.)
template <bool TIMED, bool CARRY = false>
__device__ __forceinline__ int geom_f64(Particle<false>& p, const CellsLds<false>& C, uint64_t* tally) {
    const int c = p.cell;
    const double sig = C.sig[c];
    const double e_lo = C.edge[c], e_hi = C.edge[c + 1];
    double s = quot(p.tau, sig, cell_recip<false>(C, c, sig));
    int ev = 0;   // 0 collision, 1 edge, 2 time
    const bool up = p.mu > 0.0;
    const double e_to = up ? e_hi : e_lo;
    const double se = quot(e_to - p.x, p.mu, p.rmu) + p.far;
    if (se < s) {
        s = se;
        ev = 1;
    }
    double tnext = 0.0;
    const bool timed = TIMED && C.n_time_bins > 0;   // a set may mix steady and timed problems
    if (timed) {
        tnext = C.tedge[p.tb + 1];
        const double st = tnext - p.t;
        if (st < s) {
            s = st;
            ev = 2;
        }
    }
    add_score<CARRY>(tally + 2 * (static_cast<uint32_t>(p.tb) * C.n_space_bins + C.bin[c]), quantise(s));
    if (timed) p.t = __builtin_fmin(p.t + s, tnext);
    p.tau = __builtin_fmax(p.tau - sig * s, 0.0);
    if (ev == 1) {
        const int nc = up ? c + 1 : c - 1;
        if (nc < 0) return END_LEAK_LEFT;
        if (nc == C.n_cells) return END_LEAK_RIGHT;
        p.cell = nc;
        p.x = e_to;
        return END_NONE;
    }
    p.x = __builtin_fmin(__builtin_fmax(p.x + p.mu * s, e_lo), e_hi);
    if (timed && ev == 2) {
        const int ntb = p.tb + 1;
        p.tb = ntb;
        p.t = tnext;
        if (ntb == C.n_time_bins) return END_CENSUS;
        return END_NONE;
    }
    return STEP_COLLIDE;
}

// FP32 geometry with the position measured from the cell's left edge and
// the time from the time bin's start (W = cell width, DT = bin duration);
// the remaining optical depth tau stays double (a float tau would lose
// absolute precision over a flight's many subtractions, and the flight's
// last segment, their small remainder, would carry it):
//   s = R(tau) / sig[c];  se = (W[c] - x)/mu (mu > 0), (0 - x)/mu (mu < 0),
//   +inf (mu == 0);  timed: st = DT[tb] - t;  strict-less order as in FP64
//   score q(double(s));  timed: t = t + s, clamped to DT[tb]
//   tau = tau - double(sig) double(s) (exact product), clamped at 0
//   edge: mu > 0: c + 1, x = 0;  mu < 0: c - 1, x = W[c - 1]
//   other: x = x + mu s clamped to [0, W[c]];  time: tb + 1, t = 0
template <bool TIMED, bool CARRY = false>
__device__ __forceinline__ int geom_f32(Particle<true>& p, const CellsLds<true>& C, uint64_t* tally) {
    const int c = p.cell;
    const float sig = C.sig[c];
    const float w = C.edge[c];
    float s = quot(static_cast<float>(p.tau), sig, cell_recip<true>(C, c, sig));
    int ev = 0;
    const bool up = p.mu > 0.0f;
    const float e_to = up ? w : 0.0f;
    const float se = quot(e_to - p.x, p.mu, p.rmu) + p.far;
    if (se < s) {
        s = se;
        ev = 1;
    }
    float dtb = 0.0f;
    const bool timed = TIMED && C.n_time_bins > 0;
    if (timed) {
        dtb = C.tedge[p.tb];
        const float st = dtb - p.t;
        if (st < s) {
            s = st;
            ev = 2;
        }
    }
    add_score<CARRY>(tally + 2 * (static_cast<uint32_t>(p.tb) * C.n_space_bins + C.bin[c]),
                     quantise(static_cast<double>(s)));
    if (timed) p.t = __builtin_fminf(p.t + s, dtb);
    p.tau = __builtin_fmax(p.tau - static_cast<double>(sig) * static_cast<double>(s), 0.0);
    if (ev == 1) {
        if (up) {
            const int nc = c + 1;
            if (nc == C.n_cells) return END_LEAK_RIGHT;
            p.cell = nc;
            p.x = 0.0f;
        } else {
            if (c == 0) return END_LEAK_LEFT;
            p.cell = c - 1;
            p.x = C.edge[c - 1];
        }
        return END_NONE;
    }
    p.x = __builtin_fminf(__builtin_fmaxf(p.x + p.mu * s, 0.0f), w);
    if (timed && ev == 2) {
        const int ntb = p.tb + 1;
        p.tb = ntb;
        p.t = 0.0f;
        if (ntb == C.n_time_bins) return END_CENSUS;
        return END_NONE;
    }
    return STEP_COLLIDE;
}

// CARRY: the tally is a global pair array scored with carry_add.
template <bool F32, bool TIMED, bool CARRY = false>
__device__ __forceinline__ int geom_step(Particle<F32>& p, const CellsLds<F32>& C, uint64_t* tally) {
    if constexpr (F32)
        return geom_f32<TIMED, CARRY>(p, C, tally);
    else
        return geom_f64<TIMED, CARRY>(p, C, tally);
}

// Collision at the current site: u1 decides absorption (double compare with
// the cell's scattering ratio), u2 the new direction mu = R(2 u2 - 1)
// (computed in double, exact, then rounded once).  The next flight is
// sampled by sample_tau.
template <bool F32>
__device__ __forceinline__ int collide(Particle<F32>& p, const CellsLds<F32>& C, const LcgDev& L) {
    using R = typename Particle<F32>::R;
    p.X = lcg_next_wide(L, p.X);
    p.hdraws++;
    const double u1 = to_uniform(L, p.X);
    if (!(u1 < C.scat[p.cell])) return END_ABSORBED;
    p.X = lcg_next_wide(L, p.X);
    p.hdraws++;
    const double u2 = to_uniform(L, p.X);
    p.mu = static_cast<R>(2.0 * u2 - 1.0);
    set_direction<F32>(p);
    p.need_tau = true;
    return END_NONE;
}

// One whole event (the event-sorted schedule's unit of work), counted.
template <bool F32, bool TIMED, bool CARRY = false>
__device__ __forceinline__ int step_particle(Particle<F32>& p, const CellsLds<F32>& C, const LcgDev& L,
                                             uint64_t* tally, LaneCounters& cnt) {
    if (p.need_tau) sample_tau<F32>(p, L);
    cnt.events++;
    const int r = geom_step<F32, TIMED, CARRY>(p, C, tally);
    if (r != STEP_COLLIDE) return r;
    cnt.collisions++;
    return collide<F32>(p, C, L);
}

// A new history whose stream starts at state X: source at the left face
// moving right, at the first time edge; its first flight is sampled before
// its first geometry step.
template <bool F32, bool TIMED>
__device__ __forceinline__ void init_particle_at(Particle<F32>& p, const CellsLds<F32>& C, uint64_t X) {
    using R = typename Particle<F32>::R;
    p.X = X;
    if constexpr (F32) {
        p.x = 0.0f;
        p.t = 0.0f;
    } else {
        p.x = C.edge[0];
        p.t = (TIMED && C.n_time_bins > 0) ? C.tedge[0] : 0.0;
    }
    p.mu = R(1);
    p.rmu = R(1);   // recip_refined(1) is exactly 1
    p.far = R(0);
    p.tau = 0.0;
    p.cell = 0;
    p.tb = 0;
    p.hdraws = 0;
    p.need_tau = true;
}

// History j (global index) of a problem with seeding S.
template <bool F32, bool TIMED>
__device__ __forceinline__ void init_particle(Particle<F32>& p, const CellsLds<F32>& C, const LcgDev& L,
                                              const SeedDev& S, uint64_t j) {
    init_particle_at<F32, TIMED>(p, C, stream_start(L, S, j));
}

}  // namespace mcrng
