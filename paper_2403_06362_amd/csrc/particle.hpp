// One particle event: the per-history arithmetic shared by the history-based
// and the event-sorted schedules, so that both run the identical operation
// sequence for every particle.
#pragma once

#include <type_traits>

#include "internal.hpp"

namespace mcrng {

template <bool F32>
struct Particle {
    using R = typename std::conditional<F32, float, double>::type;
    R x, mu, t, tau;
    uint64_t X;         // LCG state
    int32_t cell, tb;
    uint32_t hdraws;    // numbers drawn by this history
    bool need_tau;      // the next step starts by sampling a flight
};

// Cell data of the current problem, staged in LDS.
template <bool F32>
struct CellsLds {
    using R = typename std::conditional<F32, float, double>::type;
    const R* edge;      // n_cells + 1
    const R* sig;       // n_cells
    const double* scat; // n_cells (the absorption test stays in double)
    const int32_t* bin; // n_cells
    const R* tedge;     // n_time_bins + 1
    int32_t n_cells;
    int32_t n_time_bins;
    int32_t n_space_bins;
};

enum : int { END_NONE = 0, END_LEAK_LEFT, END_LEAK_RIGHT, END_ABSORBED, END_CENSUS };

struct LaneCounters {
    uint64_t events = 0, draws = 0, collisions = 0;
    uint32_t histories = 0, leak_left = 0, leak_right = 0, absorbed = 0, census = 0;
    uint32_t max_draws = 0, over_stride = 0;
};

__device__ __forceinline__ void lds_score(uint64_t* slot, uint64_t q) {
    atomicAdd(reinterpret_cast<unsigned long long*>(slot), static_cast<unsigned long long>(q & 0xffffffffull));
    atomicAdd(reinterpret_cast<unsigned long long*>(slot + 1), static_cast<unsigned long long>(q >> 32));
}

// One event of one particle in global double coordinates.  Returns END_*
// (END_NONE while the history continues).  Operation sequence (every
// operation rounded to nearest, no fused multiply-add):
//   [need_tau]  X = lcg(X); u = uniform(X); tau = R(-ln(u))   (ln in double)
//   s = tau / sig[cell]                                     -> collision
//   se = (E[cell+1] - x) / mu if mu > 0, (E[cell] - x) / mu if mu < 0,
//        +inf if mu == 0;  if se < s: s = se               -> edge
//   timed: st = T[tb+1] - t;  if st < s: s = st             -> time
//   score q(double(s)) into (tb, bin[cell])
//   timed: t = t + s; if t > T[tb+1]: t = T[tb+1]
//   tau = tau - sig * s; if tau < 0: tau = 0
//   edge:  mu > 0: cell + 1 (leak right past the last), x = E[cell]
//          mu < 0: x = E[cell], cell - 1 (leak left past the first)
//   other: x = x + mu * s, clamped to [E[cell], E[cell+1]]
//   time:  tb + 1, t = T[tb]; census past the last time edge
//   collision: X = lcg(X), u1: absorbed unless u1 < scat[cell] (double);
//          X = lcg(X), u2: mu = R(2 u2 - 1) (computed in double, exact);
//          the next step samples tau from the following draw.
template <bool F32, bool TIMED>
__device__ __forceinline__ int step_global(Particle<F32>& p, const CellsLds<F32>& C, const LcgDev& L,
                                           uint64_t* tally, LaneCounters& cnt) {
    using R = typename Particle<F32>::R;
    if (p.need_tau) {
        p.X = lcg_next(L, p.X);
        p.hdraws++;
        const double lg = fixed_log(to_uniform(L, p.X));
        p.tau = static_cast<R>(-lg);
        p.need_tau = false;
    }
    const int c = p.cell;
    const R sig = C.sig[c];
    R s = p.tau / sig;
    int ev = 0;   // 0 collision, 1 edge, 2 time
    R se;
    if (p.mu > R(0))
        se = (C.edge[c + 1] - p.x) / p.mu;
    else if (p.mu < R(0))
        se = (C.edge[c] - p.x) / p.mu;
    else
        se = __builtin_huge_val();
    if (se < s) {
        s = se;
        ev = 1;
    }
    R tnext = R(0);
    const bool timed = TIMED && C.n_time_bins > 0;   // a set may mix steady and timed problems
    if (timed) {
        tnext = C.tedge[p.tb + 1];
        const R st = tnext - p.t;
        if (st < s) {
            s = st;
            ev = 2;
        }
    }
    lds_score(tally + 2 * (static_cast<uint32_t>(p.tb) * C.n_space_bins + C.bin[c]),
              quantise(static_cast<double>(s)));
    cnt.events++;
    if (timed) {
        R tn = p.t + s;
        if (tn > tnext) tn = tnext;
        p.t = tn;
    }
    const R dtau = sig * s;
    R tau = p.tau - dtau;
    if (tau < R(0)) tau = R(0);
    p.tau = tau;
    if (ev == 1) {
        if (p.mu > R(0)) {
            const int nc = c + 1;
            if (nc == C.n_cells) return END_LEAK_RIGHT;
            p.cell = nc;
            p.x = C.edge[nc];
        } else {
            p.x = C.edge[c];
            if (c == 0) return END_LEAK_LEFT;
            p.cell = c - 1;
        }
        return END_NONE;
    }
    const R step = p.mu * s;
    R nx = p.x + step;
    const R lo = C.edge[c], hi = C.edge[c + 1];
    if (nx < lo) nx = lo;
    if (nx > hi) nx = hi;
    p.x = nx;
    if (timed && ev == 2) {
        const int ntb = p.tb + 1;
        p.tb = ntb;
        p.t = tnext;
        if (ntb == C.n_time_bins) return END_CENSUS;
        return END_NONE;
    }
    cnt.collisions++;
    p.X = lcg_next(L, p.X);
    p.hdraws++;
    const double u1 = to_uniform(L, p.X);
    if (!(u1 < C.scat[c])) return END_ABSORBED;
    p.X = lcg_next(L, p.X);
    p.hdraws++;
    const double u2 = to_uniform(L, p.X);
    p.mu = static_cast<R>(2.0 * u2 - 1.0);
    p.need_tau = true;
    return END_NONE;
}

// FP32 flight mode: x is the position from the cell's left edge, t the time
// from the time bin's start; C.edge[c] holds the width of cell c and
// C.tedge[tb] the duration of time bin tb (floats rounded once from double
// differences).  Operation sequence (every operation one IEEE single
// operation unless marked double):
//   [need_tau]  X = lcg(X); tau = float(-ln(uniform(X)))      (ln in double)
//   s = tau / sig[c];  se = (W[c] - x)/mu (mu > 0), (0 - x)/mu (mu < 0),
//   +inf (mu == 0);  timed: st = DT[tb] - t;  strict-less order as above
//   score q(double(s));  timed: t = t + s, clamped to DT[tb]
//   tau = tau - sig * s, clamped at 0
//   edge: mu > 0: c + 1, x = 0;  mu < 0: c - 1, x = W[c - 1]
//   other: x = x + mu s clamped to [0, W[c]];  time: tb + 1, t = 0
//   collision: as in FP64 mode (u1 < scat in double; mu = float(2 u2 - 1)).
template <bool TIMED>
__device__ __forceinline__ int step_local_f32(Particle<true>& p, const CellsLds<true>& C, const LcgDev& L,
                                              uint64_t* tally, LaneCounters& cnt) {
    if (p.need_tau) {
        p.X = lcg_next(L, p.X);
        p.hdraws++;
        const double lg = fixed_log(to_uniform(L, p.X));
        p.tau = static_cast<float>(-lg);
        p.need_tau = false;
    }
    const int c = p.cell;
    const float sig = C.sig[c];
    const float w = C.edge[c];
    float s = p.tau / sig;
    int ev = 0;
    float se;
    if (p.mu > 0.0f)
        se = (w - p.x) / p.mu;
    else if (p.mu < 0.0f)
        se = (0.0f - p.x) / p.mu;
    else
        se = __builtin_huge_valf();
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
    lds_score(tally + 2 * (static_cast<uint32_t>(p.tb) * C.n_space_bins + C.bin[c]),
              quantise(static_cast<double>(s)));
    cnt.events++;
    if (timed) {
        float tn = p.t + s;
        if (tn > dtb) tn = dtb;
        p.t = tn;
    }
    const float dtau = sig * s;
    float tau = p.tau - dtau;
    if (tau < 0.0f) tau = 0.0f;
    p.tau = tau;
    if (ev == 1) {
        if (p.mu > 0.0f) {
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
    const float step = p.mu * s;
    float nx = p.x + step;
    if (nx < 0.0f) nx = 0.0f;
    if (nx > w) nx = w;
    p.x = nx;
    if (timed && ev == 2) {
        const int ntb = p.tb + 1;
        p.tb = ntb;
        p.t = 0.0f;
        if (ntb == C.n_time_bins) return END_CENSUS;
        return END_NONE;
    }
    cnt.collisions++;
    p.X = lcg_next(L, p.X);
    p.hdraws++;
    const double u1 = to_uniform(L, p.X);
    if (!(u1 < C.scat[c])) return END_ABSORBED;
    p.X = lcg_next(L, p.X);
    p.hdraws++;
    const double u2 = to_uniform(L, p.X);
    p.mu = static_cast<float>(2.0 * u2 - 1.0);
    p.need_tau = true;
    return END_NONE;
}

// One event of one particle: global FP64 coordinates, or cell-local FP32.
template <bool F32, bool TIMED>
__device__ __forceinline__ int step_particle(Particle<F32>& p, const CellsLds<F32>& C, const LcgDev& L,
                                             uint64_t* tally, LaneCounters& cnt) {
    if constexpr (F32)
        return step_local_f32<TIMED>(p, C, L, tally, cnt);
    else
        return step_global<F32, TIMED>(p, C, L, tally, cnt);
}

template <bool F32, bool TIMED>
__device__ __forceinline__ void init_particle(Particle<F32>& p, const CellsLds<F32>& C, const LcgDev& L,
                                              const SeedDev& S, uint64_t j) {
    using R = typename Particle<F32>::R;
    p.X = stream_start(L, S, j);
    if constexpr (F32) {
        p.x = 0.0f;   // cell-local position and bin-local time
        p.t = 0.0f;
    } else {
        p.x = C.edge[0];
        p.t = (TIMED && C.n_time_bins > 0) ? C.tedge[0] : 0.0;
    }
    p.mu = R(1);
    p.tau = R(0);
    p.cell = 0;
    p.tb = 0;
    p.hdraws = 0;
    p.need_tau = true;
}

}  // namespace mcrng
