// Internal types of the pulse-problem kernels (pulse.hip) shared with the
// host-side API.  Not part of the public C ABI (include/mcrng.h).
#pragma once

#include "internal.hpp"

namespace mcrng {

// Diagnostics of the pulse problem, same order as the MCRNG_PD_* words.
enum PulseDiagWord {
    PD_SOURCES = 0, PD_COLLISIONS, PD_TALLIED, PD_SCATTERS, PD_ABSORBED, PD_CENSUS,
    PD_SECONDARIES, PD_DRAWS, PD_MAX_DRAWS, PD_OVER_STRIDE
};

// Particle bank (structure of arrays): particles waiting to start.
struct PulseBankView {
    double* x;
    double* t;
    uint64_t* X;         // start state of the particle's stream
    uint32_t* batch;
    int32_t* tb;
};

// Per-lane stack entry of the family schedule: the siblings of one
// scattering that have not started yet (keys next .. n).
struct PulseStackEntry {
    double x, t;
    uint64_t key;        // hash seeding: the parent's state X_p
    int32_t tb;
    uint16_t next, n;
};

struct PulseParams {
    LcgDev lcg;
    SeedDev seed;            // hash: base = the global seed s; stride: skip table etc.
    uint64_t first_batch;
    uint64_t per_batch;
    uint32_t n_batches;
    uint32_t n_time_bins;
    uint32_t hash;           // 1: hash seeding (secondaries seeded by eq. 5)
    uint32_t n_floor;        // floor(nu)
    double nu_frac;          // nu - floor(nu)
    double sigma_t, scatter, x_lo, x_hi, t_end;
    int32_t tb0;             // time bin of t = 0
    uint32_t stack_depth;    // family schedule: entries per lane
    const double* t_edges;   // device, n_time_bins + 1
    uint64_t* counts;        // n_batches x n_time_bins
    uint32_t n_counters;     // n_batches x n_time_bins
    uint32_t lds_tally;      // 1: each block counts into an LDS copy of all counters
    uint64_t* diag;          // kNDiag words (PD_*)
    uint64_t stride_q;       // stride: Q (over-stride count)
    uint64_t src_begin, src_end;   // sources of this launch (0-based over the run)
    PulseBankView in, out;   // bank schedule
    uint64_t n_in;
    uint64_t* out_count;
    uint64_t out_cap;
    uint64_t* item_counter;  // bank schedule: next input particle (taken 256 per wave)
    uint64_t cont_budget;    // bank schedule: appends of continuing lines stay within this
    uint32_t* overflow;      // set if an append or a stack push found no room
    uint64_t* family_counter;
    PulseStackEntry* stack;  // family schedule: stack_depth entries per lane
};

// Bank launches: the grid (resident blocks, at most one 256-item chunk per
// wave) is chosen first, so that the caller can size the output for it.
uint32_t pulse_bank_grid(const PulseParams& p, bool sources, int block, uint64_t items);
constexpr uint32_t kPulseLdsCounters = 2048;   // block-local tally copies up to this many counters (16 KiB)
hipError_t launch_pulse_bank(const PulseParams& p, bool sources, int block, uint32_t grid, hipStream_t st);
uint32_t pulse_family_grid(int block);
hipError_t launch_pulse_family(const PulseParams& p, int block, uint32_t grid, hipStream_t st);
hipError_t launch_pulse_flux(const PulseParams& p, double* flux, hipStream_t st);

}  // namespace mcrng
