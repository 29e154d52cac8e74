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

// A census arrival, or a census copy, of a population-controlled run (32 B).
struct PulseCensusEntry {
    double x, mu;        // census point and direction
    uint64_t X;          // arrival: stream state after its draws; copy: its start state
    uint32_t batch;      // batch of the run (0-based)
    uint32_t pad;
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
    uint32_t tally_slots;    // family schedule over sources, counters not in LDS: per-wave LDS
                             // slots, one per chunk of sources in flight (0: HBM atomics)
    uint64_t* diag;          // kNDiag words (PD_*)
    uint64_t stride_q;       // stride: Q (over-stride count)
    uint64_t src_begin, src_end;   // sources of this launch (0-based over the run)
    PulseBankView in, out;   // bank schedule
    uint64_t n_in;
    uint64_t* out_count;
    uint64_t out_cap;
    uint64_t* item_counter;  // bank schedule: next input particle (taken `chunk` per wave)
    uint32_t chunk;          // bank schedule: input particles a wave takes per atomic
    uint64_t cont_budget;    // bank schedule: appends of continuing lines stay within this
    uint32_t* overflow;      // set if an append or a stack push found no room
    uint64_t* family_counter;
    PulseStackEntry* stack;  // family schedule: stack_depth entries per lane of the launch,
                             // depth-major (entry d of lane l at d * lanes + l)
    // population control (t_end is then the census time of the epoch)
    PulseCensusEntry* cen;   // census arrivals of the epoch
    uint64_t* cen_count;
    uint64_t cen_cap;
    const PulseCensusEntry* copies;   // copies starting the epoch (taken as items)
    double t_start;          // the census time the copies start at
    int32_t tb_start;        // its time bin
    uint32_t census;         // split: census index c
    uint32_t n_census;       // census points of the run
    uint32_t census_every;   // time bins per epoch (census c at edge (c+1) census_every)
    uint32_t batch_lo;       // split / count: first batch of the chunk (LDS histogram base)
    uint32_t n_chunk_batches;
    uint64_t pc_target, pc_seed;
    uint64_t* pop;           // n_batches x n_census x 2: arrivals, copies
    uint64_t* copy_count;
    uint64_t copy_cap;
    PulseCensusEntry* copies_out;
    uint32_t lane_budget;    // finish launches: particles per input particle before the rest is banked
};

enum PulseItems : int { PULSE_ITEMS_SOURCES = 0, PULSE_ITEMS_BANK = 1, PULSE_ITEMS_COPIES = 2 };
constexpr uint32_t kPulsePcChunkBatches = 4096;   // batches per chunk of a population-controlled run

// Bank launches: the grid (resident blocks, at most one chunk of items per
// wave) is chosen first, so that the caller can size the output for it.
// `items` is a PulseItems value; `pc`: the launch's census is a census of
// population control (arrivals are banked in p.cen).
uint32_t pulse_bank_grid(const PulseParams& p, int items_kind, bool pc, int block, uint64_t items);
constexpr uint32_t kPulseLdsCounters = 2048;   // block-local tally copies up to this many counters (16 KiB)
constexpr uint32_t kPulseTallySlots = 16;      // most tally slots per wave of the family kernel
// Entries of a wave's LDS stage of appends in k_pulse_bank (output slack).
uint32_t pulse_bank_stage(int block);
hipError_t launch_pulse_bank(const PulseParams& p, int items_kind, bool pc, int block, uint32_t grid,
                             hipStream_t st);
// Population control at census p.census: arrival counts per batch into
// p.pop, then the copies of every arrival into p.copies_out.
hipError_t launch_pulse_census_count(const PulseParams& p, uint64_t n_arrivals, hipStream_t st);
hipError_t launch_pulse_split(const PulseParams& p, uint64_t n_arrivals, hipStream_t st);
uint32_t pulse_family_grid(int block);
// Finish launch (hash seeding): the generation bank p.in (p.n_in particles)
// run depth first per lane with p.stack (p.stack_depth entries per lane),
// at most p.lane_budget particles per input particle, the rest banked in
// p.out (p.out_count); one 256-thread block per 256 inputs, at most 8 per CU.
uint32_t pulse_finish_grid(uint64_t items);
hipError_t launch_pulse_finish(const PulseParams& p, bool pc, uint32_t grid, hipStream_t st);
hipError_t launch_pulse_family(const PulseParams& p, int block, uint32_t grid, hipStream_t st);
hipError_t launch_pulse_flux(const PulseParams& p, double* flux, hipStream_t st);

}  // namespace mcrng
