// Internal types shared by the library's kernels and its host-side API.
// Not part of the public C ABI (include/mcrng.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_rng.hpp"

namespace mcrng {

constexpr int kNDiag = 10;   // same order as the MCRNG_D_* words of the C ABI
enum DiagWord {
    D_HISTORIES = 0, D_LEAK_LEFT, D_LEAK_RIGHT, D_ABSORBED, D_CENSUS,
    D_EVENTS, D_COLLISIONS, D_DRAWS, D_MAX_DRAWS, D_OVER_STRIDE
};

enum SeedMode : int { SEED_LOAD = 0, SEED_HASH = 1, SEED_STRIDE = 2 };

// Stride skip-ahead table: for digit d (base 16) and value v, the affine map
// of Q * v * 16^d LCG steps, stored as (G, C) word pairs at
// table[(d * 16 + v) * 2].
constexpr int kStrideRadixBits = 4;
constexpr int kStrideRadix = 1 << kStrideRadixBits;
constexpr int kStrideDigits = 64 / kStrideRadixBits;

struct SeedDev {
    int kind;                  // SEED_HASH or SEED_STRIDE
    uint32_t stride_digits;    // base-16 digits of the largest stream index
    uint64_t base;             // stride: X_0 (masked); hash: subhash(parent ^ 8M)
    uint64_t first_index;      // global index of stream 0
    const uint64_t* table;     // stride: skip table of this Q
};

__device__ __forceinline__ uint64_t stream_start(const LcgDev& L, const SeedDev& S, uint64_t i) {
    const uint64_t idx = S.first_index + i;
    if (S.kind == SEED_HASH) return murmur_with_seed_part(idx + 1ull, S.base) & L.mask;
    uint64_t x = S.base;
    for (uint32_t d = 0; d < S.stride_digits; ++d) {
        const uint32_t v = static_cast<uint32_t>(idx >> (kStrideRadixBits * d)) & (kStrideRadix - 1);
        const uint64_t* e = S.table + 2 * (d * kStrideRadix + v);
        x = affine_apply(e[0], e[1], L.mask, x);
    }
    return x;
}

// ------------------------------------------------------------ draw kernels

// Round alignment of a stream (the draw kernel for m = 63 and 64 with an odd
// multiplier): a stream of n draws runs rounds = ceil(n / D) whole rounds of
// D steps and starts h = rounds D - n steps before its own start state X_0,
// so that it ends on a round boundary.  Entry h holds the affine maps, modulo
// 2^64, of that rewind, X_{-h} = a X_0 + b, and of minus the sum of the h
// outputs drawn before X_1 (X_{-h+1} .. X_0): na X_0 + nb.
struct __align__(16) AlignEntry {
    uint64_t a, b;
    uint64_t na, nb;
};

constexpr int kMaxRound = 32;
// The table holds kMaxRound alignment entries, then kSkipMaps skip-ahead
// maps: entry kMaxRound + e has (a, b) = the map of 2^e rounds (2^e D steps,
// modulo 2^64), Y -> a Y + b; na and nb are 0.
constexpr int kSkipMaps = 32;

struct DrawParams {
    LcgDev lcg;
    SeedDev seed;
    uint64_t n;
    const uint32_t* count;
    uint64_t* state;      // SEED_LOAD: in/out; else optional out (may be null)
    uint64_t* checksum;
    const AlignEntry* align;   // round alignment and skip maps for the round length (null: the generic kernel)
};

hipError_t launch_init_streams(const LcgDev& L, const SeedDev& S, uint64_t n, uint64_t* out,
                               hipStream_t st);
hipError_t launch_draw(const DrawParams& p, int seed_mode, hipStream_t st, int blocks_per_cu, int round);

// ------------------------------------------------------------ transport

struct DevProblem {
    uint32_t cell_off;       // first cell in the flat cell arrays
    uint32_t n_cells;
    uint32_t tedge_off;      // first time edge in the flat time-edge arrays
    uint32_t n_time_bins;    // 0 = steady state
    uint32_t n_space_bins;
    uint32_t slice_bins;     // max(n_time_bins, 1) * n_space_bins
    uint32_t seed_kind;      // SEED_HASH or SEED_STRIDE
    uint32_t stride_digits;
    uint64_t seed_base;
    uint64_t first_index;
    uint64_t stride_q;       // stride seeding: Q (for the over-stride count); else 0
    const uint64_t* table;   // stride seeding: skip table of this Q (device memory)
    uint32_t edge_off;       // first edge in the flat edge arrays (n_cells + 1 edges)
    uint32_t pad_;
};

struct WorkUnit {
    uint32_t problem;
    uint32_t batch;
    uint64_t j0;             // first history (0-based within the problem)
    uint32_t count;          // histories in the unit
    uint32_t slice_bins;
    uint64_t slot;           // first word of the unit's partial tally (2 words per bin)
};

struct TransportParams {
    LcgDev lcg;
    const DevProblem* problems;
    const WorkUnit* units;
    const uint32_t* order;       // schedule: units in the order blocks take them
    uint32_t n_units;
    uint32_t max_cells;          // LDS sizing: largest n_cells of the set
    uint32_t max_tedges;         // largest n_time_bins + 1 (0 if all steady)
    uint32_t max_slice;          // largest slice_bins
    uint32_t tally_copies;       // 1 or waves per block
    uint32_t coll_batch;         // run a wave's collision phase once this many of its lanes wait (>= 1)
    const double* edges64;       // flat cell arrays
    const double* sig64;
    const double* scat64;
    const int32_t* cbin;
    const float* edges32;
    const float* sig32;
    const double* tedges64;
    const float* tedges32;
    uint64_t* partial;           // per-unit partial tallies (low-half sum, high-half sum)
    uint64_t* unit_diag;         // n_units x kNDiag
    uint32_t* unit_counter;      // persistent scheduling counter (zeroed before launch)
};

// Largest work unit (histories): a unit's LDS tally words take plain 64-bit
// adds of 32-bit halves, exact while fewer than 2^32 of its scores fall in
// one bin.
constexpr uint32_t kMaxUnitHistories = 1u << 18;

struct LaunchShape {
    int block;           // threads per block
    int hist_per_lane;   // 1, 2 or 4
    int grid;            // 0 = fill the device
    int f32;             // 1 = FP32 flight mode
    int timed;           // 1 = time-dependent problems present
    int chain;           // 1 = k_transport_chain (one problem, one history per lane, two tally slices)
};

size_t transport_lds_bytes(const TransportParams& p, int f32);
// LDS k_transport declares statically for a block size (skip table, the
// waves' rings of seeded histories, block words).
size_t transport_static_lds_bytes(int block);
// Whether k_transport_chain (with `chained`, whose tally_copies is 2: the
// block's two unit slices) keeps at least k_transport's blocks per CU with
// `single` (one history per lane).
hipError_t transport_chain_fits(const TransportParams& single, const TransportParams& chained, const LaunchShape& s,
                                bool* fits);
hipError_t launch_transport(const TransportParams& p, const LaunchShape& s, hipStream_t st,
                            int* grid_used);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st);
hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t st);

// ------------------------------------------------------------ event schedule

// Structure-of-arrays particle bank (capacity entries per array).  The
// FP64 or FP32 position arrays are used according to the precision.
struct EventBank {
    double* x64; double* mu64; double* t64; double* tau64;
    float* x32; float* mu32; float* t32; float* tau32;
    uint64_t* X;             // LCG state
    int32_t* cell;           // bit 31: the next step samples a flight
    int32_t* tb;
    uint32_t* hdraws;        // numbers drawn by the history so far
    uint32_t* events;        // events of the history so far
    uint32_t* colls;         // collisions of the history so far
    uint32_t* unit;          // work unit (partial-tally slot, problem)
    uint32_t* rec;           // index of the history's outcome record
};

// Outcome of one history, written once when it ends.
struct HistoryRecord {
    uint32_t events;
    uint32_t collisions;
    uint32_t draws;
    uint32_t end;            // END_LEAK_LEFT .. END_CENSUS
};

struct EventParams {
    TransportParams tp;      // tables, units, partial slots (atomically accumulated)
    EventBank in, out;
    uint32_t n_in;           // init: particles of the slice; step / finish: a bound on the live count (grid size)
    // step / finish: device words rotated by the host over the launches of a
    // slice: the live count of `in`, the append counter of `out` (zero at the
    // start), and the next launch's append counter, which block 0 zeroes
    const uint32_t* n_live;
    uint32_t* n_out;
    uint32_t* n_clear;
    HistoryRecord* records;  // one per history of the run
    const uint64_t* rec_begin;   // per unit: index of its first record
    // init: the histories of units [unit_begin, unit_end), n_in in total
    uint32_t unit_begin;
    uint32_t unit_end;
    // the slice holds one (problem, batch): its particles all score into the
    // slice's first unit (global adds then carry, carry_add)
    uint32_t one_group;
};

hipError_t launch_event_init(const EventParams& p, int f32, int timed, hipStream_t st);
hipError_t launch_event_step(const EventParams& p, int f32, int timed, hipStream_t st);
hipError_t launch_event_unit_diag(const EventParams& p, hipStream_t st);

// ------------------------------------------------------------ reduction

struct ReduceGroup {         // one (problem, batch): a contiguous run of units
    uint32_t problem;
    uint32_t unit_begin;
    uint32_t unit_end;
    uint32_t slice_bins;
    uint32_t n_space_bins;
    uint32_t n_time_bins;    // 0 = steady
    uint64_t out_off;        // first output bin
    uint64_t n_hist;         // histories of the batch (flux normalisation)
    uint32_t dx_off;         // first space-bin width of the problem
    uint32_t dt_off;         // first time-bin width of the problem
};

struct ReduceParams {
    const ReduceGroup* groups;
    uint32_t n_groups;
    uint32_t max_slice;
    const WorkUnit* units;
    const uint64_t* partial;
    const double* dx;
    const double* dt;
    uint64_t* raw;           // 2 words per bin
    double* flux;
    // diagnostics: problem p owns units [pu_begin[p], pu_begin[p+1])
    const uint32_t* pu_begin;
    uint32_t n_problems;
    const uint64_t* unit_diag;
    uint64_t* diag;          // n_problems x kNDiag, may be null
};

hipError_t launch_reduce(const ReduceParams& p, hipStream_t st);

}  // namespace mcrng
