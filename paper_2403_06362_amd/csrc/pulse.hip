// Pulse in an infinite multiplying medium with secondary particles, for
// gfx950 (the paper's test problem, Sec. "Implementation and Results").
//
// One particle's life (pulse_particle): direction from its first draw,
// flight tau = -ln(u) / sigma_t, census if t + s reaches the last time edge,
// else move, collision-estimator score (an integer count per batch and time
// bin) when x_lo <= x <= x_hi, absorption draw, and on a scattering the
// multiplicity draw n = floor(nu) + (u < nu - floor(nu)).  The n emerging
// particles start at the collision site:
//   hash seeding   the k-th starts its own stream at hash(k, X_p) mod 2^m
//                  (eq. 5; X_p the parent's state after its draws), so any
//                  particle can run anywhere, in any order;
//   stride seeding they continue the source's one stream, depth first.
//
// Schedules:
//   k_pulse_bank (hash only)  one launch per generation.  A wave takes a chunk
//       of input particles (or sources) at a time through one atomic and hands
//       them to its idle lanes; a lane runs each one's line of descent: at a
//       scattering it keeps the first emerging particle in registers and
//       banks its siblings (staged per wave in LDS, copied to the output bank
//       with one atomic per flush) while the wave's view of the output count
//       (its last flush plus its staged entries) is within the launch's
//       budget; past it, a scattering banks all n particles and ends the
//       line.  Appends are thus at most budget + n_max per input particle +
//       one stage and one iteration's appends per wave (the view lags by at
//       most a stage), which the output capacity covers.  With no budget
//       (the event-based schedule) every scattering banks all n particles:
//       each launch advances every live particle by one flight.
//   k_pulse_family            one source family per lane (sources taken 64
//       per wave and atomic), walked depth first with a per-lane stack (its
//       top entry in registers, the rest in HBM planes, one per depth); a
//       stack entry holds the siblings still to start of one scattering
//       (stride: a count; hash: X_p and the next key), so the depth is at
//       most the number of scatterings on the current line of descent.  With bank items (hash seeding) the same kernel finishes
//       a bank schedule's tail: up to a budget of particles per item, the
//       rest banked for the next launch.
// Counts are integers added with 64-bit atomics (into a per-block LDS copy
// of every counter when they fit, else one HBM atomic per distinct counter
// of a wave), so every schedule, launch shape and order gives the same
// counts.
//
// Population control (hash seeding, bank schedule; Sec. "Hierarchical Seed
// Splitting": one-off hashed values where no full stream is needed): the
// run is cut into epochs at census times T[(c+1) K].  A particle whose
// flight reaches the census stops at x + mu (C - t) with its direction and
// state (staged per wave in LDS like the appends).  Per batch, N particles
// arrive and M = target leave: arrival X leaves q + [u < r/N] copies
// (q = floor(M/N), r = M mod N) with the one-off value
// u = U(hash(X, hash(c+1, hash(B+1, pc_seed)))) compared exactly in
// integers, and copy k starts the stream hash(k, X) (eq. 5).  All
// particles of a batch share the epoch's weight, so counts stay integers
// and the flux applies the weights.
#include <cstdlib>

#include "pulse.hpp"

namespace mcrng {

struct PulseLane {
    uint64_t sources = 0, collisions = 0, tallied = 0, scatters = 0, absorbed = 0, census = 0;
    uint64_t secondaries = 0, draws = 0, max_draws = 0, over_stride = 0;
};

struct PParticle {
    double x, t;
    uint64_t X;        // stream state
    int32_t tb;        // time bin of t (-1 before the first time edge)
    uint32_t batch;
    double mu;         // direction: a census copy's, or the last flight's
    bool has_mu;       // a census copy keeps its direction; others draw it first
};

enum : uint32_t { PULSE_CENSUS = 0, PULSE_ABSORBED = 1, PULSE_SCATTERED = 2 };

// Runs the particle from its start to its end.  Returns PULSE_CENSUS,
// PULSE_ABSORBED or PULSE_SCATTERED, with *n the number of particles
// emerging (0 unless it scattered); p then holds the collision site and the
// state after the particle's draws (at a census: its start, its state and,
// with DIR, its direction in p.mu).  *draws counts the numbers drawn; a
// scored collision sets *tally to its counter index (the caller adds it
// with wave_tally).  DIR: the particle may carry a direction (census copies).
template <bool DIR>
__device__ __forceinline__ uint32_t pulse_flight(const PulseParams& P, PParticle& p, PulseLane& c,
                                                 uint32_t* draws, uint32_t* n, int64_t* tally) {
    const LcgDev& L = P.lcg;
    *n = 0;
    double mu;
    if (DIR && p.has_mu) {
        mu = p.mu;
    } else {
        p.X = lcg_next_wide(L, p.X);
        mu = 2.0 * to_uniform(L, p.X) - 1.0;
        *draws += 1;
    }
    p.X = lcg_next_wide(L, p.X);
    const double tau = -fixed_log(to_uniform(L, p.X));
    *draws += 1;
    const double s = quot(tau, P.sigma_t, recip_refined(P.sigma_t));   // the reciprocal is loop-invariant
    const double tn = p.t + s;
    if (!(tn < P.t_end)) {
        if (DIR) p.mu = mu;
        return PULSE_CENSUS;
    }
    const double step = mu * s;
    p.x = p.x + step;
    p.t = tn;
    while (p.tb + 1 < static_cast<int32_t>(P.n_time_bins) && P.t_edges[p.tb + 1] <= p.t) p.tb++;
    c.collisions++;
    if (p.tb >= 0 && P.x_lo <= p.x && p.x <= P.x_hi) {
        *tally = static_cast<int64_t>(p.batch) * P.n_time_bins + p.tb;
        c.tallied++;
    }
    p.X = lcg_next_wide(L, p.X);
    *draws += 1;
    if (!(to_uniform(L, p.X) < P.scatter)) return PULSE_ABSORBED;
    p.X = lcg_next_wide(L, p.X);
    *draws += 1;
    *n = P.n_floor + (to_uniform(L, p.X) < P.nu_frac ? 1u : 0u);
    return PULSE_SCATTERED;
}

// pulse_flight plus the end counters (kept out of the branches above so that
// the compiler does not fold them into an indexed array in scratch memory).
// *census is set when the particle reached the census.
template <bool DIR = false>
__device__ __forceinline__ uint32_t pulse_particle(const PulseParams& P, PParticle& p, PulseLane& c,
                                                   uint32_t* draws, int64_t* tally, bool* census = nullptr) {
    uint32_t n = 0;
    const uint32_t r = pulse_flight<DIR>(P, p, c, draws, &n, tally);
    if (census) *census = r == PULSE_CENSUS;
    c.census += static_cast<uint64_t>(r == PULSE_CENSUS);
    c.absorbed += static_cast<uint64_t>(r == PULSE_ABSORBED);
    c.scatters += static_cast<uint64_t>(r == PULSE_SCATTERED);
    c.secondaries += n;
    return n;
}

// Start state of source i of the run (0-based over all batches).
__device__ __forceinline__ uint64_t pulse_source_state(const PulseParams& P, uint64_t j, uint32_t* batch) {
    const uint64_t b = j / P.per_batch;
    const uint64_t i = j - b * P.per_batch;
    *batch = static_cast<uint32_t>(b);
    if (P.hash) {
        const uint64_t parent = murmur_hash(P.first_batch + b + 1ull, P.seed.base);
        return murmur_hash(i + 1ull, parent) & P.lcg.mask;
    }
    return stream_start(P.lcg, P.seed, j);
}

__device__ __forceinline__ void note_stream(const PulseParams& P, PulseLane& c, uint64_t draws) {
    c.draws += draws;
    if (draws > c.max_draws) c.max_draws = draws;
    if (!P.hash && draws > P.stride_q) c.over_stride++;
}

template <int BLOCK>
__device__ __forceinline__ void tally_lds_begin(const PulseParams& P, unsigned long long* lds_counts) {
    if (P.lds_tally)
        for (uint32_t i = threadIdx.x; i < P.n_counters; i += BLOCK) lds_counts[i] = 0;
    __syncthreads();
}

template <int BLOCK>
__device__ __forceinline__ void tally_lds_end(const PulseParams& P, const unsigned long long* lds_counts) {
    if (!P.lds_tally) return;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < P.n_counters; i += BLOCK)
        if (lds_counts[i] != 0) atomicAdd(reinterpret_cast<unsigned long long*>(P.counts) + i, lds_counts[i]);
}

// Block-level sum of the lane counters into P.diag (one atomic per word
// per block).
template <int BLOCK>
__device__ __forceinline__ void flush_lane_counters(const PulseParams& P, const PulseLane& c) {
    __shared__ unsigned long long acc[kNDiag];
    if (threadIdx.x < kNDiag) acc[threadIdx.x] = 0;
    __syncthreads();
    atomicAdd(&acc[PD_SOURCES], c.sources);
    atomicAdd(&acc[PD_COLLISIONS], c.collisions);
    atomicAdd(&acc[PD_TALLIED], c.tallied);
    atomicAdd(&acc[PD_SCATTERS], c.scatters);
    atomicAdd(&acc[PD_ABSORBED], c.absorbed);
    atomicAdd(&acc[PD_CENSUS], c.census);
    atomicAdd(&acc[PD_SECONDARIES], c.secondaries);
    atomicAdd(&acc[PD_DRAWS], c.draws);
    atomicMax(&acc[PD_MAX_DRAWS], c.max_draws);
    atomicAdd(&acc[PD_OVER_STRIDE], c.over_stride);
    __syncthreads();
    if (threadIdx.x < kNDiag) {
        unsigned long long* d = reinterpret_cast<unsigned long long*>(P.diag) + threadIdx.x;
        if (threadIdx.x == PD_MAX_DRAWS)
            atomicMax(d, acc[threadIdx.x]);
        else
            atomicAdd(d, acc[threadIdx.x]);
    }
}

__device__ __forceinline__ uint32_t lane_prefix(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// Adds the wave's scored collisions (tally = counter index, or -1).  When
// all counters fit in LDS (P.lds_tally) each block counts into its own copy
// and adds it to HBM once at its end (tally_lds_begin / tally_lds_end);
// otherwise one 64-bit HBM atomic per distinct counter of the wave.  Either
// way same-address atomics from every wave of the GPU, which serialise, are
// avoided.  Called by the whole wave.
// Lane l's value of v as a wave-uniform (scalar) value: the compiler then
// treats what depends on it (loop exits included) as uniform, where a lane
// shuffle's result would count as divergent.
__device__ __forceinline__ uint64_t lane_value(uint64_t v, int l) {
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v)), l));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v >> 32)), l));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ void wave_tally(const PulseParams& P, int64_t tally, uint32_t lane,
                                           unsigned long long* lds_counts) {
    if (P.lds_tally) {
        // the block's own copy of every counter (added to HBM at the end)
        if (tally >= 0) atomicAdd(lds_counts + tally, 1ull);
        return;
    }
    uint64_t pending = __ballot(tally >= 0);
    while (pending != 0) {
        const int leader = __ffsll(static_cast<long long>(pending)) - 1;
        const int64_t key = static_cast<int64_t>(lane_value(static_cast<uint64_t>(tally), leader));
        const uint64_t same = __ballot(tally == key);
        if (lane == static_cast<uint32_t>(leader))
            atomicAdd(reinterpret_cast<unsigned long long*>(P.counts) + key,
                      static_cast<unsigned long long>(__popcll(same)));
        pending &= ~same;
    }
}

// ------------------------------------------------------------ bank schedule

// Wave prefix sum of per-lane values v < 16 (one ballot per bit).
__device__ __forceinline__ uint32_t wave_prefix16(uint32_t v, uint32_t* total) {
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int bit = 0; bit < 4; ++bit) {
        const uint64_t m = __ballot((v >> bit) & 1u);
        off += lane_prefix(m) << bit;
        tot += static_cast<uint32_t>(__popcll(m)) << bit;
    }
    *total = tot;
    return off;
}

// Per-wave staging of appends in LDS: a wave collects the particles it
// banks here and copies them to the output bank with one atomic per
// flush, so the output counter sees one atomic per few iterations of a
// wave instead of one per iteration.
// Entries of a wave's bank stage: 16 KiB per wave (8 KiB at 512 threads,
// 4 KiB at 1024, so that a block fits in LDS).  Larger stages mean fewer
// flushes, each an atomic on the one output counter: 512 entries took the
// 1000 x 1000 problem from 6.1 to 5.7 ms and the event-based passes from
// 7.6 to 6.3 ms against 256.
constexpr uint32_t bank_stage_entries(int block) { return block >= 1024 ? 128u : (block >= 512 ? 256u : 512u); }

uint32_t pulse_bank_stage(int block) { return bank_stage_entries(block); }

template <uint32_t CAP>
struct BankStage {
    static constexpr uint32_t kCap = CAP;   // 32 B per entry
    double x[kCap];
    double t[kCap];
    uint64_t X[kCap];
    uint32_t batch[kCap];
    int32_t tb[kCap];
};

__device__ __forceinline__ void bank_store(const PulseParams& P, uint64_t o, double x, double t, uint64_t X,
                                           uint32_t batch, int32_t tb) {
    if (o < P.out_cap) {
        P.out.x[o] = x;
        P.out.t[o] = t;
        P.out.X[o] = X;
        P.out.batch[o] = batch;
        P.out.tb[o] = tb;
    } else {
        atomicOr(P.overflow, 1u);
    }
}

// Copies the wave's staged entries to the output bank (one atomic) and
// returns the output count just after them.
template <class Stage>
__device__ __forceinline__ uint64_t bank_flush(const PulseParams& P, Stage& S, uint32_t count,
                                               uint32_t lane) {
    __builtin_amdgcn_wave_barrier();
    uint64_t base = 0;
    if (lane == 0) base = atomicAdd(reinterpret_cast<unsigned long long*>(P.out_count), count);
    base = lane_value(base, 0);
    for (uint32_t i = lane; i < count; i += 64) bank_store(P, base + i, S.x[i], S.t[i], S.X[i], S.batch[i], S.tb[i]);
    __builtin_amdgcn_wave_barrier();
    return base + count;
}

// Per-wave staging of census arrivals (population control), flushed to
// P.cen with one atomic per flush.
struct CensusStage {
    static constexpr uint32_t kCap = 128;   // 28 B per entry: 3.5 KiB per wave
    double x[kCap];
    double mu[kCap];
    uint64_t X[kCap];
    uint32_t batch[kCap];
};

__device__ __forceinline__ void census_flush(const PulseParams& P, CensusStage& S, uint32_t count, uint32_t lane) {
    __builtin_amdgcn_wave_barrier();
    uint64_t base = 0;
    if (lane == 0) base = atomicAdd(reinterpret_cast<unsigned long long*>(P.cen_count), count);
    base = lane_value(base, 0);
    for (uint32_t i = lane; i < count; i += 64) {
        const uint64_t o = base + i;
        if (o < P.cen_cap) {
            PulseCensusEntry e;
            e.x = S.x[i];
            e.mu = S.mu[i];
            e.X = S.X[i];
            e.batch = S.batch[i];
            e.pad = 0;
            P.cen[o] = e;
        } else {
            atomicOr(P.overflow, 1u);
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// Stages the wave's census arrivals (lanes with at_census) in CS: the point
// x + mu (C - t), the direction and the state.  Called by the whole wave.
__device__ __forceinline__ void census_stage(const PulseParams& P, CensusStage& CS, uint32_t& cstaged,
                                             bool at_census, const PParticle& p, uint32_t lane) {
    const uint64_t cm = __ballot(at_census);
    if (cm == 0) return;
    const uint32_t cnt = static_cast<uint32_t>(__popcll(cm));
    if (cstaged + cnt > CensusStage::kCap) {
        census_flush(P, CS, cstaged, lane);
        cstaged = 0;
    }
    if (at_census) {
        const uint32_t e = cstaged + lane_prefix(cm);
        const double rest = P.t_end - p.t;
        const double step = p.mu * rest;
        CS.x[e] = p.x + step;
        CS.mu[e] = p.mu;
        CS.X[e] = p.X;
        CS.batch[e] = p.batch;
    }
    cstaged += cnt;
}

// Loads input item j of a bank or copies launch into p.
template <int ITEMS>
__device__ __forceinline__ void load_item(const PulseParams& P, uint64_t j, PParticle& p) {
    if (ITEMS == PULSE_ITEMS_COPIES) {
        const PulseCensusEntry e = P.copies[j];
        p.x = e.x;
        p.mu = e.mu;
        p.has_mu = true;
        p.X = e.X;
        p.batch = e.batch;
        p.t = P.t_start;
        p.tb = P.tb_start;
    } else {
        p.x = P.in.x[j];
        p.t = P.in.t[j];
        p.X = P.in.X[j];
        p.batch = P.in.batch[j];
        p.tb = P.in.tb[j];
        p.has_mu = false;
    }
}

// ITEMS: what a launch takes as input (sources, a generation bank, or the
// census copies starting an epoch).  PC: the launch's census (P.t_end) is a
// census of population control, whose arrivals go to P.cen.
template <int ITEMS, bool PC, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_pulse_bank(PulseParams P) {
    constexpr bool SOURCES = ITEMS == PULSE_ITEMS_SOURCES;
    constexpr bool COPIES = ITEMS == PULSE_ITEMS_COPIES;
    constexpr bool DIR = PC || COPIES;   // particles may carry a direction
    const uint32_t chunk = P.chunk;   // items a wave takes per atomic
    using Stage = BankStage<bank_stage_entries(BLOCK)>;
    __shared__ Stage stage[BLOCK / 64];
    __shared__ CensusStage cstage[PC ? BLOCK / 64 : 1];
    extern __shared__ unsigned long long lds_counts[];
    tally_lds_begin<BLOCK>(P, lds_counts);
    PulseLane c;
    const uint64_t n_items = SOURCES ? P.src_end - P.src_begin : P.n_in;
    const uint32_t lane = threadIdx.x & 63u;
    Stage& S = stage[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)];
    CensusStage& CS = cstage[PC ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0];
    uint32_t cstaged = 0;              // wave-uniform: entries in CS
    uint64_t wnext = 0, wend = 0;      // wave-uniform: the wave's unassigned items [wnext, wend)
    bool exhausted = false;            // wave-uniform
    uint32_t staged = 0;               // wave-uniform: entries in S
    uint64_t seen = 0;                 // wave-uniform: output count after this wave's last flush
    PParticle p;
    p.x = p.t = 0.0;
    p.X = 0;
    p.tb = -1;
    p.batch = 0;
    p.mu = 0.0;
    p.has_mu = false;
    bool active = false;
    for (;;) {
        const uint64_t need = __ballot(!active);
        if (need != 0 && wnext == wend && !exhausted) {
            uint64_t b = 0;
            if (lane == 0) b = atomicAdd(reinterpret_cast<unsigned long long*>(P.item_counter), chunk);
            b = lane_value(b, 0);
            if (b + chunk >= n_items) exhausted = true;
            wnext = b < n_items ? b : n_items;
            wend = b + chunk < n_items ? b + chunk : n_items;
        }
        const uint64_t avail = wend - wnext;
        const uint32_t nneed = static_cast<uint32_t>(__popcll(need));
        const uint32_t take = avail < nneed ? static_cast<uint32_t>(avail) : nneed;
        const uint32_t rank = lane_prefix(need);
        const uint64_t mine = wnext + rank;
        wnext += take;
        if (!active && rank < take) {
            const uint64_t j = mine;
            if (SOURCES) {
                p.X = pulse_source_state(P, P.src_begin + j, &p.batch);
                p.x = 0.0;
                p.t = 0.0;
                p.tb = P.tb0;
                c.sources++;
            } else {
                load_item<ITEMS>(P, j, p);
            }
            active = true;
        }
        if (__ballot(active) == 0 && wnext == wend && exhausted) break;
        uint32_t n = 0;
        int64_t tally = -1;
        bool at_census = false;
        if (active) {
            uint32_t draws = 0;
            n = pulse_particle<DIR>(P, p, c, &draws, &tally, &at_census);
            note_stream(P, c, draws);   // every particle has its own stream
            if (n == 0) active = false;
        }
        wave_tally(P, tally, lane, lds_counts);
        if (PC) census_stage(P, CS, cstaged, at_census, p, lane);
        // siblings (keys 2..n) are banked and the line runs on with key 1
        // while this wave's view of the output count (last flush + staged)
        // is within the budget; past it (or with no budget: the event
        // schedule), a scattering banks all n and ends the line
        uint32_t sib_total = 0;
        wave_prefix16(n > 1 ? n - 1 : 0, &sib_total);
        const bool keep = P.cont_budget != 0 && seen + staged + sib_total <= P.cont_budget;   // 0: event based
        const uint32_t k0 = keep ? 2u : 1u;
        const uint32_t npush = n >= k0 ? n - k0 + 1 : 0;
        uint32_t total = 0;
        const uint32_t off = wave_prefix16(npush, &total);
        if (total != 0) {
            if (staged + total > Stage::kCap) {
                seen = bank_flush(P, S, staged, lane);
                staged = 0;
            }
            if (total <= Stage::kCap) {
                for (uint32_t k = k0; k <= n; ++k) {
                    const uint32_t e = staged + off + (k - k0);
                    S.x[e] = p.x;
                    S.t[e] = p.t;
                    S.X[e] = murmur_hash(k, p.X) & P.lcg.mask;
                    S.batch[e] = p.batch;
                    S.tb[e] = p.tb;
                }
                staged += total;
            } else {
                // more than the stage holds (large multiplicities): straight to the bank
                uint64_t base = 0;
                if (lane == 0) base = atomicAdd(reinterpret_cast<unsigned long long*>(P.out_count), total);
                base = lane_value(base, 0);
                for (uint32_t k = k0; k <= n; ++k)
                    bank_store(P, base + off + (k - k0), p.x, p.t, murmur_hash(k, p.X) & P.lcg.mask, p.batch, p.tb);
                seen = base + total;
            }
        }
        if (n > 0) {
            if (keep) {
                p.X = murmur_hash(1ull, p.X) & P.lcg.mask;   // the first emerging particle runs on here
                p.has_mu = false;
            } else {
                active = false;
            }
        }
    }
    if (staged != 0) bank_flush(P, S, staged, lane);
    if (PC && cstaged != 0) census_flush(P, CS, cstaged, lane);
    tally_lds_end<BLOCK>(P, lds_counts);
    flush_lane_counters<BLOCK>(P, c);
}

// ------------------------------------------------------------ family schedule

// Banks the particles of keys k0..k1 emerging from a scattering of state
// key at (x, t, tb): a finish launch leaves them to the next generation.
__device__ __forceinline__ void spill(const PulseParams& P, double x, double t, int32_t tb, uint32_t batch,
                                      uint64_t key, uint32_t k0, uint32_t k1) {
    if (k1 < k0) return;
    const uint64_t base = atomicAdd(reinterpret_cast<unsigned long long*>(P.out_count),
                                    static_cast<unsigned long long>(k1 - k0 + 1));
    for (uint32_t k = k0; k <= k1; ++k)
        bank_store(P, base + (k - k0), x, t, murmur_hash(k, key) & P.lcg.mask, batch, tb);
}

// ITEMS = sources: the family schedule.  ITEMS = a generation bank (hash
// seeding): a finish launch, which runs each input particle's descendants
// depth first as well, up to P.lane_budget particles per input particle;
// what is left then (the first emerging particle and the stack), and
// siblings that find the stack full, go to the output bank.  So a finish
// launch appends at most (budget + stack_depth + 1) n_max particles and
// banks at most `budget` census arrivals per input particle.
constexpr uint32_t kFamilyChunk = 64;   // items a wave of the family kernel takes per atomic

// A source of the family schedule, seeded when its wave takes the chunk.
struct __align__(16) FamilySource {
    uint64_t X;
    uint32_t batch;
    uint32_t pad;
};

// A family of a chunk with a tally slot has ended: the lane whose end leaves
// the chunk with no family marks the slot for its wave's flush.
__device__ __forceinline__ void family_ended(uint32_t* slot_alive, int32_t& lsl) {
    if (lsl < 0) return;
    const int32_t s = lsl >> 16;
    lsl = atomicSub(slot_alive + s, 1u) == 1u ? -2 - s : -1;
}

// Banks a lane's whole stack, bottom entry first: the sp entries in HBM,
// then the top entry.
__device__ __forceinline__ void spill_stack(const PulseParams& P, const PulseStackEntry* stack, uint64_t sstride,
                                            uint32_t sp, const PulseStackEntry& top, bool has_top, uint32_t batch) {
    for (uint32_t i = 0; i < sp; ++i) {
        const PulseStackEntry& e = stack[static_cast<uint64_t>(i) * sstride];
        spill(P, e.x, e.t, e.tb, batch, e.key, e.next, e.n);
    }
    if (has_top) spill(P, top.x, top.t, top.tb, batch, top.key, top.next, top.n);
}

template <bool HASH, int ITEMS, bool PC, int BLOCK, bool DEEP, bool SLOTS>
__global__ void __launch_bounds__(BLOCK) k_pulse_family(PulseParams P) {
    constexpr bool SOURCES = ITEMS == PULSE_ITEMS_SOURCES;
    constexpr bool SPILL = !SOURCES;
    constexpr bool DIR = PC || ITEMS == PULSE_ITEMS_COPIES;
    __shared__ CensusStage cstage[PC ? BLOCK / 64 : 1];
    extern __shared__ unsigned long long lds_counts[];
    tally_lds_begin<BLOCK>(P, lds_counts);
    PulseLane c;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t gl = static_cast<uint64_t>(blockIdx.x) * BLOCK + threadIdx.x;
    // The lane's stack.  DEEP (many families per lane): its top entry in
    // registers (top, valid if has_top), the entries below it in HBM, entry d
    // of every lane of the launch in one plane (stack[d * sstride]), so that
    // a wave's lanes at one depth share lines and the planes in use are a few
    // dense regions.  Otherwise every entry in HBM, the lane's own entries
    // contiguous (stack[d]), the top updated in place: a lane that runs alone
    // on its SIMD waits for each entry anyway, and the registers the top
    // would take cost occupancy.
    PulseStackEntry* const stack = DEEP ? P.stack + gl : P.stack + gl * P.stack_depth;
    const uint64_t sstride = DEEP ? static_cast<uint64_t>(gridDim.x) * BLOCK : 1ull;
    // sources: the wave's current chunk, seeded at once (one per lane) when
    // the chunk is taken, so that a lane taking a source reads it from LDS
    __shared__ FamilySource s_src[SOURCES ? BLOCK / 64 : 1][SOURCES ? kFamilyChunk : 1];
    FamilySource* const ring = s_src[SOURCES ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0];
    uint64_t cbase = 0;        // wave-uniform: the item of ring[0]
    // Tally slots (SLOTS: sources, counters that do not fit one LDS copy per
    // block): each chunk of sources the wave takes gets a slot of
    // 2 x n_time_bins counters in LDS (its sources span at most two batches);
    // its families count there, and the slot goes to HBM once the chunk's
    // last family has ended.  With no slot free the chunk counts straight
    // into HBM.
    constexpr bool SL = SOURCES && SLOTS;
    const uint32_t nslots = SL ? P.tally_slots : 0u;
    const uint32_t nt = P.n_time_bins;
    __shared__ uint32_t s_slot[SL ? BLOCK / 64 : 1][SL ? 2 * kPulseTallySlots : 1];
    uint32_t* const slot_alive = s_slot[SL ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0];
    uint32_t* const slot_b0 = slot_alive + (SL ? kPulseTallySlots : 0);   // first batch of the slot's chunk
    unsigned long long* const wslots =
        lds_counts + static_cast<size_t>(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * nslots * 2u * nt;
    if (SL)
        for (uint32_t i = lane; i < nslots * 2u * nt; i += 64u) wslots[i] = 0ull;
    uint32_t free_mask = nslots >= 32 ? 0xffffffffu : (1u << nslots) - 1u;   // wave-uniform
    int32_t cur_slot = -1;     // wave-uniform: the current chunk's slot
    uint32_t cur_b0 = 0;       // wave-uniform: the current chunk's first batch
    // the lane's family: slot s and the counter of its batch's time bin 0
    // in wslots as (s << 16) | base; -1: counts go to HBM; -2 - s: the lane
    // ended the last family of slot s's chunk (flushed at the next top)
    int32_t lsl = -1;
    CensusStage& CS = cstage[PC ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0];
    uint32_t cstaged = 0;      // wave-uniform: entries in CS
    uint32_t sp = 0;           // entries in HBM (DEEP: below the top)
    PulseStackEntry top{};
    bool has_top = false;
    const uint64_t n_items = SOURCES ? P.src_end - P.src_begin : P.n_in;

    PParticle p;
    p.x = p.t = 0.0;
    p.X = 0;
    p.tb = -1;
    p.batch = 0;
    p.mu = 0.0;
    p.has_mu = false;
    bool active = false;       // the lane holds a particle of a family
    bool exhausted = false;    // wave-uniform: the item counter has passed the end
    uint64_t wnext = 0, wend = 0;   // wave-uniform: the wave's untaken items [wnext, wend)
    uint32_t pdraws = 0;       // draws of the current stream (hash: particle; stride: family)
    uint32_t budget = 0;       // finish: particles the current item may still start

    for (;;) {
        if (SL) {
            // slots whose chunk has no family left: add them to HBM, clear, free
            uint64_t fm = __ballot(lsl <= -2);
            while (fm != 0) {
                const int leader = __ffsll(static_cast<long long>(fm)) - 1;
                const uint32_t s = static_cast<uint32_t>(-2 - __builtin_amdgcn_readlane(lsl, leader));
                const uint64_t c0 = static_cast<uint64_t>(slot_b0[s]) * nt;
                unsigned long long* const sc = wslots + static_cast<size_t>(s) * 2u * nt;
                for (uint32_t i = lane; i < 2u * nt; i += 64u) {
                    const unsigned long long v = sc[i];
                    if (v != 0ull) {
                        if (c0 + i < P.n_counters) atomicAdd(reinterpret_cast<unsigned long long*>(P.counts) + c0 + i, v);
                        sc[i] = 0ull;
                    }
                }
                free_mask |= 1u << s;
                fm &= fm - 1ull;
            }
            if (lsl <= -2) lsl = -1;
        }
        // lanes without a family take the next items from the wave's chunk
        // (one atomic per kFamilyChunk items: the counter is one address
        // for the whole GPU)
        const uint64_t need = __ballot(!active);
        if (need != 0 && wnext == wend && !exhausted) {
            uint64_t b = 0;
            if (lane == 0) b = atomicAdd(reinterpret_cast<unsigned long long*>(P.family_counter), kFamilyChunk);
            b = lane_value(b, 0);
            if (b + kFamilyChunk >= n_items) exhausted = true;
            wnext = b < n_items ? b : n_items;
            wend = b + kFamilyChunk < n_items ? b + kFamilyChunk : n_items;
            if (SOURCES) {
                const uint64_t j = wnext + lane;
                if (j < wend) {
                    FamilySource e;
                    e.X = pulse_source_state(P, P.src_begin + j, &e.batch);
                    e.pad = 0;
                    ring[lane] = e;
                }
                cbase = wnext;
                __builtin_amdgcn_wave_barrier();
                cur_slot = -1;
                if (SL && nslots != 0 && free_mask != 0 && wend > wnext) {
                    cur_slot = __builtin_ctz(free_mask);
                    free_mask &= free_mask - 1u;
                    cur_b0 = ring[0].batch;
                    if (lane == 0) {
                        slot_alive[cur_slot] = static_cast<uint32_t>(wend - wnext);
                        slot_b0[cur_slot] = cur_b0;
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
        }
        if (need != 0 && wnext != wend) {
            const uint64_t avail = wend - wnext;
            const uint32_t nneed = static_cast<uint32_t>(__popcll(need));
            const uint32_t take = avail < nneed ? static_cast<uint32_t>(avail) : nneed;
            const uint32_t rank = lane_prefix(need);
            const uint64_t wbase = wnext;
            wnext += take;
            if (!active && rank < take) {
                const uint64_t j = wbase + rank;
                if (SOURCES) {
                    const FamilySource e = ring[j - cbase];
                    p.X = e.X;
                    p.batch = e.batch;
                    if (SL)
                        lsl = cur_slot >= 0 ? (cur_slot << 16) | static_cast<int32_t>(static_cast<uint32_t>(cur_slot) * 2u * nt +
                                                                                    (e.batch - cur_b0) * nt)
                                            : -1;
                    p.x = 0.0;
                    p.t = 0.0;
                    p.tb = P.tb0;
                    c.sources++;
                } else {
                    load_item<ITEMS>(P, j, p);
                }
                pdraws = 0;
                sp = 0;
                has_top = false;
                budget = P.lane_budget;
                active = true;
            }
        }
        if (__ballot(active) == 0 && wnext == wend && exhausted) break;
        uint32_t n = 0;
        int64_t tally = -1;
        bool at_census = false;
        if (active) n = pulse_particle<DIR>(P, p, c, &pdraws, &tally, &at_census);
        if (SL) {
            if (tally >= 0 && lsl >= 0)
                atomicAdd(wslots + (lsl & 0xffff) + static_cast<uint32_t>(tally - static_cast<int64_t>(p.batch) * nt), 1ull);
            wave_tally(P, lsl >= 0 ? -1 : tally, lane, lds_counts);   // chunks without a slot
        } else {
            wave_tally(P, tally, lane, lds_counts);
        }
        if (PC) census_stage(P, CS, cstaged, at_census, p, lane);
        if (!active) continue;
        if (HASH) {
            // the particle's own stream ends here
            note_stream(P, c, pdraws);
            pdraws = 0;
        }
        if (SPILL) budget--;
        if (n > 0) {
            if (n > 1) {
                if (sp + (has_top ? 1u : 0u) == P.stack_depth) {   // has_top is false unless DEEP
                    if (SPILL) {
                        spill(P, p.x, p.t, p.tb, p.batch, p.X, 2, n);
                    } else {
                        atomicOr(P.overflow, 1u);
                        active = false;   // the family is abandoned; the run reports an error
                        if (SL) family_ended(slot_alive, lsl);
                        continue;
                    }
                } else {
                    PulseStackEntry e;
                    e.x = p.x;
                    e.t = p.t;
                    e.key = p.X;
                    e.tb = p.tb;
                    e.next = 2;
                    e.n = static_cast<uint16_t>(n);
                    if (DEEP) {
                        if (has_top) stack[static_cast<uint64_t>(sp++) * sstride] = top;
                        top = e;
                        has_top = true;
                    } else {
                        stack[sp++] = e;
                    }
                }
            }
            if (SPILL && budget == 0) {
                // out of budget: the first emerging particle and the stack go to the bank
                spill(P, p.x, p.t, p.tb, p.batch, p.X, 1, 1);
                spill_stack(P, stack, sstride, sp, top, has_top, p.batch);
                sp = 0;
                has_top = false;
                active = false;
                continue;
            }
            if (HASH) p.X = murmur_hash(1ull, p.X) & P.lcg.mask;
            p.has_mu = false;
            continue;   // the first emerging particle starts at once
        }
        if (DEEP ? !has_top : sp == 0) {
            if (!HASH) note_stream(P, c, pdraws);
            active = false;
            if (SL) family_ended(slot_alive, lsl);
            continue;
        }
        if (SPILL && budget == 0) {
            spill_stack(P, stack, sstride, sp, top, has_top, p.batch);
            sp = 0;
            has_top = false;
            active = false;
            continue;
        }
        PulseStackEntry& e = DEEP ? top : stack[sp - 1];
        p.x = e.x;
        p.t = e.t;
        p.tb = e.tb;
        p.has_mu = false;
        if (HASH) p.X = murmur_hash(e.next, e.key) & P.lcg.mask;
        if (e.next != e.n) {
            e.next++;
        } else if (!DEEP) {
            --sp;
        } else if (sp > 0) {
            // the entry's last sibling: the entry below becomes the top (its
            // load is in flight while this sibling's line runs)
            top = stack[static_cast<uint64_t>(--sp) * sstride];
        } else {
            has_top = false;
        }
    }
    if (PC && cstaged != 0) census_flush(P, CS, cstaged, lane);
    tally_lds_end<BLOCK>(P, lds_counts);
    flush_lane_counters<BLOCK>(P, c);
}

// ------------------------------------------------------------ population control

// Arrivals per batch at census P.census: a block-local histogram over the
// chunk's batches, added to P.pop once per block.
__global__ void __launch_bounds__(256) k_pulse_census_count(PulseParams P, uint64_t n) {
    __shared__ uint32_t hist[kPulsePcChunkBatches];
    for (uint32_t i = threadIdx.x; i < P.n_chunk_batches; i += 256) hist[i] = 0;
    __syncthreads();
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * 256) {
        const uint32_t k = P.cen[i].batch - P.batch_lo;
        if (k < P.n_chunk_batches)
            atomicAdd(&hist[k], 1u);
        else
            atomicOr(P.overflow, 2u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < P.n_chunk_batches; i += 256)
        if (hist[i] != 0)
            atomicAdd(reinterpret_cast<unsigned long long*>(P.pop) +
                          (static_cast<uint64_t>(P.batch_lo + i) * P.n_census + P.census) * 2,
                      static_cast<unsigned long long>(hist[i]));
}

// Copies left by arrival a: q + [u < r/N] with u the one-off value of the
// arrival's state under the phase seed of (batch, census); the comparison
// ((S >> (m-53)) + 1) N < r 2^53 is exact in 128 bits.
__device__ __forceinline__ uint64_t split_copies(const PulseParams& P, const PulseCensusEntry& a) {
    const LcgDev& L = P.lcg;
    const uint64_t N = P.pop[(static_cast<uint64_t>(a.batch) * P.n_census + P.census) * 2];
    const uint64_t M = P.pc_target;
    const uint64_t q = M / N, r = M - q * N;
    const uint64_t phase = murmur_hash(P.census + 1ull, murmur_hash(P.first_batch + a.batch + 1ull, P.pc_seed));
    const uint64_t S = murmur_hash(a.X, phase) & L.mask;
    const uint64_t j1 = (S >> L.shift53) + 1ull;
    const uint64_t lo = j1 * N, hi = __umul64hi(j1, N);
    const uint64_t rlo = r << 53, rhi = r >> 11;
    const bool extra = hi < rhi || (hi == rhi && lo < rlo);
    return q + (extra ? 1ull : 0ull);
}

// Block exclusive scan of one value per thread (BLOCK = 256).
__device__ __forceinline__ uint64_t block_scan256(uint64_t v, uint64_t* total, uint64_t* s_wave) {
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    uint64_t incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t o = __shfl_up(incl, off);
        if (lane >= static_cast<uint32_t>(off)) incl += o;
    }
    if (lane == 63) s_wave[w] = incl;
    __syncthreads();
    uint64_t before = 0, all = 0;
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
        if (i < w) before += s_wave[i];
        all += s_wave[i];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

// The copies of every arrival of census P.census.  A block takes a tile of
// 256 x 16 arrivals, counts their copies, reserves room for all of them with
// one atomic, and writes copy k of arrival X as (x, mu, hash(k, X), batch).
__global__ void __launch_bounds__(256) k_pulse_split(PulseParams P, uint64_t n) {
    constexpr uint32_t kPer = 16;
    __shared__ unsigned long long hist[kPulsePcChunkBatches];
    __shared__ uint64_t s_wave[4];
    __shared__ uint64_t s_base;
    for (uint32_t i = threadIdx.x; i < P.n_chunk_batches; i += 256) hist[i] = 0;
    __syncthreads();
    const uint64_t tile = 256ull * kPer;
    for (uint64_t t0 = static_cast<uint64_t>(blockIdx.x) * tile; t0 < n; t0 += static_cast<uint64_t>(gridDim.x) * tile) {
        uint64_t mine = 0;
        for (uint32_t t = 0; t < kPer; ++t) {
            const uint64_t i = t0 + t * 256ull + threadIdx.x;
            if (i < n) mine += split_copies(P, P.cen[i]);
        }
        uint64_t total = 0;
        uint64_t o = block_scan256(mine, &total, s_wave);
        if (threadIdx.x == 0) s_base = atomicAdd(reinterpret_cast<unsigned long long*>(P.copy_count), total);
        __syncthreads();
        o += s_base;
        for (uint32_t t = 0; t < kPer; ++t) {
            const uint64_t i = t0 + t * 256ull + threadIdx.x;
            if (i >= n) continue;
            const PulseCensusEntry a = P.cen[i];
            const uint64_t nk = split_copies(P, a);
            for (uint64_t k = 1; k <= nk; ++k, ++o) {
                if (o < P.copy_cap) {
                    PulseCensusEntry e;
                    e.x = a.x;
                    e.mu = a.mu;
                    e.X = murmur_hash(k, a.X) & P.lcg.mask;
                    e.batch = a.batch;
                    e.pad = 0;
                    P.copies_out[o] = e;
                } else {
                    atomicOr(P.overflow, 1u);
                }
            }
            const uint32_t kb = a.batch - P.batch_lo;
            if (kb < P.n_chunk_batches)
                atomicAdd(&hist[kb], static_cast<unsigned long long>(nk));
            else
                atomicOr(P.overflow, 2u);
        }
        __syncthreads();   // s_base and s_wave are reused by the next tile
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < P.n_chunk_batches; i += 256)
        if (hist[i] != 0)
            atomicAdd(reinterpret_cast<unsigned long long*>(P.pop) +
                          (static_cast<uint64_t>(P.batch_lo + i) * P.n_census + P.census) * 2 + 1,
                      hist[i]);
}

// ------------------------------------------------------------ flux

// count / (((sigma_t N_b) dx) dt); with population control the count is
// first multiplied by its epoch's weight w_e (w_0 = 1,
// w_{c+1} = (w_c N_c) / M, N_c the batch's arrivals at census c).
__global__ void __launch_bounds__(256) k_pulse_flux(PulseParams P, double* flux) {
    const uint64_t n = static_cast<uint64_t>(P.n_batches) * P.n_time_bins;
    const double dx = P.x_hi - P.x_lo;
    const double nb = static_cast<double>(P.per_batch);
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * 256) {
        const uint32_t k = static_cast<uint32_t>(i % P.n_time_bins);
        const double dt = P.t_edges[k + 1] - P.t_edges[k];
        const double den = ((P.sigma_t * nb) * dx) * dt;
        if (P.n_census == 0) {
            flux[i] = static_cast<double>(P.counts[i]) / den;
        } else {
            const uint64_t b = i / P.n_time_bins;
            double w = 1.0;
            for (uint32_t e = 0; e < P.n_census && k >= (e + 1) * P.census_every; ++e)
                w = (w * static_cast<double>(P.pop[(b * P.n_census + e) * 2])) / static_cast<double>(P.pc_target);
            flux[i] = (static_cast<double>(P.counts[i]) * w) / den;
        }
    }
}

// ------------------------------------------------------------ launchers

static int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
    return cus > 0 ? cus : 256;
}

template <int BLOCK>
static const void* bank_kernel_b(int items, bool pc) {
    switch (items) {
        case PULSE_ITEMS_SOURCES:
            return pc ? reinterpret_cast<const void*>(k_pulse_bank<PULSE_ITEMS_SOURCES, true, BLOCK>)
                      : reinterpret_cast<const void*>(k_pulse_bank<PULSE_ITEMS_SOURCES, false, BLOCK>);
        case PULSE_ITEMS_COPIES:
            return pc ? reinterpret_cast<const void*>(k_pulse_bank<PULSE_ITEMS_COPIES, true, BLOCK>)
                      : reinterpret_cast<const void*>(k_pulse_bank<PULSE_ITEMS_COPIES, false, BLOCK>);
        default:
            return pc ? reinterpret_cast<const void*>(k_pulse_bank<PULSE_ITEMS_BANK, true, BLOCK>)
                      : reinterpret_cast<const void*>(k_pulse_bank<PULSE_ITEMS_BANK, false, BLOCK>);
    }
}

static const void* bank_kernel(int block, int items, bool pc) {
    switch (block) {
        case 64: return bank_kernel_b<64>(items, pc);
        case 128: return bank_kernel_b<128>(items, pc);
        case 512: return bank_kernel_b<512>(items, pc);
        case 1024: return bank_kernel_b<1024>(items, pc);
        default: return bank_kernel_b<256>(items, pc);
    }
}

static int bank_block(int block) {
    return (block == 64 || block == 128 || block == 512 || block == 1024) ? block : 256;
}

size_t pulse_tally_lds_bytes(const PulseParams& p) { return p.lds_tally ? 8ull * p.n_counters : 0; }

static uint64_t bank_items(const PulseParams& p, int items_kind) {
    return items_kind == PULSE_ITEMS_SOURCES ? p.src_end - p.src_begin : p.n_in;
}

uint32_t pulse_bank_grid(const PulseParams& p, int items_kind, bool pc, int block, uint64_t items) {
    // resident blocks only: waves keep taking chunks of items, so a launch
    // ends with one tail instead of one per wave
    block = bank_block(block);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bank_kernel(block, items_kind, pc), block,
                                                     pulse_tally_lds_bytes(p)) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const uint64_t per_block = static_cast<uint64_t>(p.chunk) * static_cast<uint64_t>(block / 64);
    uint64_t blocks = (items + per_block - 1) / per_block;   // a chunk per wave at least
    const uint64_t cap = static_cast<uint64_t>(device_cus()) * static_cast<uint64_t>(per_cu);
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    return static_cast<uint32_t>(blocks);
}

hipError_t launch_pulse_bank(const PulseParams& p, int items_kind, bool pc, int block, uint32_t grid,
                             hipStream_t st) {
    if (bank_items(p, items_kind) == 0) return hipSuccess;
    block = bank_block(block);
    PulseParams arg = p;
    void* args[] = {&arg};
    return hipLaunchKernel(bank_kernel(block, items_kind, pc), dim3(grid), dim3(block), args,
                           pulse_tally_lds_bytes(p), st);
}

static uint32_t stream_grid(uint64_t work, uint64_t per_block) {
    uint64_t blocks = (work + per_block - 1) / per_block;
    const uint64_t cap = static_cast<uint64_t>(device_cus()) * 8;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    return static_cast<uint32_t>(blocks);
}

hipError_t launch_pulse_census_count(const PulseParams& p, uint64_t n_arrivals, hipStream_t st) {
    if (n_arrivals == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pulse_census_count, dim3(stream_grid(n_arrivals, 256ull * 16)), dim3(256), 0, st, p,
                       n_arrivals);
    return hipGetLastError();
}

hipError_t launch_pulse_split(const PulseParams& p, uint64_t n_arrivals, hipStream_t st) {
    if (n_arrivals == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pulse_split, dim3(stream_grid(n_arrivals, 256ull * 16)), dim3(256), 0, st, p, n_arrivals);
    return hipGetLastError();
}

// Tally slots per wave of the family kernel over sources: when the counters
// do not fit one LDS copy per block, a chunk of 64 sources spans at most two
// batches (at least 64 sources per batch) and the slots of a block fit in
// 32 KiB.  MCRNG_PULSE_SLOTS sets the number (0: per-wave HBM atomics).
template <int BLOCK>
static uint32_t family_tally_slots(const PulseParams& p) {
    if (p.lds_tally || p.per_batch < kFamilyChunk || p.n_time_bins > 64) return 0;
    uint32_t k = kPulseTallySlots;
    if (const char* env = getenv("MCRNG_PULSE_SLOTS")) k = static_cast<uint32_t>(atoi(env));
    if (k > kPulseTallySlots) k = kPulseTallySlots;
    while (k > 0 && static_cast<size_t>(BLOCK / 64) * k * 2u * p.n_time_bins * 8u > 32768u) k /= 2;
    return k;
}

template <bool HASH, int BLOCK>
static hipError_t launch_family_b(const PulseParams& p_in, uint32_t grid, hipStream_t st) {
    PulseParams p = p_in;
    p.tally_slots = family_tally_slots<BLOCK>(p);
    const size_t lds = static_cast<size_t>(BLOCK / 64) * p.tally_slots * 2u * p.n_time_bins * 8u;
    // the register-top stack once every lane has many families to run
    // (MCRNG_PULSE_DEEP = 0 or 1 forces one form: both give the same counts)
    bool deep = p.src_end - p.src_begin >= 16ull * grid * BLOCK;
    if (const char* env = getenv("MCRNG_PULSE_DEEP")) deep = atoi(env) != 0;
    // the slot form only for the default block (other blocks count into HBM)
    constexpr bool kSlots = BLOCK == 256;
    if (!kSlots) p.tally_slots = 0;
    if (p.tally_slots != 0) {
        if (deep)
            hipLaunchKernelGGL((k_pulse_family<HASH, PULSE_ITEMS_SOURCES, false, BLOCK, true, kSlots>), dim3(grid),
                               dim3(BLOCK), lds, st, p);
        else
            hipLaunchKernelGGL((k_pulse_family<HASH, PULSE_ITEMS_SOURCES, false, BLOCK, false, kSlots>), dim3(grid),
                               dim3(BLOCK), lds, st, p);
    } else {
        if (deep)
            hipLaunchKernelGGL((k_pulse_family<HASH, PULSE_ITEMS_SOURCES, false, BLOCK, true, false>), dim3(grid),
                               dim3(BLOCK), pulse_tally_lds_bytes(p), st, p);
        else
            hipLaunchKernelGGL((k_pulse_family<HASH, PULSE_ITEMS_SOURCES, false, BLOCK, false, false>), dim3(grid),
                               dim3(BLOCK), pulse_tally_lds_bytes(p), st, p);
    }
    return hipGetLastError();
}

uint32_t pulse_finish_grid(uint64_t items) {
    uint64_t blocks = (items + 255) / 256;
    const uint64_t cap = static_cast<uint64_t>(device_cus()) * 8;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    return static_cast<uint32_t>(blocks);
}

hipError_t launch_pulse_finish(const PulseParams& p, bool pc, uint32_t grid, hipStream_t st) {
    if (p.n_in == 0) return hipSuccess;
    if (pc)
        hipLaunchKernelGGL((k_pulse_family<true, PULSE_ITEMS_BANK, true, 256, false, false>), dim3(grid), dim3(256),
                           pulse_tally_lds_bytes(p), st, p);
    else
        hipLaunchKernelGGL((k_pulse_family<true, PULSE_ITEMS_BANK, false, 256, false, false>), dim3(grid), dim3(256),
                           pulse_tally_lds_bytes(p), st, p);
    return hipGetLastError();
}

uint32_t pulse_family_grid(int block) {
    // persistent lanes: 2048 per CU (the stack buffer is sized from this);
    // a run of few sources has its waves spread over the whole chip
    return static_cast<uint32_t>(device_cus()) * static_cast<uint32_t>(2048 / block);
}

hipError_t launch_pulse_family(const PulseParams& p, int block, uint32_t grid, hipStream_t st) {
    if (p.src_end == p.src_begin) return hipSuccess;
    switch (block) {
        case 64: return p.hash ? launch_family_b<true, 64>(p, grid, st) : launch_family_b<false, 64>(p, grid, st);
        case 128: return p.hash ? launch_family_b<true, 128>(p, grid, st) : launch_family_b<false, 128>(p, grid, st);
        case 512: return p.hash ? launch_family_b<true, 512>(p, grid, st) : launch_family_b<false, 512>(p, grid, st);
        case 1024:
            return p.hash ? launch_family_b<true, 1024>(p, grid, st) : launch_family_b<false, 1024>(p, grid, st);
        default: return p.hash ? launch_family_b<true, 256>(p, grid, st) : launch_family_b<false, 256>(p, grid, st);
    }
}

hipError_t launch_pulse_flux(const PulseParams& p, double* flux, hipStream_t st) {
    const uint64_t n = static_cast<uint64_t>(p.n_batches) * p.n_time_bins;
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_pulse_flux, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, p, flux);
    return hipGetLastError();
}

}  // namespace mcrng
