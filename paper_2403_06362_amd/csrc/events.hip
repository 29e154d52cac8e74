// Event-sorted schedule for gfx950.
//
// The live particles sit in a structure-of-arrays bank in HBM.  One launch of
// k_event_step advances every live particle by exactly one event (the same
// step_particle as the history-based kernel, so the per-particle operation
// sequence is identical); survivors are appended to the other bank through
// one atomic per 1024-thread block, so each launch compacts the bank.  A
// particle scores into the partial-tally slot of its score unit: its own work
// unit, or, when the slice holds a single (problem, batch), the slice's first
// unit.  The reduction adds every unit slot of a (problem, batch), so any
// slot of it gives the same sum; with one slot for the whole slice every
// block's particles share its home slot (below) however the compaction
// orders them.  That slot may collect more than 2^32 additions per word, so
// its global adds carry a wrap of the low word into the high one
// (carry_add).  The slots are zeroed first and the sums are exact, so the
// result is the same as the history-based schedule's bit for bit.  (Scoring
// a mixed slice by (problem, batch) as well measured 12x slower on 64
// problems: its particles are mostly away from home, and one slot per
// problem concentrates their atomics.)  A history that ends writes one
// outcome record; k_event_unit_diag reduces the records of each unit in
// history order into the unit's diagnostics slot.  Once a slice's bank is
// small, k_event_finish runs its remaining particles to their ends (one per
// thread, the same per-event calls), which saves a launch per remaining
// event generation.
#include "particle.hpp"

namespace mcrng {

template <bool F32>
struct BankView {
    using R = typename std::conditional<F32, float, double>::type;
    R* x; R* mu; R* t;
    double* tau;   // the remaining optical depth is double in both modes
};

template <bool F32>
__device__ __forceinline__ BankView<F32> view(const EventBank& b) {
    BankView<F32> v;
    if constexpr (F32) {
        v.x = b.x32; v.mu = b.mu32; v.t = b.t32; v.tau = b.tau64;
    } else {
        v.x = b.x64; v.mu = b.mu64; v.t = b.t64; v.tau = b.tau64;
    }
    return v;
}

template <bool F32>
__device__ __forceinline__ CellsLds<F32> global_cells(const TransportParams& P, const DevProblem& PR) {
    CellsLds<F32> C;
    if constexpr (F32) {
        C.edge = P.edges32 + PR.edge_off;
        C.sig = P.sig32 + PR.cell_off;
        C.tedge = P.tedges32 + PR.tedge_off;
    } else {
        C.edge = P.edges64 + PR.edge_off;
        C.sig = P.sig64 + PR.cell_off;
        C.tedge = P.tedges64 + PR.tedge_off;
    }
    C.rsig = nullptr;   // each event refines its cell's reciprocal
    C.scat = P.scat64 + PR.cell_off;
    C.bin = P.cbin + PR.cell_off;
    C.n_cells = static_cast<int32_t>(PR.n_cells);
    C.n_time_bins = static_cast<int32_t>(PR.n_time_bins);
    C.n_space_bins = static_cast<int32_t>(PR.n_space_bins);
    return C;
}

// A bank particle's cell word carries its need-a-flight flag in bit 31
// (cell indices stay below 2^31): no separate flag word to read and write
// per event.
constexpr uint32_t kNeedTauBit = 0x80000000u;

template <bool F32>
__device__ __forceinline__ void load_cell(const EventBank& b, uint32_t i, Particle<F32>& p) {
    const uint32_t w = static_cast<uint32_t>(b.cell[i]);
    p.cell = static_cast<int32_t>(w & ~kNeedTauBit);
    p.need_tau = (w & kNeedTauBit) != 0;
}

// TIMED false: no problem of the set is timed, so a particle's time is never
// read and is not stored.
template <bool F32, bool TIMED>
__device__ __forceinline__ void store_particle(const EventBank& b, uint32_t i, const Particle<F32>& p, uint32_t ev,
                                               uint32_t co, uint32_t unit, uint32_t rec) {
    BankView<F32> v = view<F32>(b);
    v.x[i] = p.x;
    v.mu[i] = p.mu;
    if (TIMED) v.t[i] = p.t;
    v.tau[i] = p.tau;
    b.X[i] = p.X;
    b.cell[i] = static_cast<int32_t>(static_cast<uint32_t>(p.cell) | (p.need_tau ? kNeedTauBit : 0u));
    b.tb[i] = p.tb;
    b.hdraws[i] = p.hdraws;
    b.events[i] = ev;
    b.colls[i] = co;
    b.unit[i] = unit;
    b.rec[i] = rec;
}

// Particle i of the slice [unit_begin, unit_end): the unit is found by binary
// search over the units' first-record indices.
template <bool F32, bool TIMED>
__global__ void __launch_bounds__(256) k_event_init(EventParams E) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E.n_in) return;
    const uint64_t r = E.rec_begin[E.unit_begin] + i;
    uint32_t lo = E.unit_begin, hi = E.unit_end;   // last unit with rec_begin <= r
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (E.rec_begin[mid] <= r) lo = mid; else hi = mid;
    }
    const WorkUnit U = E.tp.units[lo];
    const DevProblem PR = E.tp.problems[U.problem];
    const CellsLds<F32> C = global_cells<F32>(E.tp, PR);
    const uint32_t su = E.one_group ? E.unit_begin : lo;   // score unit
    SeedDev S;
    S.kind = static_cast<int>(PR.seed_kind);
    S.stride_digits = PR.stride_digits;
    S.base = PR.seed_base;
    S.first_index = PR.first_index;
    S.table = PR.table;
    Particle<F32> p;
    init_particle<F32, TIMED>(p, C, E.tp.lcg, S, U.j0 + (r - E.rec_begin[lo]));
    store_particle<F32, TIMED>(E.in, i, p, 0u, 0u, su, static_cast<uint32_t>(r));
}

constexpr int kEventStepBlock = 1024;
constexpr int kEventStepPer = 4;             // particles per thread: a block takes 4096 consecutive ones
constexpr uint32_t kEventLdsBins = 2048;     // home-unit tally bins a block keeps in LDS (32 KiB)

// A block advances the 4096 consecutive bank particles from
// blockIdx * 4096 by one event each.  Particles of the score unit of the
// block's first particle (its home unit: all of them when the slice holds one
// (problem, batch)) score into an LDS copy of that unit's tally, added to the
// unit's slot once at the end; other particles' scores go straight to their
// slots.  Integer sums, so the bits do not depend on where a score is added
// first.  (An LDS copy of the home problem's cells as well measured no
// faster.)  Global adds into a one-group slice's slot carry; a unit's own
// slot takes at most its histories' scores, as in the history schedule.
template <bool F32, bool TIMED>
__global__ void __launch_bounds__(kEventStepBlock) k_event_step(EventParams E) {
    constexpr int kWaves = kEventStepBlock / 64;
    __shared__ uint32_t s_wave_count[kWaves];
    __shared__ uint32_t s_base;
    __shared__ unsigned long long s_tally[2 * kEventLdsBins];
    __shared__ uint32_t s_home, s_home_words;
    __shared__ uint64_t s_home_slot;
    const uint32_t b0 = blockIdx.x * (kEventStepBlock * kEventStepPer);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wid = threadIdx.x >> 6;
    if (blockIdx.x == 0 && threadIdx.x == 0) *E.n_clear = 0;
    // the grid covers a bound on the live count: blocks past it leave at once
    const uint32_t n_in = *E.n_live;
    if (b0 >= n_in) return;
    if (threadIdx.x == 0) {
        const uint32_t u = E.in.unit[b0];
        const WorkUnit U = E.tp.units[u];
        const bool fits = U.slice_bins <= kEventLdsBins;
        s_home = fits ? u : 0xffffffffu;
        s_home_words = fits ? 2 * U.slice_bins : 0u;
        s_home_slot = U.slot;
    }
    __syncthreads();
    const uint32_t home = s_home;
    for (uint32_t w = threadIdx.x; w < s_home_words; w += kEventStepBlock) s_tally[w] = 0;
    __syncthreads();

    for (int k = 0; k < kEventStepPer; ++k) {
        const uint32_t i = b0 + static_cast<uint32_t>(k) * kEventStepBlock + threadIdx.x;
        bool alive = false;
        Particle<F32> p;
        uint32_t unit = 0, rec = 0;
        LaneCounters cnt;
        if (i < n_in) {
            BankView<F32> v = view<F32>(E.in);
            p.x = v.x[i];
            p.mu = v.mu[i];
        set_direction<F32>(p);
            set_direction<F32>(p);
            p.t = TIMED ? v.t[i] : 0;
            p.tau = v.tau[i];
            p.X = E.in.X[i];
            load_cell<F32>(E.in, i, p);
            p.tb = E.in.tb[i];
            p.hdraws = E.in.hdraws[i];
            cnt.events = E.in.events[i];
            cnt.collisions = E.in.colls[i];
            unit = E.in.unit[i];
            rec = E.in.rec[i];
            const WorkUnit U = E.tp.units[unit];
            const DevProblem PR = E.tp.problems[U.problem];
            const CellsLds<F32> C = global_cells<F32>(E.tp, PR);
            const int end = (unit == home)  ? step_particle<F32, TIMED>(p, C, E.tp.lcg, reinterpret_cast<uint64_t*>(s_tally), cnt)
                            : E.one_group   ? step_particle<F32, TIMED, true>(p, C, E.tp.lcg, E.tp.partial + U.slot, cnt)
                                            : step_particle<F32, TIMED>(p, C, E.tp.lcg, E.tp.partial + U.slot, cnt);
            if (end != END_NONE) {
                HistoryRecord h;
                h.events = static_cast<uint32_t>(cnt.events);
                h.collisions = static_cast<uint32_t>(cnt.collisions);
                h.draws = p.hdraws;
                h.end = static_cast<uint32_t>(end);
                E.records[rec] = h;
            } else {
                alive = true;
            }
        }
        // compaction: the block's survivors go to consecutive slots of `out`
        // through one atomic per block and pass (a single counter hit once
        // per wave by every wave of the GPU serialises)
        const uint64_t mask = __ballot(alive);
        if (lane == 0) s_wave_count[wid] = static_cast<uint32_t>(__popcll(mask));
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t total = 0;
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t c = s_wave_count[w];
                s_wave_count[w] = total;
                total += c;
            }
            s_base = total ? atomicAdd(E.n_out, total) : 0u;
        }
        __syncthreads();
        if (alive) {
            const uint32_t lt = static_cast<uint32_t>(__popcll(mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane)))));
            store_particle<F32, TIMED>(E.out, s_base + s_wave_count[wid] + lt, p, static_cast<uint32_t>(cnt.events),
                                static_cast<uint32_t>(cnt.collisions), unit, rec);
        }
        __syncthreads();   // s_wave_count and s_base are reused by the next pass
    }
    // a block's LDS words stay below 4096 x 2^32; the slot's may wrap
    for (uint32_t w = 2 * threadIdx.x; w < s_home_words; w += 2 * kEventStepBlock)
        if ((s_tally[w] | s_tally[w + 1]) != 0) carry_add(E.tp.partial + s_home_slot + w, s_tally[w], s_tally[w + 1]);
}

// The particles of a small bank run to the end of their histories, one per
// thread (the same step_particle calls, event after event): the tail of a
// slice without one launch per remaining event.  In a one-group slice every
// particle has the same score unit, whose tally the block keeps in LDS (when
// it fits) and adds to the slot once, with carries.
template <bool F32, bool TIMED>
__global__ void __launch_bounds__(256) k_event_finish(EventParams E) {
    __shared__ unsigned long long s_tally[2 * kEventLdsBins];
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    const uint32_t n_in = *E.n_live;
    if (blockIdx.x * 256 >= n_in) return;   // the grid covers a bound on the live count
    const WorkUnit H = E.tp.units[E.unit_begin];
    const uint32_t words = (E.one_group && H.slice_bins <= kEventLdsBins) ? 2 * H.slice_bins : 0u;
    for (uint32_t w = threadIdx.x; w < words; w += 256) s_tally[w] = 0;
    __syncthreads();
    if (i < n_in) {
        BankView<F32> v = view<F32>(E.in);
        Particle<F32> p;
        LaneCounters cnt;
        p.x = v.x[i];
        p.mu = v.mu[i];
        set_direction<F32>(p);
        p.t = TIMED ? v.t[i] : 0;
        p.tau = v.tau[i];
        p.X = E.in.X[i];
        load_cell<F32>(E.in, i, p);
        p.tb = E.in.tb[i];
        p.hdraws = E.in.hdraws[i];
        cnt.events = E.in.events[i];
        cnt.collisions = E.in.colls[i];
        const uint32_t unit = E.in.unit[i];
        const uint32_t rec = E.in.rec[i];
        const WorkUnit U = E.tp.units[unit];
        const DevProblem PR = E.tp.problems[U.problem];
        const CellsLds<F32> C = global_cells<F32>(E.tp, PR);
        uint64_t* tally = E.tp.partial + U.slot;
        int end = END_NONE;
        if (words != 0)
            while (end == END_NONE)
                end = step_particle<F32, TIMED>(p, C, E.tp.lcg, reinterpret_cast<uint64_t*>(s_tally), cnt);
        else if (E.one_group)
            while (end == END_NONE) end = step_particle<F32, TIMED, true>(p, C, E.tp.lcg, tally, cnt);
        else
            while (end == END_NONE) end = step_particle<F32, TIMED>(p, C, E.tp.lcg, tally, cnt);
        HistoryRecord h;
        h.events = static_cast<uint32_t>(cnt.events);
        h.collisions = static_cast<uint32_t>(cnt.collisions);
        h.draws = p.hdraws;
        h.end = static_cast<uint32_t>(end);
        E.records[rec] = h;
    }
    __syncthreads();
    for (uint32_t w = 2 * threadIdx.x; w < words; w += 2 * 256)
        if ((s_tally[w] | s_tally[w + 1]) != 0) carry_add(E.tp.partial + H.slot + w, s_tally[w], s_tally[w + 1]);
}

// One block per unit: the unit's records, in history order, into its
// diagnostics slot.
__global__ void __launch_bounds__(256) k_event_unit_diag(EventParams E) {
    const uint32_t u = blockIdx.x;
    const WorkUnit U = E.tp.units[u];
    const DevProblem PR = E.tp.problems[U.problem];
    __shared__ unsigned long long acc[kNDiag];
    if (threadIdx.x < kNDiag) acc[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long loc[kNDiag];
#pragma unroll
    for (int k = 0; k < kNDiag; ++k) loc[k] = 0;
    const uint64_t r0 = E.rec_begin[u];
    for (uint32_t j = threadIdx.x; j < U.count; j += blockDim.x) {
        const HistoryRecord h = E.records[r0 + j];
        loc[D_HISTORIES] += 1;
        loc[D_LEAK_LEFT] += (h.end == END_LEAK_LEFT);
        loc[D_LEAK_RIGHT] += (h.end == END_LEAK_RIGHT);
        loc[D_ABSORBED] += (h.end == END_ABSORBED);
        loc[D_CENSUS] += (h.end == END_CENSUS);
        loc[D_EVENTS] += h.events;
        loc[D_COLLISIONS] += h.collisions;
        loc[D_DRAWS] += h.draws;
        loc[D_MAX_DRAWS] = h.draws > loc[D_MAX_DRAWS] ? h.draws : loc[D_MAX_DRAWS];
        loc[D_OVER_STRIDE] += (PR.stride_q != 0 && h.draws > PR.stride_q);
    }
#pragma unroll
    for (int k = 0; k < kNDiag; ++k) {
        if (k == D_MAX_DRAWS)
            atomicMax(&acc[k], loc[k]);
        else
            atomicAdd(&acc[k], loc[k]);
    }
    __syncthreads();
    if (threadIdx.x < kNDiag) E.tp.unit_diag[static_cast<size_t>(u) * kNDiag + threadIdx.x] = acc[threadIdx.x];
}

template <bool F32, bool TIMED>
static hipError_t init_t(const EventParams& p, hipStream_t st) {
    hipLaunchKernelGGL((k_event_init<F32, TIMED>), dim3((p.n_in + 255) / 256), dim3(256), 0, st, p);
    return hipGetLastError();
}

template <bool F32, bool TIMED>
static hipError_t step_t(const EventParams& p, hipStream_t st) {
    constexpr uint32_t per_block = kEventStepBlock * kEventStepPer;
    hipLaunchKernelGGL((k_event_step<F32, TIMED>), dim3((p.n_in + per_block - 1) / per_block), dim3(kEventStepBlock),
                       0, st, p);
    return hipGetLastError();
}

hipError_t launch_event_init(const EventParams& p, int f32, int timed, hipStream_t st) {
    if (p.n_in == 0) return hipSuccess;
    if (f32) return timed ? init_t<true, true>(p, st) : init_t<true, false>(p, st);
    return timed ? init_t<false, true>(p, st) : init_t<false, false>(p, st);
}

hipError_t launch_event_step(const EventParams& p, int f32, int timed, hipStream_t st) {
    if (p.n_in == 0) return hipSuccess;
    if (f32) return timed ? step_t<true, true>(p, st) : step_t<true, false>(p, st);
    return timed ? step_t<false, true>(p, st) : step_t<false, false>(p, st);
}

template <bool F32, bool TIMED>
static hipError_t finish_t(const EventParams& p, hipStream_t st) {
    hipLaunchKernelGGL((k_event_finish<F32, TIMED>), dim3((p.n_in + 255) / 256), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_event_finish(const EventParams& p, int f32, int timed, hipStream_t st) {
    if (p.n_in == 0) return hipSuccess;
    if (f32) return timed ? finish_t<true, true>(p, st) : finish_t<true, false>(p, st);
    return timed ? finish_t<false, true>(p, st) : finish_t<false, false>(p, st);
}

hipError_t launch_event_unit_diag(const EventParams& p, hipStream_t st) {
    if (p.tp.n_units == 0) return hipSuccess;
    hipLaunchKernelGGL(k_event_unit_diag, dim3(p.tp.n_units), dim3(256), 0, st, p);
    return hipGetLastError();
}

}  // namespace mcrng
