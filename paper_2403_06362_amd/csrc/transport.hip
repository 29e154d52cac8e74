// Fixed-source 1-D slab transport kernels for gfx950 (history-based schedule).
//
// k_transport (history-based, persistent).  A block takes work units (a run
// of histories of one batch of one problem) from a global counter.  For each
// unit it stages the problem's cells in LDS, zeroes an LDS tally slice and
// runs the unit's histories one per lane: a lane whose history ended takes
// the next history index of the unit through a wave ballot, a prefix count
// and one LDS atomic per wave.  Every track length is scored as the integer
// q = round-half-even(s 2^56) into the LDS slice (64-bit LDS atomics on its
// low and high 32-bit halves, exact while fewer than 2^32 of the unit's
// scores fall in one bin), so the unit's partial tally is an exact integer
// whatever order the lanes score in.  At the end of the unit the block adds
// its tally copies (carrying a wrap of the low word) and writes the slice to
// the unit's own partial-tally slot in HBM.  (Carrying every score's wrap,
// with a returning low-word atomic, measured 5-6% slower.)
//
// k_reduce sums the partial slots of each (problem, batch) in unit order
// (a fixed order; integer addition makes any order give the same bits),
// converts the 128-bit sums to double with round-half-even, normalises the
// flux and reduces per-problem diagnostics.
//
// The per-history arithmetic (flight sampling, cell / time marching,
// collision, scoring) follows the same fixed IEEE operation sequence in FP64
// mode and in FP32-flight mode; it is spelled out in step_particle (particle.hpp).
#include "particle.hpp"

namespace mcrng {

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v) {
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3(static_cast<unsigned>(b)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3(static_cast<unsigned>(b)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// LDS layout: [tally: copies x max_slice x 2 u64][edges][sig][rsig][scat f64][bin i32][tedges]
__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~static_cast<size_t>(15); }

size_t transport_lds_bytes(const TransportParams& p, int f32) {
    const size_t rs = f32 ? sizeof(float) : sizeof(double);
    size_t b = align16(static_cast<size_t>(p.tally_copies) * p.max_slice * 2 * sizeof(uint64_t));
    b += align16((p.max_cells + 1) * rs);
    b += align16(p.max_cells * rs);
    b += align16(p.max_cells * rs);
    b += align16(p.max_cells * sizeof(double));
    b += align16(p.max_cells * sizeof(int32_t));
    b += align16((p.max_tedges > 0 ? p.max_tedges : 1) * rs);
    return b;
}

size_t transport_static_lds_bytes(int block) {
    // skip table, rings, ring slice tags (k_transport_chain), block words
    return static_cast<size_t>(kStrideDigits) * kStrideRadix * 2 * sizeof(uint64_t) +
           static_cast<size_t>(block / 64) * 128 * (sizeof(uint64_t) + 1) + 512;
}

// Phase of a lane's history slot.
enum : int {
    PH_EMPTY = 0,   // no history: refilled at the next collision pass
    PH_GEOM = 1,    // has a flight: takes geometry steps
    PH_COLL = 2,    // stands at a collision site
    PH_NEW = 3      // a new history or a scattered particle: samples its next flight
};

__device__ __forceinline__ uint32_t wave_count(bool c) {
    return static_cast<uint32_t>(__popcll(__builtin_amdgcn_ballot_w64(c)));
}

// One history per lane: seven waves per SIMD (72 VGPRs, a few spilled)
// measured faster than five (FP64) or six (FP32) without spills, except
// FP64 with time bins, where six (80 VGPRs) is best.
template <bool F32, bool TIMED, int H, int BLOCK>
__global__ void __launch_bounds__(BLOCK, (H == 1) ? ((F32 || !TIMED) ? 7 : 6) : 1) k_transport(TransportParams P) {
    using R = typename Particle<F32>::R;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_unit;
    __shared__ uint32_t s_next;
    __shared__ unsigned long long s_diag[kNDiag];
    // the current problem's stride skip table: a history's start is a chain
    // of dependent table reads, cheaper from LDS than from the cache
    __shared__ uint64_t s_skip[kStrideDigits * kStrideRadix * 2];
    // per wave: start states of the next histories, seeded 64 at a time
    __shared__ uint64_t s_ring[BLOCK / 64][128];

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wid = tid >> 6;

    uint64_t* tally_all = reinterpret_cast<uint64_t*>(smem);
    size_t off = align16(static_cast<size_t>(P.tally_copies) * P.max_slice * 2 * sizeof(uint64_t));
    R* l_edge = reinterpret_cast<R*>(smem + off);
    off += align16((P.max_cells + 1) * sizeof(R));
    R* l_sig = reinterpret_cast<R*>(smem + off);
    off += align16(P.max_cells * sizeof(R));
    R* l_rsig = reinterpret_cast<R*>(smem + off);
    off += align16(P.max_cells * sizeof(R));
    double* l_scat = reinterpret_cast<double*>(smem + off);
    off += align16(P.max_cells * sizeof(double));
    int32_t* l_bin = reinterpret_cast<int32_t*>(smem + off);
    off += align16(P.max_cells * sizeof(int32_t));
    R* l_tedge = reinterpret_cast<R*>(smem + off);

    const R* g_edge;
    const R* g_sig;
    const R* g_tedge;
    if constexpr (F32) {
        g_edge = P.edges32;
        g_sig = P.sig32;
        g_tedge = P.tedges32;
    } else {
        g_edge = P.edges64;
        g_sig = P.sig64;
        g_tedge = P.tedges64;
    }

    const uint32_t copy = (P.tally_copies > 1) ? (wid % P.tally_copies) : 0u;
    int32_t cur_problem = -1;

    for (;;) {
        if (tid == 0) {
            s_unit = atomicAdd(P.unit_counter, 1u);
            s_next = 0;
        }
        if (tid < kNDiag) s_diag[tid] = 0;
        __syncthreads();
        const uint32_t pos = s_unit;
        if (pos >= P.n_units) break;
        const uint32_t ui = P.order[pos];
        const WorkUnit U = P.units[ui];
        const DevProblem PR = P.problems[U.problem];
        const uint32_t slice = PR.slice_bins;

        for (uint32_t c = 0; c < P.tally_copies; ++c)
            for (uint32_t i = tid; i < 2 * slice; i += BLOCK) tally_all[static_cast<size_t>(c) * P.max_slice * 2 + i] = 0;
        if (static_cast<int32_t>(U.problem) != cur_problem) {
            for (uint32_t i = tid; i <= PR.n_cells; i += BLOCK) l_edge[i] = g_edge[PR.edge_off + i];
            for (uint32_t i = tid; i < PR.n_cells; i += BLOCK) {
                const R sg = g_sig[PR.cell_off + i];
                l_sig[i] = sg;
                l_rsig[i] = recip_refined(sg);
                l_scat[i] = P.scat64[PR.cell_off + i];
                l_bin[i] = P.cbin[PR.cell_off + i];
            }
            if (TIMED)
                for (uint32_t i = tid; i <= PR.n_time_bins; i += BLOCK) l_tedge[i] = g_tedge[PR.tedge_off + i];
            if (PR.seed_kind == SEED_STRIDE)
                for (uint32_t i = tid; i < PR.stride_digits * kStrideRadix * 2u; i += BLOCK) s_skip[i] = PR.table[i];
            cur_problem = static_cast<int32_t>(U.problem);
        }
        __syncthreads();

        CellsLds<F32> C;
        C.edge = l_edge;
        C.sig = l_sig;
        C.rsig = l_rsig;
        C.scat = l_scat;
        C.bin = l_bin;
        C.tedge = l_tedge;
        C.n_cells = static_cast<int32_t>(PR.n_cells);
        C.n_time_bins = static_cast<int32_t>(PR.n_time_bins);
        C.n_space_bins = static_cast<int32_t>(PR.n_space_bins);
        SeedDev S;
        S.kind = static_cast<int>(PR.seed_kind);
        S.stride_digits = PR.stride_digits;
        S.base = PR.seed_base;
        S.first_index = PR.first_index;
        S.table = s_skip;
        uint64_t* tally = tally_all + static_cast<size_t>(copy) * P.max_slice * 2;
        const uint64_t stride_q = PR.stride_q;

        Particle<F32> p[H];
        int ph[H];
#pragma unroll
        for (int h = 0; h < H; ++h) ph[h] = PH_EMPTY;
        // wave-uniform counts of the unit (scalar registers)
        uint64_t w_events = 0, w_colls = 0;
        uint32_t w_ll = 0, w_lr = 0, w_abs = 0, w_cen = 0;
        // per lane, over the histories this lane ended (their total draws
        // follow from the wave counts: one for each history's first flight,
        // one per collision for the absorption test and two more per scatter)
        uint32_t l_maxd = 0, l_over = 0;
        bool exhausted = false;   // wave-uniform: no history of the unit left for this wave
        // the wave's ring of seeded histories (positions & 127): [r_next, r_filled)
        uint64_t* ring = s_ring[__builtin_amdgcn_readfirstlane(wid)];
        uint32_t r_next = 0, r_filled = 0;   // wave-uniform
        bool unit_taken = false;             // wave-uniform: s_next has passed the unit's end

        // Each iteration: one geometry step for every lane with a flight;
        // then, once enough lanes wait at a collision site (or stand empty
        // while histories remain), or none can move, the collision pass:
        // empty lanes take new histories, and every waiting particle runs its
        // collision draws and samples its next flight.  Every particle still
        // runs its own operations in its own order.
        for (;;) {
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const bool g = ph[h] == PH_GEOM;
                w_events += wave_count(g);
                int r = END_NONE;
                if (g) {
                    r = geom_step<F32, TIMED>(p[h], C, tally);
                    if (r == STEP_COLLIDE) {
                        ph[h] = PH_COLL;
                    } else if (r != END_NONE) {
                        ph[h] = PH_EMPTY;
                        const uint32_t d = p[h].hdraws;
                        l_maxd = d > l_maxd ? d : l_maxd;
                        if (stride_q != 0 && d > stride_q) l_over++;
                    }
                }
                if (__builtin_amdgcn_ballot_w64(r > END_NONE) != 0) {
                    w_ll += wave_count(r == END_LEAK_LEFT);
                    w_lr += wave_count(r == END_LEAK_RIGHT);
                    if (TIMED) w_cen += wave_count(r == END_CENSUS);
                }
            }
            uint32_t nwait = 0, ngeom = 0;
#pragma unroll
            for (int h = 0; h < H; ++h) {
                nwait += wave_count(ph[h] == PH_COLL || (ph[h] == PH_EMPTY && !exhausted));
                ngeom += wave_count(ph[h] == PH_GEOM);
            }
            if (nwait < P.coll_batch && ngeom != 0) continue;

            // collision pass: refill the empty lanes first
#pragma unroll
            for (int h = 0; h < H; ++h) {
                if (exhausted) continue;
                const uint64_t need = __builtin_amdgcn_ballot_w64(ph[h] == PH_EMPTY);
                if (need == 0) continue;
                const uint32_t nneed = static_cast<uint32_t>(__popcll(need));
                if (r_filled - r_next < nneed && !unit_taken) {
                    // seed the next 64 histories of the unit at once (one per
                    // lane), so that a refill is an LDS read
                    uint32_t base = 0;
                    if (lane == 0) base = atomicAdd(&s_next, 64u);
                    base = __builtin_amdgcn_readfirstlane(base);
                    if (base + 64u >= U.count) unit_taken = true;
                    const uint32_t got = base < U.count ? (U.count - base < 64u ? U.count - base : 64u) : 0u;
                    if (lane < got) ring[(r_filled + lane) & 127u] = stream_start(P.lcg, S, U.j0 + base + lane);
                    r_filled += got;
                    __builtin_amdgcn_wave_barrier();
                }
                const uint32_t avail = r_filled - r_next;
                const uint32_t take = avail < nneed ? avail : nneed;
                if (ph[h] == PH_EMPTY) {
                    const uint32_t rank = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(need >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(need), 0u));
                    if (rank < take) {
                        init_particle_at<F32, TIMED>(p[h], C, ring[(r_next + rank) & 127u]);
                        ph[h] = PH_NEW;
                    }
                }
                r_next += take;
                if (unit_taken && r_next == r_filled) exhausted = true;
                __builtin_amdgcn_wave_barrier();
            }
            uint32_t nlive = 0;
#pragma unroll
            for (int h = 0; h < H; ++h) nlive += wave_count(ph[h] != PH_EMPTY);
            if (nlive == 0) break;
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const bool cl = ph[h] == PH_COLL;
                w_colls += wave_count(cl);
                bool absorbed = false;
                if (cl) {
                    if (collide<F32>(p[h], C, P.lcg) != END_NONE) {
                        absorbed = true;
                        ph[h] = PH_EMPTY;
                        const uint32_t d = p[h].hdraws;
                        l_maxd = d > l_maxd ? d : l_maxd;
                        if (stride_q != 0 && d > stride_q) l_over++;
                    } else {
                        ph[h] = PH_NEW;
                    }
                }
                w_abs += wave_count(absorbed);
                if (ph[h] == PH_NEW) {
                    sample_tau<F32>(p[h], P.lcg);
                    ph[h] = PH_GEOM;
                }
            }
        }

        // unit diagnostics: the wave's counts and the lanes' into LDS
        if (lane == 0) {
            const unsigned long long ends = static_cast<unsigned long long>(w_ll) + w_lr + w_abs + w_cen;
            atomicAdd(&s_diag[D_HISTORIES], ends);
            atomicAdd(&s_diag[D_LEAK_LEFT], static_cast<unsigned long long>(w_ll));
            atomicAdd(&s_diag[D_LEAK_RIGHT], static_cast<unsigned long long>(w_lr));
            atomicAdd(&s_diag[D_ABSORBED], static_cast<unsigned long long>(w_abs));
            atomicAdd(&s_diag[D_CENSUS], static_cast<unsigned long long>(w_cen));
            atomicAdd(&s_diag[D_EVENTS], static_cast<unsigned long long>(w_events));
            atomicAdd(&s_diag[D_COLLISIONS], static_cast<unsigned long long>(w_colls));
            atomicAdd(&s_diag[D_DRAWS], ends + 3ull * w_colls - 2ull * w_abs);
        }
        atomicMax(&s_diag[D_MAX_DRAWS], static_cast<unsigned long long>(l_maxd));
        atomicAdd(&s_diag[D_OVER_STRIDE], static_cast<unsigned long long>(l_over));
        __syncthreads();

        uint64_t* dst = P.partial + U.slot;
        for (uint32_t i = tid; i < slice; i += BLOCK) {
            uint64_t lo = 0, hi = 0;
            for (uint32_t c = 0; c < P.tally_copies; ++c) {
                const uint64_t l = tally_all[(static_cast<size_t>(c) * P.max_slice + i) * 2];
                hi += tally_all[(static_cast<size_t>(c) * P.max_slice + i) * 2 + 1];
                if (lo + l < lo) hi += 1ull << 32;   // a wrap of the low word: 2^64 = 2^32 x 2^32
                lo += l;
            }
            dst[2 * i] = lo;
            dst[2 * i + 1] = hi;
        }
        if (tid < kNDiag) P.unit_diag[static_cast<size_t>(ui) * kNDiag + tid] = s_diag[tid];
        __syncthreads();
    }
}

// Chained units (a set of one problem, one history per lane).  In k_transport
// a block's lanes fall idle while the slowest histories of its unit finish
// (history lengths are heavy-tailed: the long-chain slab has a median of 23
// events and a longest of about 1750), and the block's next unit starts only
// after a barrier.  Here a block holds two units at once, each
// with its own LDS tally slice: once every history of the feeding unit has
// been handed out, the block takes its next unit into the other slice and
// the lanes go on without a pause.  A unit's slice is written to the unit's
// HBM slot by the wave that ends its last history, and the slice is then free
// for the block's next unit.  Each particle still runs its own operations in
// its own order and the counts are integer sums, so every output equals
// k_transport's.  The problem's diagnostics are summed over the block's
// units and written to the block's last unit (the per-unit words start at
// zero; the reduction sums a problem's units).
//
// Block state in LDS (only lane 0 of a wave touches it, with
// workgroup-scope atomics):
//   s_w     bit s (s = 0, 1): slice s holds a unit; kWant: the feeding unit
//           has been handed out and the block wants its next unit; kNoMore:
//           the launch's counter has passed its last unit
//   s_feed  (claim number << 1) | slice of the unit handed out now, or kNone
//   s_cs[s] the unit in slice s: first index, HBM slot, the histories not
//           yet ended, and the hand-out word (claim number, size, handed
//           out)
// Claims are serial: kWant is set once per unit, by the wave that hands out
// its last histories, and cleared by the compare-exchange that takes a free
// slice, so exactly one wave claims; that wave is the one that finds both
// conditions (kWant set, a slice free), whichever of the two came last.
// A wave with nothing to run waits only while no unit is being handed out
// and the counter is not exhausted: then kWant is set and both slices are
// busy (or a claim is under way), a busy slice's live histories run in other
// waves' lanes, the last of them frees the slice and that wave claims.  So
// every wave ends once the counter has passed the last unit and its own
// lanes and ring are empty.
namespace chain {
constexpr uint32_t kWant = 4u, kNoMore = 8u, kNone = 0xffffffffu;
// A slice's hand-out word: claim number (24 bits, mod 2^24) | the unit's
// histories (20 bits) | histories handed out (20 bits).  A wave takes
// histories by compare-exchange on the whole word, so a wave that read a
// stale feed word (its unit replaced in the meantime) fails the exchange and
// changes nothing, and a unit's size is read with the word, never from a
// field a new claim could have overwritten.
constexpr int kWordCount = 20, kWordGen = 40;
constexpr uint64_t kWordMask = (1ull << kWordCount) - 1ull;
static_assert(kMaxUnitHistories + 64u < (1u << kWordCount), "a unit's size and hand-out count fit their fields");
struct Slot {
    uint64_t j0;
    uint64_t hslot;
    uint64_t word;
    uint32_t alive;
    uint32_t pad;
};
}  // namespace chain

#define CH_ACQ_REL(op, p, v) __hip_atomic_##op((p), (v), __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP)

template <bool F32, bool TIMED, int BLOCK>
__global__ void __launch_bounds__(BLOCK, (F32 || !TIMED) ? 7 : 6) k_transport_chain(TransportParams P) {
    using R = typename Particle<F32>::R;
    using chain::kNone;
    using chain::kNoMore;
    using chain::kWant;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint64_t s_skip[kStrideDigits * kStrideRadix * 2];
    __shared__ uint64_t s_ring[BLOCK / 64][128];
    __shared__ uint8_t s_rslice[BLOCK / 64][128];   // the slice of each ring entry's unit
    __shared__ chain::Slot s_cs[2];
    __shared__ uint32_t s_w, s_feed, s_seq, s_last_ui;
    __shared__ unsigned long long s_diag[kNDiag];

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(tid >> 6);

    uint64_t* tally_all = reinterpret_cast<uint64_t*>(smem);
    size_t off = align16(static_cast<size_t>(P.tally_copies) * P.max_slice * 2 * sizeof(uint64_t));
    R* l_edge = reinterpret_cast<R*>(smem + off);
    off += align16((P.max_cells + 1) * sizeof(R));
    R* l_sig = reinterpret_cast<R*>(smem + off);
    off += align16(P.max_cells * sizeof(R));
    R* l_rsig = reinterpret_cast<R*>(smem + off);
    off += align16(P.max_cells * sizeof(R));
    double* l_scat = reinterpret_cast<double*>(smem + off);
    off += align16(P.max_cells * sizeof(double));
    int32_t* l_bin = reinterpret_cast<int32_t*>(smem + off);
    off += align16(P.max_cells * sizeof(int32_t));
    R* l_tedge = reinterpret_cast<R*>(smem + off);

    const R* g_edge;
    const R* g_sig;
    const R* g_tedge;
    if constexpr (F32) {
        g_edge = P.edges32;
        g_sig = P.sig32;
        g_tedge = P.tedges32;
    } else {
        g_edge = P.edges64;
        g_sig = P.sig64;
        g_tedge = P.tedges64;
    }

    const DevProblem PR = P.problems[0];
    const uint32_t slice = PR.slice_bins;
    uint64_t* const tsl0 = tally_all;
    uint64_t* const tsl1 = tally_all + static_cast<size_t>(P.max_slice) * 2;
    for (uint32_t i = tid; i <= PR.n_cells; i += BLOCK) l_edge[i] = g_edge[PR.edge_off + i];
    for (uint32_t i = tid; i < PR.n_cells; i += BLOCK) {
        const R sg = g_sig[PR.cell_off + i];
        l_sig[i] = sg;
        l_rsig[i] = recip_refined(sg);
        l_scat[i] = P.scat64[PR.cell_off + i];
        l_bin[i] = P.cbin[PR.cell_off + i];
    }
    if (TIMED)
        for (uint32_t i = tid; i <= PR.n_time_bins; i += BLOCK) l_tedge[i] = g_tedge[PR.tedge_off + i];
    if (PR.seed_kind == SEED_STRIDE)
        for (uint32_t i = tid; i < PR.stride_digits * kStrideRadix * 2u; i += BLOCK) s_skip[i] = PR.table[i];
    for (uint32_t i = tid; i < 2u * slice; i += BLOCK) {
        tsl0[i] = 0ull;
        tsl1[i] = 0ull;
    }
    if (tid < kNDiag) s_diag[tid] = 0;

    // lane 0 of a wave: puts the launch's next unit into free slice f
    auto take_unit = [&](uint32_t f) {
        const uint32_t pos = atomicAdd(P.unit_counter, 1u);
        if (pos >= P.n_units) {
            CH_ACQ_REL(fetch_or, &s_w, kNoMore);
            CH_ACQ_REL(fetch_and, &s_w, ~(1u << f));
            return;
        }
        const uint32_t ui = P.order[pos];
        const WorkUnit U = P.units[ui];
        const uint32_t seq = s_seq + 1u;
        s_seq = seq;
        s_last_ui = ui;
        s_cs[f].j0 = U.j0;
        s_cs[f].hslot = U.slot;
        s_cs[f].alive = U.count;
        __hip_atomic_store(&s_cs[f].word,
                           (static_cast<uint64_t>(seq & 0xffffffu) << chain::kWordGen) |
                               (static_cast<uint64_t>(U.count) << chain::kWordCount),
                           __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_store(&s_feed, (seq << 1) | f, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    // lane 0 of a wave: claims a free slice if the block wants a unit
    auto try_claim = [&]() {
        uint32_t old = __hip_atomic_load(&s_w, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
        for (;;) {
            if (!(old & kWant) || (old & kNoMore)) return;
            const int f = !(old & 1u) ? 0 : (!(old & 2u) ? 1 : -1);
            if (f < 0) return;
            if (__hip_atomic_compare_exchange_strong(&s_w, &old, (old & ~kWant) | (1u << f), __ATOMIC_ACQ_REL,
                                                     __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) {
                take_unit(static_cast<uint32_t>(f));
                return;
            }
        }
    };
    if (tid == 0) {
        s_w = 1u;
        s_seq = 0;
        s_last_ui = kNone;
        s_feed = kNone;
        take_unit(0);
    }
    __syncthreads();

    CellsLds<F32> C;
    C.edge = l_edge;
    C.sig = l_sig;
    C.rsig = l_rsig;
    C.scat = l_scat;
    C.bin = l_bin;
    C.tedge = l_tedge;
    C.n_cells = static_cast<int32_t>(PR.n_cells);
    C.n_time_bins = static_cast<int32_t>(PR.n_time_bins);
    C.n_space_bins = static_cast<int32_t>(PR.n_space_bins);
    SeedDev S;
    S.kind = static_cast<int>(PR.seed_kind);
    S.stride_digits = PR.stride_digits;
    S.base = PR.seed_base;
    S.first_index = PR.first_index;
    S.table = s_skip;
    const uint64_t stride_q = PR.stride_q;
    uint64_t* const ring = s_ring[wid];
    uint8_t* const rsl = s_rslice[wid];

    // The lanes in `ended` have ended their histories.  A wave counts its
    // ended histories per slice and subtracts them from the unit's live
    // count once none of its lanes runs a history of that slice (so about
    // once per unit and wave, not at every end); the wave whose subtraction
    // reaches zero writes the unit's slice to HBM, clears it and frees it.
    uint64_t live = 0;     // wave-uniform: lanes running a history
    uint64_t s1mask = 0;   // wave-uniform: lanes whose history is in slice 1
    uint32_t acc0 = 0, acc1 = 0;
    auto report = [&](uint32_t sl, uint32_t n) {
        uint32_t old = 0;
        if (lane == 0) old = CH_ACQ_REL(fetch_sub, &s_cs[sl].alive, n);
        old = __builtin_amdgcn_readfirstlane(old);
        if (old != n) return;
        uint64_t* t = sl ? tsl1 : tsl0;
        uint64_t* dst = P.partial + s_cs[sl].hslot;
        for (uint32_t i = lane; i < 2u * slice; i += 64u) {
            dst[i] = t[i];
            t[i] = 0ull;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (lane == 0) {
            CH_ACQ_REL(fetch_and, &s_w, ~(1u << sl));
            try_claim();
        }
        __builtin_amdgcn_wave_barrier();
    };
    auto ends = [&](uint64_t ended) {
        const uint32_t e1 = static_cast<uint32_t>(__popcll(ended & s1mask));
        acc1 += e1;
        acc0 += static_cast<uint32_t>(__popcll(ended)) - e1;
        live &= ~ended;
        s1mask &= ~ended;
        if (acc0 != 0 && (live & ~s1mask) == 0) {
            report(0, acc0);
            acc0 = 0;
        }
        if (acc1 != 0 && (live & s1mask) == 0) {
            report(1, acc1);
            acc1 = 0;
        }
    };
    // seeds up to 64 histories of the feeding unit into the ring; returns
    // false when no unit is feeding or it has been handed out
    uint32_t r_next = 0, r_filled = 0;   // wave-uniform: the ring holds [r_next, r_filled)
    auto fetch = [&]() -> bool {
        // lane 0: takes up to 64 histories of the feeding unit, if it has any left
        uint32_t fd = kNone, base = 0, cnt = 0;
        if (lane == 0) {
            fd = __hip_atomic_load(&s_feed, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (fd != kNone) {
                uint64_t* w = &s_cs[fd & 1u].word;
                const uint64_t gen = (fd >> 1) & 0xffffffu;
                uint64_t cur = __hip_atomic_load(w, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
                for (;;) {
                    const uint32_t c = static_cast<uint32_t>(cur >> chain::kWordCount) & chain::kWordMask;
                    const uint32_t h = static_cast<uint32_t>(cur) & chain::kWordMask;
                    if ((cur >> chain::kWordGen) != gen || h >= c) {   // replaced, or handed out
                        fd = kNone;
                        break;
                    }
                    if (__hip_atomic_compare_exchange_strong(w, &cur, cur + 64u, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE,
                                                             __HIP_MEMORY_SCOPE_WORKGROUP)) {
                        base = h;
                        cnt = c;
                        break;
                    }
                }
            }
        }
        fd = __builtin_amdgcn_readfirstlane(fd);
        if (fd == kNone) return false;
        const uint32_t f = fd & 1u;
        base = __builtin_amdgcn_readfirstlane(base);
        cnt = __builtin_amdgcn_readfirstlane(cnt);
        const uint32_t got = cnt - base < 64u ? cnt - base : 64u;
        if (lane < got) {
            ring[(r_filled + lane) & 127u] = stream_start(P.lcg, S, s_cs[f].j0 + base + lane);
            rsl[(r_filled + lane) & 127u] = static_cast<uint8_t>(f);
        }
        r_filled += got;
        if (base + 64u >= cnt && lane == 0) {
            // this wave took the unit's last histories
            __hip_atomic_store(&s_feed, kNone, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            CH_ACQ_REL(fetch_or, &s_w, kWant);
            try_claim();
        }
        __builtin_amdgcn_wave_barrier();
        return true;
    };

    Particle<F32> p;
    int ph = PH_EMPTY;
    uint64_t* tl = tsl0;   // the slice of the lane's history
    uint64_t w_events = 0, w_colls = 0;
    uint32_t w_ll = 0, w_lr = 0, w_abs = 0, w_cen = 0;
    uint32_t l_maxd = 0, l_over = 0;
    bool starved = false;   // wave-uniform: the last refill found no history to take

    for (;;) {
        {
            const bool g = ph == PH_GEOM;
            w_events += wave_count(g);
            int r = END_NONE;
            if (g) {
                r = geom_step<F32, TIMED>(p, C, tl);
                if (r == STEP_COLLIDE) {
                    ph = PH_COLL;
                } else if (r != END_NONE) {
                    ph = PH_EMPTY;
                    const uint32_t d = p.hdraws;
                    l_maxd = d > l_maxd ? d : l_maxd;
                    if (stride_q != 0 && d > stride_q) l_over++;
                }
            }
            const uint64_t ended = __builtin_amdgcn_ballot_w64(r > END_NONE);
            if (ended != 0) {
                w_ll += wave_count(r == END_LEAK_LEFT);
                w_lr += wave_count(r == END_LEAK_RIGHT);
                if (TIMED) w_cen += wave_count(r == END_CENSUS);
                ends(ended);
            }
        }
        const uint32_t nwait = wave_count(ph == PH_COLL || (ph == PH_EMPTY && !starved));
        const uint32_t ngeom = wave_count(ph == PH_GEOM);
        if (nwait < P.coll_batch && ngeom != 0) continue;

        // collision pass: refill the empty lanes first
        const uint64_t need = __builtin_amdgcn_ballot_w64(ph == PH_EMPTY);
        if (need != 0) {
            const uint32_t nneed = static_cast<uint32_t>(__popcll(need));
            starved = false;
            while (r_filled - r_next < nneed) {
                if (!fetch()) {
                    starved = true;
                    break;
                }
            }
            const uint32_t avail = r_filled - r_next;
            const uint32_t take = avail < nneed ? avail : nneed;
            bool in1 = false;
            if (ph == PH_EMPTY) {
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(need >> 32),
                                                                __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(need), 0u));
                if (rank < take) {
                    const uint32_t e = (r_next + rank) & 127u;
                    init_particle_at<F32, TIMED>(p, C, ring[e]);
                    in1 = rsl[e] != 0;
                    tl = in1 ? tsl1 : tsl0;
                    ph = PH_NEW;
                }
            }
            s1mask |= __builtin_amdgcn_ballot_w64(in1);
            live = __builtin_amdgcn_ballot_w64(ph != PH_EMPTY);
            r_next += take;
            __builtin_amdgcn_wave_barrier();
        }
        if (live == 0) {
            // nothing to run: done once the launch has no unit left, else
            // wait for a unit (another wave frees a slice or is claiming)
            uint32_t w = 0;
            if (lane == 0) w = __hip_atomic_load(&s_w, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
            w = __builtin_amdgcn_readfirstlane(w);
            if ((w & kNoMore) && r_next == r_filled) break;
            __builtin_amdgcn_s_sleep(4);
        }
        {
            const bool cl = ph == PH_COLL;
            w_colls += wave_count(cl);
            bool absorbed = false;
            if (cl) {
                if (collide<F32>(p, C, P.lcg) != END_NONE) {
                    absorbed = true;
                    ph = PH_EMPTY;
                    const uint32_t d = p.hdraws;
                    l_maxd = d > l_maxd ? d : l_maxd;
                    if (stride_q != 0 && d > stride_q) l_over++;
                } else {
                    ph = PH_NEW;
                }
            }
            const uint64_t ab = __builtin_amdgcn_ballot_w64(absorbed);
            if (ab != 0) {
                w_abs += static_cast<uint32_t>(__popcll(ab));
                ends(ab);
            }
            if (ph == PH_NEW) {
                sample_tau<F32>(p, P.lcg);
                ph = PH_GEOM;
            }
        }
    }

    // the problem's diagnostics: the block's sums, into its last unit's words
    if (lane == 0) {
        const unsigned long long nend = static_cast<unsigned long long>(w_ll) + w_lr + w_abs + w_cen;
        atomicAdd(&s_diag[D_HISTORIES], nend);
        atomicAdd(&s_diag[D_LEAK_LEFT], static_cast<unsigned long long>(w_ll));
        atomicAdd(&s_diag[D_LEAK_RIGHT], static_cast<unsigned long long>(w_lr));
        atomicAdd(&s_diag[D_ABSORBED], static_cast<unsigned long long>(w_abs));
        atomicAdd(&s_diag[D_CENSUS], static_cast<unsigned long long>(w_cen));
        atomicAdd(&s_diag[D_EVENTS], static_cast<unsigned long long>(w_events));
        atomicAdd(&s_diag[D_COLLISIONS], static_cast<unsigned long long>(w_colls));
        atomicAdd(&s_diag[D_DRAWS], nend + 3ull * w_colls - 2ull * w_abs);
    }
    atomicMax(&s_diag[D_MAX_DRAWS], static_cast<unsigned long long>(l_maxd));
    atomicAdd(&s_diag[D_OVER_STRIDE], static_cast<unsigned long long>(l_over));
    __syncthreads();
    if (tid < kNDiag && s_last_ui != kNone) P.unit_diag[static_cast<size_t>(s_last_ui) * kNDiag + tid] = s_diag[tid];
}
#undef CH_ACQ_REL

template <bool F32, bool TIMED, int H, int BLOCK>
static hipError_t launch_t(const TransportParams& p, int grid, size_t lds, hipStream_t st, int* used) {
    auto kern = k_transport<F32, TIMED, H, BLOCK>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    if (grid <= 0) {
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), BLOCK, lds);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
        grid = cus * per_cu;
    }
    if (static_cast<uint32_t>(grid) > p.n_units) grid = static_cast<int>(p.n_units);
    if (grid < 1) grid = 1;
    if (used) *used = grid;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(BLOCK), lds, st, p);
    return hipGetLastError();
}

template <bool F32, bool TIMED, int H>
static hipError_t launch_b(const TransportParams& p, int block, int grid, size_t lds, hipStream_t st, int* used) {
    switch (block) {
        case 64: return launch_t<F32, TIMED, H, 64>(p, grid, lds, st, used);
        case 128: return launch_t<F32, TIMED, H, 128>(p, grid, lds, st, used);
        case 512: return launch_t<F32, TIMED, H, 512>(p, grid, lds, st, used);
        case 1024: return launch_t<F32, TIMED, H, 1024>(p, grid, lds, st, used);
        default: return launch_t<F32, TIMED, H, 256>(p, grid, lds, st, used);
    }
}

template <bool F32, bool TIMED>
static hipError_t launch_h(const TransportParams& p, const LaunchShape& s, size_t lds, hipStream_t st, int* used) {
    switch (s.hist_per_lane) {
        case 2: return launch_b<F32, TIMED, 2>(p, s.block, s.grid, lds, st, used);
        case 4: return launch_b<F32, TIMED, 4>(p, s.block, s.grid, lds, st, used);
        default: return launch_b<F32, TIMED, 1>(p, s.block, s.grid, lds, st, used);
    }
}

// Blocks of `kern` that fit on one CU with `lds` bytes of dynamic LDS.
static hipError_t blocks_per_cu(const void* kern, int block, size_t lds, int* out) {
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, kern, block, lds);
}

template <bool F32, bool TIMED, int BLOCK>
static hipError_t launch_chain_t(const TransportParams& p, int grid, size_t lds, hipStream_t st, int* used) {
    auto kern = k_transport_chain<F32, TIMED, BLOCK>;
    if (grid <= 0) {
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        e = blocks_per_cu(reinterpret_cast<const void*>(kern), BLOCK, lds, &per_cu);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
        grid = cus * per_cu;
    } else if (lds > 64 * 1024) {
        int per_cu = 0;
        hipError_t e = blocks_per_cu(reinterpret_cast<const void*>(kern), BLOCK, lds, &per_cu);
        if (e != hipSuccess) return e;
    }
    if (static_cast<uint32_t>(grid) > p.n_units) grid = static_cast<int>(p.n_units);
    if (grid < 1) grid = 1;
    if (used) *used = grid;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(BLOCK), lds, st, p);
    return hipGetLastError();
}

template <bool F32, bool TIMED>
static hipError_t launch_chain_b(const TransportParams& p, const LaunchShape& s, size_t lds, hipStream_t st,
                                 int* used) {
    switch (s.block) {
        case 64: return launch_chain_t<F32, TIMED, 64>(p, s.grid, lds, st, used);
        case 128: return launch_chain_t<F32, TIMED, 128>(p, s.grid, lds, st, used);
        case 512: return launch_chain_t<F32, TIMED, 512>(p, s.grid, lds, st, used);
        case 1024: return launch_chain_t<F32, TIMED, 1024>(p, s.grid, lds, st, used);
        default: return launch_chain_t<F32, TIMED, 256>(p, s.grid, lds, st, used);
    }
}

template <bool F32, bool TIMED, int BLOCK>
static hipError_t chain_fits_t(const TransportParams& a, const TransportParams& b, int f32, bool* fits) {
    int na = 0, nb = 0;
    hipError_t e = blocks_per_cu(reinterpret_cast<const void*>(k_transport<F32, TIMED, 1, BLOCK>), BLOCK,
                                 transport_lds_bytes(a, f32), &na);
    if (e != hipSuccess) return e;
    e = blocks_per_cu(reinterpret_cast<const void*>(k_transport_chain<F32, TIMED, BLOCK>), BLOCK,
                      transport_lds_bytes(b, f32), &nb);
    if (e != hipSuccess) return e;
    *fits = nb >= 1 && nb >= na;
    return hipSuccess;
}

template <bool F32, bool TIMED>
static hipError_t chain_fits_b(const TransportParams& a, const TransportParams& b, const LaunchShape& s, bool* fits) {
    switch (s.block) {
        case 64: return chain_fits_t<F32, TIMED, 64>(a, b, s.f32, fits);
        case 128: return chain_fits_t<F32, TIMED, 128>(a, b, s.f32, fits);
        case 512: return chain_fits_t<F32, TIMED, 512>(a, b, s.f32, fits);
        case 1024: return chain_fits_t<F32, TIMED, 1024>(a, b, s.f32, fits);
        default: return chain_fits_t<F32, TIMED, 256>(a, b, s.f32, fits);
    }
}

hipError_t transport_chain_fits(const TransportParams& single, const TransportParams& chained, const LaunchShape& s,
                                bool* fits) {
    *fits = false;
    if (s.f32)
        return s.timed ? chain_fits_b<true, true>(single, chained, s, fits)
                       : chain_fits_b<true, false>(single, chained, s, fits);
    return s.timed ? chain_fits_b<false, true>(single, chained, s, fits)
                   : chain_fits_b<false, false>(single, chained, s, fits);
}

hipError_t launch_transport(const TransportParams& p, const LaunchShape& s, hipStream_t st, int* grid_used) {
    if (p.n_units == 0) return hipSuccess;
    const size_t lds = transport_lds_bytes(p, s.f32);
    if (s.chain) {
        if (s.f32)
            return s.timed ? launch_chain_b<true, true>(p, s, lds, st, grid_used)
                           : launch_chain_b<true, false>(p, s, lds, st, grid_used);
        return s.timed ? launch_chain_b<false, true>(p, s, lds, st, grid_used)
                       : launch_chain_b<false, false>(p, s, lds, st, grid_used);
    }
    if (s.f32) {
        return s.timed ? launch_h<true, true>(p, s, lds, st, grid_used)
                       : launch_h<true, false>(p, s, lds, st, grid_used);
    }
    return s.timed ? launch_h<false, true>(p, s, lds, st, grid_used)
                   : launch_h<false, false>(p, s, lds, st, grid_used);
}

// ------------------------------------------------------------------ reduction

// Round-half-even conversion of the 128-bit integer (hi, lo) to double:
// keep the top 53 bits, round on the dropped bits, scale back exactly.
__device__ __forceinline__ double u128_to_double(uint64_t lo, uint64_t hi) {
    typedef unsigned __int128 u128;
    const u128 v = (static_cast<u128>(hi) << 64) | lo;
    if ((v >> 53) == 0) return static_cast<double>(lo);
    const int nbits = (hi != 0) ? 128 - __clzll(static_cast<long long>(hi)) : 64 - __clzll(static_cast<long long>(lo));
    const int sh = nbits - 53;
    u128 mant = v >> sh;
    const u128 rem = v - (mant << sh);
    const u128 half = static_cast<u128>(1) << (sh - 1);
    if (rem > half || (rem == half && (mant & 1))) mant += 1;
    return __builtin_ldexp(static_cast<double>(static_cast<uint64_t>(mant)), sh);
}

// Block = (group, tile of 32 bins); 8 unit lanes per bin.  A group's units
// are consecutive with consecutive partial slots (2 x slice_bins words each),
// so unit u's words for bin i sit at slot0 + (u - u0) 2 slice + 2 i.  Unit
// lane l sums units u0 + l, u0 + l + 8, ...; the 8 partial sums are then
// added in lane order (integers: any order gives the same bits).
constexpr int kRedBins = 32, kRedLanes = 8;

__global__ void __launch_bounds__(256) k_reduce_bins(ReduceParams P) {
    typedef unsigned __int128 u128;
    __shared__ uint64_t part[kRedLanes][kRedBins][2];
    const ReduceGroup G = P.groups[blockIdx.y];
    const uint32_t bl = threadIdx.x % kRedBins, ul = threadIdx.x / kRedBins;
    const uint32_t i = blockIdx.x * kRedBins + bl;
    u128 acc = 0;
    if (i < G.slice_bins && G.unit_end > G.unit_begin) {
        const uint64_t slot0 = P.units[G.unit_begin].slot;
        const uint64_t stride = 2ull * G.slice_bins;
        for (uint32_t u = ul; u < G.unit_end - G.unit_begin; u += kRedLanes) {
            const uint64_t* s = P.partial + slot0 + u * stride + 2ull * i;
            acc += static_cast<u128>(s[0]);
            acc += static_cast<u128>(s[1]) << 32;
        }
    }
    part[ul][bl][0] = static_cast<uint64_t>(acc);
    part[ul][bl][1] = static_cast<uint64_t>(acc >> 64);
    __syncthreads();
    if (ul != 0 || i >= G.slice_bins) return;
    u128 tot = 0;
#pragma unroll
    for (int l = 0; l < kRedLanes; ++l)
        tot += (static_cast<u128>(part[l][bl][1]) << 64) | part[l][bl][0];
    const uint64_t lo = static_cast<uint64_t>(tot), hi = static_cast<uint64_t>(tot >> 64);
    const uint64_t o = G.out_off + i;
    P.raw[2 * o] = lo;
    P.raw[2 * o + 1] = hi;
    const uint32_t sb = i % G.n_space_bins;
    const uint32_t tb = i / G.n_space_bins;
    const double r = u128_to_double(lo, hi) * 0x1p-56;
    double d = static_cast<double>(G.n_hist) * P.dx[G.dx_off + sb];
    if (G.n_time_bins > 0) d = d * P.dt[G.dt_off + tb];
    P.flux[o] = (d != 0.0) ? r / d : 0.0;
}

__global__ void __launch_bounds__(256) k_reduce_diag(ReduceParams P) {
    const uint32_t pb = blockIdx.x;
    __shared__ unsigned long long acc[kNDiag];
    if (threadIdx.x < kNDiag) acc[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t u0 = P.pu_begin[pb], u1 = P.pu_begin[pb + 1];
    unsigned long long loc[kNDiag];
#pragma unroll
    for (int k = 0; k < kNDiag; ++k) loc[k] = 0;
    for (uint32_t u = u0 + threadIdx.x; u < u1; u += blockDim.x) {
#pragma unroll
        for (int k = 0; k < kNDiag; ++k) {
            const unsigned long long v = P.unit_diag[static_cast<size_t>(u) * kNDiag + k];
            if (k == D_MAX_DRAWS)
                loc[k] = v > loc[k] ? v : loc[k];
            else
                loc[k] += v;
        }
    }
#pragma unroll
    for (int k = 0; k < kNDiag; ++k) {
        if (k == D_MAX_DRAWS)
            atomicMax(&acc[k], loc[k]);
        else
            atomicAdd(&acc[k], loc[k]);
    }
    __syncthreads();
    if (threadIdx.x < kNDiag) P.diag[static_cast<size_t>(pb) * kNDiag + threadIdx.x] = acc[threadIdx.x];
}

hipError_t launch_reduce(const ReduceParams& p, hipStream_t st) {
    if (p.n_groups > 0) {
        uint32_t bx = (p.max_slice + kRedBins - 1) / kRedBins;
        if (bx < 1) bx = 1;
        hipLaunchKernelGGL(k_reduce_bins, dim3(bx, p.n_groups), dim3(kRedBins * kRedLanes), 0, st, p);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (p.diag != nullptr && p.n_problems > 0) {
        hipLaunchKernelGGL(k_reduce_diag, dim3(p.n_problems), dim3(256), 0, st, p);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace mcrng
