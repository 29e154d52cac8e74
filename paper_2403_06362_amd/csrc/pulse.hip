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
// Two schedules:
//   k_pulse_bank (hash only)  one launch per generation: every particle of
//       the input bank (or every source) runs one flight; the particles
//       emerging from it are appended to the output bank through one atomic
//       per wave (wave prefix sum of the per-lane counts).  Output capacity
//       is n_max per input particle, so no append can overflow.
//   k_pulse_family            one source family per lane (taken from a
//       global counter, one atomic per wave), walked depth first with a
//       per-lane stack in HBM; a stack entry holds the siblings still to
//       start of one scattering (stride: a count; hash: X_p and the next
//       key), so the depth is at most the number of scatterings on the
//       current line of descent.
// Counts are 64-bit integer atomics, so every schedule, launch shape and
// order gives the same counts.
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
};

// Runs the particle from its start to its end.  Returns the number of
// particles emerging from it (0 unless it scattered); p then holds the
// collision site and the state after the particle's draws.  *draws counts
// the numbers drawn.
__device__ __forceinline__ uint32_t pulse_particle(const PulseParams& P, PParticle& p, PulseLane& c,
                                                   uint32_t* draws) {
    const LcgDev& L = P.lcg;
    p.X = lcg_next(L, p.X);
    const double mu = 2.0 * to_uniform(L, p.X) - 1.0;
    p.X = lcg_next(L, p.X);
    const double tau = -fixed_log(to_uniform(L, p.X));
    *draws += 2;
    const double s = tau / P.sigma_t;
    const double tn = p.t + s;
    if (!(tn < P.t_end)) {
        c.census++;
        return 0;
    }
    const double step = mu * s;
    p.x = p.x + step;
    p.t = tn;
    while (p.tb + 1 < static_cast<int32_t>(P.n_time_bins) && P.t_edges[p.tb + 1] <= p.t) p.tb++;
    c.collisions++;
    if (p.tb >= 0 && P.x_lo <= p.x && p.x <= P.x_hi) {
        atomicAdd(reinterpret_cast<unsigned long long*>(P.counts) +
                      static_cast<size_t>(p.batch) * P.n_time_bins + p.tb,
                  1ull);
        c.tallied++;
    }
    p.X = lcg_next(L, p.X);
    *draws += 1;
    if (!(to_uniform(L, p.X) < P.scatter)) {
        c.absorbed++;
        return 0;
    }
    p.X = lcg_next(L, p.X);
    *draws += 1;
    const uint32_t n = P.n_floor + (to_uniform(L, p.X) < P.nu_frac ? 1u : 0u);
    c.scatters++;
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

// ------------------------------------------------------------ bank schedule

template <bool SOURCES, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_pulse_bank(PulseParams P) {
    PulseLane c;
    const uint64_t n_items = SOURCES ? P.src_end - P.src_begin : P.n_in;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * BLOCK;
    const uint32_t lane = threadIdx.x & 63u;
    // every lane of a wave runs the same number of rounds (the ballots below need the whole wave)
    const uint64_t first = static_cast<uint64_t>(blockIdx.x) * BLOCK + (threadIdx.x & ~63u);
    for (uint64_t base = first; base < n_items; base += stride) {
        const uint64_t item = base + lane;
        uint32_t n = 0;
        PParticle p;
        if (item < n_items) {
            if (SOURCES) {
                p.X = pulse_source_state(P, P.src_begin + item, &p.batch);
                p.x = 0.0;
                p.t = 0.0;
                p.tb = P.tb0;
                c.sources++;
            } else {
                p.x = P.in.x[item];
                p.t = P.in.t[item];
                p.X = P.in.X[item];
                p.batch = P.in.batch[item];
                p.tb = P.in.tb[item];
            }
            uint32_t draws = 0;
            n = pulse_particle(P, p, c, &draws);
            note_stream(P, c, draws);
        }
        // wave prefix sum of n (n < 16) from one ballot per bit
        uint32_t off = 0, total = 0;
#pragma unroll
        for (int bit = 0; bit < 4; ++bit) {
            const uint64_t m = __ballot((n >> bit) & 1u);
            off += lane_prefix(m) << bit;
            total += static_cast<uint32_t>(__popcll(m)) << bit;
        }
        uint64_t wbase = 0;
        if (total != 0) {
            if (lane == 0) wbase = atomicAdd(reinterpret_cast<unsigned long long*>(P.out_count), total);
            wbase = __shfl(wbase, 0);
        }
        for (uint32_t k = 1; k <= n; ++k) {
            const uint64_t o = wbase + off + (k - 1);
            if (o < P.out_cap) {
                P.out.x[o] = p.x;
                P.out.t[o] = p.t;
                P.out.X[o] = murmur_hash(k, p.X) & P.lcg.mask;
                P.out.batch[o] = p.batch;
                P.out.tb[o] = p.tb;
            } else {
                atomicOr(P.overflow, 1u);
            }
        }
    }
    flush_lane_counters<BLOCK>(P, c);
}

// ------------------------------------------------------------ family schedule

template <bool HASH, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_pulse_family(PulseParams P) {
    PulseLane c;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t gl = static_cast<uint64_t>(blockIdx.x) * BLOCK + threadIdx.x;
    PulseStackEntry* stack = P.stack + gl * P.stack_depth;
    uint32_t sp = 0;
    const uint64_t n_sources = P.src_end - P.src_begin;

    PParticle p;
    p.x = p.t = 0.0;
    p.X = 0;
    p.tb = -1;
    p.batch = 0;
    bool active = false;       // the lane holds a particle of a family
    bool exhausted = false;    // wave-uniform: no sources left
    uint32_t pdraws = 0;       // draws of the current stream (hash: particle; stride: family)

    for (;;) {
        // lanes without a family take the next sources (one atomic per wave)
        const uint64_t need = __ballot(!active);
        if (need != 0 && !exhausted) {
            const uint32_t cnt = static_cast<uint32_t>(__popcll(need));
            uint64_t wbase = 0;
            if (lane == 0) wbase = atomicAdd(reinterpret_cast<unsigned long long*>(P.family_counter), cnt);
            wbase = __shfl(wbase, 0);
            if (wbase + cnt >= n_sources) exhausted = true;
            if (!active) {
                const uint64_t j = wbase + lane_prefix(need);
                if (j < n_sources) {
                    p.X = pulse_source_state(P, P.src_begin + j, &p.batch);
                    p.x = 0.0;
                    p.t = 0.0;
                    p.tb = P.tb0;
                    pdraws = 0;
                    sp = 0;
                    c.sources++;
                    active = true;
                }
            }
        }
        if (__ballot(active) == 0) break;
        if (!active) continue;
        uint32_t n = pulse_particle(P, p, c, &pdraws);
        if (HASH) {
            // the particle's own stream ends here
            note_stream(P, c, pdraws);
            pdraws = 0;
        }
        if (n > 0) {
            if (n > 1) {
                if (sp == P.stack_depth) {
                    atomicOr(P.overflow, 1u);
                    active = false;   // the family is abandoned; the run reports an error
                    continue;
                }
                PulseStackEntry& e = stack[sp++];
                e.x = p.x;
                e.t = p.t;
                e.key = p.X;
                e.tb = p.tb;
                e.next = 2;
                e.n = n;
            }
            if (HASH) p.X = murmur_hash(1ull, p.X) & P.lcg.mask;
            continue;   // the first emerging particle starts at once
        }
        if (sp == 0) {
            if (!HASH) note_stream(P, c, pdraws);
            active = false;
            continue;
        }
        PulseStackEntry& e = stack[sp - 1];
        p.x = e.x;
        p.t = e.t;
        p.tb = e.tb;
        if (HASH) p.X = murmur_hash(e.next, e.key) & P.lcg.mask;
        if (e.next == e.n)
            --sp;
        else
            e.next++;
    }
    flush_lane_counters<BLOCK>(P, c);
}

// ------------------------------------------------------------ flux

__global__ void __launch_bounds__(256) k_pulse_flux(PulseParams P, double* flux) {
    const uint64_t n = static_cast<uint64_t>(P.n_batches) * P.n_time_bins;
    const double dx = P.x_hi - P.x_lo;
    const double nb = static_cast<double>(P.per_batch);
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * 256) {
        const uint32_t k = static_cast<uint32_t>(i % P.n_time_bins);
        const double dt = P.t_edges[k + 1] - P.t_edges[k];
        const double den = ((P.sigma_t * nb) * dx) * dt;
        flux[i] = static_cast<double>(P.counts[i]) / den;
    }
}

// ------------------------------------------------------------ launchers

static int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
    return cus > 0 ? cus : 256;
}

template <bool SOURCES, int BLOCK>
static hipError_t launch_bank_b(const PulseParams& p, uint64_t items, hipStream_t st) {
    uint64_t blocks = (items + BLOCK - 1) / BLOCK;
    const uint64_t cap = static_cast<uint64_t>(device_cus()) * (2048 / BLOCK) * 2;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((k_pulse_bank<SOURCES, BLOCK>), dim3(static_cast<unsigned>(blocks)), dim3(BLOCK), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_pulse_bank(const PulseParams& p, bool sources, int block, hipStream_t st) {
    const uint64_t items = sources ? p.src_end - p.src_begin : p.n_in;
    if (items == 0) return hipSuccess;
    switch (block) {
        case 64: return sources ? launch_bank_b<true, 64>(p, items, st) : launch_bank_b<false, 64>(p, items, st);
        case 128: return sources ? launch_bank_b<true, 128>(p, items, st) : launch_bank_b<false, 128>(p, items, st);
        case 512: return sources ? launch_bank_b<true, 512>(p, items, st) : launch_bank_b<false, 512>(p, items, st);
        case 1024: return sources ? launch_bank_b<true, 1024>(p, items, st) : launch_bank_b<false, 1024>(p, items, st);
        default: return sources ? launch_bank_b<true, 256>(p, items, st) : launch_bank_b<false, 256>(p, items, st);
    }
}

template <bool HASH, int BLOCK>
static hipError_t launch_family_b(const PulseParams& p, uint32_t grid, hipStream_t st) {
    hipLaunchKernelGGL((k_pulse_family<HASH, BLOCK>), dim3(grid), dim3(BLOCK), 0, st, p);
    return hipGetLastError();
}

uint32_t pulse_family_grid(int block) {
    // persistent lanes: 2048 per CU (the stack buffer is sized from this)
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
