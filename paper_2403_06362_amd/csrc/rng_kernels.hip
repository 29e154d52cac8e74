// Stream seeding and LCG draw kernels for gfx950.
//
// k_init_streams: one stream per lane, grid-stride; writes S_i.
// k_draw: persistent waves, one active stream per lane, refilled from a
//   per-wave queue of pre-seeded streams (see the kernel).  The state, sum and
//   remaining count never leave registers; HBM sees 4 bytes of count in and
//   8 bytes of checksum (+ 8 of state) out per stream.
#include "internal.hpp"

namespace mcrng {

// The k-step map of stride seeding, A_{Qk} = x -> G x + C, composed from
// the skip table's entries for the base-16 digits of k.
__device__ __forceinline__ void stride_map(const SeedDev& S, uint64_t k, uint64_t* G, uint64_t* C) {
    uint64_t g = 1, c = 0;
    for (uint32_t d = 0; d < kStrideDigits && (k >> (kStrideRadixBits * d)) != 0; ++d) {
        const uint32_t v = static_cast<uint32_t>(k >> (kStrideRadixBits * d)) & (kStrideRadix - 1);
        const uint64_t* e = S.table + 2 * (d * kStrideRadix + v);
        c = e[0] * c + e[1];
        g = e[0] * g;
    }
    *G = g;
    *C = c;
}

// Stride seeding (256-thread blocks): thread t of block b writes the streams
// i = b 256 + t + j stride; from the block's first stream X_{Q b 256} (one
// digit walk) the thread applies A_{Q t} (two table entries), and moves the
// block base on by A_{Q stride} for the next i.  Same states as
// stream_start, one affine step per stream.
__global__ void __launch_bounds__(256) k_init_streams(LcgDev L, SeedDev S, uint64_t n, uint64_t* out) {
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * 256;
    const uint64_t b0 = static_cast<uint64_t>(blockIdx.x) * 256;
    if (S.kind == SEED_STRIDE) {
        if (b0 >= n) return;
        const uint64_t* a = S.table + 2 * (threadIdx.x & (kStrideRadix - 1));
        const uint64_t* b = S.table + 2 * (kStrideRadix + (threadIdx.x >> kStrideRadixBits));
        const uint64_t lg = a[0] * b[0], lc = a[0] * b[1] + a[1];
        uint64_t jg = 0, jc = 0;
        stride_map(S, stride, &jg, &jc);
        uint64_t base = stream_start(L, S, b0);
        for (uint64_t i = b0 + threadIdx.x; i < n; i += stride) {
            out[i] = affine_apply(lg, lc, L.mask, base);
            base = affine_apply(jg, jc, L.mask, base);
        }
        return;
    }
    for (uint64_t i = b0 + threadIdx.x; i < n; i += stride) out[i] = stream_start(L, S, i);
}

hipError_t launch_init_streams(const LcgDev& L, const SeedDev& S, uint64_t n, uint64_t* out, hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    // hash: many short blocks (HBM-bound); stride: fewer, longer-lived
    // threads, so that each amortises its start (two chains of dependent
    // table reads) over more streams
    uint64_t cap = 65536;
    if (S.kind == SEED_STRIDE) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            cap = static_cast<uint64_t>(cus) * 16;
        else
            cap = 4096;
    }
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(k_init_streams, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, L, S, n, out);
    return hipGetLastError();
}

// One LCG step for m = 63, c = 1: with the increment and the mask known at
// compile time this is one v_mad_u64_u32 (g_lo * x_lo + 1), two
// v_mul_lo_u32 (cross products), one v_add3_u32 and one v_and_b32.
template <bool M63C1>
__device__ __forceinline__ uint64_t draw_step(const LcgDev& L, uint64_t x, uint64_t g) {
    if (M63C1) return (g * x + 1ull) & 0x7fffffffffffffffull;
    return lcg_next(L, x);
}

template <int MODE>
__device__ __forceinline__ uint64_t queue_seed(const DrawParams& P, uint64_t j) {
    if (MODE == SEED_LOAD) return P.state[j];
    return stream_start(P.lcg, P.seed, j);
}

// A ring entry's start state for stream j0 + lane (j0 wave-uniform): X, or
// 2X on the halves path (m = 63, c = 1, no stored states).  There a hashed
// start needs no mask (((h mod 2^63) 2) mod 2^64 = 2h mod 2^64), and the
// hash's first product (k0 + lane) M, k0 = first_index + j0 + 1, is
// k0 M (scalar) plus the lane's lane M.
template <int MODE, bool HALVES>
__device__ __forceinline__ uint64_t ring_state(const DrawParams& P, uint64_t j0, uint32_t lane, uint64_t lane_m) {
    if constexpr (HALVES && MODE == SEED_HASH) {
        const uint64_t k0m = (P.seed.first_index + j0 + 1ull) * kMurmurM;
        return murmur_from_product(k0m + lane_m, P.seed.base) << 1;
    } else {
        return queue_seed<MODE>(P, j0 + lane) << (HALVES ? 1 : 0);
    }
}

// Stride seeding of a batch of 64 consecutive streams s0 + l (l = lane):
// X_{Q(s0 + l)} = A_{Ql}(X_{Q s0}), with A_k the k-step map x -> G_k x + C_k
// (eq. 2).  A_{Ql} composes the skip table's digit-0 entry for l & 15 and
// its digit-1 entry for l >> 4; the next batch's base is A_{64Q} (digit 1,
// value 4) of this one.  Same states as the digit walk of stream_start.
struct StrideLanes {
    uint64_t g, c;        // A_{Q lane}
    uint64_t g64, c64;    // A_{64 Q}
};

__device__ __forceinline__ StrideLanes stride_lanes(const SeedDev& S, uint32_t lane) {
    const uint64_t* a = S.table + 2 * (lane & (kStrideRadix - 1));
    const uint64_t* b = S.table + 2 * (kStrideRadix + (lane >> kStrideRadixBits));
    const uint64_t* q = S.table + 2 * (kStrideRadix + 4);
    StrideLanes r;
    r.g = a[0] * b[0];
    r.c = a[0] * b[1] + a[1];
    r.g64 = q[0];
    r.c64 = q[1];
    return r;
}

// One ring entry: a stream's start state and its draw count (one LDS read).
struct __align__(16) RingEntry {
    uint64_t state;
    uint32_t count;
    uint32_t pad;
};

// Persistent seed + draw kernel.  Each wave owns the streams [lo, hi)
// (fewer than 2^28) and keeps the next streams ready in a 128-entry LDS ring
// (start state and draw count at position j & 127 for stream j), seeded 64 at
// a time by all 64 lanes at once (stride seeding: one affine step per lane
// from the batch's base), the counts loaded one batch ahead.  Each
// lane carries one active stream; a round draws D steps (only the checksum is
// masked by the remaining count); after a round, lanes whose stream ended
// store its checksum and take the next ring entries in order (ballot, prefix
// count, one ring entry read).  Up to 64 lanes are served per round without a
// loop, and the refill path never waits on vector memory (one wait per 64
// streams, when a batch is seeded).
template <int MODE, int D, bool STORE_STATE, bool M63C1>
__global__ void __launch_bounds__(256) k_draw(DrawParams P) {
    __shared__ RingEntry s_ring[4][128];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave in block
    const uint64_t wave = static_cast<uint64_t>(blockIdx.x) * (blockDim.x >> 6) + wib;
    const uint64_t nwaves = static_cast<uint64_t>(gridDim.x) * (blockDim.x >> 6);
    const uint64_t lo = wave * P.n / nwaves;
    const uint32_t nw = static_cast<uint32_t>((wave + 1) * P.n / nwaves - lo);   // streams of this wave
    const uint64_t g = P.lcg.g;
    RingEntry* ring = s_ring[wib];
    // HALVES (m = 63, c = 1, state not stored): a lane holds 2 X, which
    // follows 2X <- g (2X) + 2 mod 2^64 with no mask; the ring holds 2 X too.
    // The checksum is kept as the exact sums of the low and the high 32-bit
    // words of 2X (each below 2^64 for fewer than 2^32 draws), so sum X mod
    // 2^64 = (lo_sum >> 1) + (hi_sum << 31).  A masked draw slot then costs a
    // bit-field extract and two 32 x 32 + 64 multiply-adds.
    constexpr bool HALVES = M63C1 && !STORE_STATE;
    constexpr int SH = HALVES ? 1 : 0;
    // wave-uniform base of the wave's checksums; a store adds a 32-bit byte
    // offset (the launcher keeps a wave below 2^28 streams)
    char* const cbase = reinterpret_cast<char*>(P.checksum + lo);
    const uint64_t lane_m = static_cast<uint64_t>(lane) * kMurmurM;   // hashed ring entries

    // ring bookkeeping, wave-uniform: streams [next, filled) are seeded and
    // not yet handed out; c_next holds the counts of the batch after them
    uint32_t next = 0, filled = 128;
    uint32_t c_next = 0;
    // stride seeding: this lane's map A_{Q lane} and the base X_{Q s0} of the
    // next batch to seed (wave-uniform)
    StrideLanes sl{};
    uint64_t sbase = 0;
    if (MODE == SEED_STRIDE) {
        sl = stride_lanes(P.seed, lane);
        sbase = stream_start(P.lcg, P.seed, lo);
    }
    {
        const uint32_t ja = lane, jb = 64u + lane, jn = 128u + lane;
        ring[ja].count = (ja < nw) ? P.count[lo + ja] : 0u;
        ring[jb].count = (jb < nw) ? P.count[lo + jb] : 0u;
        if (MODE == SEED_STRIDE) {
            const uint64_t b1 = affine_apply(sl.g64, sl.c64, P.lcg.mask, sbase);
            ring[ja].state = (ja < nw) ? affine_apply(sl.g, sl.c, P.lcg.mask, sbase) << SH : 0ull;
            ring[jb].state = (jb < nw) ? affine_apply(sl.g, sl.c, P.lcg.mask, b1) << SH : 0ull;
            sbase = affine_apply(sl.g64, sl.c64, P.lcg.mask, b1);
        } else {
            ring[ja].state = (ja < nw) ? ring_state<MODE, HALVES>(P, lo, lane, lane_m) : 0ull;
            ring[jb].state = (jb < nw) ? ring_state<MODE, HALVES>(P, lo + 64u, lane, lane_m) : 0ull;
        }
        if (jn < nw) c_next = P.count[lo + jn];
    }

    uint64_t x = 0, sum = 0, hsum = 0;
    uint32_t sid = 0, rem = 0;
    bool active = false;
    for (;;) {
        if (active && rem == 0) {
            *reinterpret_cast<uint64_t*>(cbase + (sid << 3)) = HALVES ? (sum >> 1) + (hsum << 31) : sum;
            if (STORE_STATE) P.state[lo + sid] = x;
            active = false;
        }
        next = __builtin_amdgcn_readfirstlane(next);   // wave-uniform: kept in a scalar register
        const uint64_t need = __builtin_amdgcn_ballot_w64(!active);
        const uint32_t left = nw - next;   // streams not yet handed out
        if (need != 0 && left != 0) {
            const uint32_t nneed = static_cast<uint32_t>(__popcll(need));
            const uint32_t take = __builtin_amdgcn_readfirstlane(nneed < left ? nneed : left);
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(need >> 32),
                                                            __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(need), 0u));
            if (!active && rank < take) {
                const uint32_t e = (next + rank) & 127u;
                const RingEntry r = ring[e];
                x = r.state;
                rem = r.count;
                sid = next + rank;
                sum = 0;
                hsum = 0;
                active = true;
            }
            next = __builtin_amdgcn_readfirstlane(next + take);
            if (filled - next < 64u && filled < nw) {
                // fewer than 64 ready: seed the next batch of 64 (its ring
                // positions hold no stream that is still to be handed out)
                const uint32_t j = filled + lane;
                if (MODE == SEED_STRIDE) {
                    ring[j & 127u].state = (j < nw) ? affine_apply(sl.g, sl.c, P.lcg.mask, sbase) << SH : 0ull;
                    sbase = affine_apply(sl.g64, sl.c64, P.lcg.mask, sbase);
                } else {
                    ring[j & 127u].state = (j < nw) ? ring_state<MODE, HALVES>(P, lo + filled, lane, lane_m) : 0ull;
                }
                ring[j & 127u].count = c_next;   // the one wait on vector memory per 64 streams
                const uint32_t jn = j + 64u;
                c_next = (jn < nw) ? P.count[lo + jn] : 0u;
                filled += 64u;
            }
        }
        if (__builtin_amdgcn_ballot_w64(active) == 0) break;
        // a lane without a stream has rem == 0
        const uint32_t k = rem < static_cast<uint32_t>(D) ? rem : static_cast<uint32_t>(D);
        if (STORE_STATE) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                if (static_cast<uint32_t>(d) < k) {
                    x = draw_step<M63C1>(P.lcg, x, g);
                    sum += x;
                }
            }
        } else if (HALVES) {
            const uint32_t fb = (D < 32 || k < 32u) ? __builtin_amdgcn_ubfe(0xffffffffu, 0u, k) : 0xffffffffu;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                x = g * x + 2ull;
                uint32_t f = __builtin_amdgcn_ubfe(fb, static_cast<uint32_t>(d), 1u);
                // hides that f <= 1, so that each product-sum stays one
                // v_mad_u64_u32 (not a 32-bit multiply and a 64-bit add)
                asm("" : "+v"(f));
                sum += static_cast<uint64_t>(static_cast<uint32_t>(x)) * f;
                hsum += static_cast<uint64_t>(static_cast<uint32_t>(x >> 32)) * f;
            }
        } else {
            // the state may run past the end of the stream (it is not
            // stored); only the checksum is masked
#pragma unroll
            for (int d = 0; d < D; ++d) {
                x = draw_step<M63C1>(P.lcg, x, g);
                if (static_cast<uint32_t>(d) < k) sum += x;
            }
        }
        rem -= k;
    }
}

template <int MODE, int D, bool M63C1>
static hipError_t launch_draw_t(const DrawParams& p, hipStream_t st, int blocks) {
    if (p.state != nullptr)
        hipLaunchKernelGGL((k_draw<MODE, D, true, M63C1>), dim3(blocks), dim3(256), 0, st, p);
    else
        hipLaunchKernelGGL((k_draw<MODE, D, false, M63C1>), dim3(blocks), dim3(256), 0, st, p);
    return hipGetLastError();
}

template <int MODE, bool M63C1>
static hipError_t launch_draw_d(const DrawParams& p, hipStream_t st, int blocks, int d) {
    // rounds of 20 draws: measured 1% faster than 16 or 24, 3% faster than 12 or 32
    switch (d) {
        case 8: return launch_draw_t<MODE, 8, M63C1>(p, st, blocks);
        case 16: return launch_draw_t<MODE, 16, M63C1>(p, st, blocks);
        case 32: return launch_draw_t<MODE, 32, M63C1>(p, st, blocks);
        default: return launch_draw_t<MODE, 20, M63C1>(p, st, blocks);
    }
}

template <int MODE>
static hipError_t launch_draw_m(const DrawParams& p, hipStream_t st, int blocks, int d) {
    const bool m63c1 = p.lcg.m == 63 && p.lcg.c == 1;
    return m63c1 ? launch_draw_d<MODE, true>(p, st, blocks, d) : launch_draw_d<MODE, false>(p, st, blocks, d);
}

hipError_t launch_draw(const DrawParams& p, int seed_mode, hipStream_t st, int blocks_per_cu, int round) {
    if (p.n == 0) return hipSuccess;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (blocks_per_cu <= 0) blocks_per_cu = 16;
    uint64_t blocks = static_cast<uint64_t>(cus) * blocks_per_cu;
    // at least one queue of streams per wave on average
    const uint64_t max_blocks = (p.n + 255) / 256;
    if (blocks > max_blocks) blocks = max_blocks;
    if (blocks < 1) blocks = 1;
    // fewer than 2^28 streams per wave (4 per block): its checksum offsets fit 32 bits
    const uint64_t min_blocks = (p.n >> 30) + 1;
    if (blocks < min_blocks) blocks = min_blocks;
    switch (seed_mode) {
        case SEED_LOAD: return launch_draw_m<SEED_LOAD>(p, st, static_cast<int>(blocks), round);
        case SEED_HASH: return launch_draw_m<SEED_HASH>(p, st, static_cast<int>(blocks), round);
        default: return launch_draw_m<SEED_STRIDE>(p, st, static_cast<int>(blocks), round);
    }
}

}  // namespace mcrng
