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

template <int MODE>
__device__ __forceinline__ uint64_t queue_seed(const DrawParams& P, uint64_t j) {
    if (MODE == SEED_LOAD) return P.state[j];
    return stream_start(P.lcg, P.seed, j);
}

// Start state of stream j0 + lane (j0 wave-uniform).  Hashed: the hash's
// first product (k0 + lane) M, k0 = first_index + j0 + 1, is k0 M (scalar)
// plus the lane's lane M.
template <int MODE>
__device__ __forceinline__ uint64_t lane_start(const DrawParams& P, uint64_t j0, uint32_t lane, uint64_t lane_m) {
    if constexpr (MODE == SEED_HASH) {
        const uint64_t k0m = (P.seed.first_index + j0 + 1ull) * kMurmurM;
        return murmur_from_product(k0m + lane_m, P.seed.base) & P.lcg.mask;
    } else {
        return queue_seed<MODE>(P, j0 + lane);
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

// ------------------------------------------------------------------ generic kernel

// One ring entry of the generic kernel: a stream's start state and its draw
// count (one LDS read).
struct __align__(16) RingEntry {
    uint64_t state;
    uint32_t count;
    uint32_t pad;
};

// Persistent seed + draw kernel for any generator (the round-aligned kernel
// below serves m = 63 and 64 with an odd multiplier).  Each wave owns the
// streams [lo, hi) (fewer than 2^28) and keeps the next streams ready in a
// 128-entry LDS ring (start state and draw count at position j & 127 for
// stream j), seeded 64 at a time by all 64 lanes at once (stride seeding:
// one affine step per lane from the batch's base), the counts loaded one
// batch ahead.  Each lane carries one active stream; a round draws D steps,
// the checksum (and, with STORE_STATE, the state) masked by the remaining
// count; after a round, lanes whose stream ended store its checksum and take
// the next ring entries in order (ballot, prefix count, one ring entry read).
template <int MODE, int D, bool STORE_STATE>
__global__ void __launch_bounds__(256) k_draw(DrawParams P) {
    __shared__ RingEntry s_ring[4][128];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave in block
    const uint64_t wave = static_cast<uint64_t>(blockIdx.x) * (blockDim.x >> 6) + wib;
    const uint64_t nwaves = static_cast<uint64_t>(gridDim.x) * (blockDim.x >> 6);
    const uint64_t lo = wave * P.n / nwaves;
    const uint32_t nw = static_cast<uint32_t>((wave + 1) * P.n / nwaves - lo);   // streams of this wave
    RingEntry* ring = s_ring[wib];
    char* const cbase = reinterpret_cast<char*>(P.checksum + lo);
    const uint64_t lane_m = static_cast<uint64_t>(lane) * kMurmurM;

    uint32_t next = 0, filled = 128;
    uint32_t c_next = 0;
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
            ring[ja].state = (ja < nw) ? affine_apply(sl.g, sl.c, P.lcg.mask, sbase) : 0ull;
            ring[jb].state = (jb < nw) ? affine_apply(sl.g, sl.c, P.lcg.mask, b1) : 0ull;
            sbase = affine_apply(sl.g64, sl.c64, P.lcg.mask, b1);
        } else {
            ring[ja].state = (ja < nw) ? lane_start<MODE>(P, lo, lane, lane_m) : 0ull;
            ring[jb].state = (jb < nw) ? lane_start<MODE>(P, lo + 64u, lane, lane_m) : 0ull;
        }
        if (jn < nw) c_next = P.count[lo + jn];
    }

    uint64_t x = 0, sum = 0;
    uint32_t sid = 0, rem = 0;
    bool active = false;
    for (;;) {
        if (active && rem == 0) {
            *reinterpret_cast<uint64_t*>(cbase + (sid << 3)) = sum;
            if (STORE_STATE) P.state[lo + sid] = x;
            active = false;
        }
        next = __builtin_amdgcn_readfirstlane(next);
        const uint64_t need = __builtin_amdgcn_ballot_w64(!active);
        const uint32_t left = nw - next;
        if (need != 0 && left != 0) {
            const uint32_t nneed = static_cast<uint32_t>(__popcll(need));
            const uint32_t take = __builtin_amdgcn_readfirstlane(nneed < left ? nneed : left);
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(need >> 32),
                                                            __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(need), 0u));
            if (!active && rank < take) {
                const RingEntry r = ring[(next + rank) & 127u];
                x = r.state;
                rem = r.count;
                sid = next + rank;
                sum = 0;
                active = true;
            }
            next = __builtin_amdgcn_readfirstlane(next + take);
            if (filled - next < 64u && filled < nw) {
                const uint32_t j = filled + lane;
                if (MODE == SEED_STRIDE) {
                    ring[j & 127u].state = (j < nw) ? affine_apply(sl.g, sl.c, P.lcg.mask, sbase) : 0ull;
                    sbase = affine_apply(sl.g64, sl.c64, P.lcg.mask, sbase);
                } else {
                    ring[j & 127u].state = (j < nw) ? lane_start<MODE>(P, lo + filled, lane, lane_m) : 0ull;
                }
                ring[j & 127u].count = c_next;   // the one wait on vector memory per 64 streams
                const uint32_t jn = j + 64u;
                c_next = (jn < nw) ? P.count[lo + jn] : 0u;
                filled += 64u;
            }
        }
        if (__builtin_amdgcn_ballot_w64(active) == 0) break;
        const uint32_t k = rem < static_cast<uint32_t>(D) ? rem : static_cast<uint32_t>(D);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (STORE_STATE) {
                if (static_cast<uint32_t>(d) < k) {
                    x = lcg_next(P.lcg, x);
                    sum += x;
                }
            } else {
                // the state may run past the end of the stream (it is not
                // stored); only the checksum is masked
                x = lcg_next(P.lcg, x);
                if (static_cast<uint32_t>(d) < k) sum += x;
            }
        }
        rem -= k;
    }
}

// ------------------------------------------------------------------ round-aligned kernel

// Ring entry of the round-aligned kernel: the stream's state h steps before
// its start, its initial sum (minus its h leading outputs), its number of
// whole rounds and the parity mask of its first round.
struct __align__(16) RoundEntry {
    uint64_t y;
    uint64_t s;
    uint32_t rounds;
    uint32_t pm;
    uint64_t pad;
};

// The ring entry of a stream with start state x0 and n draws.
template <int D>
__device__ __forceinline__ RoundEntry round_entry(const AlignEntry* al, uint64_t x0, uint32_t n) {
    const uint32_t q = n / static_cast<uint32_t>(D);
    const uint32_t r = n - q * static_cast<uint32_t>(D);
    const uint32_t h = r ? static_cast<uint32_t>(D) - r : 0u;
    const AlignEntry e = al[h];
    RoundEntry t;
    t.y = e.a * x0 + e.b;
    t.s = e.na * x0 + e.nb;
    t.rounds = q + (r ? 1u : 0u);
    // slot d of a round leaves its top bit at position D - 1 - d: the first
    // round counts the slots d >= h only (a 64-bit shift: D - h may be 32)
    t.pm = static_cast<uint32_t>((1ull << (static_cast<uint32_t>(D) - h)) - 1ull);
    t.pad = 0;
    return t;
}

// Seed + draw for m = 63 or 64 and an odd multiplier.  The lane keeps the
// state Y modulo 2^64 with no mask, Y <- g Y + c: its low m bits are the
// LCG's state X (2^m divides 2^64), so X_n = Y_n mod 2^m.  Then
//   sum of X_n = sum of Y_n - 2^63 (number of top bits set)   (m = 63)
// modulo 2^64, and only the parity of that number matters: a draw slot is
// the step (one 64-bit multiply-add on 32-bit halves, two cross products, a
// three-way add), one 64-bit add into the sum and (m = 63) one funnel shift
// that collects the top bit, with no mask.  Rounds carry no per-slot mask
// either: each stream starts h steps early (the rewound state of its ring
// entry) so that its last draw ends a round, its initial sum removes its h
// leading outputs, and its first round's parity mask drops their top bits.
// Work distribution, ring and refill as in the generic kernel; the ring
// entries are computed when a batch of 64 streams is seeded (all lanes).
template <int MODE, int D, bool STORE_STATE, bool TOPBIT>
__global__ void __launch_bounds__(256) k_draw_rounds(DrawParams P) {
    // splitting the last streams between lanes (below) leaves a stream's
    // final state in whichever lane ran its last part: not with final states
    constexpr bool SPLIT = !STORE_STATE;
    __shared__ RoundEntry s_ring[4][128];
    __shared__ AlignEntry s_align[kMaxRound];
    __shared__ uint64_t s_skip[SPLIT ? kSkipMaps : 1][2];
    if (threadIdx.x < static_cast<uint32_t>(D)) s_align[threadIdx.x] = P.align[threadIdx.x];
    if (SPLIT && threadIdx.x < static_cast<uint32_t>(kSkipMaps)) {
        s_skip[threadIdx.x][0] = P.align[kMaxRound + threadIdx.x].a;
        s_skip[threadIdx.x][1] = P.align[kMaxRound + threadIdx.x].b;
    }
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t wave = static_cast<uint64_t>(blockIdx.x) * (blockDim.x >> 6) + wib;
    const uint64_t nwaves = static_cast<uint64_t>(gridDim.x) * (blockDim.x >> 6);
    const uint64_t lo = wave * P.n / nwaves;
    const uint32_t nw = static_cast<uint32_t>((wave + 1) * P.n / nwaves - lo);
    const uint64_t g = P.lcg.g, c = P.lcg.c;
    RoundEntry* ring = s_ring[wib];
    char* const cbase = reinterpret_cast<char*>(P.checksum + lo);
    const uint64_t lane_m = static_cast<uint64_t>(lane) * kMurmurM;
    constexpr uint32_t kFull = (D >= 32) ? 0xffffffffu : ((1u << (D & 31)) - 1u);

    uint32_t next = 0, filled = 128;
    uint32_t c_next = 0;
    StrideLanes sl{};
    uint64_t sbase = 0;
    if (MODE == SEED_STRIDE) {
        sl = stride_lanes(P.seed, lane);
        sbase = stream_start(P.lcg, P.seed, lo);
    }
    {
        const uint32_t ja = lane, jb = 64u + lane, jn = 128u + lane;
        const uint32_t na = (ja < nw) ? P.count[lo + ja] : 0u;
        const uint32_t nb = (jb < nw) ? P.count[lo + jb] : 0u;
        uint64_t xa, xb;
        if (MODE == SEED_STRIDE) {
            const uint64_t b1 = affine_apply(sl.g64, sl.c64, P.lcg.mask, sbase);
            xa = affine_apply(sl.g, sl.c, P.lcg.mask, sbase);
            xb = affine_apply(sl.g, sl.c, P.lcg.mask, b1);
            sbase = affine_apply(sl.g64, sl.c64, P.lcg.mask, b1);
        } else {
            xa = (ja < nw) ? lane_start<MODE>(P, lo, lane, lane_m) : 0ull;
            xb = (jb < nw) ? lane_start<MODE>(P, lo + 64u, lane, lane_m) : 0ull;
        }
        ring[ja] = round_entry<D>(s_align, xa, na);
        ring[jb] = round_entry<D>(s_align, xb, nb);
        if (jn < nw) c_next = P.count[lo + jn];
    }

    // a lane's stream is live while rounds > 0.  A lane whose stream ended
    // has rounds == 0 at the top of the loop, stores its checksum there and
    // then counts on downwards (idle lanes have rounds < 0 from the next
    // round on; a stream of no draws is stored when it is taken and leaves
    // the lane idle).  The wave ends once no lane is live and every stream
    // of its range has been taken: a take that hands out only streams of no
    // draws leaves no lane live, but streams may remain.
    // The wave's tail: once every stream of its range is taken, a lane with
    // two or more rounds left hands its last rounds to an idle lane (the
    // idle lane starts 2^e rounds ahead through a skip map; the parts' sums
    // and parities add).  The parts of a split stream add their checksums
    // into a record, ring[r] (s: the sum, rounds: the parts still running),
    // r the lane that first split it; the last part stores the total.  The
    // ring holds no untaken stream by then: records use ring[0..63], the
    // hand-over ring[64..127].
    uint64_t y = 0, s = 0;
    uint32_t sid = 0, pm = 0, par = 0, bits = 0;
    int32_t rounds = -1;
    int32_t rec = -1;          // SPLIT: the record of the stream's parts (-1: the stream is whole here)
    for (;;) {
        if (rounds == 0) {
            uint64_t chk = s;
            if (TOPBIT) chk += static_cast<uint64_t>(par & 1u) << 63;
            if (SPLIT && rec >= 0) {
                RoundEntry* const r = ring + rec;
                atomicAdd(reinterpret_cast<unsigned long long*>(&r->s), static_cast<unsigned long long>(chk));
                if (atomicSub(&r->rounds, 1u) == 1u) *reinterpret_cast<uint64_t*>(cbase + (sid << 3)) = r->s;
                rec = -1;
            } else {
                *reinterpret_cast<uint64_t*>(cbase + (sid << 3)) = chk;
                if (STORE_STATE) P.state[lo + sid] = y & P.lcg.mask;
            }
        }
        next = __builtin_amdgcn_readfirstlane(next);
        const uint64_t need = __builtin_amdgcn_ballot_w64(rounds <= 0);
        const uint32_t left = nw - next;
        if (need != 0 && left != 0) {
            const uint32_t nneed = static_cast<uint32_t>(__popcll(need));
            const uint32_t take = __builtin_amdgcn_readfirstlane(nneed < left ? nneed : left);
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(need >> 32),
                                                            __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(need), 0u));
            if (rounds <= 0 && rank < take) {
                const RoundEntry r = ring[(next + rank) & 127u];
                y = r.y;
                s = r.s;
                rounds = static_cast<int32_t>(r.rounds);
                pm = r.pm;
                par = 0;
                sid = next + rank;
                if (rounds == 0) {
                    // no draws: the checksum is 0 and the state its start
                    *reinterpret_cast<uint64_t*>(cbase + (sid << 3)) = 0ull;
                    if (STORE_STATE) P.state[lo + sid] = y;
                    rounds = -1;
                }
            }
            next = __builtin_amdgcn_readfirstlane(next + take);
            if (filled - next < 64u && filled < nw) {
                const uint32_t j = filled + lane;
                uint64_t x0;
                if (MODE == SEED_STRIDE) {
                    x0 = affine_apply(sl.g, sl.c, P.lcg.mask, sbase);
                    sbase = affine_apply(sl.g64, sl.c64, P.lcg.mask, sbase);
                } else {
                    x0 = (j < nw) ? lane_start<MODE>(P, lo + filled, lane, lane_m) : 0ull;
                }
                ring[j & 127u] = round_entry<D>(s_align, x0, c_next);   // the one wait on vector memory per 64 streams
                const uint32_t jn = j + 64u;
                c_next = (jn < nw) ? P.count[lo + jn] : 0u;
                filled += 64u;
            }
        }
        if (SPLIT && next >= nw) {
            const uint64_t idle = __builtin_amdgcn_ballot_w64(rounds <= 0);
            const uint64_t cand = __builtin_amdgcn_ballot_w64(rounds >= 2);
            if (idle != 0 && cand != 0) {
                const uint32_t ni = static_cast<uint32_t>(__popcll(idle));
                const uint32_t nc = static_cast<uint32_t>(__popcll(cand));
                const uint32_t np = ni < nc ? ni : nc;
                if (rounds >= 2) {
                    const uint32_t cr = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(cand >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(cand), 0u));
                    if (cr < np) {
                        // keep the first 2^e rounds, 2^e <= rounds / 2; hand over the rest
                        const uint32_t e = 31u - static_cast<uint32_t>(__builtin_clz(static_cast<uint32_t>(rounds) >> 1));
                        const int32_t keep = 1 << e;
                        if (rec < 0) {
                            rec = static_cast<int32_t>(lane);
                            ring[lane].s = 0ull;
                            ring[lane].rounds = 2u;
                        } else {
                            atomicAdd(&ring[rec].rounds, 1u);
                        }
                        RoundEntry h;
                        h.y = s_skip[e][0] * y + s_skip[e][1];
                        h.s = (static_cast<uint64_t>(sid) << 32) | static_cast<uint32_t>(rec);
                        h.rounds = static_cast<uint32_t>(rounds - keep);
                        h.pm = kFull;
                        h.pad = 0;
                        ring[64u + cr] = h;
                        rounds = keep;
                    }
                }
                __builtin_amdgcn_wave_barrier();
                if (rounds <= 0) {
                    const uint32_t ir = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(idle >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(idle), 0u));
                    if (ir < np) {
                        const RoundEntry h = ring[64u + ir];
                        y = h.y;
                        sid = static_cast<uint32_t>(h.s >> 32);
                        rec = static_cast<int32_t>(static_cast<uint32_t>(h.s));
                        rounds = static_cast<int32_t>(h.rounds);
                        pm = h.pm;
                        s = 0ull;
                        par = 0u;
                    }
                }
            }
        }
        const bool live = __builtin_amdgcn_ballot_w64(rounds > 0) != 0;
        if (!live && next >= nw) break;
        if (live) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                y = g * y + c;
                s += y;
                if (TOPBIT) bits = __builtin_amdgcn_alignbit(bits, static_cast<uint32_t>(y >> 32), 31u);
            }
            if (TOPBIT) {
                par = static_cast<uint32_t>(__builtin_popcount(bits & pm)) + par;
                pm = kFull;
            }
            rounds -= 1;
        }
    }
}

template <int MODE, int D>
static hipError_t launch_draw_t(const DrawParams& p, hipStream_t st, int blocks) {
    const bool rounds = p.align != nullptr;
    const bool top = p.lcg.m == 63;
    if (p.state != nullptr) {
        if (!rounds)
            hipLaunchKernelGGL((k_draw<MODE, D, true>), dim3(blocks), dim3(256), 0, st, p);
        else if (top)
            hipLaunchKernelGGL((k_draw_rounds<MODE, D, true, true>), dim3(blocks), dim3(256), 0, st, p);
        else
            hipLaunchKernelGGL((k_draw_rounds<MODE, D, true, false>), dim3(blocks), dim3(256), 0, st, p);
    } else {
        if (!rounds)
            hipLaunchKernelGGL((k_draw<MODE, D, false>), dim3(blocks), dim3(256), 0, st, p);
        else if (top)
            hipLaunchKernelGGL((k_draw_rounds<MODE, D, false, true>), dim3(blocks), dim3(256), 0, st, p);
        else
            hipLaunchKernelGGL((k_draw_rounds<MODE, D, false, false>), dim3(blocks), dim3(256), 0, st, p);
    }
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_draw_m(const DrawParams& p, hipStream_t st, int blocks, int d) {
    switch (d) {
        case 8: return launch_draw_t<MODE, 8>(p, st, blocks);
        case 16: return launch_draw_t<MODE, 16>(p, st, blocks);
        case 24: return launch_draw_t<MODE, 24>(p, st, blocks);
        case 32: return launch_draw_t<MODE, 32>(p, st, blocks);
        default: return launch_draw_t<MODE, 20>(p, st, blocks);
    }
}

hipError_t launch_draw(const DrawParams& p, int seed_mode, hipStream_t st, int blocks_per_cu, int round) {
    if (p.n == 0) return hipSuccess;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (blocks_per_cu <= 0) blocks_per_cu = 32;
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
