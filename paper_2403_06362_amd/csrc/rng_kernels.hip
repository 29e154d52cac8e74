// Stream seeding and LCG draw kernels for gfx950.
//
// k_init_streams: one stream per lane, grid-stride; writes S_i.
// k_draw: persistent waves.  Each wave owns a contiguous range of streams and
//   keeps one stream per lane.  A lane draws from its stream in blocks of D
//   LCG steps (masked by the remaining count); between blocks the lanes whose
//   stream ended store its checksum and take the next streams of the wave's
//   range in order (ballot + prefix count), seeding them in registers.  The
//   state, sum and remaining count never leave registers; HBM sees 4 bytes of
//   count in and 8 bytes of checksum (+ 8 of state) out per stream.
#include "internal.hpp"

namespace mcrng {

__global__ void __launch_bounds__(256) k_init_streams(LcgDev L, SeedDev S, uint64_t n, uint64_t* out) {
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = stream_start(L, S, i);
}

hipError_t launch_init_streams(const LcgDev& L, const SeedDev& S, uint64_t n, uint64_t* out, hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_init_streams, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, L, S, n, out);
    return hipGetLastError();
}

template <int MODE, int D, bool STORE_STATE>
__global__ void __launch_bounds__(256) k_draw(DrawParams P) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
    const uint64_t lo = wave * P.n / nwaves;
    const uint64_t hi = (wave + 1) * P.n / nwaves;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    uint64_t head = lo;          // wave-uniform: next unassigned stream
    uint64_t x = 0, sum = 0, sid = 0;
    uint32_t rem = 0;
    bool active = false;
    for (;;) {
        if (active && rem == 0) {
            P.checksum[sid] = sum;
            if (STORE_STATE) P.state[sid] = x;
            active = false;
        }
        const uint64_t need = __ballot(!active);
        if (need != 0 && head < hi) {
            const uint64_t j = head + static_cast<uint64_t>(__popcll(need & lt_mask));
            if (!active && j < hi) {
                sid = j;
                if (MODE == SEED_LOAD)
                    x = P.state[j];
                else
                    x = stream_start(P.lcg, P.seed, j);
                rem = P.count[j];
                sum = 0;
                active = true;
            }
            head += static_cast<uint64_t>(__popcll(need));
        }
        if (__ballot(active) == 0) break;
        const uint32_t k = active ? (rem < static_cast<uint32_t>(D) ? rem : static_cast<uint32_t>(D)) : 0u;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (static_cast<uint32_t>(d) < k) {
                x = lcg_next(P.lcg, x);
                sum += x;
            }
        }
        rem -= k;
    }
}

template <int MODE, int D>
static hipError_t launch_draw_t(const DrawParams& p, hipStream_t st, int blocks) {
    if (p.state != nullptr)
        hipLaunchKernelGGL((k_draw<MODE, D, true>), dim3(blocks), dim3(256), 0, st, p);
    else
        hipLaunchKernelGGL((k_draw<MODE, D, false>), dim3(blocks), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_draw(const DrawParams& p, int seed_mode, hipStream_t st, int blocks_per_cu) {
    if (p.n == 0) return hipSuccess;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (blocks_per_cu <= 0) blocks_per_cu = 8;
    uint64_t blocks = static_cast<uint64_t>(cus) * blocks_per_cu;
    // at least one stream per lane on average
    const uint64_t max_blocks = (p.n + 255) / 256;
    if (blocks > max_blocks) blocks = max_blocks;
    if (blocks < 1) blocks = 1;
    constexpr int D = 8;
    switch (seed_mode) {
        case SEED_LOAD: return launch_draw_t<SEED_LOAD, D>(p, st, static_cast<int>(blocks));
        case SEED_HASH: return launch_draw_t<SEED_HASH, D>(p, st, static_cast<int>(blocks));
        default: return launch_draw_t<SEED_STRIDE, D>(p, st, static_cast<int>(blocks));
    }
}

}  // namespace mcrng
