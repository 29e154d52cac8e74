// Uniform random numbers of many streams, for gfx950.
//
// k_uniforms: stream i (grid-stride) starts at its seed (stride skip-ahead
// or hash seed, or a state loaded from HBM), takes k LCG steps (eq. 1) and
// writes the uniform of its j-th output to u[(j - 1) n + i].  The layout is
// draw-major, so a wave's 64 stores of one draw are one contiguous 512-byte
// run; the stores are non-temporal (the output is not read back by the
// kernel).  The kernel is bound by HBM writes: 8 bytes per number against
// about a dozen VALU operations.
#include "internal.hpp"
#include "uniforms.hpp"

namespace mcrng {

template <int MODE>
__global__ void __launch_bounds__(256) k_uniforms(LcgDev L, SeedDev S, uint64_t n, uint32_t k, uint64_t* state,
                                                  double* u) {
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * 256;
    const uint64_t b0 = static_cast<uint64_t>(blockIdx.x) * 256;
    // stride seeding: stream b0 + t + j stride starts at A_{Q t} of the
    // block's base, which moves on by A_{Q stride} (one affine step each)
    uint64_t lg = 1, lc = 0, jg = 1, jc = 0, base = 0;
    if (MODE == SEED_STRIDE && b0 < n) {
        const uint64_t* a = S.table + 2 * (threadIdx.x & (kStrideRadix - 1));
        const uint64_t* b = S.table + 2 * (kStrideRadix + (threadIdx.x >> kStrideRadixBits));
        lg = a[0] * b[0];
        lc = a[0] * b[1] + a[1];
        for (uint32_t d = 0; d < kStrideDigits && (stride >> (kStrideRadixBits * d)) != 0; ++d) {
            const uint32_t v = static_cast<uint32_t>(stride >> (kStrideRadixBits * d)) & (kStrideRadix - 1);
            const uint64_t* e = S.table + 2 * (d * kStrideRadix + v);
            jc = e[0] * jc + e[1];
            jg = e[0] * jg;
        }
        base = stream_start(L, S, b0);
    }
    for (uint64_t i = b0 + threadIdx.x; i < n; i += stride) {
        uint64_t x;
        if (MODE == SEED_LOAD) {
            x = state[i];
        } else if (MODE == SEED_STRIDE) {
            x = affine_apply(lg, lc, L.mask, base);
            base = affine_apply(jg, jc, L.mask, base);
        } else {
            x = stream_start(L, S, i);
        }
        double* out = u + i;
        for (uint32_t j = 0; j < k; ++j) {
            x = lcg_next(L, x);
            __builtin_nontemporal_store(to_uniform(L, x), out);
            out += n;
        }
        if (state) state[i] = x;
    }
}

hipError_t launch_uniforms(const LcgDev& L, const SeedDev& S, int mode, uint64_t n, uint32_t k, uint64_t* state,
                           double* u, hipStream_t st) {
    if (n == 0 || k == 0) return hipSuccess;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    // many short-lived blocks: 256 per CU wrote 5.3 TB/s, 16 per CU 4.6 TB/s
    uint64_t blocks = (n + 255) / 256;
    const uint64_t cap = static_cast<uint64_t>(cus > 0 ? cus : 256) * 256;
    if (blocks > cap) blocks = cap;
    const dim3 grid(static_cast<unsigned>(blocks)), block(256);
    switch (mode) {
        case SEED_LOAD: hipLaunchKernelGGL(k_uniforms<SEED_LOAD>, grid, block, 0, st, L, S, n, k, state, u); break;
        case SEED_HASH: hipLaunchKernelGGL(k_uniforms<SEED_HASH>, grid, block, 0, st, L, S, n, k, state, u); break;
        default: hipLaunchKernelGGL(k_uniforms<SEED_STRIDE>, grid, block, 0, st, L, S, n, k, state, u); break;
    }
    return hipGetLastError();
}

}  // namespace mcrng
