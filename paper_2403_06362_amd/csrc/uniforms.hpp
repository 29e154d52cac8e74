// Launcher of the uniforms kernel (uniforms.hip), used by the host-side API.
#pragma once

#include "internal.hpp"

namespace mcrng {

// mode: SEED_LOAD (start states from `state`), SEED_HASH or SEED_STRIDE.
hipError_t launch_uniforms(const LcgDev& L, const SeedDev& S, int mode, uint64_t n, uint32_t k, uint64_t* state,
                           double* u, hipStream_t st);

}  // namespace mcrng
