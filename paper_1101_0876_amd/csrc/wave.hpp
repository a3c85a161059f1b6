// wave.hpp -- a wave64 sum in registers for per-sweep reductions.
//
// The kernels that run several sweeps per launch (LDS-resident lattices,
// multi-sweep tiles) reduce a record every sweep; there wave_sum's shuffles,
// one LDS round trip each, sit on the sweep's critical path.  This form adds
// within each row of 16 lanes by DPP (two quad permutations, then the half-row
// and row mirrors) and reads the four row sums out.  It needs the whole wave
// active and returns the same (wave-uniform) total in every lane.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace potts {

__device__ __forceinline__ uint32_t wave_sum_rows(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);  // row_mirror
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) + (uint32_t)__builtin_amdgcn_readlane((int)v, 16) +
         (uint32_t)__builtin_amdgcn_readlane((int)v, 32) + (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

}  // namespace potts
