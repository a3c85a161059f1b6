// cubic.hpp -- launch parameters of the colour-split simple-cubic half sweep
// (cubic_packed.hip), used by the state code in cubic.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace potts {
namespace cube {

struct CubeThr {
  uint32_t v[6];  // thr[d-1], d = 1..6
};

struct CubeLaunch {
  uint8_t *planes;         // plane 0, then plane 1 (plane_bytes each)
  uint64_t plane_bytes;    // L^3 / 2
  uint32_t L, q;
  uint32_t ipr;            // L / 32 items (16 packed bytes) per row
  uint32_t rows;           // R: rows of one item's walk (even, divides L)
  uint32_t nitems;         // ipr * L * (L / R)
  uint32_t xcd_stride;     // grid / 8 when the grid is a multiple of 8, else 0 (set by packed_grid)
  uint32_t k0, k1;         // Philox key
  uint32_t t_lo, t_hi;     // sweep index
  CubeThr thr;
  unsigned long long *rec;        // this sweep's record {e_sat, hist[q]} (both colours add to it)
  unsigned long long *rec_clear;  // zeroed by the colour-1 launch (the next sweep's record), or null
};

// Workgroups for l (also sets l.xcd_stride).
unsigned packed_grid(CubeLaunch &l);
hipError_t launch_packed(const CubeLaunch &l, int colour, unsigned grid, hipStream_t stream);
// Row-major cube (L^3 bytes) <-> the two colour planes; L % 32 == 0.
hipError_t launch_pack(const uint8_t *cube, uint8_t *planes, uint32_t L, hipStream_t stream);
hipError_t launch_unpack(const uint8_t *planes, uint8_t *cube, uint32_t L, hipStream_t stream);

}  // namespace cube
}  // namespace potts
