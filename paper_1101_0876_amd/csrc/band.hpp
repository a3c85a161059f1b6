// band.hpp -- parameter block and launcher of the persistent band kernel
// (band.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace potts {

// Persistent colour-split sweeps on LDS bands (band.hip): workgroup b keeps
// rows b*rows .. b*rows + rows - 1 of both colour planes of a packed L x L
// lattice (L % 32 == 0) in LDS for nsweeps <= kBandMaxSweeps sweeps and
// trades its edge rows with bands b-1 and b+1 (mod bands) through xbuf and
// flags.  The record of sweep t0 + s is added into partial-record set s as
// for the tile kernel (launch_fold_sets).
constexpr uint32_t kBandMaxSweeps = 64;
constexpr size_t kBandMaxLds = 136u * 1024u;   // dynamic LDS of one band (static LDS up to 20 KB)

struct BandParams {
  uint8_t *planes;            // the packed lattice: plane 0, then plane 1 (L*L/2 bytes each)
  uint8_t *xbuf;              // edge rows: [plane][band][top, bottom][L/2 bytes]
  uint32_t *flags;            // [band][part]: epoch + half sweeps published
  uint32_t *err;              // host-visible: set to 1 when a neighbour wait outlived wait_ticks
  unsigned long long *stripes;
  uint32_t nstripes;          // a power of two
  uint32_t L, q;
  uint32_t rows, bands;       // rows per band (even), bands = L / rows
  uint32_t parts;             // flag words per band: waves holding edge items
  uint32_t prow_magic;        // ceil(2^32 / (L / 32))
  uint32_t k0, k1;            // Philox key = seed
  Thresholds thr;
  uint64_t t0;                // sweep index of the launch's first sweep
  uint32_t nsweeps;
  uint32_t epoch;             // flag value before the launch
  uint64_t wait_ticks;        // bound on one wait, in wall_clock64 ticks
};

size_t band_lds_bytes(uint32_t L, uint32_t rows);
uint32_t band_parts(uint32_t L);
bool band_shape_ok(uint32_t L, uint32_t rows, uint32_t block);
// whether a grid of L / rows workgroups of `block` lanes can be resident at once
hipError_t band_resident(uint32_t L, uint32_t q, uint32_t rows, uint32_t block, bool *fits);
hipError_t launch_band(const BandParams &p, uint32_t block, hipStream_t stream);

}  // namespace potts
