// drawn.hpp -- single small lattices swept with their random words drawn
// beforehand by the whole GPU (resident.hip).
//
// A lattice small enough for one workgroup's LDS runs on one CU, and its half
// sweeps are latency-bound there: each item's two Philox blocks are a chain of
// ten dependent rounds.  The words depend only on (seed, site, sweep), so a
// generator kernel spread over every CU draws them for a chunk of sweeps
// first (per 8-byte item and half sweep: the four proposals scaled to q and
// packed, and the four acceptance words), and the LDS-resident kernel loads
// them a few half sweeps ahead instead of computing them.  Same words, same
// chain: results are identical to every other kernel's.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "kernels.hpp"

namespace potts {

// one 8-byte item per lane of a 512-lane workgroup: L*L/8 <= 512 (L <= 64)
constexpr uint32_t kDrawnMaxItems = 512;
// sweeps drawn per generator launch
constexpr uint32_t kDrawnChunk = 1024;
// the resident kernel loads the words this many half sweeps ahead; the
// generator draws that many sweeps past the chunk's end (2 sweeps cover it)
constexpr uint32_t kDrawnAhead = 3;
constexpr uint32_t kDrawnPad = 2;

bool drawn_fits(uint32_t L, uint32_t q);
// bytes of the word buffer for chunks of up to kDrawnChunk sweeps
size_t drawn_words_bytes(uint32_t L);
// Draws the words of sweeps j.t0 .. j.t0 + j.nsweeps + kDrawnPad - 1 into
// words (j.nsweeps <= kDrawnChunk).
hipError_t launch_draw_words(const ResidentJob &j, uint32_t *words, hipStream_t stream);
// Runs sweeps j.t0 .. j.t0 + j.nsweeps - 1 of the single lattice j with the
// words launch_draw_words wrote for the same j.
hipError_t launch_resident_drawn(const ResidentJob &j, const uint32_t *words, bool wide, hipStream_t stream);

}  // namespace potts
