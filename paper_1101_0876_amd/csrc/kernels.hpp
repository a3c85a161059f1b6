// kernels.hpp -- parameter blocks and launchers of the Potts sweep kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace potts {

struct Thresholds {
  uint32_t v[4];  // v[d-1] for dE = d = 1..4
};

struct SweepParams {
  uint8_t *spins;
  uint32_t L, q;
  uint64_t nchunks;               // L*L/4
  uint32_t t_lo, t_hi;            // sweep index
  uint32_t k0, k1;                // Philox key = seed
  Thresholds thr;
  unsigned long long *rec;        // record of this sweep: [0] e_sat, [1+v] N_v
  unsigned long long *rec_clear;  // record slot to zero for the next sweep, or null
};

// Main path (L % 16 == 0, L <= 65536): a work item is a 16-byte-wide strip of
// `rows` consecutive rows (rows even, L % rows == 0).
struct StripParams {
  uint8_t *spins;
  uint32_t L, q;
  uint32_t ipr;         // items per row band = L/16
  uint32_t rows;        // rows per item
  uint32_t nitems;      // (L/rows) * (L/16)
  int32_t item_shift;   // log2(ipr) when ipr is a power of two, else -1
  uint64_t item_magic;  // ceil(2^64 / ipr) otherwise
  uint32_t row_words;   // L/4: Philox counter stride between rows
  uint32_t t_lo, t_hi;
  uint32_t k0, k1;
  Thresholds thr;
  unsigned long long *rec;
  unsigned long long *rec_clear;
};

// populations are counted in lane-private LDS columns up to this many states
constexpr uint32_t kPrivateHistMaxQ = 64;

struct InitParams {
  uint8_t *spins;
  uint32_t L, q;
  uint64_t nchunks;
  uint32_t k0, k1;
  int random;
};

struct MeasureParams {
  const uint8_t *spins;
  uint32_t L, q;
  uint64_t nchunks;
  unsigned long long *out;  // [0] e_sat, [1+v] N_v; must start zeroed
};

struct StatsParams {
  const unsigned long long *ring;  // record ring, cap slots of (1+q) int64
  int64_t cap, slot0, n;           // window: n records starting at slot0 (wrapping)
  uint32_t q;
  uint64_t N;
  double beta;
  double *out;                     // e, C, V_L, m, chi
};

hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long value,
                           hipStream_t stream);
hipError_t launch_init(const InitParams &p, hipStream_t stream);
hipError_t launch_half_sweep(const SweepParams &p, int colour, hipStream_t stream);
hipError_t launch_strip(const StripParams &p, int colour, unsigned max_groups, hipStream_t stream);
size_t strip_lds_bytes(uint32_t q, int colour);
hipError_t launch_measure(const MeasureParams &p, hipStream_t stream);
hipError_t launch_stats(const StatsParams &p, hipStream_t stream);

}  // namespace potts
