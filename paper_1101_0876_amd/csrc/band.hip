// band.hip -- persistent colour-split sweeps for mid-size single lattices.
//
// Each workgroup owns a band of R whole rows of both colour planes (the
// layout of packed.hip) and keeps it in LDS for a run of up to
// kBandMaxSweeps sweeps.  A half sweep updates the band's rows of the active
// plane from LDS alone: the only values another workgroup changes are the
// two rows just outside the band (the last row of the band above, the first
// row of the band below), held in two halo rows.  After a half sweep every
// band publishes the two edge rows of the plane it updated, and its
// neighbours copy them into their halo rows before the next half sweep reads
// them.  A half sweep then costs no kernel boundary; a site is still updated
// once per half sweep from its four neighbours with its own Philox words
// (Sec. 3.2, counter-based here), so the result is the same bit pattern as
// every other kernel's.
//
// Publication: the waves holding the edge rows update them first, at raised
// priority, store them into the exchange buffer, wait until those stores
// have completed and raise one flag per wave.  Wave 0 then waits for the
// neighbours' flags and copies their edges into its halo rows while the
// other waves are still updating the interior; a workgroup barrier ends the
// half sweep.  Flags count half sweeps from an epoch the host advances by
// 2 x sweeps per launch, so they are never cleared.  Every wait is bounded
// in time: on expiry the workgroup stops and raises a host-visible error
// word, and the neighbours waiting on it stop the same way, so the grid
// always drains.  All workgroups must be resident at once (a neighbour wait
// on a workgroup that has not started would never end): the launch is
// cooperative, which the runtime refuses when the grid cannot be resident.
//
// Ordering without L2 fences: every exchanged word (edge rows and flags) is
// written and read only with agent-scope atomic accesses, which gfx950
// performs coherently across its XCDs instead of in an XCD's own L2; a
// store has completed (vmcnt) once it is visible at that scope.  So edge
// stores, then a wait for their completion, then the flag store, read in the
// opposite order with agent-scope loads, hand over the edge rows exactly.
// An agent-scope release / acquire pair would instead write back and
// invalidate the whole L2 of the XCD at every publication and every fetch:
// measured on MI355X at L = 4096, 2.63 against 1.08 ps per site update.
//
// Records: the colour-0 pass counts the band's new colour-0 values, the
// colour-1 pass its new colour-1 values and the differing neighbours of its
// colour-1 sites (every bond once); per sweep the workgroup adds them into
// partial-record set s (striped by workgroup), folded into ring slot t0 + s
// after the launch as for the tile kernel.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "band.hpp"
#include "kernels.hpp"
#include "sweep_row.hpp"

namespace potts {
namespace {

using namespace row;

__device__ __forceinline__ u32x4 lds16(const uint8_t *p) { return *reinterpret_cast<const u32x4 *>(p); }
__device__ __forceinline__ uint32_t lds4(const uint8_t *p) { return *reinterpret_cast<const uint32_t *>(p); }

// Per-workgroup constants of a launch.
struct BandCtx {
  uint8_t *lds;          // plane c at c * plane; local row j at j * half
  const uint8_t *table;  // acceptance table
  uint8_t *hist;         // value counters
  uint32_t plane;        // LDS bytes of one plane: (R + 2) * half
  uint32_t half;         // bytes of one plane row: L / 2
  uint32_t prow;         // 16-byte items per plane row: L / 32
  uint32_t prow_magic;   // ceil(2^32 / prow): item -> row by one multiply
  uint32_t R, nitems, nedge;
  uint32_t b, up, dn;    // this band, the band above, the band below
  uint32_t y0;           // global row of local row 1
  uint32_t lane, wave, lane_off;
};

// One 16-byte item: active bytes of local row j at byte column col, updated
// from the passive rows j-1, j, j+1 (and the passive dword beside the item)
// exactly as packed_row does from HBM.  edge: exchange-buffer address of the
// item when row j is an edge row, else null.
template <int COLOUR, int O, int CMP, bool PRIV, bool WIDE>
__device__ __forceinline__ uint32_t band_item(const BandCtx &x, uint32_t q, const PhiloxHead &h, uint32_t j,
                                              uint32_t col, uint32_t ctr, uint8_t *edge) {
  uint8_t *act = x.lds + COLOUR * x.plane + j * x.half;
  const uint8_t *pas = x.lds + (COLOUR ^ 1) * x.plane + j * x.half;
  const u32x4 a = lds16(act + col);
  const u32x4 pp = lds16(pas + col);
  const u32x4 u = lds16(pas - x.half + col);
  const u32x4 d = lds16(pas + x.half + col);
  const uint32_t side = O == 0 ? lds4(pas + (col == 0 ? x.half - 4u : col - 4u))
                               : lds4(pas + (col + 16u == x.half ? 0u : col + 16u));
  const Row8 r0 = update8<COLOUR, O, CMP, WIDE>(a.x, a.y, pp.x, pp.y, u.x, u.y, d.x, d.y, O == 0 ? side : pp.z,
                                                ctr, h, q, x.table);
  const Row8 r1 = update8<COLOUR, O, CMP, WIDE>(a.z, a.w, pp.z, pp.w, u.z, u.w, d.z, d.w, O == 0 ? pp.y : side,
                                                ctr + 4u, h, q, x.table);
  u32x4 out;
  out.x = r0.ns_lo;
  out.y = r0.ns_hi;
  out.z = r1.ns_lo;
  out.w = r1.ns_hi;
  *reinterpret_cast<u32x4 *>(act + col) = out;
  if (edge) {
    uint32_t *e = reinterpret_cast<uint32_t *>(edge);
    __hip_atomic_store(e + 0, out.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(e + 1, out.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(e + 2, out.z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(e + 3, out.w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (PRIV) {
    count_active_private(x.hist, x.lane_off, r0.ns_lo, r0.ns_hi);
    count_active_private(x.hist, x.lane_off, r1.ns_lo, r1.ns_hi);
  } else {
    count_active_shared(reinterpret_cast<uint32_t *>(x.hist), r0.ns_lo, r0.ns_hi);
    count_active_shared(reinterpret_cast<uint32_t *>(x.hist), r1.ns_lo, r1.ns_hi);
  }
  if (COLOUR == 1)
    return __popc(r0.nz_lo & 0xF0F0F0F0u) + __popc(r0.nz_hi & 0xF0F0F0F0u) + __popc(r1.nz_lo & 0xF0F0F0F0u) +
           __popc(r1.nz_hi & 0xF0F0F0F0u);
  return 0;
}

// Item i of a half sweep: the top edge row's items first, then the bottom
// edge row's, then the interior rows 2 .. R-1 in order.
template <int COLOUR, int CMP, bool PRIV, bool WIDE>
__device__ __forceinline__ uint32_t band_step(const BandParams &p, const BandCtx &x, const PhiloxHead &h,
                                              uint32_t i) {
  uint32_t j, k;
  if (i < x.nedge) {
    const uint32_t bottom = i >= x.prow;
    j = bottom ? x.R : 1u;
    k = i - bottom * x.prow;
  } else {
    const uint32_t r = __umulhi(i - x.nedge, x.prow_magic);
    j = 2u + r;
    k = i - x.nedge - r * x.prow;
  }
  const uint32_t y = x.y0 + j - 1u;  // global row; y0 is even
  const uint32_t col = 16u * k;
  const uint32_t ctr = y * (p.L >> 2) + (col >> 1);
  uint8_t *edge = nullptr;
  if (i < x.nedge)
    edge = p.xbuf + ((size_t)(COLOUR * p.bands + x.b) * 2u + (j == 1u ? 0u : 1u)) * x.half + col;
  if (((COLOUR + j - 1u) & 1u) == 0)
    return band_item<COLOUR, 0, CMP, PRIV, WIDE>(x, p.q, h, j, col, ctr, edge);
  return band_item<COLOUR, 1, CMP, PRIV, WIDE>(x, p.q, h, j, col, ctr, edge);
}

// Wave 0: waits until both neighbours have published half sweep hs (all
// their flag words reach epoch + hs + 1), then copies the edge rows of plane
// COLOUR they published into this band's halo rows of that plane (the band
// above's bottom row into local row 0, the band below's top row into local
// row R + 1).  Those rows are read by no item of the current half sweep.
// Returns false when the wait outlived its bound.
template <int COLOUR>
__device__ __forceinline__ bool band_fetch(const BandParams &p, const BandCtx &x, uint32_t hs) {
  const uint32_t target = p.epoch + hs + 1u;
  const uint32_t np = 2u * p.parts;
  const uint32_t *f =
      p.flags + (x.lane < p.parts ? x.up * p.parts + x.lane : x.dn * p.parts + (x.lane - p.parts) % p.parts);
  const uint64_t start = wall_clock64();
  bool ok = true;
  for (;;) {
    bool seen = true;
    if (x.lane < np)
      seen = (int32_t)(__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) >= 0;
    if (__all(seen)) break;
    if (wall_clock64() - start > p.wait_ticks) {
      ok = false;
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  // the edge loads stay after the flag loads (the loop exit depends on them)
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  if (!ok) return false;
  uint8_t *act = x.lds + COLOUR * x.plane;
  for (uint32_t k = x.lane; k < 2u * x.prow; k += 64u) {
    const uint32_t below = k >= x.prow;  // the band below's top row -> local row R + 1
    const uint32_t kk = k - below * x.prow;
    const uint8_t *src =
        p.xbuf + ((size_t)(COLOUR * p.bands + (below ? x.dn : x.up)) * 2u + (below ? 0u : 1u)) * x.half + 16u * kk;
    const uint32_t *e = reinterpret_cast<const uint32_t *>(src);
    u32x4 v;
    v.x = __hip_atomic_load(e + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v.y = __hip_atomic_load(e + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v.z = __hip_atomic_load(e + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v.w = __hip_atomic_load(e + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *reinterpret_cast<u32x4 *>(act + (below ? (x.R + 1u) * x.half : 0u) + 16u * kk) = v;
  }
  return true;
}

// Half sweep hs (colour COLOUR of sweep t) of the band.  Ends with a
// workgroup barrier; sets stop[hs & 1] when a neighbour wait failed (two
// words: a wave still reading the word of half sweep hs after the barrier
// cannot see a write of half sweep hs + 1, which only wave 0 makes, before
// every wave reached the next barrier).
template <int COLOUR, int CMP, bool PRIV, bool WIDE, int BLOCK>
__device__ __forceinline__ uint32_t band_half(const BandParams &p, const BandCtx &x, uint32_t hs, uint64_t t,
                                              uint32_t *stop) {
  const PhiloxHead h = philox_head((uint32_t)t, (uint32_t)(t >> 32), (uint32_t)COLOUR, p.k0, p.k1);
  uint32_t nz = 0;
  // round 0 holds every edge item (nedge <= BLOCK); their waves go first
  const bool edge_wave = x.wave < p.parts;
  if (edge_wave) __builtin_amdgcn_s_setprio(2);
  if (threadIdx.x < x.nitems) nz += band_step<COLOUR, CMP, PRIV, WIDE>(p, x, h, threadIdx.x);
  if (edge_wave) {
    // the wave's edge stores complete before its flag is raised
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    if (x.lane == 0)
      __hip_atomic_store(p.flags + x.b * p.parts + x.wave, p.epoch + hs + 1u, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_setprio(0);
  }
  if (x.wave == 0 && hs + 1u < 2u * p.nsweeps && !band_fetch<COLOUR>(p, x, hs)) {
    if (x.lane == 0) {
      stop[hs & 1u] = 1u;
      __hip_atomic_store(p.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
  for (uint32_t i = threadIdx.x + BLOCK; i < x.nitems; i += BLOCK) nz += band_step<COLOUR, CMP, PRIV, WIDE>(p, x, h, i);
  __syncthreads();
  return nz;
}

template <int CMP, bool PRIV, bool WIDE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void band_kernel(BandParams p) {
  constexpr uint32_t kWaves = BLOCK / 64;
  __shared__ __align__(16) uint32_t table_words[512];
  constexpr uint32_t kHistWords = PRIV ? 64u * (CMP == 0 ? 16u : kPrivateHistMaxQ) : 256u;
  __shared__ __align__(16) uint32_t hist[kHistWords];
  __shared__ uint32_t partial[256 + kWaves];
  __shared__ uint32_t stop[2];
  extern __shared__ __align__(16) uint32_t lds_words[];

  BandCtx x;
  x.lds = reinterpret_cast<uint8_t *>(lds_words);
  x.table = reinterpret_cast<const uint8_t *>(table_words);
  x.hist = reinterpret_cast<uint8_t *>(hist);
  const uint32_t L = p.L, q = p.q, R = p.rows;
  x.half = L >> 1;
  x.prow = L >> 5;
  x.prow_magic = p.prow_magic;
  x.plane = (R + 2u) * x.half;
  x.R = R;
  x.nitems = R * x.prow;
  x.nedge = 2u * x.prow;
  x.b = blockIdx.x;
  x.up = x.b == 0 ? p.bands - 1u : x.b - 1u;
  x.dn = x.b + 1u == p.bands ? 0u : x.b + 1u;
  x.y0 = x.b * R;
  x.lane = threadIdx.x & 63u;
  x.wave = threadIdx.x >> 6;
  x.lane_off = x.lane * 4u;
  const size_t gplane = (size_t)x.half * L;

  fill_accept_table<WIDE>(reinterpret_cast<uint8_t *>(table_words), p.thr);
  const uint32_t nh = PRIV ? 64u * q : q;
  for (uint32_t i = threadIdx.x; i < nh; i += BLOCK) hist[i] = 0;
  if (threadIdx.x == 0) stop[0] = stop[1] = 0;
  // both planes, local rows 0 .. R+1 = global rows y0-1 .. y0+R (mod L)
  const uint32_t rows2 = R + 2u;
  for (uint32_t i = threadIdx.x; i < 2u * rows2 * x.prow; i += BLOCK) {
    const uint32_t pr = __umulhi(i, x.prow_magic);  // c * (R + 2) + j
    const uint32_t k = i - pr * x.prow;
    const uint32_t c = pr >= rows2;
    const uint32_t j = pr - c * rows2;
    uint32_t gy = x.y0 + j + L - 1u;
    gy = gy >= L ? gy - L : gy;
    gy = gy >= L ? gy - L : gy;
    *reinterpret_cast<u32x4 *>(x.lds + c * x.plane + j * x.half + 16u * k) =
        *reinterpret_cast<const u32x4 *>(p.planes + c * gplane + (size_t)gy * x.half + 16u * k);
  }
  __syncthreads();

  const uint32_t sw = stripe_words(q);
  const unsigned long long bonds = 2ull * R * L;  // 4 bonds per colour-1 site of the band
  bool failed = false;
  for (uint32_t s = 0; s < p.nsweeps; ++s) {
    const uint64_t t = p.t0 + s;
    band_half<0, CMP, PRIV, WIDE, BLOCK>(p, x, 2u * s, t, stop);
    failed = stop[0] != 0;
    if (failed) break;
    const uint32_t nz = band_half<1, CMP, PRIV, WIDE, BLOCK>(p, x, 2u * s + 1u, t, stop);
    failed = stop[1] != 0;
    if (failed) break;
    const uint32_t nz_w = wave_sum(nz);
    if (PRIV) {
      for (uint32_t v = x.wave; v < q; v += kWaves) {
        const uint32_t c = wave_sum(hist[v * 64u + x.lane]);
        hist[v * 64u + x.lane] = 0;
        if (x.lane == 0) partial[v] = c;
      }
    } else {
      for (uint32_t v = threadIdx.x; v < q; v += BLOCK) {
        partial[v] = hist[v];
        hist[v] = 0;
      }
    }
    if (x.lane == 0) partial[q + x.wave] = nz_w;
    __syncthreads();
    unsigned long long *dst =
        p.stripes + ((uint64_t)s * p.nstripes + (x.b & (p.nstripes - 1u))) * (uint64_t)sw;
    for (uint32_t v = threadIdx.x; v < q; v += BLOCK)
      if (partial[v]) atomicAdd(&dst[1 + v], (unsigned long long)partial[v]);
    if (threadIdx.x == 0) {
      unsigned long long nzt = 0;
      for (uint32_t w = 0; w < kWaves; ++w) nzt += partial[q + w];
      atomicAdd(&dst[0], bonds - nzt);
    }
  }
  if (failed) return;
  // the band's rows of both planes back to the lattice
  for (uint32_t i = threadIdx.x; i < 2u * R * x.prow; i += BLOCK) {
    const uint32_t pr = __umulhi(i, x.prow_magic);  // c * R + (j - 1)
    const uint32_t k = i - pr * x.prow;
    const uint32_t c = pr >= R;
    const uint32_t j = pr - c * R + 1u;
    *reinterpret_cast<u32x4 *>(p.planes + c * gplane + (size_t)(x.y0 + j - 1u) * x.half + 16u * k) =
        lds16(x.lds + c * x.plane + j * x.half + 16u * k);
  }
}

template <int CMP, bool PRIV, bool WIDE, int BLOCK>
const void *kernel_of() {
  return reinterpret_cast<const void *>(&band_kernel<CMP, PRIV, WIDE, BLOCK>);
}

template <int BLOCK>
const void *pick_b(uint32_t q, bool wide) {
  if (q <= 16) return wide ? kernel_of<0, true, true, BLOCK>() : kernel_of<0, true, false, BLOCK>();
  if (q <= kPrivateHistMaxQ) return wide ? kernel_of<1, true, true, BLOCK>() : kernel_of<1, true, false, BLOCK>();
  if (q <= 128) return wide ? kernel_of<1, false, true, BLOCK>() : kernel_of<1, false, false, BLOCK>();
  return wide ? kernel_of<2, false, true, BLOCK>() : kernel_of<2, false, false, BLOCK>();
}

const void *pick(uint32_t q, bool wide, uint32_t block) {
  if (block == 256) return pick_b<256>(q, wide);
  if (block == 512) return pick_b<512>(q, wide);
  if (block == 1024) return pick_b<1024>(q, wide);
  return nullptr;
}

}  // namespace

size_t band_lds_bytes(uint32_t L, uint32_t rows) { return (size_t)(rows + 2u) * L; }

uint32_t band_parts(uint32_t L) { return (L / 16u + 63u) / 64u; }

bool band_shape_ok(uint32_t L, uint32_t rows, uint32_t block) {
  if (L % 32 || L < 64 || rows < 2 || rows % 2 || L % rows || L / rows < 2) return false;
  if (block != 256 && block != 512 && block != 1024) return false;
  // every edge item in round 0; parts flags per neighbour polled by one wave
  if (L / 16u > block || 2u * band_parts(L) > 64u) return false;
  // item -> row by a multiply with ceil(2^32 / prow): exact below 2^32 / prow^2
  const uint64_t prow = L / 32u;
  if (2ull * (rows + 2u) * prow * prow >= (1ull << 32)) return false;
  return band_lds_bytes(L, rows) <= kBandMaxLds;
}

hipError_t band_resident(uint32_t L, uint32_t q, uint32_t rows, uint32_t block, bool *fits) {
  *fits = false;
  if (!band_shape_ok(L, rows, block)) return hipSuccess;
  // both table forms: a call may take either (the wide one holds more registers)
  const size_t lds = band_lds_bytes(L, rows);
  int per_cu = 1 << 30;
  for (bool wide : {false, true}) {
    const void *k = pick(q, wide, block);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int n = 0;
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, (int)block, lds);
    if (e != hipSuccess) return e;
    per_cu = n < per_cu ? n : per_cu;
  }
  int dev = 0, cus = 0, coop = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
  if (e != hipSuccess) return e;
  *fits = coop != 0 && (uint64_t)per_cu * (uint64_t)cus >= L / rows;
  return hipSuccess;
}

hipError_t launch_band(const BandParams &p, uint32_t block, hipStream_t stream) {
  if (p.nsweeps == 0) return hipSuccess;
  if (!band_shape_ok(p.L, p.rows, block) || p.bands != p.L / p.rows || p.parts != band_parts(p.L) ||
      p.nsweeps > kBandMaxSweeps || !p.planes || !p.xbuf || !p.flags || !p.err || !p.stripes ||
      (p.nstripes & (p.nstripes - 1)) || p.q < 2 || p.q > 256)
    return hipErrorInvalidValue;
  const bool wide = !p.thr.v[0] || !p.thr.v[1] || !p.thr.v[2] || !p.thr.v[3];
  const void *k = pick(p.q, wide, block);
  const size_t lds = band_lds_bytes(p.L, p.rows);
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  BandParams arg = p;
  void *args[] = {&arg};
  return hipLaunchCooperativeKernel(k, dim3(p.bands), dim3(block), args, (unsigned)lds, stream);
}

}  // namespace potts
