// resident.hip -- LDS-resident multi-sweep kernel for small lattices
// (L % 16 == 0, L*L <= 64 KiB).
//
// One workgroup owns one lattice: it copies the lattice into LDS once, runs
// all requested sweeps there (colour 0, barrier, colour 1, barrier, records),
// and writes the lattice back at the end.  Every sweep's record {e_sat,
// hist[q]} is reduced inside the workgroup and stored directly in its ring
// slot, so one launch replaces 2 x nsweeps launches of the streaming kernel.
// A launch may hold many jobs (one per workgroup), which is how batches of
// small lattices run.
//
// Work item: 8 bytes of one row (4 active sites), updated by the shared
// 4-site row routine (sweep_row.hpp); 512 lanes, so a 64 x 64 lattice gives
// every lane one item per half sweep and each SIMD two waves to overlap.
// Items are ordered so that all rows of one parity come first: a wave then
// usually sees a single byte parity and the parity branch is uniform.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"
#include "sweep_row.hpp"

namespace potts {
namespace {

using namespace row;

// A single lattice runs 8-byte items on 512 lanes (latency first: a 64 x 64
// lattice gives each lane one item per half sweep and each SIMD two waves);
// a batch runs 16-byte items on 256 lanes per lattice (fewer instructions per
// site, many workgroups per CU).
constexpr int kMaxWaves = 8;

__device__ __forceinline__ u32x4 lds16(const uint8_t *lat, uint32_t off) {
  return *reinterpret_cast<const u32x4 *>(lat + off);
}
__device__ __forceinline__ uint32_t lds4(const uint8_t *lat, uint32_t off) {
  return *reinterpret_cast<const uint32_t *>(lat + off);
}

__device__ __forceinline__ uint2 lds8(const uint8_t *lat, uint32_t off) {
  return *reinterpret_cast<const uint2 *>(lat + off);
}

// One 8-byte row item of the LDS lattice (row y, byte column col): 4 active
// sites.  Returns the differing-neighbour count of its new spins (colour 1).
template <int COLOUR, int O, int CMP, bool PRIV, bool WIDE>
__device__ __forceinline__ uint32_t item_update(uint8_t *lat, const ResidentJob &j, uint32_t y,
                                                uint32_t col, const PhiloxHead &h,
                                                const uint8_t *table, uint8_t *hist,
                                                uint32_t lane_off) {
  const uint32_t L = j.L;
  const uint32_t ro = y * L;
  const uint32_t ru = (y == 0 ? L - 1 : y - 1) * L;
  const uint32_t rd = (y + 1 == L ? 0 : y + 1) * L;
  const uint2 cur = lds8(lat, ro + col);
  const uint2 up = lds8(lat, ru + col);
  const uint2 dn = lds8(lat, rd + col);
  const uint32_t side = O == 0 ? lds4(lat, ro + (col == 0 ? L - 4 : col - 4))
                               : lds4(lat, ro + (col + 8 == L ? 0u : col + 8));
  const Row4 r = update4<COLOUR, O, CMP, WIDE>(
      perm(cur.y, cur.x, kSel<O>), perm(cur.y, cur.x, kSel<O ^ 1>), perm(up.y, up.x, kSel<O>),
      perm(dn.y, dn.x, kSel<O>), side, y * (L >> 2) + (col >> 2), h, j.q, table);
  *reinterpret_cast<uint2 *>(lat + ro + col) = make_uint2(r.out_x, r.out_y);
  if (COLOUR == 1) {
    // every site is final after colour 1: count all 8 bytes
    if (PRIV)
      count_active_private(hist, lane_off, r.out_x, r.out_y);
    else
      count_active_shared(reinterpret_cast<uint32_t *>(hist), r.out_x, r.out_y);
    return __popc(r.nz & 0xF0F0F0F0u);
  }
  return 0;
}

template <int COLOUR, int CMP, bool PRIV, bool WIDE, int BLOCK>
__device__ __forceinline__ uint32_t half_sweep8(uint8_t *lat, const ResidentJob &j, uint64_t t,
                                               const uint8_t *table, uint8_t *hist, uint32_t lane_off) {
  const PhiloxHead h = philox_head((uint32_t)t, (uint32_t)(t >> 32), (uint32_t)COLOUR, j.k0, j.k1);
  const uint32_t L = j.L;
  const uint32_t cpr = L >> 3;                  // 8-byte items per row
  const uint32_t per_parity = (L >> 1) * cpr;   // items in the rows of one parity
  uint32_t nz = 0;
  for (uint32_t i = threadIdx.x; i < 2 * per_parity; i += BLOCK) {
    const uint32_t par = i >= per_parity;
    const uint32_t k = i - par * per_parity;
    const uint32_t rr = k / cpr;
    const uint32_t y = 2 * rr + par;
    const uint32_t col = (k - rr * cpr) * 8u;
    if (((COLOUR + y) & 1u) == 0)
      nz += item_update<COLOUR, 0, CMP, PRIV, WIDE>(lat, j, y, col, h, table, hist, lane_off);
    else
      nz += item_update<COLOUR, 1, CMP, PRIV, WIDE>(lat, j, y, col, h, table, hist, lane_off);
  }
  return nz;
}


// One 16-byte row item of the LDS lattice (row y, byte column col): 8 active
// sites (batches: many lattices per launch, throughput first).
template <int COLOUR, int O, int CMP, bool PRIV, bool WIDE>
__device__ __forceinline__ uint32_t item_update16(uint8_t *lat, const ResidentJob &j, uint32_t y,
                                                uint32_t col, const PhiloxHead &h,
                                                const uint8_t *table, uint8_t *hist,
                                                uint32_t lane_off) {
  const uint32_t L = j.L;
  const uint32_t ro = y * L;
  const uint32_t ru = (y == 0 ? L - 1 : y - 1) * L;
  const uint32_t rd = (y + 1 == L ? 0 : y + 1) * L;
  const u32x4 cur = lds16(lat, ro + col);
  const u32x4 up = lds16(lat, ru + col);
  const u32x4 dn = lds16(lat, rd + col);
  const uint32_t side = O == 0 ? lds4(lat, ro + (col == 0 ? L - 4 : col - 4))
                               : lds4(lat, ro + (col + 16 == L ? 0u : col + 16));
  const Row8 r = update8<COLOUR, O, CMP, WIDE>(
      perm(cur.y, cur.x, kSel<O>), perm(cur.w, cur.z, kSel<O>),
      perm(cur.y, cur.x, kSel<O ^ 1>), perm(cur.w, cur.z, kSel<O ^ 1>),
      perm(up.y, up.x, kSel<O>), perm(up.w, up.z, kSel<O>),
      perm(dn.y, dn.x, kSel<O>), perm(dn.w, dn.z, kSel<O>), side,
      y * (L >> 2) + (col >> 2), h, j.q, table);
  *reinterpret_cast<u32x4 *>(lat + ro + col) = r.out;
  if (COLOUR == 1) {
    if (PRIV)
      count_row_private(hist, lane_off, r.out);
    else
      count_row_shared(reinterpret_cast<uint32_t *>(hist), r.out);
    return __popc(r.nz_lo & 0xF0F0F0F0u) + __popc(r.nz_hi & 0xF0F0F0F0u);
  }
  return 0;
}

template <int COLOUR, int CMP, bool PRIV, bool WIDE, int BLOCK>
__device__ __forceinline__ uint32_t half_sweep16(uint8_t *lat, const ResidentJob &j, uint64_t t,
                                               const uint8_t *table, uint8_t *hist, uint32_t lane_off) {
  const PhiloxHead h = philox_head((uint32_t)t, (uint32_t)(t >> 32), (uint32_t)COLOUR, j.k0, j.k1);
  const uint32_t L = j.L;
  const uint32_t cpr = L >> 4;                  // 16-byte items per row
  const uint32_t per_parity = (L >> 1) * cpr;   // items in the rows of one parity
  uint32_t nz = 0;
  for (uint32_t i = threadIdx.x; i < 2 * per_parity; i += BLOCK) {
    const uint32_t par = i >= per_parity;
    const uint32_t k = i - par * per_parity;
    const uint32_t rr = k / cpr;
    const uint32_t y = 2 * rr + par;
    const uint32_t col = (k - rr * cpr) * 16u;
    if (((COLOUR + y) & 1u) == 0)
      nz += item_update16<COLOUR, 0, CMP, PRIV, WIDE>(lat, j, y, col, h, table, hist, lane_off);
    else
      nz += item_update16<COLOUR, 1, CMP, PRIV, WIDE>(lat, j, y, col, h, table, hist, lane_off);
  }
  return nz;
}


template <int CMP, bool PRIV, bool WIDE, bool NARROW>
__global__ __launch_bounds__(NARROW ? 512 : 256) void resident_kernel(ResidentLaunch p) {
  constexpr int kBlock = NARROW ? 512 : 256;
  constexpr int kWaves = kBlock / 64;
  // table, counters and totals in static LDS (addresses fold into the LDS
  // instructions' offsets); the lattice in dynamic LDS
  __shared__ __align__(16) uint32_t table_words[512];
  constexpr uint32_t kHistWords = PRIV ? 64u * (CMP == 0 ? 16u : kPrivateHistMaxQ) : 256u;
  __shared__ __align__(16) uint32_t hist[kHistWords];  // PRIV: q x 64 lane columns; else q bins
  __shared__ uint32_t partial[256 + kMaxWaves];        // q totals, then kWaves bond sums
  extern __shared__ __align__(16) uint32_t lds[];
  const ResidentJob j = p.jobs ? p.jobs[blockIdx.x] : p.single;
  const uint32_t L = j.L, q = j.q, nbytes = L * L;
  uint8_t *lat = reinterpret_cast<uint8_t *>(lds);
  uint8_t *table = reinterpret_cast<uint8_t *>(table_words);
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t lane_off = lane * 4u;

  fill_accept_table<WIDE>(table, j.thr);
  for (uint32_t off = threadIdx.x * 16u; off < nbytes; off += kBlock * 16u)
    *reinterpret_cast<u32x4 *>(lat + off) = *reinterpret_cast<const u32x4 *>(j.spins + off);
  __syncthreads();

  const uint32_t nh = PRIV ? 64 * q : q;
  for (uint32_t s = 0; s < j.nsweeps; ++s) {
    const uint64_t t = j.t0 + s;
    for (uint32_t i = threadIdx.x; i < nh; i += kBlock) hist[i] = 0;
    uint8_t *hb = reinterpret_cast<uint8_t *>(hist);
    if (NARROW)
      half_sweep8<0, CMP, PRIV, WIDE, kBlock>(lat, j, t, table, hb, lane_off);
    else
      half_sweep16<0, CMP, PRIV, WIDE, kBlock>(lat, j, t, table, hb, lane_off);
    __syncthreads();
    const uint32_t nz = NARROW ? half_sweep8<1, CMP, PRIV, WIDE, kBlock>(lat, j, t, table, hb, lane_off)
                               : half_sweep16<1, CMP, PRIV, WIDE, kBlock>(lat, j, t, table, hb, lane_off);
    const uint32_t nz_w = wave_sum(nz);
    __syncthreads();
    if (PRIV) {
      for (uint32_t v = wave; v < q; v += kWaves) {
        const uint32_t c = wave_sum(hist[v * 64u + lane]);
        if (lane == 0) partial[v] = c;
      }
    } else {
      for (uint32_t v = threadIdx.x; v < q; v += kBlock) partial[v] = hist[v];
    }
    if (lane == 0) partial[q + wave] = nz_w;
    __syncthreads();
    unsigned long long *rec = j.ring + (t & (j.cap - 1)) * (uint64_t)(q + 1);
    for (uint32_t v = threadIdx.x; v < q; v += kBlock) rec[1 + v] = partial[v];
    if (threadIdx.x == 0) {
      uint32_t nzt = 0;
      for (int w = 0; w < kWaves; ++w) nzt += partial[q + w];
      // each colour-1 site has 4 bonds; e_sat = 4 * (N/2) - differing neighbours
      rec[0] = (unsigned long long)(2u * nbytes - nzt);
    }
  }

  __syncthreads();
  for (uint32_t off = threadIdx.x * 16u; off < nbytes; off += kBlock * 16u)
    *reinterpret_cast<u32x4 *>(j.spins + off) = *reinterpret_cast<const u32x4 *>(lat + off);
}

template <int CMP, bool PRIV, bool WIDE>
hipError_t launch_t(const ResidentLaunch &p, unsigned n, size_t lds, hipStream_t stream) {
  if (p.jobs)
    hipLaunchKernelGGL((resident_kernel<CMP, PRIV, WIDE, false>), dim3(n), dim3(256), lds, stream, p);
  else
    hipLaunchKernelGGL((resident_kernel<CMP, PRIV, WIDE, true>), dim3(n), dim3(512), lds, stream, p);
  return hipGetLastError();
}

template <bool WIDE>
hipError_t launch_w(const ResidentLaunch &p, unsigned n, uint32_t q, size_t lds, hipStream_t stream) {
  if (q <= 16) return launch_t<0, true, WIDE>(p, n, lds, stream);
  if (q <= kPrivateHistMaxQ) return launch_t<1, true, WIDE>(p, n, lds, stream);
  if (q <= 128) return launch_t<1, false, WIDE>(p, n, lds, stream);
  return launch_t<2, false, WIDE>(p, n, lds, stream);
}

}  // namespace

// dynamic LDS: the lattice (the rest is static, at most 19 KB)
size_t resident_lds_bytes(uint32_t L, uint32_t q) {
  (void)q;
  return (size_t)L * L;
}

bool resident_fits(uint32_t L, uint32_t q) {
  return L % 16 == 0 && (uint64_t)L * L <= 65536 && q >= 2 && q <= 256;
}

hipError_t launch_resident(const ResidentLaunch &p, unsigned njobs, uint32_t max_L, uint32_t max_q,
                           bool wide, hipStream_t stream) {
  if (njobs == 0) return hipSuccess;
  const size_t lds = resident_lds_bytes(max_L, max_q);
  return wide ? launch_w<true>(p, njobs, max_q, lds, stream)
              : launch_w<false>(p, njobs, max_q, lds, stream);
}

}  // namespace potts
