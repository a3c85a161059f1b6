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
#include "drawn.hpp"
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

// ---- pre-drawn words (drawn.hpp) ---------------------------------------------

// Item i of a half sweep (the order of half_sweep8): row y, byte column col.
__device__ __forceinline__ void item_geometry(uint32_t L, uint32_t i, uint32_t &y, uint32_t &col) {
  const uint32_t cpr = L >> 3, per_parity = (L >> 1) * cpr;
  const uint32_t par = i >= per_parity;
  const uint32_t k = i - par * per_parity;
  const uint32_t rr = k / cpr;
  y = 2 * rr + par;
  col = (k - rr * cpr) * 8u;
}

// Word buffer of H half sweeps of n items: acceptance words (one u32x4 per
// item, site j's word in component j) first, then the packed proposals.
__host__ __device__ inline size_t drawn_acc_words(uint32_t H, uint32_t n) { return (size_t)H * n * 4u; }

// One thread per (item, half sweep of the chunk): half sweep hs is colour
// hs & 1 of sweep t0 + hs / 2.
__global__ __launch_bounds__(256) void draw_words_kernel(ResidentJob j, uint32_t nitems, uint32_t H, uint32_t *words) {
  const uint32_t hs = blockIdx.y;
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= nitems) return;
  const uint64_t t = j.t0 + (hs >> 1);
  const PhiloxHead h = philox_head((uint32_t)t, (uint32_t)(t >> 32), hs & 1u, j.k0, j.k1);
  uint32_t y, col;
  item_geometry(j.L, i, y, col);
  // the blocks of update4: chunk ctr (even) and ctr + 1 == ctr ^ 1
  const uint32_t x0 = h.a0 ^ (y * (j.L >> 2) + (col >> 2));
  const Words b0 = philox_tail(x0, h);
  const Words b1 = philox_tail(x0 ^ 1u, h);
  const uint32_t q = j.q;
  reinterpret_cast<u32x4 *>(words)[(size_t)hs * nitems + i] = u32x4{b0.w1, b0.w3, b1.w1, b1.w3};
  words[drawn_acc_words(H, nitems) + (size_t)hs * nitems + i] =
      pack4(scale_to_q(b0.w0, q), scale_to_q(b0.w2, q), scale_to_q(b1.w0, q), scale_to_q(b1.w2, q));
}

// Item (y, col)'s part of a colour-COLOUR half sweep with its drawn words: k
// the packed proposals, a the acceptance words.  Colour 1 counts the final
// values of all 8 bytes and returns the differing-neighbour flags of its 4
// sites.
template <int COLOUR, int CMP, bool PRIV, bool WIDE>
__device__ __forceinline__ uint32_t drawn_half(uint8_t *lat, uint32_t L, uint32_t y, uint32_t col, bool has,
                                               uint32_t k, const u32x4 &a, const uint8_t *table, uint8_t *hist,
                                               uint32_t lane_off) {
  if (!has) return 0;
  const uint32_t ro = y * L;
  const uint32_t ru = (y == 0 ? L - 1 : y - 1) * L;
  const uint32_t rd = (y + 1 == L ? 0 : y + 1) * L;
  const uint2 cur = lds8(lat, ro + col);
  const uint2 up = lds8(lat, ru + col);
  const uint2 dn = lds8(lat, rd + col);
  Row4 r;
  if (((COLOUR + y) & 1u) == 0) {
    const uint32_t side = lds4(lat, ro + (col == 0 ? L - 4 : col - 4));
    r = update4_drawn<COLOUR, 0, CMP, WIDE>(perm(cur.y, cur.x, kSel<0>), perm(cur.y, cur.x, kSel<1>),
                                            perm(up.y, up.x, kSel<0>), perm(dn.y, dn.x, kSel<0>), side, k, a.x, a.y,
                                            a.z, a.w, table);
  } else {
    const uint32_t side = lds4(lat, ro + (col + 8 == L ? 0u : col + 8));
    r = update4_drawn<COLOUR, 1, CMP, WIDE>(perm(cur.y, cur.x, kSel<1>), perm(cur.y, cur.x, kSel<0>),
                                            perm(up.y, up.x, kSel<1>), perm(dn.y, dn.x, kSel<1>), side, k, a.x, a.y,
                                            a.z, a.w, table);
  }
  *reinterpret_cast<uint2 *>(lat + ro + col) = make_uint2(r.out_x, r.out_y);
  if (COLOUR == 1) {
    if (PRIV)
      count_active_private(hist, lane_off, r.out_x, r.out_y);
    else
      count_active_shared(reinterpret_cast<uint32_t *>(hist), r.out_x, r.out_y);
    return __popc(r.nz & 0xF0F0F0F0u);
  }
  return 0;
}

// One lattice, 512 lanes, lane i owns item i of every half sweep.  The words
// of half sweep h sit in register slot h % 4 and are loaded kDrawnAhead half
// sweeps before use; the loop body spans two sweeps so every slot is a fixed
// set of registers.  Two barriers per sweep: the counters of sweep s - 1 (one
// of two sets, by sweep parity) are reduced into its record, and cleared,
// while colour 0 of sweep s runs.
template <int CMP, bool PRIV, bool WIDE>
__global__ __launch_bounds__(512) void resident_drawn_kernel(ResidentJob j, const uint32_t *words) {
  constexpr int kBlock = 512, kWaves = kBlock / 64;
  __shared__ __align__(16) uint32_t table_words[512];
  constexpr uint32_t kHistWords = PRIV ? 64u * (CMP == 0 ? 16u : kPrivateHistMaxQ) : 256u;
  __shared__ __align__(16) uint32_t hist[2][kHistWords];
  __shared__ uint32_t nzw[2][kWaves];  // colour-1 differing-neighbour sums per wave
  extern __shared__ __align__(16) uint32_t lds[];
  const uint32_t L = j.L, q = j.q, nbytes = L * L, nitems = nbytes >> 3;
  const uint32_t H = 2u * (j.nsweeps + kDrawnPad);
  uint8_t *lat = reinterpret_cast<uint8_t *>(lds);
  uint8_t *table = reinterpret_cast<uint8_t *>(table_words);
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t lane_off = lane * 4u;
  const bool has = threadIdx.x < nitems;
  const uint32_t me = has ? threadIdx.x : 0u;  // lanes without an item load item 0's words
  uint32_t y = 0, col = 0;
  item_geometry(L, me, y, col);
  const u32x4 *aw = reinterpret_cast<const u32x4 *>(words) + me;
  const uint32_t *kw = words + drawn_acc_words(H, nitems) + me;
  const uint32_t nh = PRIV ? 64 * q : q;

  fill_accept_table<WIDE>(table, j.thr);
  for (uint32_t off = threadIdx.x * 16u; off < nbytes; off += kBlock * 16u)
    *reinterpret_cast<u32x4 *>(lat + off) = *reinterpret_cast<const u32x4 *>(j.spins + off);
  for (uint32_t i = threadIdx.x; i < nh; i += kBlock) {
    hist[0][i] = 0;
    hist[1][i] = 0;
  }

  // slots 0 .. 2 in the order the loop reloads them (each slot's two loads
  // together), so the loads in flight at each use are counted the same way on
  // the first pass as on later ones
  u32x4 a0, a1, a2, a3;
  uint32_t k0, k1, k2, k3;
  a0 = aw[0];
  k0 = kw[0];
  __builtin_amdgcn_sched_barrier(0);
  a1 = aw[nitems];
  k1 = kw[nitems];
  __builtin_amdgcn_sched_barrier(0);
  a2 = aw[2 * nitems];
  k2 = kw[2 * nitems];
  __builtin_amdgcn_sched_barrier(0);
  __syncthreads();

  // the record of sweep t from counter set b, which is then cleared.  Fixed
  // trip counts (no loop around the stores: the compiler would wait for every
  // word load in flight before entering one)
  auto record = [&](uint64_t t, uint32_t b) {
    unsigned long long *rec = j.ring + (t & (j.cap - 1)) * (uint64_t)(q + 1);
    if (PRIV) {
      constexpr uint32_t kRounds = kHistWords / 64u / kWaves;
#pragma unroll
      for (uint32_t r = 0; r < kRounds; ++r) {
        const uint32_t v = wave + r * kWaves;
        if (v < q) {
          const uint32_t c = wave_sum(hist[b][v * 64u + lane]);
          hist[b][v * 64u + lane] = 0;
          if (lane == 0) rec[1 + v] = c;
        }
      }
    } else if (threadIdx.x < q) {  // q <= 256 < kBlock
      rec[1 + threadIdx.x] = hist[b][threadIdx.x];
      hist[b][threadIdx.x] = 0;
    }
    if (threadIdx.x == 0) {
      uint32_t nzt = 0;
      for (int w = 0; w < kWaves; ++w) nzt += nzw[b][w];
      // each colour-1 site has 4 bonds; e_sat = 4 * (N/2) - differing neighbours
      rec[0] = (unsigned long long)(2u * nbytes - nzt);
    }
  };
  // sweep s: colour 0 (and the record of sweep s - 1), colour 1 counting
  // into set s & 1
  auto colour0 = [&](uint32_t s, const u32x4 &a, uint32_t k) {
    drawn_half<0, CMP, PRIV, WIDE>(lat, L, y, col, has, k, a, table, nullptr, lane_off);
    if (s > 0) record(j.t0 + s - 1, (s - 1) & 1u);
    __syncthreads();
  };
  auto colour1 = [&](uint32_t s, const u32x4 &a, uint32_t k) {
    const uint32_t b = s & 1u;
    const uint32_t nz =
        drawn_half<1, CMP, PRIV, WIDE>(lat, L, y, col, has, k, a, table, reinterpret_cast<uint8_t *>(hist[b]), lane_off);
    const uint32_t nz_w = wave_sum(nz);
    if (lane == 0) nzw[b][wave] = nz_w;
    __syncthreads();
  };
  // half sweeps h .. h + 3 of two sweeps use slots 0 .. 3; a slot is reloaded
  // (kDrawnAhead half sweeps ahead) right after the half sweep that used it.
  // The body always runs both sweeps (an odd last one follows the loop), so
  // the loads in flight at every use are the same three slots.
  const uint32_t pairs = j.nsweeps >> 1;
  for (uint32_t m = 0; m < pairs; ++m) {
    const size_t h = 4u * (size_t)m;
    a3 = aw[(h + 3) * nitems];
    k3 = kw[(h + 3) * nitems];
    colour0(2u * m, a0, k0);
    a0 = aw[(h + 4) * nitems];
    k0 = kw[(h + 4) * nitems];
    colour1(2u * m, a1, k1);
    a1 = aw[(h + 5) * nitems];
    k1 = kw[(h + 5) * nitems];
    colour0(2u * m + 1u, a2, k2);
    a2 = aw[(h + 6) * nitems];
    k2 = kw[(h + 6) * nitems];
    colour1(2u * m + 1u, a3, k3);
  }
  if (j.nsweeps & 1u) {
    colour0(j.nsweeps - 1u, a0, k0);
    colour1(j.nsweeps - 1u, a1, k1);
  }
  record(j.t0 + j.nsweeps - 1u, (j.nsweeps - 1u) & 1u);
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

bool drawn_fits(uint32_t L, uint32_t q) { return resident_fits(L, q) && (L * L >> 3) <= kDrawnMaxItems; }

size_t drawn_words_bytes(uint32_t L) {
  // per item and half sweep: four acceptance words and the packed proposals
  return (size_t)2u * (kDrawnChunk + kDrawnPad) * (L * L >> 3) * 20u;
}

hipError_t launch_draw_words(const ResidentJob &j, uint32_t *words, hipStream_t stream) {
  if (j.nsweeps == 0) return hipSuccess;
  if (!drawn_fits(j.L, j.q) || j.nsweeps > kDrawnChunk) return hipErrorInvalidValue;
  const uint32_t nitems = j.L * j.L >> 3, H = 2u * (j.nsweeps + kDrawnPad);
  hipLaunchKernelGGL(draw_words_kernel, dim3((nitems + 255) / 256, H), dim3(256), 0, stream, j, nitems, H, words);
  return hipGetLastError();
}

template <int CMP, bool PRIV, bool WIDE>
hipError_t launch_d(const ResidentJob &j, const uint32_t *words, hipStream_t stream) {
  hipLaunchKernelGGL((resident_drawn_kernel<CMP, PRIV, WIDE>), dim3(1), dim3(512), (size_t)j.L * j.L, stream, j,
                     words);
  return hipGetLastError();
}

template <bool WIDE>
hipError_t launch_dw(const ResidentJob &j, const uint32_t *words, hipStream_t stream) {
  if (j.q <= 16) return launch_d<0, true, WIDE>(j, words, stream);
  if (j.q <= kPrivateHistMaxQ) return launch_d<1, true, WIDE>(j, words, stream);
  if (j.q <= 128) return launch_d<1, false, WIDE>(j, words, stream);
  return launch_d<2, false, WIDE>(j, words, stream);
}

hipError_t launch_resident_drawn(const ResidentJob &j, const uint32_t *words, bool wide, hipStream_t stream) {
  if (j.nsweeps == 0) return hipSuccess;
  if (!drawn_fits(j.L, j.q) || j.nsweeps > kDrawnChunk) return hipErrorInvalidValue;
  return wide ? launch_dw<true>(j, words, stream) : launch_dw<false>(j, words, stream);
}

hipError_t launch_resident(const ResidentLaunch &p, unsigned njobs, uint32_t max_L, uint32_t max_q,
                           bool wide, hipStream_t stream) {
  if (njobs == 0) return hipSuccess;
  const size_t lds = resident_lds_bytes(max_L, max_q);
  return wide ? launch_w<true>(p, njobs, max_q, lds, stream)
              : launch_w<false>(p, njobs, max_q, lds, stream);
}

}  // namespace potts
