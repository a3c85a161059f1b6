// packed.hip -- the single-lattice half sweep on a checkerboard-split copy of
// the lattice (the paper's cell packing, Sec. 3.3, in its simplest form).
//
// Layout: two planes of N/2 bytes.  Row y of plane c holds the L/2 sites of
// colour c ((x + y) & 1 == c) of lattice row y in increasing x: packed index i
// is site x = 2i + ((c + y) & 1).  A colour-c half sweep then reads plane c
// (active) and plane c^1 (neighbours) and writes only plane c: 1.5 N bytes
// per half sweep instead of 2 N, and no byte shuffling to separate or merge
// the colours.  The neighbours of active index i are the passive bytes at
// index i in rows y-1 and y+1, and at i and i-1 (O = 0) or i+1 (O = 1) in row
// y, with O = (c + y) & 1: exactly the packed operands the row update of
// sweep_row.hpp takes, which is reused unchanged (its Philox block and word
// for active index i, chunk y*(L/4) + i/2 and pair i & 1, are the contract's).
//
// A single lattice is packed into the state's second buffer before its first
// colour-split sweep and unpacked when the row-major lattice is read, or at the
// end of every call when the caller owns the buffers (capi.hip); batches pack
// their jobs before a run and unpack them after it.
// Both copies are plain streaming kernels.
//
// Work item: 16 packed bytes (16 active sites) of R consecutive rows of the
// active plane, walked downwards like the strip kernel: each passive row is
// loaded once and serves as the down, the same-row and the up neighbour.
// Batches of lattices run the same kernel through a tile table.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"
#include "sweep_row.hpp"

namespace potts {
namespace {

constexpr int kBlock = 256;

using namespace row;

struct PCarry {
  u32x4 u;  // passive row y-1
  u32x4 p;  // passive row y
};

struct PSums {
  uint32_t nz;
  uint32_t sites;
};

// One packed row: active bytes at a_off, the passive row below at d_off, the
// passive dword beside the item at side_off (left of it when O == 0, right
// when O == 1).  ctr: Philox chunk of the item's first active byte.
template <int COLOUR, int O, int CMP, bool PRIV, bool WIDE>
__device__ __forceinline__ void packed_row(const StripParams &p, const PhiloxHead &h,
                                           __amdgpu_buffer_rsrc_t rs, const uint8_t *table, uint8_t *hist,
                                           uint32_t lane_off, uint32_t a_off, uint32_t d_off, uint32_t side_off,
                                           uint32_t ctr, PCarry &cy, PSums &sums) {
  const u32x4 a = load16(rs, a_off);
  const u32x4 dn = load16(rs, d_off);
  const uint32_t side = load4(rs, side_off);
  // two groups of 8 sites; each needs the passive dword beyond its own pair
  const Row8 r0 = update8<COLOUR, O, CMP, WIDE>(a.x, a.y, cy.p.x, cy.p.y, cy.u.x, cy.u.y, dn.x, dn.y,
                                                O == 0 ? side : cy.p.z, ctr, h, p.q, table);
  const Row8 r1 = update8<COLOUR, O, CMP, WIDE>(a.z, a.w, cy.p.z, cy.p.w, cy.u.z, cy.u.w, dn.z, dn.w,
                                                O == 0 ? cy.p.y : side, ctr + 4u, h, p.q, table);
  u32x4 out;
  out.x = r0.ns_lo;
  out.y = r0.ns_hi;
  out.z = r1.ns_lo;
  out.w = r1.ns_hi;
  store16(rs, a_off, out);
  if (COLOUR == 1) {
    sums.nz += __popc(r0.nz_lo & 0xF0F0F0F0u) + __popc(r0.nz_hi & 0xF0F0F0F0u) +
               __popc(r1.nz_lo & 0xF0F0F0F0u) + __popc(r1.nz_hi & 0xF0F0F0F0u);
    sums.sites += 16;
  }
  if (PRIV) {
    count_active_private(hist, lane_off, r0.ns_lo, r0.ns_hi);
    count_active_private(hist, lane_off, r1.ns_lo, r1.ns_hi);
  } else {
    count_active_shared(reinterpret_cast<uint32_t *>(hist), r0.ns_lo, r0.ns_hi);
    count_active_shared(reinterpret_cast<uint32_t *>(hist), r1.ns_lo, r1.ns_hi);
  }
  cy.u = cy.p;
  cy.p = dn;
}

// p.spins: the packed lattice; p.ipr = L/32 items per row band; the whole
// lattice (no slab mode); records through p.stripes when set, else the slot.
// TILED: workgroup -> (job, item range) from the tile table (batched
// lattices, as in the strip kernel); otherwise the single descriptor with a
// grid-stride loop.
template <int COLOUR, int CMP, bool PRIV, bool WIDE, bool TILED, int BLOCK>
__device__ __forceinline__ void packed_body(const StripLaunch &launch) {
  constexpr int kWaves = BLOCK / 64;
  __shared__ __align__(16) uint32_t table_words[512];
  constexpr uint32_t kHistWords = PRIV ? 64u * (CMP == 0 ? 16u : kPrivateHistMaxQ) : 256u;
  __shared__ __align__(16) uint32_t hist[kHistWords];
  __shared__ uint32_t partial[257];
  // colour 1 walks the workgroups bottom-up (see strip.hip)
  const uint32_t bid = COLOUR == 1 ? gridDim.x - 1 - blockIdx.x : blockIdx.x;
  const StripTile tile = TILED ? launch.tiles[bid] : StripTile{0, 0, 0, 0};
  const StripParams &p = TILED ? launch.jobs[tile.job] : launch.single;
  const uint32_t first = TILED ? tile.first + threadIdx.x : bid * BLOCK + threadIdx.x;
  const uint32_t end = TILED ? tile.first + tile.count : p.nitems;
  const uint32_t stride = TILED ? (uint32_t)BLOCK : gridDim.x * BLOCK;
  const bool lead = TILED ? tile.lead != 0 : bid == 0;
  if (launch.sweep >= p.nsweeps) return;
  const uint64_t t = p.t0 + launch.sweep;
  const PhiloxHead h = philox_head((uint32_t)t, (uint32_t)(t >> 32), (uint32_t)COLOUR, p.k0, p.k1);
  uint8_t *table = reinterpret_cast<uint8_t *>(table_words);
  const uint32_t q = p.q;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = threadIdx.x >> 6;

  fill_accept_table<WIDE>(table, p.thr);
  const uint32_t nh = PRIV ? 64 * q : q;
  for (uint32_t i = threadIdx.x; i < nh; i += BLOCK) hist[i] = 0;
  // a workgroup's bond count reaches 2N / grid, beyond 32 bits on the largest
  // lattices with few workgroups: counted in 64 bits
  __shared__ unsigned long long esum;
  if (threadIdx.x == 0) esum = 0;
  if (p.stripes) {
    __shared__ unsigned long long fold_acc[COLOUR == 0 ? 257 : 1];
    if (COLOUR == 0 && lead && launch.sweep > 0) fold_stripes<BLOCK>(p, t - 1, fold_acc);
  } else if (COLOUR == 1 && lead) {
    unsigned long long *rec_next = p.ring + ((t + 1) & (p.cap - 1)) * (uint64_t)(q + 1);
    for (uint32_t i = threadIdx.x; i < q + 1; i += BLOCK) rec_next[i] = 0;
  }
  __syncthreads();

  const __amdgpu_buffer_rsrc_t rs = lattice_rsrc(p.spins);
  uint8_t *hist_bytes = reinterpret_cast<uint8_t *>(hist);
  const uint32_t lane_off = lane * 4u;
  const uint32_t L = p.L;
  const uint32_t half = L >> 1;           // bytes per plane row
  const uint32_t plane = half * L;        // bytes per plane
  const uint32_t a_base = COLOUR == 0 ? 0u : plane;
  const uint32_t p_base = COLOUR == 0 ? plane : 0u;
  const uint32_t rows = p.rows;
  PSums sums{0, 0};

  for (uint32_t item = first; item < end; item += stride) {
    const uint32_t rb = p.item_shift >= 0 ? item >> p.item_shift
                                          : (uint32_t)__umul64hi((uint64_t)item, p.item_magic);
    const uint32_t xi = item - rb * p.ipr;
    const uint32_t col = xi * 16u;
    const uint32_t left_col = col == 0 ? half - 4 : col - 4;
    const uint32_t right_col = col + 16 == half ? 0u : col + 16;
    const uint32_t r0 = rb * rows;  // even, so row r0 has O = COLOUR
    const uint32_t rp = r0 == 0 ? L - 1 : r0 - 1;
    PCarry cy;
    cy.u = load16(rs, p_base + rp * half + col);
    cy.p = load16(rs, p_base + r0 * half + col);
    uint32_t ctr = r0 * p.row_words + (col >> 1);
    constexpr bool kLeftFirst = COLOUR == 0;  // row parity 0: O = COLOUR
    for (uint32_t k = 0; k < rows; k += 2) {
      const uint32_t y = r0 + k;
      packed_row<COLOUR, COLOUR, CMP, PRIV, WIDE>(
          p, h, rs, table, hist_bytes, lane_off, a_base + y * half + col, p_base + (y + 1) * half + col,
          p_base + y * half + (kLeftFirst ? left_col : right_col), ctr, cy, sums);
      ctr += p.row_words;
      const uint32_t yd = k + 2 == rows ? (r0 + rows == L ? 0u : r0 + rows) : y + 2;
      packed_row<COLOUR, COLOUR ^ 1, CMP, PRIV, WIDE>(
          p, h, rs, table, hist_bytes, lane_off, a_base + (y + 1) * half + col, p_base + yd * half + col,
          p_base + (y + 1) * half + (kLeftFirst ? right_col : left_col), ctr, cy, sums);
      ctr += p.row_words;
    }
  }

  unsigned long long *rec = p.ring + (t & (p.cap - 1)) * (uint64_t)(q + 1);
  if (COLOUR == 1) {
    // at most 4 x 2^29 bonds per wave (L < 2^16): 32 bits suffice up to here
    const uint32_t e = wave_sum(4u * sums.sites - sums.nz);
    if (lane == 0 && e) atomicAdd(&esum, (unsigned long long)e);
  }
  __syncthreads();
  if (PRIV) {
    for (uint32_t v = wave; v < q; v += kWaves) {
      const uint32_t s = wave_sum(hist[v * 64u + lane]);
      if (lane == 0) partial[v] = s;
    }
    __syncthreads();
  }
  unsigned long long *dst =
      p.stripes ? p.stripes + ((t & 1) * p.nstripes + (bid & (p.nstripes - 1))) * (uint64_t)stripe_words(q) : rec;
  for (uint32_t v = threadIdx.x; v < q; v += BLOCK) {
    const uint32_t s = PRIV ? partial[v] : hist[v];
    if (s) atomicAdd(&dst[1 + v], (unsigned long long)s);
  }
  if (COLOUR == 1 && threadIdx.x == 0 && esum) atomicAdd(&dst[0], esum);
}

// BLOCK lanes per workgroup (tiled launches: BLOCK items per tile); the _w8
// form asks the compiler for at least 8 waves per SIMD (at most 64 VGPRs), the
// occupancy the tuner may pick.
template <int COLOUR, int CMP, bool PRIV, bool WIDE, bool TILED, int BLOCK>
__global__ __launch_bounds__(BLOCK) void packed_kernel(StripLaunch launch) {
  packed_body<COLOUR, CMP, PRIV, WIDE, TILED, BLOCK>(launch);
}

template <int COLOUR, int CMP, bool PRIV, bool WIDE, bool TILED, int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8))) void packed_kernel_w8(
    StripLaunch launch) {
  packed_body<COLOUR, CMP, PRIV, WIDE, TILED, BLOCK>(launch);
}

// Graph replay of a single lattice's sweeps (capi.hip): the captured launches
// read the lattice's descriptor from device memory; set_desc_kernel writes it
// before the first replay of a call, and fold_advance_kernel, the last node of
// the graph, folds the partial records of the graph's last sweep into their
// ring slot and moves the descriptor's first sweep on by the graph's length.
__global__ void set_desc_kernel(StripParams *d, StripParams p) {
  if (threadIdx.x == 0) *d = p;
}

__global__ __launch_bounds__(kBlock) void fold_advance_kernel(StripParams *d, uint32_t sweeps) {
  __shared__ unsigned long long acc[257];
  const StripParams p = *d;
  fold_stripes<kBlock>(p, p.t0 + sweeps - 1, acc);
  __syncthreads();  // every thread has read the descriptor
  if (threadIdx.x == 0) d->t0 = p.t0 + sweeps;
}

// Row-major lattice <-> two colour planes; one thread per 32 bytes of a row
// (16 sites of each colour).
__global__ __launch_bounds__(kBlock) void pack_kernel(const uint8_t *src, uint8_t *dst, uint32_t L) {
  const uint32_t groups = L >> 5;
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= (uint64_t)groups * L) return;
  const uint32_t y = (uint32_t)(g / groups), j = (uint32_t)(g - (uint64_t)y * groups);
  const u32x4 *in = reinterpret_cast<const u32x4 *>(src + (size_t)y * L + 32u * j);
  const u32x4 lo = in[0], hi = in[1];
  u32x4 even, odd;
  even.x = perm(lo.y, lo.x, kSel<0>);
  even.y = perm(lo.w, lo.z, kSel<0>);
  even.z = perm(hi.y, hi.x, kSel<0>);
  even.w = perm(hi.w, hi.z, kSel<0>);
  odd.x = perm(lo.y, lo.x, kSel<1>);
  odd.y = perm(lo.w, lo.z, kSel<1>);
  odd.z = perm(hi.y, hi.x, kSel<1>);
  odd.w = perm(hi.w, hi.z, kSel<1>);
  const size_t plane = (size_t)(L >> 1) * L;
  const size_t row = (size_t)y * (L >> 1) + 16u * j;
  // even x has colour y & 1
  *reinterpret_cast<u32x4 *>(dst + (y & 1) * plane + row) = even;
  *reinterpret_cast<u32x4 *>(dst + ((y & 1) ^ 1) * plane + row) = odd;
}

__global__ __launch_bounds__(kBlock) void unpack_kernel(const uint8_t *src, uint8_t *dst, uint32_t L) {
  const uint32_t groups = L >> 5;
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= (uint64_t)groups * L) return;
  const uint32_t y = (uint32_t)(g / groups), j = (uint32_t)(g - (uint64_t)y * groups);
  const size_t plane = (size_t)(L >> 1) * L;
  const size_t row = (size_t)y * (L >> 1) + 16u * j;
  const u32x4 even = *reinterpret_cast<const u32x4 *>(src + (y & 1) * plane + row);
  const u32x4 odd = *reinterpret_cast<const u32x4 *>(src + ((y & 1) ^ 1) * plane + row);
  u32x4 lo, hi;
  lo.x = perm(odd.x, even.x, 0x05010400u);
  lo.y = perm(odd.x, even.x, 0x07030602u);
  lo.z = perm(odd.y, even.y, 0x05010400u);
  lo.w = perm(odd.y, even.y, 0x07030602u);
  hi.x = perm(odd.z, even.z, 0x05010400u);
  hi.y = perm(odd.z, even.z, 0x07030602u);
  hi.z = perm(odd.w, even.w, 0x05010400u);
  hi.w = perm(odd.w, even.w, 0x07030602u);
  u32x4 *out = reinterpret_cast<u32x4 *>(dst + (size_t)y * L + 32u * j);
  out[0] = lo;
  out[1] = hi;
}

template <int COLOUR, bool WIDE, bool TILED>
hipError_t launch_w(const StripLaunch &l, unsigned grid, uint32_t q, hipStream_t stream) {
  if (q <= 16)
    hipLaunchKernelGGL((packed_kernel<COLOUR, 0, true, WIDE, TILED, kBlock>), dim3(grid), dim3(kBlock), 0, stream, l);
  else if (q <= kPrivateHistMaxQ)
    hipLaunchKernelGGL((packed_kernel<COLOUR, 1, true, WIDE, TILED, kBlock>), dim3(grid), dim3(kBlock), 0, stream, l);
  else if (q <= 128)
    hipLaunchKernelGGL((packed_kernel<COLOUR, 1, false, WIDE, TILED, kBlock>), dim3(grid), dim3(kBlock), 0, stream, l);
  else
    hipLaunchKernelGGL((packed_kernel<COLOUR, 2, false, WIDE, TILED, kBlock>), dim3(grid), dim3(kBlock), 0, stream, l);
  return hipGetLastError();
}

template <bool TILED>
hipError_t launch_c(const StripLaunch &l, int colour, unsigned grid, uint32_t qmax, bool wide, hipStream_t stream) {
  if (colour == 0)
    return wide ? launch_w<0, true, TILED>(l, grid, qmax, stream) : launch_w<0, false, TILED>(l, grid, qmax, stream);
  return wide ? launch_w<1, true, TILED>(l, grid, qmax, stream) : launch_w<1, false, TILED>(l, grid, qmax, stream);
}

// Tiled launches of q <= 16 in the tuner's other shapes.
template <int COLOUR, bool WIDE>
hipError_t launch_shape(const StripLaunch &l, unsigned ntiles, const TileShape &shape, hipStream_t stream) {
  if (shape.block == 128) {
    if (shape.wpe)
      hipLaunchKernelGGL((packed_kernel_w8<COLOUR, 0, true, WIDE, true, 128>), dim3(ntiles), dim3(128), 0, stream, l);
    else
      hipLaunchKernelGGL((packed_kernel<COLOUR, 0, true, WIDE, true, 128>), dim3(ntiles), dim3(128), 0, stream, l);
  } else {
    hipLaunchKernelGGL((packed_kernel_w8<COLOUR, 0, true, WIDE, true, 256>), dim3(ntiles), dim3(256), 0, stream, l);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_packed(const StripLaunch &l, int colour, unsigned grid, uint32_t qmax, bool wide,
                         hipStream_t stream) {
  if (grid == 0) return hipSuccess;
  return l.tiles ? launch_c<true>(l, colour, grid, qmax, wide, stream)
                 : launch_c<false>(l, colour, grid, qmax, wide, stream);
}

hipError_t launch_packed_single(const StripLaunch &l, int colour, unsigned grid, uint32_t qmax, bool wide,
                                uint32_t wpe, hipStream_t stream) {
  if (wpe == 0 || qmax > 16 || l.tiles) return launch_packed(l, colour, grid, qmax, wide, stream);
  if (grid == 0) return hipSuccess;
  if (colour == 0) {
    if (wide)
      hipLaunchKernelGGL((packed_kernel_w8<0, 0, true, true, false, kBlock>), dim3(grid), dim3(kBlock), 0, stream, l);
    else
      hipLaunchKernelGGL((packed_kernel_w8<0, 0, true, false, false, kBlock>), dim3(grid), dim3(kBlock), 0, stream, l);
  } else {
    if (wide)
      hipLaunchKernelGGL((packed_kernel_w8<1, 0, true, true, false, kBlock>), dim3(grid), dim3(kBlock), 0, stream, l);
    else
      hipLaunchKernelGGL((packed_kernel_w8<1, 0, true, false, false, kBlock>), dim3(grid), dim3(kBlock), 0, stream, l);
  }
  return hipGetLastError();
}

hipError_t launch_packed_tiled(const StripLaunch &l, int colour, unsigned ntiles, const TileShape &shape,
                               uint32_t qmax, bool wide, hipStream_t stream) {
  if (!shape_ok(shape, qmax) || !l.tiles) return hipErrorInvalidValue;
  if (ntiles == 0) return hipSuccess;
  if (shape.block == 256 && shape.wpe == 0) return launch_c<true>(l, colour, ntiles, qmax, wide, stream);
  if (colour == 0) return wide ? launch_shape<0, true>(l, ntiles, shape, stream) : launch_shape<0, false>(l, ntiles, shape, stream);
  return wide ? launch_shape<1, true>(l, ntiles, shape, stream) : launch_shape<1, false>(l, ntiles, shape, stream);
}

hipError_t launch_set_desc(StripParams *d, const StripParams &p, hipStream_t stream) {
  hipLaunchKernelGGL(set_desc_kernel, dim3(1), dim3(64), 0, stream, d, p);
  return hipGetLastError();
}

hipError_t launch_fold_advance(StripParams *d, uint32_t sweeps, hipStream_t stream) {
  hipLaunchKernelGGL(fold_advance_kernel, dim3(1), dim3(kBlock), 0, stream, d, sweeps);
  return hipGetLastError();
}

hipError_t launch_pack(const uint8_t *row_major, uint8_t *packed, uint32_t L, hipStream_t stream) {
  const uint64_t n = (uint64_t)(L >> 5) * L;
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream, row_major,
                     packed, L);
  return hipGetLastError();
}

hipError_t launch_unpack(const uint8_t *packed, uint8_t *row_major, uint32_t L, hipStream_t stream) {
  const uint64_t n = (uint64_t)(L >> 5) * L;
  hipLaunchKernelGGL(unpack_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream, packed,
                     row_major, L);
  return hipGetLastError();
}

}  // namespace potts
