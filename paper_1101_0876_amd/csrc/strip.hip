// strip.hip -- the main gfx950 half-sweep kernel (L % 16 == 0).
//
// Work item: a 16-byte-wide column strip of R consecutive rows (R even).  A
// lane walks down its strip one row at a time, so each row is loaded once and
// its bytes serve three times: as the active row, and as the up and down
// neighbours of the rows around it.  Rows alternate between the two byte
// parities, so the loop is unrolled by two and the parity is a compile-time
// constant in each half (no per-lane selects).
//
// The per-row update itself is in sweep_row.hpp.
//
// Each pass counts the final values of the sites it updates into the
// population histogram (lane-private LDS columns), which spreads that work
// over both passes; the colour-1 pass, which sees every site's final value,
// also counts the satisfied bonds (sum over colour-1 sites of equal
// neighbours).  Each workgroup then adds its totals to the sweep's record with
// one 64-bit atomic per bin.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"
#include "sweep_row.hpp"

namespace potts {
namespace {

constexpr int kBlock = 256;

using namespace row;

struct Carry {
  uint32_t s_lo, s_hi;  // active bytes of the current row
  uint32_t p_lo, p_hi;  // passive bytes of the current row
  uint32_t u_lo, u_hi;  // bytes of the row above at the active offset
};

struct Sums {
  uint32_t nz;     // differing neighbours of colour-1 sites (energy)
  uint32_t sites;  // colour-1 sites seen
};

// One row at byte offset ro (next row at rn).  O = (colour + y) & 1 is the
// byte offset of the active sites inside every dword; side_col is the column
// of the dword holding the one horizontal neighbour outside the strip.
template <int COLOUR, int O, int CMP, bool PRIV, bool WIDE>
__device__ __forceinline__ void do_row(const StripParams &p, const PhiloxHead &h,
                                       __amdgpu_buffer_rsrc_t rs, const uint8_t *table, uint8_t *hist,
                                       uint32_t lane_off, uint32_t ro, uint32_t rn, uint32_t col,
                                       uint32_t side_col, uint32_t ctr, Carry &cy, Sums &sums) {
  const u32x4 nxt = load16(rs, rn + col);
  const uint32_t side = load4(rs, ro + side_col);
  const uint32_t d_lo = perm(nxt.y, nxt.x, kSel<O>), d_hi = perm(nxt.w, nxt.z, kSel<O>);
  const Row8 r = update8<COLOUR, O, CMP, WIDE>(cy.s_lo, cy.s_hi, cy.p_lo, cy.p_hi, cy.u_lo, cy.u_hi,
                                               d_lo, d_hi, side, ctr, h, p.q, table);
  store16(rs, ro + col, r.out);
  if (COLOUR == 1) {
    sums.nz += __popc(r.nz_lo & 0xF0F0F0F0u) + __popc(r.nz_hi & 0xF0F0F0F0u);
    sums.sites += 8;
  }
  if (PRIV)
    count_active_private(hist, lane_off, r.ns_lo, r.ns_hi);
  else
    count_active_shared(reinterpret_cast<uint32_t *>(hist), r.ns_lo, r.ns_hi);
  // the row below becomes current: its active bytes sit at the other offset,
  // its passive bytes are exactly d; this row's passive bytes are the next "up"
  cy.u_lo = cy.p_lo;
  cy.u_hi = cy.p_hi;
  cy.p_lo = d_lo;
  cy.p_hi = d_hi;
  cy.s_lo = perm(nxt.y, nxt.x, kSel<O ^ 1>);
  cy.s_hi = perm(nxt.w, nxt.z, kSel<O ^ 1>);
}

// TILED: workgroup -> (job, item range) from the tile table (batched
// lattices); otherwise the single descriptor in the kernel arguments with a
// grid-stride loop.  Two instantiations keep the descriptor in scalar
// registers in both cases.
template <int COLOUR, int CMP, bool PRIV, bool WIDE, bool TILED, int BLOCK>
__device__ __forceinline__ void strip_body(const StripLaunch &launch) {
  constexpr int kWaves = BLOCK / 64;
  // acceptance table in static LDS, so its address folds into the ds_read offset
  __shared__ __align__(16) uint32_t table_words[512];
  // colour 1 walks the lattice bottom-up, so it starts on the rows colour 0
  // wrote last (still in the memory-side cache), and the next colour 0 starts
  // on the rows colour 1 wrote last
  const uint32_t bid = COLOUR == 1 ? gridDim.x - 1 - blockIdx.x : blockIdx.x;
  const StripTile tile = TILED ? launch.tiles[bid] : StripTile{0, 0, 0, 0};
  const StripParams &p = TILED ? launch.jobs[tile.job] : launch.single;
  const uint32_t first = TILED ? tile.first + threadIdx.x : bid * BLOCK + threadIdx.x;
  const uint32_t end = TILED ? tile.first + tile.count : p.nitems;
  const uint32_t stride = TILED ? (uint32_t)BLOCK : gridDim.x * BLOCK;
  const bool lead = TILED ? tile.lead != 0 : bid == 0;
  if (launch.sweep >= p.nsweeps) return;  // the whole workgroup: this job is done
  const uint64_t t = p.t0 + launch.sweep;
  const PhiloxHead h = philox_head((uint32_t)t, (uint32_t)(t >> 32), (uint32_t)COLOUR, p.k0, p.k1);

  // population counters (PRIV: q x 64 lane columns; else q bins) and totals
  // (q bins, then the bond sum), static so that their addresses fold into
  // the LDS instructions' offsets
  constexpr uint32_t kHistWords = PRIV ? 64u * (CMP == 0 ? 16u : kPrivateHistMaxQ) : 256u;
  __shared__ __align__(16) uint32_t hist[kHistWords];
  __shared__ uint32_t partial[257];
  uint8_t *table = reinterpret_cast<uint8_t *>(table_words);  // 2 KB
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
    // the previous launched sweep's partial records, complete now
    __shared__ unsigned long long fold_acc[COLOUR == 0 ? 257 : 1];
    if (COLOUR == 0 && lead && launch.sweep > 0) fold_stripes<BLOCK>(p, t - 1, fold_acc);
  } else if (COLOUR == 1 && lead) {
    // the slot of sweep t+1, zeroed before the next colour-0 launch starts
    unsigned long long *rec_next = p.ring + ((t + 1) & (p.cap - 1)) * (uint64_t)(q + 1);
    for (uint32_t i = threadIdx.x; i < q + 1; i += BLOCK) rec_next[i] = 0;
  }
  __syncthreads();

  const __amdgpu_buffer_rsrc_t rs = lattice_rsrc(p.spins);
  uint8_t *hist_bytes = reinterpret_cast<uint8_t *>(hist);
  const uint32_t lane_off = lane * 4u;
  const uint32_t L = p.L;
  const uint32_t rows = p.rows;
  Sums sums{0, 0};

  for (uint32_t item = first; item < end; item += stride) {
    const uint32_t rb = p.item_shift >= 0 ? item >> p.item_shift
                                          : (uint32_t)__umul64hi((uint64_t)item, p.item_magic);
    const uint32_t xi = item - rb * p.ipr;
    const uint32_t col = xi * 16u;
    const uint32_t left_col = col == 0 ? L - 4 : col - 4;       // dword left of the strip
    const uint32_t right_col = col + 16 == L ? 0u : col + 16;   // dword right of the strip
    const uint32_t r0 = rb * rows;  // even (as is y0), so row r0 has active offset COLOUR
    const uint32_t rp = (r0 == 0 ? p.up_row : p.first_row + r0 - 1) * L;
    const uint32_t last_next = (r0 + rows == p.nrows ? p.down_row : p.first_row + r0 + rows) * L;
    uint32_t ro = (p.first_row + r0) * L;
    const u32x4 prev = load16(rs, rp + col);
    const u32x4 cur = load16(rs, ro + col);
    Carry cy;
    cy.s_lo = perm(cur.y, cur.x, kSel<COLOUR>);
    cy.s_hi = perm(cur.w, cur.z, kSel<COLOUR>);
    cy.p_lo = perm(cur.y, cur.x, kSel<COLOUR ^ 1>);
    cy.p_hi = perm(cur.w, cur.z, kSel<COLOUR ^ 1>);
    cy.u_lo = perm(prev.y, prev.x, kSel<COLOUR>);
    cy.u_hi = perm(prev.w, prev.z, kSel<COLOUR>);
    uint32_t ctr = p.ctr0 + r0 * p.row_words + xi * 4u;
    constexpr uint32_t kSideA = COLOUR == 0 ? 0 : 1;  // row parity 0: side dword on the left
    for (uint32_t k = 0; k < rows; k += 2) {
      do_row<COLOUR, COLOUR, CMP, PRIV, WIDE>(p, h, rs, table, hist_bytes, lane_off, ro,
                                              ro + L, col, kSideA ? right_col : left_col, ctr, cy, sums);
      ro += L;
      ctr += p.row_words;
      const uint32_t rn = k + 2 == rows ? last_next : ro + L;
      do_row<COLOUR, COLOUR ^ 1, CMP, PRIV, WIDE>(p, h, rs, table, hist_bytes, lane_off, ro,
                                                  rn, col, kSideA ? left_col : right_col, ctr, cy, sums);
      ro += L;
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
__global__ __launch_bounds__(BLOCK) void strip_kernel(StripLaunch launch) {
  strip_body<COLOUR, CMP, PRIV, WIDE, TILED, BLOCK>(launch);
}

template <int COLOUR, int CMP, bool PRIV, bool WIDE, bool TILED, int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8))) void strip_kernel_w8(
    StripLaunch launch) {
  strip_body<COLOUR, CMP, PRIV, WIDE, TILED, BLOCK>(launch);
}

__global__ __launch_bounds__(kBlock) void fold_kernel(StripParams p, uint64_t t) {
  __shared__ unsigned long long acc[257];
  fold_stripes<kBlock>(p, t, acc);
}

template <int COLOUR, int CMP, bool PRIV, bool WIDE>
hipError_t launch_t(const StripLaunch &l, unsigned grid, size_t lds, hipStream_t stream) {
  if (l.tiles)
    hipLaunchKernelGGL((strip_kernel<COLOUR, CMP, PRIV, WIDE, true, kBlock>), dim3(grid), dim3(kBlock), lds, stream, l);
  else
    hipLaunchKernelGGL((strip_kernel<COLOUR, CMP, PRIV, WIDE, false, kBlock>), dim3(grid), dim3(kBlock), lds, stream, l);
  return hipGetLastError();
}

// Tiled launches of q <= 16 in the tuner's other shapes.
template <int COLOUR, bool WIDE>
hipError_t launch_shape(const StripLaunch &l, unsigned ntiles, const TileShape &shape, hipStream_t stream) {
  if (shape.block == 128) {
    if (shape.wpe)
      hipLaunchKernelGGL((strip_kernel_w8<COLOUR, 0, true, WIDE, true, 128>), dim3(ntiles), dim3(128), 0, stream, l);
    else
      hipLaunchKernelGGL((strip_kernel<COLOUR, 0, true, WIDE, true, 128>), dim3(ntiles), dim3(128), 0, stream, l);
  } else {
    hipLaunchKernelGGL((strip_kernel_w8<COLOUR, 0, true, WIDE, true, 256>), dim3(ntiles), dim3(256), 0, stream, l);
  }
  return hipGetLastError();
}

template <int COLOUR, bool WIDE>
hipError_t launch_w(const StripLaunch &l, unsigned grid, uint32_t q, size_t lds, hipStream_t stream) {
  if (q <= 16) return launch_t<COLOUR, 0, true, WIDE>(l, grid, lds, stream);
  if (q <= kPrivateHistMaxQ) return launch_t<COLOUR, 1, true, WIDE>(l, grid, lds, stream);
  if (q <= 128) return launch_t<COLOUR, 1, false, WIDE>(l, grid, lds, stream);
  return launch_t<COLOUR, 2, false, WIDE>(l, grid, lds, stream);
}

template <int COLOUR>
hipError_t launch_c(const StripLaunch &l, unsigned grid, uint32_t q, bool wide, size_t lds,
                    hipStream_t stream) {
  return wide ? launch_w<COLOUR, true>(l, grid, q, lds, stream) : launch_w<COLOUR, false>(l, grid, q, lds, stream);
}

}  // namespace

hipError_t launch_fold_stripes(const StripParams &p, uint64_t t, hipStream_t stream) {
  hipLaunchKernelGGL(fold_kernel, dim3(1), dim3(kBlock), 0, stream, p, t);
  return hipGetLastError();
}

hipError_t launch_strip(const StripLaunch &l, int colour, unsigned grid, uint32_t max_q, bool wide,
                        hipStream_t stream) {
  if (grid == 0) return hipSuccess;
  return colour == 0 ? launch_c<0>(l, grid, max_q, wide, 0, stream)
                     : launch_c<1>(l, grid, max_q, wide, 0, stream);
}

hipError_t launch_strip_tiled(const StripLaunch &l, int colour, unsigned ntiles, const TileShape &shape,
                              uint32_t max_q, bool wide, hipStream_t stream) {
  if (!shape_ok(shape, max_q) || !l.tiles) return hipErrorInvalidValue;
  if (ntiles == 0) return hipSuccess;
  if (shape.block == 256 && shape.wpe == 0) return launch_strip(l, colour, ntiles, max_q, wide, stream);
  if (colour == 0) return wide ? launch_shape<0, true>(l, ntiles, shape, stream) : launch_shape<0, false>(l, ntiles, shape, stream);
  return wide ? launch_shape<1, true>(l, ntiles, shape, stream) : launch_shape<1, false>(l, ntiles, shape, stream);
}

}  // namespace potts
