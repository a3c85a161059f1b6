// strip.hip -- the main gfx950 half-sweep kernel (L % 16 == 0).
//
// Work item: a 16-byte-wide column strip of R consecutive rows (R even).  A
// lane walks down its strip one row at a time, so each row is loaded once and
// its bytes serve three times: as the active row, and as the up and down
// neighbours of the rows around it.  Rows alternate between the two byte
// parities, so the loop is unrolled by two and the parity is a compile-time
// constant in each half (no per-lane selects).
//
// Per row, 8 active sites: four Philox4x32-10 blocks (one per 4-byte chunk, see
// device.hpp), the active and passive bytes packed into dwords with v_perm, the
// four neighbour comparisons of four sites at once as byte-wise flag patterns
// (bits 7..4 of each byte; v_xad + v_bitop3), and one LDS acceptance-table read
// plus one 64-bit compare per site.  The kernel updates one colour in place:
// the other colour's bytes are only read, and are written back unchanged.
//
// The colour-1 pass sees every site's final value of the sweep, so it alone
// accumulates the population histogram (lane-private LDS columns) and the
// number of satisfied bonds (sum over colour-1 sites of equal neighbours);
// each workgroup then adds its totals to the sweep's record with one 64-bit
// atomic per bin.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"

namespace potts {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

// (m & a) | (~m & b) as one v_bitop3_b32 (truth table 0xCA)
__device__ __forceinline__ uint32_t bfi(uint32_t m, uint32_t a, uint32_t b) {
  return __builtin_amdgcn_bitop3_b32(m, a, b, 0xCA);
}

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

__device__ __forceinline__ uint32_t alignbyte(uint32_t hi, uint32_t lo, uint32_t shift) {
  return __builtin_amdgcn_alignbyte(hi, lo, shift);
}

// selector of the bytes at offset o and o+2 of two dwords (lo dword first)
template <int O>
constexpr uint32_t kSel = 0x06040200u + (uint32_t)O * 0x01010101u;

// Byte-wise "differs from v" flags against the four neighbour dwords, at bits
// 7 (a), 6 (b), 5 (c), 4 (d) of every byte; bits 3..0 are garbage.
//   CMP 0 (q <= 16):  x = nb ^ v < 16, so x + 0x7F/0x3F/0x1F/0x0F sets exactly
//                     bit 7/6/5/4 when x != 0 and never carries above it
//   CMP 1 (q <= 128): x < 128, x + 0x7F flags bit 7; shifted into place
//   CMP 2 (q <= 256): exact zero-byte test, then shifted into place
template <int CMP>
__device__ __forceinline__ uint32_t diff_pattern(uint32_t v, uint32_t a, uint32_t b, uint32_t c,
                                                 uint32_t d) {
  if (CMP == 0) {
    const uint32_t fa = (a ^ v) + 0x7F7F7F7Fu;
    const uint32_t fb = (b ^ v) + 0x3F3F3F3Fu;
    const uint32_t fc = (c ^ v) + 0x1F1F1F1Fu;
    const uint32_t fd = (d ^ v) + 0x0F0F0F0Fu;
    return bfi(0xE0E0E0E0u, bfi(0xC0C0C0C0u, bfi(0x80808080u, fa, fb), fc), fd);
  } else {
    const uint32_t nb[4] = {a, b, c, d};
    uint32_t f[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t x = nb[i] ^ v;
      f[i] = CMP == 1 ? x + 0x7F7F7F7Fu : (((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x);
    }
    return bfi(0xE0E0E0E0u, bfi(0xC0C0C0C0u, bfi(0x80808080u, f[0], f[1] >> 1), f[2] >> 2), f[3] >> 3);
  }
}

struct Carry {
  uint32_t s_lo, s_hi;  // active bytes of the current row
  uint32_t p_lo, p_hi;  // passive bytes of the current row
  uint32_t u_lo, u_hi;  // bytes of the row above at the active offset
};

struct Sums {
  uint32_t nz;     // differing neighbours of colour-1 sites (energy)
  uint32_t sites;  // colour-1 sites seen
};

// One row: y is the row index, O = (colour + y) & 1 is the byte offset of the
// active sites inside every dword.
template <int COLOUR, int O, int CMP, bool PRIV>
__device__ __forceinline__ void do_row(const StripParams &p, const uint64_t *table, uint8_t *hist_base,
                                       uint32_t lane_off, uint32_t y, uint32_t col, uint32_t ctr,
                                       Carry &cy, Sums &sums) {
  const uint32_t L = p.L;
  const uint32_t ro = y * L;
  const uint32_t rn = y + 1 == L ? 0u : ro + L;
  const uint4 nxt = *reinterpret_cast<const uint4 *>(p.spins + rn + col);
  uint32_t side;
  if (O == 0)  // left neighbour of the first site: byte 3 of the dword before
    side = *reinterpret_cast<const uint32_t *>(p.spins + ro + (col == 0 ? L - 4 : col - 4));
  else  // right neighbour of the last site: byte 0 of the dword after
    side = *reinterpret_cast<const uint32_t *>(p.spins + ro + (col + 16 == L ? 0u : col + 16));

  const uint32_t d_lo = perm(nxt.y, nxt.x, kSel<O>), d_hi = perm(nxt.w, nxt.z, kSel<O>);
  const uint32_t x_lo = O == 0 ? alignbyte(cy.p_lo, side, 3) : alignbyte(cy.p_hi, cy.p_lo, 1);
  const uint32_t x_hi = O == 0 ? alignbyte(cy.p_hi, cy.p_lo, 3) : alignbyte(side, cy.p_hi, 1);

  const Words b0 = philox4x32_10(ctr + 0, p.t_lo, p.t_hi, (uint32_t)COLOUR, p.k0, p.k1);
  const Words b1 = philox4x32_10(ctr + 1, p.t_lo, p.t_hi, (uint32_t)COLOUR, p.k0, p.k1);
  const Words b2 = philox4x32_10(ctr + 2, p.t_lo, p.t_hi, (uint32_t)COLOUR, p.k0, p.k1);
  const Words b3 = philox4x32_10(ctr + 3, p.t_lo, p.t_hi, (uint32_t)COLOUR, p.k0, p.k1);
  const uint32_t q = p.q;
  const uint32_t k_lo = scale_to_q(b0.w0, q) | (scale_to_q(b0.w2, q) << 8) |
                        (scale_to_q(b1.w0, q) << 16) | (scale_to_q(b1.w2, q) << 24);
  const uint32_t k_hi = scale_to_q(b2.w0, q) | (scale_to_q(b2.w2, q) << 8) |
                        (scale_to_q(b3.w0, q) << 16) | (scale_to_q(b3.w2, q) << 24);
  const uint32_t acc_w[8] = {b0.w1, b0.w3, b1.w1, b1.w3, b2.w1, b2.w3, b3.w1, b3.w3};

  const uint32_t ps_lo = diff_pattern<CMP>(cy.s_lo, cy.u_lo, d_lo, cy.p_lo, x_lo);
  const uint32_t ps_hi = diff_pattern<CMP>(cy.s_hi, cy.u_hi, d_hi, cy.p_hi, x_hi);
  const uint32_t pk_lo = diff_pattern<CMP>(k_lo, cy.u_lo, d_lo, cy.p_lo, x_lo);
  const uint32_t pk_hi = diff_pattern<CMP>(k_hi, cy.u_hi, d_hi, cy.p_hi, x_hi);
  const uint32_t idx_lo = bfi(0xF0F0F0F0u, pk_lo, ps_lo >> 4);
  const uint32_t idx_hi = bfi(0xF0F0F0F0u, pk_hi, ps_hi >> 4);

  uint32_t sel_lo = 0x03020100u, sel_hi = 0x03020100u;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint64_t t_lo = table[(idx_lo >> (8 * j)) & 0xFFu];
    const uint64_t t_hi = table[(idx_hi >> (8 * j)) & 0xFFu];
    if ((uint64_t)acc_w[j] < t_lo) sel_lo |= 4u << (8 * j);
    if ((uint64_t)acc_w[4 + j] < t_hi) sel_hi |= 4u << (8 * j);
  }
  const uint32_t ns_lo = perm(k_lo, cy.s_lo, sel_lo);
  const uint32_t ns_hi = perm(k_hi, cy.s_hi, sel_hi);
  // interleave the new active bytes with the unchanged passive ones
  constexpr uint32_t sel_w0 = O ? 0x05010400u : 0x01050004u;
  constexpr uint32_t sel_w1 = O ? 0x07030602u : 0x03070206u;
  uint4 out;
  out.x = perm(ns_lo, cy.p_lo, sel_w0);
  out.y = perm(ns_lo, cy.p_lo, sel_w1);
  out.z = perm(ns_hi, cy.p_hi, sel_w0);
  out.w = perm(ns_hi, cy.p_hi, sel_w1);
  *reinterpret_cast<uint4 *>(p.spins + ro + col) = out;

  if (COLOUR == 1) {
    sums.nz += __popc(perm(pk_lo, ps_lo, sel_lo) & 0xF0F0F0F0u) +
               __popc(perm(pk_hi, ps_hi, sel_hi) & 0xF0F0F0F0u);
    sums.sites += 8;
    const uint32_t words[4] = {out.x, out.y, out.z, out.w};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if (PRIV) {
          // byte address (value << 8) | lane*4 of this lane's counter, one v_perm
          const uint32_t addr = perm(words[m], lane_off, 0x0C0C0000u | ((4u + b) << 8));
          atomicAdd(reinterpret_cast<uint32_t *>(hist_base + addr), 1u);
        } else {
          atomicAdd(reinterpret_cast<uint32_t *>(hist_base) + ((words[m] >> (8 * b)) & 0xFFu), 1u);
        }
      }
    }
  }

  // the row below becomes current: its active bytes at the other offset, its
  // passive bytes are exactly d; this row's passive bytes are the next "up"
  cy.u_lo = cy.p_lo;
  cy.u_hi = cy.p_hi;
  cy.p_lo = d_lo;
  cy.p_hi = d_hi;
  cy.s_lo = perm(nxt.y, nxt.x, kSel<O ^ 1>);
  cy.s_hi = perm(nxt.w, nxt.z, kSel<O ^ 1>);
}

__device__ __forceinline__ void fill_accept_table(uint64_t *table, const Thresholds &thr) {
  // entry (k_pattern << 4 | s_pattern): dE = popcount(k_pattern) - popcount(s_pattern)
  for (uint32_t i = threadIdx.x; i < 256; i += kBlock) {
    const int de = __popc(i >> 4) - __popc(i & 15u);
    table[i] = de <= 0 ? (1ull << 32)
                       : (uint64_t)(de == 1 ? thr.v[0] : de == 2 ? thr.v[1] : de == 3 ? thr.v[2] : thr.v[3]);
  }
}

template <int COLOUR, int CMP, bool PRIV>
__global__ __launch_bounds__(kBlock) void strip_kernel(StripParams p) {
  extern __shared__ uint32_t lds[];
  uint64_t *table = reinterpret_cast<uint64_t *>(lds);  // 256 x u64
  uint32_t *hist = lds + 512;  // PRIV: kWaves regions of q x 64 lane columns; else q bins
  const uint32_t q = p.q;
  uint32_t *partial = hist + (PRIV ? kWaves * 64 * q : q);  // kWaves x q, then the bond sum
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = threadIdx.x >> 6;

  fill_accept_table(table, p.thr);
  if (COLOUR == 1) {
    const uint32_t nh = PRIV ? kWaves * 64 * q : q;
    for (uint32_t i = threadIdx.x; i < nh; i += kBlock) hist[i] = 0;
    if (threadIdx.x == 0) partial[kWaves * q] = 0;
    if (blockIdx.x == 0 && p.rec_clear)
      for (uint32_t i = threadIdx.x; i < q + 1; i += kBlock) p.rec_clear[i] = 0;
  }
  __syncthreads();

  uint8_t *hist_base = reinterpret_cast<uint8_t *>(hist + (PRIV ? wave * 64u * q : 0u));
  const uint32_t lane_off = lane * 4u;
  const uint32_t L = p.L;
  Sums sums{0, 0};

  for (uint32_t item = blockIdx.x * kBlock + threadIdx.x; item < p.nitems;
       item += gridDim.x * kBlock) {
    const uint32_t rb = p.item_shift >= 0 ? item >> p.item_shift
                                          : (uint32_t)__umul64hi((uint64_t)item, p.item_magic);
    const uint32_t xi = item - rb * p.ipr;
    const uint32_t col = xi * 16u;
    const uint32_t r0 = rb * p.rows;  // even, so row r0 has active offset COLOUR
    const uint32_t rp = (r0 == 0 ? L - 1 : r0 - 1) * L;
    const uint4 prev = *reinterpret_cast<const uint4 *>(p.spins + rp + col);
    const uint4 cur = *reinterpret_cast<const uint4 *>(p.spins + r0 * L + col);
    Carry cy;
    cy.s_lo = perm(cur.y, cur.x, kSel<COLOUR>);
    cy.s_hi = perm(cur.w, cur.z, kSel<COLOUR>);
    cy.p_lo = perm(cur.y, cur.x, kSel<COLOUR ^ 1>);
    cy.p_hi = perm(cur.w, cur.z, kSel<COLOUR ^ 1>);
    cy.u_lo = perm(prev.y, prev.x, kSel<COLOUR>);
    cy.u_hi = perm(prev.w, prev.z, kSel<COLOUR>);
    uint32_t ctr = r0 * p.row_words + xi * 4u;
    for (uint32_t k = 0; k < p.rows; k += 2) {
      do_row<COLOUR, COLOUR, CMP, PRIV>(p, table, hist_base, lane_off, r0 + k, col, ctr, cy, sums);
      ctr += p.row_words;
      do_row<COLOUR, COLOUR ^ 1, CMP, PRIV>(p, table, hist_base, lane_off, r0 + k + 1, col, ctr, cy,
                                            sums);
      ctr += p.row_words;
    }
  }

  if (COLOUR == 1) {
    uint32_t *esum = partial + kWaves * q;
    const uint32_t e = wave_sum(4u * sums.sites - sums.nz);
    if (lane == 0 && e) atomicAdd(esum, e);
    __syncthreads();
    if (PRIV) {
      const uint32_t *mine = hist + wave * 64u * q;
      for (uint32_t v = 0; v < q; ++v) {
        const uint32_t s = wave_sum(mine[v * 64u + lane]);
        if (lane == 0) partial[wave * q + v] = s;
      }
      __syncthreads();
    }
    for (uint32_t v = threadIdx.x; v < q; v += kBlock) {
      uint32_t s = 0;
      if (PRIV) {
        for (int w = 0; w < kWaves; ++w) s += partial[w * q + v];
      } else {
        s = hist[v];
      }
      if (s) atomicAdd(&p.rec[1 + v], (unsigned long long)s);
    }
    if (threadIdx.x == 0 && *esum) atomicAdd(&p.rec[0], (unsigned long long)*esum);
  }
}

template <int COLOUR, int CMP, bool PRIV>
hipError_t launch_t(const StripParams &p, unsigned grid, size_t lds, hipStream_t stream) {
  hipLaunchKernelGGL((strip_kernel<COLOUR, CMP, PRIV>), dim3(grid), dim3(kBlock), lds, stream, p);
  return hipGetLastError();
}

template <int COLOUR>
hipError_t launch_c(const StripParams &p, unsigned grid, size_t lds, hipStream_t stream) {
  const bool priv = p.q <= kPrivateHistMaxQ;
  if (p.q <= 16)
    return priv ? launch_t<COLOUR, 0, true>(p, grid, lds, stream) : launch_t<COLOUR, 0, false>(p, grid, lds, stream);
  if (p.q <= 128)
    return priv ? launch_t<COLOUR, 1, true>(p, grid, lds, stream) : launch_t<COLOUR, 1, false>(p, grid, lds, stream);
  return launch_t<COLOUR, 2, false>(p, grid, lds, stream);
}

}  // namespace

size_t strip_lds_bytes(uint32_t q, int colour) {
  if (colour == 0) return 256 * 8;  // acceptance table only
  const bool priv = q <= kPrivateHistMaxQ;
  const size_t hist_words = priv ? (size_t)kWaves * 64 * q : q;
  return 256 * 8 + hist_words * 4 + ((size_t)kWaves * q + 1) * 4;
}

hipError_t launch_strip(const StripParams &p, int colour, unsigned max_groups, hipStream_t stream) {
  const uint64_t need = ((uint64_t)p.nitems + kBlock - 1) / kBlock;
  const unsigned grid = (unsigned)(need < max_groups ? (need ? need : 1) : max_groups);
  const size_t lds = strip_lds_bytes(p.q, colour);
  return colour == 0 ? launch_c<0>(p, grid, lds, stream) : launch_c<1>(p, grid, lds, stream);
}

}  // namespace potts
