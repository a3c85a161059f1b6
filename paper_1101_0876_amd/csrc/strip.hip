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

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Raw buffer access with 32-bit byte offsets (lattices below 2^32 bytes): no
// 64-bit address arithmetic per load.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t lattice_rsrc(uint8_t *spins) {
  return __builtin_amdgcn_make_buffer_rsrc(spins, 0, (int)0xFFFFFFFFu, 0x00020000);
}
__device__ __forceinline__ u32x4 load16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
}
__device__ __forceinline__ uint32_t load4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}
__device__ __forceinline__ void store16(__amdgpu_buffer_rsrc_t r, uint32_t off, u32x4 v) {
  __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, 0);
}

// Byte J of idx, scaled to a table offset (idx.byte_J << SHIFT), in one SDWA op.
template <int J, int SHIFT>
__device__ __forceinline__ uint32_t table_offset(uint32_t idx) {
  uint32_t r;
  if (J == 0)
    asm("v_lshlrev_b32_sdwa %0, %2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0" : "=v"(r) : "v"(idx), "n"(SHIFT));
  else if (J == 1)
    asm("v_lshlrev_b32_sdwa %0, %2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1" : "=v"(r) : "v"(idx), "n"(SHIFT));
  else if (J == 2)
    asm("v_lshlrev_b32_sdwa %0, %2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2" : "=v"(r) : "v"(idx), "n"(SHIFT));
  else
    asm("v_lshlrev_b32_sdwa %0, %2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3" : "=v"(r) : "v"(idx), "n"(SHIFT));
  return r;
}

// dst.byte_J = (w <= t) ? if_acc.byte_J : if_rej.byte_J, other bytes of dst
// kept: one v_cmp and one SDWA v_cndmask.
template <int J>
__device__ __forceinline__ void accept_byte(uint32_t &dst, uint32_t w, uint32_t t, uint32_t if_rej,
                                            uint32_t if_acc) {
  if (J == 0)
    asm("v_cmp_le_u32 vcc, %1, %2\n\tv_cndmask_b32_sdwa %0, %3, %4, vcc dst_sel:BYTE_0 dst_unused:UNUSED_PRESERVE src0_sel:BYTE_0 src1_sel:BYTE_0"
        : "+v"(dst) : "v"(w), "v"(t), "v"(if_rej), "v"(if_acc) : "vcc");
  else if (J == 1)
    asm("v_cmp_le_u32 vcc, %1, %2\n\tv_cndmask_b32_sdwa %0, %3, %4, vcc dst_sel:BYTE_1 dst_unused:UNUSED_PRESERVE src0_sel:BYTE_1 src1_sel:BYTE_1"
        : "+v"(dst) : "v"(w), "v"(t), "v"(if_rej), "v"(if_acc) : "vcc");
  else if (J == 2)
    asm("v_cmp_le_u32 vcc, %1, %2\n\tv_cndmask_b32_sdwa %0, %3, %4, vcc dst_sel:BYTE_2 dst_unused:UNUSED_PRESERVE src0_sel:BYTE_2 src1_sel:BYTE_2"
        : "+v"(dst) : "v"(w), "v"(t), "v"(if_rej), "v"(if_acc) : "vcc");
  else
    asm("v_cmp_le_u32 vcc, %1, %2\n\tv_cndmask_b32_sdwa %0, %3, %4, vcc dst_sel:BYTE_3 dst_unused:UNUSED_PRESERVE src0_sel:BYTE_3 src1_sel:BYTE_3"
        : "+v"(dst) : "v"(w), "v"(t), "v"(if_rej), "v"(if_acc) : "vcc");
}

// As accept_byte, selecting byte J of two pairs with one compare.
#define POTTS_ACCEPT2(J)                                                                        \
  asm("v_cmp_le_u32 vcc, %2, %3\n\t"                                                           \
      "v_cndmask_b32_sdwa %0, %4, %5, vcc dst_sel:BYTE_" #J                                     \
      " dst_unused:UNUSED_PRESERVE src0_sel:BYTE_" #J " src1_sel:BYTE_" #J "\n\t"              \
      "v_cndmask_b32_sdwa %1, %6, %7, vcc dst_sel:BYTE_" #J                                     \
      " dst_unused:UNUSED_PRESERVE src0_sel:BYTE_" #J " src1_sel:BYTE_" #J                      \
      : "+v"(dst1), "+v"(dst2)                                                                  \
      : "v"(w), "v"(t), "v"(rej1), "v"(acc1), "v"(rej2), "v"(acc2)                              \
      : "vcc")
template <int J>
__device__ __forceinline__ void accept_byte2(uint32_t &dst1, uint32_t &dst2, uint32_t w, uint32_t t,
                                             uint32_t rej1, uint32_t acc1, uint32_t rej2, uint32_t acc2) {
  if (J == 0) POTTS_ACCEPT2(0);
  else if (J == 1) POTTS_ACCEPT2(1);
  else if (J == 2) POTTS_ACCEPT2(2);
  else POTTS_ACCEPT2(3);
}
#undef POTTS_ACCEPT2

// Four 8-bit values (each < 256) packed into one dword, a in byte 0.
__device__ __forceinline__ uint32_t pack4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  return perm(b, a, 0x0C0C0400u) | perm(d, c, 0x04000C0Cu);
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

// One row at byte offset ro (next row at rn).  O = (colour + y) & 1 is the
// byte offset of the active sites inside every dword; side_col is the column
// of the dword holding the one horizontal neighbour outside the strip.
//
// Acceptance table in LDS, indexed by (proposal pattern << 4 | current
// pattern): narrow form (all thresholds >= 1) holds thr[dE-1] - 1, or
// 2^32 - 1 when dE <= 0, and a move is accepted iff w <= entry; the wide form
// (some threshold is 0) holds thr[dE-1], or 2^32, as u64 and accepts iff w < entry.
template <int COLOUR, int O, int CMP, bool PRIV, bool WIDE>
__device__ __forceinline__ void do_row(const StripParams &p, __amdgpu_buffer_rsrc_t rs,
                                       const uint8_t *table, uint8_t *hist, uint32_t lane_off,
                                       uint32_t ro, uint32_t rn, uint32_t col, uint32_t side_col,
                                       uint32_t ctr, Carry &cy, Sums &sums) {
  const u32x4 nxt = load16(rs, rn + col);
  const uint32_t side = load4(rs, ro + side_col);

  const uint32_t d_lo = perm(nxt.y, nxt.x, kSel<O>), d_hi = perm(nxt.w, nxt.z, kSel<O>);
  // horizontal neighbours: one is the passive byte at the same packed index,
  // the other the passive byte one site over (left when O == 0, right when O == 1)
  const uint32_t x_lo = O == 0 ? alignbyte(cy.p_lo, side, 3) : alignbyte(cy.p_hi, cy.p_lo, 1);
  const uint32_t x_hi = O == 0 ? alignbyte(cy.p_hi, cy.p_lo, 3) : alignbyte(side, cy.p_hi, 1);

  // block m serves dword m: (w0, w1) for its site at byte O, (w2, w3) at byte O+2
  const Words b0 = philox4x32_10(ctr + 0, p.t_lo, p.t_hi, (uint32_t)COLOUR, p.k0, p.k1);
  const Words b1 = philox4x32_10(ctr + 1, p.t_lo, p.t_hi, (uint32_t)COLOUR, p.k0, p.k1);
  const Words b2 = philox4x32_10(ctr + 2, p.t_lo, p.t_hi, (uint32_t)COLOUR, p.k0, p.k1);
  const Words b3 = philox4x32_10(ctr + 3, p.t_lo, p.t_hi, (uint32_t)COLOUR, p.k0, p.k1);
  const uint32_t q = p.q;
  const uint32_t k_lo = pack4(scale_to_q(b0.w0, q), scale_to_q(b0.w2, q), scale_to_q(b1.w0, q), scale_to_q(b1.w2, q));
  const uint32_t k_hi = pack4(scale_to_q(b2.w0, q), scale_to_q(b2.w2, q), scale_to_q(b3.w0, q), scale_to_q(b3.w2, q));

  const uint32_t ps_lo = diff_pattern<CMP>(cy.s_lo, cy.u_lo, d_lo, cy.p_lo, x_lo);
  const uint32_t ps_hi = diff_pattern<CMP>(cy.s_hi, cy.u_hi, d_hi, cy.p_hi, x_hi);
  const uint32_t pk_lo = diff_pattern<CMP>(k_lo, cy.u_lo, d_lo, cy.p_lo, x_lo);
  const uint32_t pk_hi = diff_pattern<CMP>(k_hi, cy.u_hi, d_hi, cy.p_hi, x_hi);
  const uint32_t idx_lo = bfi(0xF0F0F0F0u, pk_lo, ps_lo >> 4);
  const uint32_t idx_hi = bfi(0xF0F0F0F0u, pk_hi, ps_hi >> 4);

  uint32_t ns_lo, ns_hi;  // new active bytes
  uint32_t nz_lo = 0, nz_hi = 0;  // colour 1: flag patterns of the new spins
  if (!WIDE) {
    const uint32_t *t32 = reinterpret_cast<const uint32_t *>(table);
#define POTTS_T(J, IDX) *reinterpret_cast<const uint32_t *>(table + table_offset<J, 2>(IDX))
    const uint32_t t0 = POTTS_T(0, idx_lo), t1 = POTTS_T(1, idx_lo), t2 = POTTS_T(2, idx_lo), t3 = POTTS_T(3, idx_lo);
    const uint32_t t4 = POTTS_T(0, idx_hi), t5 = POTTS_T(1, idx_hi), t6 = POTTS_T(2, idx_hi), t7 = POTTS_T(3, idx_hi);
#undef POTTS_T
    (void)t32;
    ns_lo = cy.s_lo;
    ns_hi = cy.s_hi;
    if (COLOUR == 0) {
      accept_byte<0>(ns_lo, b0.w1, t0, cy.s_lo, k_lo);
      accept_byte<1>(ns_lo, b0.w3, t1, cy.s_lo, k_lo);
      accept_byte<2>(ns_lo, b1.w1, t2, cy.s_lo, k_lo);
      accept_byte<3>(ns_lo, b1.w3, t3, cy.s_lo, k_lo);
      accept_byte<0>(ns_hi, b2.w1, t4, cy.s_hi, k_hi);
      accept_byte<1>(ns_hi, b2.w3, t5, cy.s_hi, k_hi);
      accept_byte<2>(ns_hi, b3.w1, t6, cy.s_hi, k_hi);
      accept_byte<3>(ns_hi, b3.w3, t7, cy.s_hi, k_hi);
    } else {
      nz_lo = ps_lo;
      nz_hi = ps_hi;
      accept_byte2<0>(ns_lo, nz_lo, b0.w1, t0, cy.s_lo, k_lo, ps_lo, pk_lo);
      accept_byte2<1>(ns_lo, nz_lo, b0.w3, t1, cy.s_lo, k_lo, ps_lo, pk_lo);
      accept_byte2<2>(ns_lo, nz_lo, b1.w1, t2, cy.s_lo, k_lo, ps_lo, pk_lo);
      accept_byte2<3>(ns_lo, nz_lo, b1.w3, t3, cy.s_lo, k_lo, ps_lo, pk_lo);
      accept_byte2<0>(ns_hi, nz_hi, b2.w1, t4, cy.s_hi, k_hi, ps_hi, pk_hi);
      accept_byte2<1>(ns_hi, nz_hi, b2.w3, t5, cy.s_hi, k_hi, ps_hi, pk_hi);
      accept_byte2<2>(ns_hi, nz_hi, b3.w1, t6, cy.s_hi, k_hi, ps_hi, pk_hi);
      accept_byte2<3>(ns_hi, nz_hi, b3.w3, t7, cy.s_hi, k_hi, ps_hi, pk_hi);
    }
  } else {
    const uint64_t *t64 = reinterpret_cast<const uint64_t *>(table);
    const uint32_t acc_w[8] = {b0.w1, b0.w3, b1.w1, b1.w3, b2.w1, b2.w3, b3.w1, b3.w3};
    uint32_t sel_lo = 0x03020100u, sel_hi = 0x03020100u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if ((uint64_t)acc_w[j] < t64[(idx_lo >> (8 * j)) & 0xFFu]) sel_lo |= 4u << (8 * j);
      if ((uint64_t)acc_w[4 + j] < t64[(idx_hi >> (8 * j)) & 0xFFu]) sel_hi |= 4u << (8 * j);
    }
    ns_lo = perm(k_lo, cy.s_lo, sel_lo);
    ns_hi = perm(k_hi, cy.s_hi, sel_hi);
    if (COLOUR == 1) {
      nz_lo = perm(pk_lo, ps_lo, sel_lo);
      nz_hi = perm(pk_hi, ps_hi, sel_hi);
    }
  }
  // interleave the new active bytes with the unchanged passive ones
  constexpr uint32_t sel_w0 = O ? 0x05010400u : 0x01050004u;
  constexpr uint32_t sel_w1 = O ? 0x07030602u : 0x03070206u;
  u32x4 out;
  out.x = perm(ns_lo, cy.p_lo, sel_w0);
  out.y = perm(ns_lo, cy.p_lo, sel_w1);
  out.z = perm(ns_hi, cy.p_hi, sel_w0);
  out.w = perm(ns_hi, cy.p_hi, sel_w1);
  store16(rs, ro + col, out);

  if (COLOUR == 1) {
    // differing neighbours of the new spins, 8 sites
    sums.nz += __popc(nz_lo & 0xF0F0F0F0u) + __popc(nz_hi & 0xF0F0F0F0u);
    sums.sites += 8;
    const uint32_t words[4] = {out.x, out.y, out.z, out.w};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if (PRIV) {
          // counter of (value, lane) at byte (value << 8) | lane*4: one v_perm;
          // the four waves share the lane columns (LDS atomics)
          const uint32_t addr = perm(words[m], lane_off, 0x0C0C0000u | ((4u + b) << 8));
          atomicAdd(reinterpret_cast<uint32_t *>(hist + addr), 1u);
        } else {
          atomicAdd(reinterpret_cast<uint32_t *>(hist) + ((words[m] >> (8 * b)) & 0xFFu), 1u);
        }
      }
    }
  }

  // the row below becomes current: its active bytes sit at the other offset,
  // its passive bytes are exactly d; this row's passive bytes are the next "up"
  cy.u_lo = cy.p_lo;
  cy.u_hi = cy.p_hi;
  cy.p_lo = d_lo;
  cy.p_hi = d_hi;
  cy.s_lo = perm(nxt.y, nxt.x, kSel<O ^ 1>);
  cy.s_hi = perm(nxt.w, nxt.z, kSel<O ^ 1>);
}

template <bool WIDE>
__device__ __forceinline__ void fill_accept_table(uint8_t *table, const Thresholds &thr) {
  // entry (k_pattern << 4 | s_pattern): dE = popcount(k_pattern) - popcount(s_pattern)
  for (uint32_t i = threadIdx.x; i < 256; i += kBlock) {
    const int de = __popc(i >> 4) - __popc(i & 15u);
    const uint32_t t = de == 1 ? thr.v[0] : de == 2 ? thr.v[1] : de == 3 ? thr.v[2] : thr.v[3];
    if (WIDE)
      reinterpret_cast<uint64_t *>(table)[i] = de <= 0 ? (1ull << 32) : (uint64_t)t;
    else
      reinterpret_cast<uint32_t *>(table)[i] = de <= 0 ? 0xFFFFFFFFu : t - 1u;
  }
}

template <int COLOUR, int CMP, bool PRIV, bool WIDE>
__global__ __launch_bounds__(kBlock) void strip_kernel(StripParams p) {
  // acceptance table in static LDS, so its address folds into the ds_read offset
  __shared__ __align__(16) uint32_t table_words[512];
  extern __shared__ uint32_t lds[];
  uint8_t *table = reinterpret_cast<uint8_t *>(table_words);  // 2 KB
  uint32_t *hist = lds;  // PRIV: q x 64 lane columns; else q bins
  const uint32_t q = p.q;
  uint32_t *partial = hist + (PRIV ? 64 * q : q);  // q totals, then the bond sum
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = threadIdx.x >> 6;

  fill_accept_table<WIDE>(table, p.thr);
  if (COLOUR == 1) {
    const uint32_t nh = PRIV ? 64 * q : q;
    for (uint32_t i = threadIdx.x; i < nh; i += kBlock) hist[i] = 0;
    if (threadIdx.x == 0) partial[q] = 0;
    if (blockIdx.x == 0 && p.rec_clear)
      for (uint32_t i = threadIdx.x; i < q + 1; i += kBlock) p.rec_clear[i] = 0;
  }
  __syncthreads();

  const __amdgpu_buffer_rsrc_t rs = lattice_rsrc(p.spins);
  uint8_t *hist_bytes = reinterpret_cast<uint8_t *>(hist);
  const uint32_t lane_off = lane * 4u;
  const uint32_t L = p.L;
  const uint32_t rows = p.rows;
  Sums sums{0, 0};

  for (uint32_t item = blockIdx.x * kBlock + threadIdx.x; item < p.nitems;
       item += gridDim.x * kBlock) {
    const uint32_t rb = p.item_shift >= 0 ? item >> p.item_shift
                                          : (uint32_t)__umul64hi((uint64_t)item, p.item_magic);
    const uint32_t xi = item - rb * p.ipr;
    const uint32_t col = xi * 16u;
    const uint32_t left_col = col == 0 ? L - 4 : col - 4;       // dword left of the strip
    const uint32_t right_col = col + 16 == L ? 0u : col + 16;   // dword right of the strip
    const uint32_t r0 = rb * rows;  // even, so row r0 has active offset COLOUR
    const uint32_t rp = (r0 == 0 ? L - 1 : r0 - 1) * L;
    const uint32_t last_next = r0 + rows == L ? 0u : (r0 + rows) * L;
    uint32_t ro = r0 * L;
    const u32x4 prev = load16(rs, rp + col);
    const u32x4 cur = load16(rs, ro + col);
    Carry cy;
    cy.s_lo = perm(cur.y, cur.x, kSel<COLOUR>);
    cy.s_hi = perm(cur.w, cur.z, kSel<COLOUR>);
    cy.p_lo = perm(cur.y, cur.x, kSel<COLOUR ^ 1>);
    cy.p_hi = perm(cur.w, cur.z, kSel<COLOUR ^ 1>);
    cy.u_lo = perm(prev.y, prev.x, kSel<COLOUR>);
    cy.u_hi = perm(prev.w, prev.z, kSel<COLOUR>);
    uint32_t ctr = r0 * p.row_words + xi * 4u;
    constexpr uint32_t kSideA = COLOUR == 0 ? 0 : 1;  // row parity 0: side dword on the left
    for (uint32_t k = 0; k < rows; k += 2) {
      do_row<COLOUR, COLOUR, CMP, PRIV, WIDE>(p, rs, table, hist_bytes, lane_off, ro, ro + L, col,
                                              kSideA ? right_col : left_col, ctr, cy, sums);
      ro += L;
      ctr += p.row_words;
      const uint32_t rn = k + 2 == rows ? last_next : ro + L;
      do_row<COLOUR, COLOUR ^ 1, CMP, PRIV, WIDE>(p, rs, table, hist_bytes, lane_off, ro, rn, col,
                                                  kSideA ? left_col : right_col, ctr, cy, sums);
      ro += L;
      ctr += p.row_words;
    }
  }

  if (COLOUR == 1) {
    uint32_t *esum = partial + q;
    const uint32_t e = wave_sum(4u * sums.sites - sums.nz);
    if (lane == 0 && e) atomicAdd(esum, e);
    __syncthreads();
    if (PRIV) {
      for (uint32_t v = wave; v < q; v += kWaves) {
        const uint32_t s = wave_sum(hist[v * 64u + lane]);
        if (lane == 0) partial[v] = s;
      }
      __syncthreads();
    }
    for (uint32_t v = threadIdx.x; v < q; v += kBlock) {
      const uint32_t s = PRIV ? partial[v] : hist[v];
      if (s) atomicAdd(&p.rec[1 + v], (unsigned long long)s);
    }
    if (threadIdx.x == 0 && *esum) atomicAdd(&p.rec[0], (unsigned long long)*esum);
  }
}

template <int COLOUR, int CMP, bool PRIV, bool WIDE>
hipError_t launch_t(const StripParams &p, unsigned grid, size_t lds, hipStream_t stream) {
  hipLaunchKernelGGL((strip_kernel<COLOUR, CMP, PRIV, WIDE>), dim3(grid), dim3(kBlock), lds, stream, p);
  return hipGetLastError();
}

template <int COLOUR, bool WIDE>
hipError_t launch_w(const StripParams &p, unsigned grid, size_t lds, hipStream_t stream) {
  if (p.q <= 16) return launch_t<COLOUR, 0, true, WIDE>(p, grid, lds, stream);
  if (p.q <= kPrivateHistMaxQ) return launch_t<COLOUR, 1, true, WIDE>(p, grid, lds, stream);
  if (p.q <= 128) return launch_t<COLOUR, 1, false, WIDE>(p, grid, lds, stream);
  return launch_t<COLOUR, 2, false, WIDE>(p, grid, lds, stream);
}

template <int COLOUR>
hipError_t launch_c(const StripParams &p, unsigned grid, size_t lds, hipStream_t stream) {
  const bool wide = p.thr.v[0] == 0 || p.thr.v[1] == 0 || p.thr.v[2] == 0 || p.thr.v[3] == 0;
  return wide ? launch_w<COLOUR, true>(p, grid, lds, stream) : launch_w<COLOUR, false>(p, grid, lds, stream);
}

}  // namespace

// dynamic LDS: the population counters and totals (the table is static)
size_t strip_lds_bytes(uint32_t q, int colour) {
  if (colour == 0) return 0;
  const bool priv = q <= kPrivateHistMaxQ;
  const size_t hist_words = priv ? (size_t)64 * q : q;
  return hist_words * 4 + ((size_t)q + 1) * 4;
}

hipError_t launch_strip(const StripParams &p, int colour, unsigned max_groups, hipStream_t stream) {
  const uint64_t need = ((uint64_t)p.nitems + kBlock - 1) / kBlock;
  const unsigned grid = (unsigned)(need < max_groups ? (need ? need : 1) : max_groups);
  const size_t lds = strip_lds_bytes(p.q, colour);
  return colour == 0 ? launch_c<0>(p, grid, lds, stream) : launch_c<1>(p, grid, lds, stream);
}

}  // namespace potts
