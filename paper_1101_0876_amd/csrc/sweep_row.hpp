// sweep_row.hpp -- the per-row Metropolis update shared by the gfx950 sweep
// kernels (strip.hip: rows streamed from HBM; resident.hip: lattice in LDS).
//
// A "row" is 16 consecutive bytes of one lattice row: 8 sites of the active
// colour.  They are updated with four Philox4x32-10 blocks (device.hpp), the
// active and passive bytes packed into dwords with v_perm, the four neighbour
// comparisons of four sites at once as byte-wise flag patterns (bits 7..4 of
// each byte; v_xad + v_bitop3), one LDS acceptance-table read, one v_cmp and
// one SDWA v_cndmask per site.  Sites of one colour only have neighbours of
// the other colour (Sec. 3), so a row is updated from values no concurrent
// update changes, and its passive bytes are written back unchanged.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"
#include "kernels.hpp"

namespace potts {
namespace row {

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
// kept: one v_cmp and one SDWA v_cndmask.  gfx950 needs two wait states
// between a VALU write of VCC and a VALU read of it, and one between an SDWA
// byte write and the next read of that register: byte 3 is a byte's last
// select, whose result compiled code may read next.
#define POTTS_ACCEPT1(J, TAIL)                                                                  \
  asm("v_cmp_le_u32 vcc, %1, %2\n\ts_nop 1\n\t"                                              \
      "v_cndmask_b32_sdwa %0, %3, %4, vcc dst_sel:BYTE_" #J                                     \
      " dst_unused:UNUSED_PRESERVE src0_sel:BYTE_" #J " src1_sel:BYTE_" #J TAIL                 \
      : "+v"(dst) : "v"(w), "v"(t), "v"(if_rej), "v"(if_acc) : "vcc")
template <int J>
__device__ __forceinline__ void accept_byte(uint32_t &dst, uint32_t w, uint32_t t, uint32_t if_rej,
                                            uint32_t if_acc) {
  if (J == 0) POTTS_ACCEPT1(0, "");
  else if (J == 1) POTTS_ACCEPT1(1, "");
  else if (J == 2) POTTS_ACCEPT1(2, "");
  else POTTS_ACCEPT1(3, "\n\ts_nop 0");
}
#undef POTTS_ACCEPT1

// As accept_byte, selecting byte J of two pairs with one compare.
#define POTTS_ACCEPT2(J, TAIL)                                                                  \
  asm("v_cmp_le_u32 vcc, %2, %3\n\ts_nop 1\n\t"                                              \
      "v_cndmask_b32_sdwa %0, %4, %5, vcc dst_sel:BYTE_" #J                                     \
      " dst_unused:UNUSED_PRESERVE src0_sel:BYTE_" #J " src1_sel:BYTE_" #J "\n\t"              \
      "v_cndmask_b32_sdwa %1, %6, %7, vcc dst_sel:BYTE_" #J                                     \
      " dst_unused:UNUSED_PRESERVE src0_sel:BYTE_" #J " src1_sel:BYTE_" #J TAIL                 \
      : "+v"(dst1), "+v"(dst2)                                                                  \
      : "v"(w), "v"(t), "v"(rej1), "v"(acc1), "v"(rej2), "v"(acc2)                              \
      : "vcc")
template <int J>
__device__ __forceinline__ void accept_byte2(uint32_t &dst1, uint32_t &dst2, uint32_t w, uint32_t t,
                                             uint32_t rej1, uint32_t acc1, uint32_t rej2, uint32_t acc2) {
  if (J == 0) POTTS_ACCEPT2(0, "");
  else if (J == 1) POTTS_ACCEPT2(1, "");
  else if (J == 2) POTTS_ACCEPT2(2, "");
  else POTTS_ACCEPT2(3, "\n\ts_nop 0");
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

// Acceptance table in LDS, indexed by (proposal pattern << 4 | current
// pattern), dE = popcount(proposal pattern) - popcount(current pattern):
// narrow form (all thresholds >= 1) holds thr[dE-1] - 1, or 2^32 - 1 when
// dE <= 0, and a move is accepted iff w <= entry; the wide form (some
// threshold is 0) holds thr[dE-1], or 2^32, as u64 and accepts iff w < entry.
template <bool WIDE>
__device__ __forceinline__ void fill_accept_table(uint8_t *table, const Thresholds &thr) {
  // entry (k_pattern << 4 | s_pattern): dE = popcount(k_pattern) - popcount(s_pattern)
  for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) {
    const int de = __popc(i >> 4) - __popc(i & 15u);
    const uint32_t t = de == 1 ? thr.v[0] : de == 2 ? thr.v[1] : de == 3 ? thr.v[2] : thr.v[3];
    if (WIDE)
      reinterpret_cast<uint64_t *>(table)[i] = de <= 0 ? (1ull << 32) : (uint64_t)t;
    else
      reinterpret_cast<uint32_t *>(table)[i] = de <= 0 ? 0xFFFFFFFFu : t - 1u;
  }
}


struct Row8 {
  u32x4 out;               // the 16 bytes after the update
  uint32_t ns_lo, ns_hi;   // the 8 updated bytes, packed
  uint32_t nz_lo, nz_hi;   // colour 1: differing-neighbour flags of the new spins
};

// Update of the 8 active sites of one 16-byte row.  s/p: active/passive bytes
// of the row, u/d: bytes of the rows above/below at the active offset (all
// packed, lo = first 8 bytes); side: the dword left of the row when O == 0,
// right of it when O == 1.  ctr: chunk index (Philox counter word 1) of the
// row's first 4-byte chunk, a multiple of 4 since L % 16 == 0; h: the head of
// this half sweep's Philox blocks.
template <int COLOUR, int O, int CMP, bool WIDE>
__device__ __forceinline__ Row8 update8(uint32_t s_lo, uint32_t s_hi, uint32_t p_lo, uint32_t p_hi,
                                        uint32_t u_lo, uint32_t u_hi, uint32_t d_lo, uint32_t d_hi,
                                        uint32_t side, uint32_t ctr, const PhiloxHead &h, uint32_t q,
                                        const uint8_t *table) {
  // horizontal neighbours: one is the passive byte at the same packed index,
  // the other the passive byte one site over (left when O == 0, right when O == 1)
  const uint32_t x_lo = O == 0 ? alignbyte(p_lo, side, 3) : alignbyte(p_hi, p_lo, 1);
  const uint32_t x_hi = O == 0 ? alignbyte(p_hi, p_lo, 3) : alignbyte(side, p_hi, 1);

  // block m serves dword m: (w0, w1) for its site at byte O, (w2, w3) at byte O+2
  // ctr + m == ctr ^ m for m < 4
  const uint32_t x0 = h.a0 ^ ctr;
  const Words b0 = philox_tail(x0, h);
  const Words b1 = philox_tail(x0 ^ 1u, h);
  const Words b2 = philox_tail(x0 ^ 2u, h);
  const Words b3 = philox_tail(x0 ^ 3u, h);
  const uint32_t k_lo = pack4(scale_to_q(b0.w0, q), scale_to_q(b0.w2, q), scale_to_q(b1.w0, q), scale_to_q(b1.w2, q));
  const uint32_t k_hi = pack4(scale_to_q(b2.w0, q), scale_to_q(b2.w2, q), scale_to_q(b3.w0, q), scale_to_q(b3.w2, q));

  const uint32_t ps_lo = diff_pattern<CMP>(s_lo, u_lo, d_lo, p_lo, x_lo);
  const uint32_t ps_hi = diff_pattern<CMP>(s_hi, u_hi, d_hi, p_hi, x_hi);
  const uint32_t pk_lo = diff_pattern<CMP>(k_lo, u_lo, d_lo, p_lo, x_lo);
  const uint32_t pk_hi = diff_pattern<CMP>(k_hi, u_hi, d_hi, p_hi, x_hi);
  const uint32_t idx_lo = bfi(0xF0F0F0F0u, pk_lo, ps_lo >> 4);
  const uint32_t idx_hi = bfi(0xF0F0F0F0u, pk_hi, ps_hi >> 4);

  uint32_t ns_lo, ns_hi;          // new active bytes
  uint32_t nz_lo = 0, nz_hi = 0;  // colour 1: flag patterns of the new spins
  if (!WIDE) {
#define POTTS_T(J, IDX) *reinterpret_cast<const uint32_t *>(table + table_offset<J, 2>(IDX))
    const uint32_t t0 = POTTS_T(0, idx_lo), t1 = POTTS_T(1, idx_lo), t2 = POTTS_T(2, idx_lo), t3 = POTTS_T(3, idx_lo);
    const uint32_t t4 = POTTS_T(0, idx_hi), t5 = POTTS_T(1, idx_hi), t6 = POTTS_T(2, idx_hi), t7 = POTTS_T(3, idx_hi);
#undef POTTS_T
    // byte 0 by a whole-dword select (its other bytes are overwritten next),
    // which saves copying s into the destination first
    const bool a0 = b0.w1 <= t0, a4 = b2.w1 <= t4;
    ns_lo = a0 ? k_lo : s_lo;
    ns_hi = a4 ? k_hi : s_hi;
    if (COLOUR == 0) {
      accept_byte<1>(ns_lo, b0.w3, t1, s_lo, k_lo);
      accept_byte<2>(ns_lo, b1.w1, t2, s_lo, k_lo);
      accept_byte<3>(ns_lo, b1.w3, t3, s_lo, k_lo);
      accept_byte<1>(ns_hi, b2.w3, t5, s_hi, k_hi);
      accept_byte<2>(ns_hi, b3.w1, t6, s_hi, k_hi);
      accept_byte<3>(ns_hi, b3.w3, t7, s_hi, k_hi);
    } else {
      nz_lo = a0 ? pk_lo : ps_lo;
      nz_hi = a4 ? pk_hi : ps_hi;
      accept_byte2<1>(ns_lo, nz_lo, b0.w3, t1, s_lo, k_lo, ps_lo, pk_lo);
      accept_byte2<2>(ns_lo, nz_lo, b1.w1, t2, s_lo, k_lo, ps_lo, pk_lo);
      accept_byte2<3>(ns_lo, nz_lo, b1.w3, t3, s_lo, k_lo, ps_lo, pk_lo);
      accept_byte2<1>(ns_hi, nz_hi, b2.w3, t5, s_hi, k_hi, ps_hi, pk_hi);
      accept_byte2<2>(ns_hi, nz_hi, b3.w1, t6, s_hi, k_hi, ps_hi, pk_hi);
      accept_byte2<3>(ns_hi, nz_hi, b3.w3, t7, s_hi, k_hi, ps_hi, pk_hi);
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
    ns_lo = perm(k_lo, s_lo, sel_lo);
    ns_hi = perm(k_hi, s_hi, sel_hi);
    if (COLOUR == 1) {
      nz_lo = perm(pk_lo, ps_lo, sel_lo);
      nz_hi = perm(pk_hi, ps_hi, sel_hi);
    }
  }
  // interleave the new active bytes with the unchanged passive ones
  constexpr uint32_t sel_w0 = O ? 0x05010400u : 0x01050004u;
  constexpr uint32_t sel_w1 = O ? 0x07030602u : 0x03070206u;
  Row8 r;
  r.out.x = perm(ns_lo, p_lo, sel_w0);
  r.out.y = perm(ns_lo, p_lo, sel_w1);
  r.out.z = perm(ns_hi, p_hi, sel_w0);
  r.out.w = perm(ns_hi, p_hi, sel_w1);
  r.ns_lo = ns_lo;
  r.ns_hi = ns_hi;
  r.nz_lo = nz_lo;
  r.nz_hi = nz_hi;
  return r;
}

// The same update for the 4 active sites of 8 row bytes, given their words:
// s/p/u/d are the packed active, passive, up and down bytes, side the dword
// left (O == 0) or right (O == 1) of the 8 bytes, k the four proposals
// packed (site j in byte j) and a0..a3 the four acceptance words.
struct Row4 {
  uint32_t out_x, out_y;  // the 8 bytes after the update
  uint32_t ns;            // the 4 updated bytes, packed
  uint32_t nz;            // colour 1: differing-neighbour flags of the new spins
};

template <int COLOUR, int O, int CMP, bool WIDE>
__device__ __forceinline__ Row4 update4_drawn(uint32_t s, uint32_t p, uint32_t u, uint32_t d, uint32_t side,
                                              uint32_t k, uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3,
                                              const uint8_t *table) {
  const uint32_t x = O == 0 ? alignbyte(p, side, 3) : alignbyte(side, p, 1);
  const uint32_t ps = diff_pattern<CMP>(s, u, d, p, x);
  const uint32_t pk = diff_pattern<CMP>(k, u, d, p, x);
  const uint32_t idx = bfi(0xF0F0F0F0u, pk, ps >> 4);
  uint32_t ns = s, nz = 0;
  if (!WIDE) {
#define POTTS_T(J) *reinterpret_cast<const uint32_t *>(table + table_offset<J, 2>(idx))
    const uint32_t t0 = POTTS_T(0), t1 = POTTS_T(1), t2 = POTTS_T(2), t3 = POTTS_T(3);
#undef POTTS_T
    // byte 0 by a whole-dword select, bytes 1..3 overwritten next
    const bool acc0 = a0 <= t0;
    ns = acc0 ? k : s;
    if (COLOUR == 0) {
      accept_byte<1>(ns, a1, t1, s, k);
      accept_byte<2>(ns, a2, t2, s, k);
      accept_byte<3>(ns, a3, t3, s, k);
    } else {
      nz = acc0 ? pk : ps;
      accept_byte2<1>(ns, nz, a1, t1, s, k, ps, pk);
      accept_byte2<2>(ns, nz, a2, t2, s, k, ps, pk);
      accept_byte2<3>(ns, nz, a3, t3, s, k, ps, pk);
    }
  } else {
    const uint64_t *t64 = reinterpret_cast<const uint64_t *>(table);
    const uint32_t acc_w[4] = {a0, a1, a2, a3};
    uint32_t sel = 0x03020100u;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if ((uint64_t)acc_w[j] < t64[(idx >> (8 * j)) & 0xFFu]) sel |= 4u << (8 * j);
    ns = perm(k, s, sel);
    if (COLOUR == 1) nz = perm(pk, ps, sel);
  }
  constexpr uint32_t sel_w0 = O ? 0x05010400u : 0x01050004u;
  constexpr uint32_t sel_w1 = O ? 0x07030602u : 0x03070206u;
  Row4 r;
  r.out_x = perm(ns, p, sel_w0);
  r.out_y = perm(ns, p, sel_w1);
  r.ns = ns;
  r.nz = nz;
  return r;
}

// The update with its words drawn here (two Philox blocks): ctr is the chunk
// of the first dword (even).  Used where more, smaller work items pay (the
// LDS-resident kernel, one workgroup per small lattice).
template <int COLOUR, int O, int CMP, bool WIDE>
__device__ __forceinline__ Row4 update4(uint32_t s, uint32_t p, uint32_t u, uint32_t d, uint32_t side,
                                        uint32_t ctr, const PhiloxHead &h, uint32_t q, const uint8_t *table) {
  // ctr + 1 == ctr ^ 1 for even ctr
  const uint32_t x0 = h.a0 ^ ctr;
  const Words b0 = philox_tail(x0, h);
  const Words b1 = philox_tail(x0 ^ 1u, h);
  const uint32_t k = pack4(scale_to_q(b0.w0, q), scale_to_q(b0.w2, q), scale_to_q(b1.w0, q), scale_to_q(b1.w2, q));
  return update4_drawn<COLOUR, O, CMP, WIDE>(s, p, u, d, side, k, b0.w1, b0.w3, b1.w1, b1.w3, table);
}

// Counts the 16 final values of a row into lane-private LDS columns:
// counter (value, lane) at byte (value << 8) | lane*4 of `hist`, one v_perm
// per value.  Colours share the columns; LDS atomics keep them exact.
__device__ __forceinline__ void count_row_private(uint8_t *hist, uint32_t lane_off, const u32x4 &out) {
  const uint32_t words[4] = {out.x, out.y, out.z, out.w};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint32_t addr = perm(words[m], lane_off, 0x0C0C0000u | ((4u + b) << 8));
      atomicAdd(reinterpret_cast<uint32_t *>(hist + addr), 1u);
    }
  }
}

// The same for the 8 updated values of a row (two packed dwords).
__device__ __forceinline__ void count_active_private(uint8_t *hist, uint32_t lane_off, uint32_t lo,
                                                     uint32_t hi) {
  const uint32_t words[2] = {lo, hi};
#pragma unroll
  for (int m = 0; m < 2; ++m) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint32_t addr = perm(words[m], lane_off, 0x0C0C0000u | ((4u + b) << 8));
      atomicAdd(reinterpret_cast<uint32_t *>(hist + addr), 1u);
    }
  }
}

__device__ __forceinline__ void count_active_shared(uint32_t *bins, uint32_t lo, uint32_t hi) {
  const uint32_t words[2] = {lo, hi};
#pragma unroll
  for (int m = 0; m < 2; ++m) {
#pragma unroll
    for (int b = 0; b < 4; ++b) atomicAdd(&bins[(words[m] >> (8 * b)) & 0xFFu], 1u);
  }
}

// The same into q shared bins (any q).
__device__ __forceinline__ void count_row_shared(uint32_t *bins, const u32x4 &out) {
  const uint32_t words[4] = {out.x, out.y, out.z, out.w};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
#pragma unroll
    for (int b = 0; b < 4; ++b) atomicAdd(&bins[(words[m] >> (8 * b)) & 0xFFu], 1u);
  }
}

// Stripe set t & 1 of p summed into ring slot t, then cleared, by one whole
// workgroup (every (stripe, word) pair loaded at once; acc: 1+q words of
// LDS).  Contains barriers: call it from workgroup-uniform control flow.
template <int BLOCK>
__device__ __forceinline__ void fold_stripes(const StripParams &p, uint64_t t, unsigned long long *acc) {
  const uint32_t n = p.q + 1, sw = stripe_words(p.q), total = p.nstripes * n;
  unsigned long long *set = p.stripes + (t & 1) * (uint64_t)p.nstripes * sw;
  unsigned long long *slot = p.ring + (t & (p.cap - 1)) * (uint64_t)n;
  for (uint32_t i = threadIdx.x; i < n; i += BLOCK) acc[i] = 0;
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < total; k += BLOCK) {
    const uint32_t s = k / n, i = k - s * n;
    const unsigned long long v = set[s * sw + i];
    if (v) {
      atomicAdd(&acc[i], v);
      set[s * sw + i] = 0;
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n; i += BLOCK) slot[i] = acc[i];
}

}  // namespace row
}  // namespace potts
