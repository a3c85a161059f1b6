// cubic_packed.hip -- the simple-cubic half sweep on a colour-split copy of the
// lattice (the cell packing of Sec. 3.3 in three dimensions).
//
// Layout: two planes of N/2 bytes.  Row (y, z) of plane c holds the L/2 sites
// of colour c ((x + y + z) & 1 == c) in increasing x: packed index i is site
// x = 2i + o with o = (c + y + z) & 1, at byte ((z L + y) L/2 + i) of the
// plane.  The neighbours of active index i all sit in the other plane: index i
// of rows (y +- 1, z) and (y, z +- 1), and indices i and i - 1 (o == 0) or
// i + 1 (o == 1) of row (y, z).  A colour-c half sweep reads plane c and plane
// c^1 and writes plane c only.  Philox: index i of row (y, z) belongs to chunk
// (z L + y) L/4 + i/2, pair i & 1, exactly the contract's block and words.
//
// Energy change of a proposal: with d(v) the number of neighbours that differ
// from v, dE = n(s) - n(k) = d(k) - d(s) (Eq. 1).  For the four sites of a
// dword the six "differs" flags of each candidate are summed bitwise by two
// carry-save adders (neighbour groups A and B, three each), giving sum and
// carry bits sA, cA, sB, cB with d = sA + sB + 2 (cA + cB).  The eight bits of
// both candidates form one byte per site,
//   bit 7 sA(k), 6 sB(k), 5 sA(s), 4 sB(s), 3 cA(k), 2 cB(k), 1 cA(s), 0 cB(s),
// which indexes a 256-entry acceptance table in LDS (as the 2D kernels do
// with their four-neighbour patterns).
//
// Work item: 16 packed bytes (16 active sites) of R consecutive rows y of one
// (x-range, z), walked in y so that each passive row of the same z is loaded
// once for three roles.  Items with odd z start their walk one row lower,
// which keeps the row parity o, and with it all byte alignments, uniform
// across a wave.  Workgroups are numbered so that consecutive z-tiles run on
// the same XCD and share its L2 for the z +- 1 rows.
#include <hip/hip_runtime.h>

#include "cubic.hpp"
#include "device.hpp"
#include "kernels.hpp"
#include "sweep_row.hpp"

namespace potts {
namespace cube {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

using namespace row;

__device__ __forceinline__ uint32_t xor3b(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}

// Byte-wise "differs from v" flag of nb at bit B of every byte, other bits
// garbage.  CMP 0 (q <= 16): x = v ^ nb < 16, so x + (2^B - 1) sets bit B
// exactly when x != 0 and never carries past it (B = 4..7); CMP 1 (q <= 128):
// B = 7, x + 0x7F; CMP 2 (q <= 256): B = 7, exact zero-byte test.
template <int CMP, int B>
__device__ __forceinline__ uint32_t differs(uint32_t v, uint32_t nb) {
  const uint32_t x = v ^ nb;
  if (CMP == 0) return x + 0x01010101u * ((1u << B) - 1u);
  if (CMP == 1) return x + 0x7F7F7F7Fu;
  return ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;
}

struct Csa {
  uint32_t s, c;
};

template <int CMP, int B>
__device__ __forceinline__ Csa count3(uint32_t v, uint32_t n0, uint32_t n1, uint32_t n2) {
  const uint32_t f0 = differs<CMP, B>(v, n0), f1 = differs<CMP, B>(v, n1), f2 = differs<CMP, B>(v, n2);
  return Csa{xor3b(f0, f1, f2), maj3(f0, f1, f2)};
}

// The table index of four sites (layout in the file comment).
template <int CMP>
__device__ __forceinline__ uint32_t cube_index(uint32_t s, uint32_t k, const uint32_t a[3], const uint32_t b[3]) {
  if (CMP == 0) {
    const Csa kA = count3<0, 7>(k, a[0], a[1], a[2]);
    const Csa kB = count3<0, 6>(k, b[0], b[1], b[2]);
    const Csa sA = count3<0, 5>(s, a[0], a[1], a[2]);
    const Csa sB = count3<0, 4>(s, b[0], b[1], b[2]);
    const uint32_t S = bfi(0x80808080u, kA.s, bfi(0x40404040u, kB.s, bfi(0x20202020u, sA.s, sB.s)));
    const uint32_t C = bfi(0x80808080u, kA.c, bfi(0x40404040u, kB.c, bfi(0x20202020u, sA.c, sB.c)));
    return bfi(0xF0F0F0F0u, S, C >> 4);
  } else {
    const Csa kA = count3<CMP, 7>(k, a[0], a[1], a[2]);
    const Csa kB = count3<CMP, 7>(k, b[0], b[1], b[2]);
    const Csa sA = count3<CMP, 7>(s, a[0], a[1], a[2]);
    const Csa sB = count3<CMP, 7>(s, b[0], b[1], b[2]);
    const uint32_t S = bfi(0x80808080u, kA.s, bfi(0x40404040u, kB.s >> 1, bfi(0x20202020u, sA.s >> 2, sB.s >> 3)));
    const uint32_t C = bfi(0x80808080u, kA.c, bfi(0x40404040u, kB.c >> 1, bfi(0x20202020u, sA.c >> 2, sB.c >> 3)));
    return bfi(0xF0F0F0F0u, S, C >> 4);
  }
}

__device__ __forceinline__ uint32_t pick_thr(const CubeThr &thr, int d) {
  uint32_t t = thr.v[0];
#pragma unroll
  for (int i = 1; i < 6; ++i) t = d == i + 1 ? thr.v[i] : t;
  return t;
}

// entry i: dE = d(k) - d(s) from the bits of i; narrow form (every threshold
// >= 1): thr[dE-1] - 1, or 2^32 - 1 for dE <= 0, accept iff w <= entry; wide
// form: thr[dE-1], or 2^32, as u64, accept iff w < entry.
template <bool WIDE>
__device__ __forceinline__ void fill_cube_table(uint8_t *table, const CubeThr &thr) {
  for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) {
    const int dk = (int)(((i >> 7) & 1u) + ((i >> 6) & 1u) + 2u * (((i >> 3) & 1u) + ((i >> 2) & 1u)));
    const int ds = (int)(((i >> 5) & 1u) + ((i >> 4) & 1u) + 2u * (((i >> 1) & 1u) + (i & 1u)));
    const int de = dk - ds;
    const uint32_t t = pick_thr(thr, de);
    if (WIDE)
      reinterpret_cast<uint64_t *>(table)[i] = de <= 0 ? (1ull << 32) : (uint64_t)t;
    else
      reinterpret_cast<uint32_t *>(table)[i] = de <= 0 ? 0xFFFFFFFFu : t - 1u;
  }
}

struct Up8 {
  uint32_t ns_lo, ns_hi;  // the 8 updated sites, packed
  uint32_t nd;            // colour 1: differing neighbours of the 8 new values, summed
};

// Update of 8 active sites (two packed dwords).  s: active bytes; p: passive
// bytes at the same index of the same row; side: the passive dword left of
// them (O == 0) or right of them (O == 1); u/d: rows y-1/y+1, f/b: rows
// z+1/z-1, same index.  ctr: chunk of the first site (a multiple of 4).
template <int COLOUR, int O, int CMP, bool WIDE>
__device__ __forceinline__ Up8 update8(uint32_t s_lo, uint32_t s_hi, uint32_t p_lo, uint32_t p_hi, uint32_t side,
                                       uint32_t u_lo, uint32_t u_hi, uint32_t d_lo, uint32_t d_hi, uint32_t f_lo,
                                       uint32_t f_hi, uint32_t b_lo, uint32_t b_hi, uint32_t ctr,
                                       const PhiloxHead &h, uint32_t q, const uint8_t *table) {
  const uint32_t x_lo = O == 0 ? alignbyte(p_lo, side, 3) : alignbyte(p_hi, p_lo, 1);
  const uint32_t x_hi = O == 0 ? alignbyte(p_hi, p_lo, 3) : alignbyte(side, p_hi, 1);
  const uint32_t x0 = h.a0 ^ ctr;
  const Words b0 = philox_tail(x0, h);
  const Words b1 = philox_tail(x0 ^ 1u, h);
  const Words b2 = philox_tail(x0 ^ 2u, h);
  const Words b3 = philox_tail(x0 ^ 3u, h);
  const uint32_t k_lo = pack4(scale_to_q(b0.w0, q), scale_to_q(b0.w2, q), scale_to_q(b1.w0, q), scale_to_q(b1.w2, q));
  const uint32_t k_hi = pack4(scale_to_q(b2.w0, q), scale_to_q(b2.w2, q), scale_to_q(b3.w0, q), scale_to_q(b3.w2, q));
  const uint32_t ga_lo[3] = {p_lo, x_lo, u_lo}, gb_lo[3] = {d_lo, f_lo, b_lo};
  const uint32_t ga_hi[3] = {p_hi, x_hi, u_hi}, gb_hi[3] = {d_hi, f_hi, b_hi};
  const uint32_t idx_lo = cube_index<CMP>(s_lo, k_lo, ga_lo, gb_lo);
  const uint32_t idx_hi = cube_index<CMP>(s_hi, k_hi, ga_hi, gb_hi);
  // colour 1 keeps the bits of the chosen candidate at 5, 4, 1, 0
  const uint32_t kd_lo = idx_lo >> 2, kd_hi = idx_hi >> 2;
  uint32_t ns_lo = s_lo, ns_hi = s_hi, nd_lo = idx_lo, nd_hi = idx_hi;
  if (!WIDE) {
#define POTTS_T(J, IDX) *reinterpret_cast<const uint32_t *>(table + table_offset<J, 2>(IDX))
    const uint32_t t0 = POTTS_T(0, idx_lo), t1 = POTTS_T(1, idx_lo), t2 = POTTS_T(2, idx_lo), t3 = POTTS_T(3, idx_lo);
    const uint32_t t4 = POTTS_T(0, idx_hi), t5 = POTTS_T(1, idx_hi), t6 = POTTS_T(2, idx_hi), t7 = POTTS_T(3, idx_hi);
#undef POTTS_T
    if (COLOUR == 0) {
      accept_byte<0>(ns_lo, b0.w1, t0, s_lo, k_lo);
      accept_byte<1>(ns_lo, b0.w3, t1, s_lo, k_lo);
      accept_byte<2>(ns_lo, b1.w1, t2, s_lo, k_lo);
      accept_byte<3>(ns_lo, b1.w3, t3, s_lo, k_lo);
      accept_byte<0>(ns_hi, b2.w1, t4, s_hi, k_hi);
      accept_byte<1>(ns_hi, b2.w3, t5, s_hi, k_hi);
      accept_byte<2>(ns_hi, b3.w1, t6, s_hi, k_hi);
      accept_byte<3>(ns_hi, b3.w3, t7, s_hi, k_hi);
    } else {
      accept_byte2<0>(ns_lo, nd_lo, b0.w1, t0, s_lo, k_lo, idx_lo, kd_lo);
      accept_byte2<1>(ns_lo, nd_lo, b0.w3, t1, s_lo, k_lo, idx_lo, kd_lo);
      accept_byte2<2>(ns_lo, nd_lo, b1.w1, t2, s_lo, k_lo, idx_lo, kd_lo);
      accept_byte2<3>(ns_lo, nd_lo, b1.w3, t3, s_lo, k_lo, idx_lo, kd_lo);
      accept_byte2<0>(ns_hi, nd_hi, b2.w1, t4, s_hi, k_hi, idx_hi, kd_hi);
      accept_byte2<1>(ns_hi, nd_hi, b2.w3, t5, s_hi, k_hi, idx_hi, kd_hi);
      accept_byte2<2>(ns_hi, nd_hi, b3.w1, t6, s_hi, k_hi, idx_hi, kd_hi);
      accept_byte2<3>(ns_hi, nd_hi, b3.w3, t7, s_hi, k_hi, idx_hi, kd_hi);
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
      nd_lo = perm(kd_lo, idx_lo, sel_lo);
      nd_hi = perm(kd_hi, idx_hi, sel_hi);
    }
  }
  Up8 r;
  r.ns_lo = ns_lo;
  r.ns_hi = ns_hi;
  r.nd = COLOUR == 1 ? __popc(nd_lo & 0x30303030u) + __popc(nd_hi & 0x30303030u) +
                           2u * (__popc(nd_lo & 0x03030303u) + __popc(nd_hi & 0x03030303u))
                     : 0u;
  return r;
}

__device__ __forceinline__ u32x4 ld16(const uint8_t *base, uint64_t off) {
  return *reinterpret_cast<const u32x4 *>(base + off);
}

// One row of the walk: active row (y, z) at a_off; passive rows at p_off
// (y, z), dn_off (y+1, z), f_off (y, z+1), b_off (y, z-1); side dword at
// s_off.  cy_u / cy_p carry the passive rows y-1 and y.
template <int COLOUR, int O, int CMP, bool PRIV, bool WIDE>
__device__ __forceinline__ void cube_row(const CubeLaunch &p, const PhiloxHead &h, uint8_t *act,
                                         const uint8_t *pas, const uint8_t *table, uint8_t *hist,
                                         uint32_t lane_off, uint64_t a_off, uint64_t dn_off, uint64_t f_off,
                                         uint64_t b_off, uint64_t s_off, uint32_t ctr, u32x4 &cy_u, u32x4 &cy_p,
                                         uint32_t &nd) {
  const u32x4 a = ld16(act, a_off);
  const u32x4 dn = ld16(pas, dn_off);
  const u32x4 f = ld16(pas, f_off);
  const u32x4 b = ld16(pas, b_off);
  const uint32_t side = *reinterpret_cast<const uint32_t *>(pas + s_off);
  const Up8 r0 = update8<COLOUR, O, CMP, WIDE>(a.x, a.y, cy_p.x, cy_p.y, O == 0 ? side : cy_p.z, cy_u.x, cy_u.y,
                                               dn.x, dn.y, f.x, f.y, b.x, b.y, ctr, h, p.q, table);
  const Up8 r1 = update8<COLOUR, O, CMP, WIDE>(a.z, a.w, cy_p.z, cy_p.w, O == 0 ? cy_p.y : side, cy_u.z, cy_u.w,
                                               dn.z, dn.w, f.z, f.w, b.z, b.w, ctr + 4u, h, p.q, table);
  u32x4 out;
  out.x = r0.ns_lo;
  out.y = r0.ns_hi;
  out.z = r1.ns_lo;
  out.w = r1.ns_hi;
  *reinterpret_cast<u32x4 *>(act + a_off) = out;
  if (COLOUR == 1) nd += r0.nd + r1.nd;
  if (PRIV) {
    count_active_private(hist, lane_off, r0.ns_lo, r0.ns_hi);
    count_active_private(hist, lane_off, r1.ns_lo, r1.ns_hi);
  } else {
    count_active_shared(reinterpret_cast<uint32_t *>(hist), r0.ns_lo, r0.ns_hi);
    count_active_shared(reinterpret_cast<uint32_t *>(hist), r1.ns_lo, r1.ns_hi);
  }
  cy_u = cy_p;
  cy_p = dn;
}

template <int COLOUR, int CMP, bool PRIV, bool WIDE>
__global__ __launch_bounds__(kBlock) void cube_packed_kernel(CubeLaunch p) {
  __shared__ __align__(16) uint32_t table_words[512];
  constexpr uint32_t kHistWords = PRIV ? 64u * (CMP == 0 ? 16u : kPrivateHistMaxQ) : 256u;
  __shared__ __align__(16) uint32_t hist[kHistWords];
  __shared__ uint32_t partial[257];
  const PhiloxHead h = philox_head(p.t_lo, p.t_hi, (uint32_t)COLOUR + 8u, p.k0, p.k1);
  uint8_t *table = reinterpret_cast<uint8_t *>(table_words);
  const uint32_t q = p.q;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = threadIdx.x >> 6;
  // consecutive logical workgroups on one XCD (workgroups go round-robin over 8)
  const uint32_t bid = p.xcd_stride ? (blockIdx.x & 7u) * p.xcd_stride + (blockIdx.x >> 3) : blockIdx.x;

  fill_cube_table<WIDE>(table, p.thr);
  const uint32_t nh = PRIV ? 64 * q : q;
  for (uint32_t i = threadIdx.x; i < nh; i += kBlock) hist[i] = 0;
  if (threadIdx.x == 0) partial[q] = 0;
  if (COLOUR == 1 && blockIdx.x == 0 && p.rec_clear)
    for (uint32_t i = threadIdx.x; i < q + 1; i += kBlock) p.rec_clear[i] = 0;
  __syncthreads();

  uint8_t *hist_bytes = reinterpret_cast<uint8_t *>(hist);
  const uint32_t lane_off = lane * 4u;
  uint32_t nd = 0, sites = 0;
  const uint32_t g = bid * kBlock + threadIdx.x;
  if (g < p.nitems) {
    const uint32_t L = p.L, half = L >> 1, R = p.rows;
    const uint32_t rest = g / p.ipr;
    const uint32_t ix = g - rest * p.ipr;
    const uint32_t z = rest % L, yb = rest / L;
    const uint32_t col = ix * 16u;
    const uint32_t left_col = col == 0 ? half - 4 : col - 4;
    const uint32_t right_col = col + 16 == half ? 0u : col + 16;
    const uint32_t zf = z + 1 == L ? 0u : z + 1, zb = z == 0 ? L - 1 : z - 1;
    uint8_t *act = p.planes + (COLOUR == 0 ? 0 : p.plane_bytes);
    const uint8_t *pas = p.planes + (COLOUR == 0 ? p.plane_bytes : 0);
    const uint64_t zrow = (uint64_t)z * L, frow = (uint64_t)zf * L, brow = (uint64_t)zb * L;
    uint32_t y = yb * R + (z & 1u);
    if (y >= L) y -= L;
    const uint32_t yu = y == 0 ? L - 1 : y - 1;
    u32x4 cy_u = ld16(pas, (zrow + yu) * half + col);
    u32x4 cy_p = ld16(pas, (zrow + y) * half + col);
    const uint32_t qL = L >> 2;
    for (uint32_t k = 0; k < R; k += 2) {
      // row y: o = COLOUR; row y + 1: o = COLOUR ^ 1
      uint32_t y1 = y + 1 == L ? 0u : y + 1;
      cube_row<COLOUR, COLOUR, CMP, PRIV, WIDE>(
          p, h, act, pas, table, hist_bytes, lane_off, (zrow + y) * half + col, (zrow + y1) * half + col,
          (frow + y) * half + col, (brow + y) * half + col,
          (zrow + y) * half + (COLOUR == 0 ? left_col : right_col), (uint32_t)((zrow + y) * qL) + (col >> 1), cy_u,
          cy_p, nd);
      y = y1;
      y1 = y + 1 == L ? 0u : y + 1;
      cube_row<COLOUR, COLOUR ^ 1, CMP, PRIV, WIDE>(
          p, h, act, pas, table, hist_bytes, lane_off, (zrow + y) * half + col, (zrow + y1) * half + col,
          (frow + y) * half + col, (brow + y) * half + col,
          (zrow + y) * half + (COLOUR == 0 ? right_col : left_col), (uint32_t)((zrow + y) * qL) + (col >> 1), cy_u,
          cy_p, nd);
      y = y1;
    }
    sites = 16u * R;
  }

  uint32_t *esum = partial + q;
  if (COLOUR == 1) {
    const uint32_t e = wave_sum(6u * sites - nd);
    if (lane == 0 && e) atomicAdd(esum, e);
  }
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
  if (COLOUR == 1 && threadIdx.x == 0 && *esum) atomicAdd(&p.rec[0], (unsigned long long)*esum);
}

// Row-major cube <-> two colour planes; one thread per 32 bytes of a row.
__global__ __launch_bounds__(kBlock) void cube_pack_kernel(const uint8_t *src, uint8_t *dst, uint32_t L,
                                                           uint64_t plane_bytes) {
  const uint32_t groups = L >> 5;
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= (uint64_t)groups * L * L) return;
  const uint64_t r = g / groups;  // z L + y
  const uint32_t j = (uint32_t)(g - r * groups);
  const uint32_t par = (uint32_t)((r % L) + r / L) & 1u;  // colour of even x
  const u32x4 *in = reinterpret_cast<const u32x4 *>(src + r * L + 32u * j);
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
  const uint64_t row = r * (L >> 1) + 16u * j;
  *reinterpret_cast<u32x4 *>(dst + par * plane_bytes + row) = even;
  *reinterpret_cast<u32x4 *>(dst + (par ^ 1u) * plane_bytes + row) = odd;
}

__global__ __launch_bounds__(kBlock) void cube_unpack_kernel(const uint8_t *src, uint8_t *dst, uint32_t L,
                                                             uint64_t plane_bytes) {
  const uint32_t groups = L >> 5;
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= (uint64_t)groups * L * L) return;
  const uint64_t r = g / groups;
  const uint32_t j = (uint32_t)(g - r * groups);
  const uint32_t par = (uint32_t)((r % L) + r / L) & 1u;
  const uint64_t row = r * (L >> 1) + 16u * j;
  const u32x4 even = *reinterpret_cast<const u32x4 *>(src + par * plane_bytes + row);
  const u32x4 odd = *reinterpret_cast<const u32x4 *>(src + (par ^ 1u) * plane_bytes + row);
  u32x4 lo, hi;
  lo.x = perm(odd.x, even.x, 0x05010400u);
  lo.y = perm(odd.x, even.x, 0x07030602u);
  lo.z = perm(odd.y, even.y, 0x05010400u);
  lo.w = perm(odd.y, even.y, 0x07030602u);
  hi.x = perm(odd.z, even.z, 0x05010400u);
  hi.y = perm(odd.z, even.z, 0x07030602u);
  hi.z = perm(odd.w, even.w, 0x05010400u);
  hi.w = perm(odd.w, even.w, 0x07030602u);
  u32x4 *out = reinterpret_cast<u32x4 *>(dst + r * L + 32u * j);
  out[0] = lo;
  out[1] = hi;
}

template <int COLOUR, bool WIDE>
void launch_w(const CubeLaunch &l, unsigned grid, hipStream_t stream) {
  const uint32_t q = l.q;
  if (q <= 16)
    hipLaunchKernelGGL((cube_packed_kernel<COLOUR, 0, true, WIDE>), dim3(grid), dim3(kBlock), 0, stream, l);
  else if (q <= kPrivateHistMaxQ)
    hipLaunchKernelGGL((cube_packed_kernel<COLOUR, 1, true, WIDE>), dim3(grid), dim3(kBlock), 0, stream, l);
  else if (q <= 128)
    hipLaunchKernelGGL((cube_packed_kernel<COLOUR, 1, false, WIDE>), dim3(grid), dim3(kBlock), 0, stream, l);
  else
    hipLaunchKernelGGL((cube_packed_kernel<COLOUR, 2, false, WIDE>), dim3(grid), dim3(kBlock), 0, stream, l);
}

}  // namespace

unsigned packed_grid(CubeLaunch &l) {
  const uint64_t groups = ((uint64_t)l.nitems + kBlock - 1) / kBlock;
  l.xcd_stride = groups % 8 == 0 ? (uint32_t)(groups / 8) : 0u;
  return (unsigned)groups;
}

hipError_t launch_packed(const CubeLaunch &l, int colour, unsigned grid, hipStream_t stream) {
  if (grid == 0) return hipSuccess;
  bool wide = false;  // some threshold is 0 (tables need not be monotone)
  for (int i = 0; i < 6; ++i) wide = wide || l.thr.v[i] == 0;
  if (colour == 0)
    wide ? launch_w<0, true>(l, grid, stream) : launch_w<0, false>(l, grid, stream);
  else
    wide ? launch_w<1, true>(l, grid, stream) : launch_w<1, false>(l, grid, stream);
  return hipGetLastError();
}

hipError_t launch_pack(const uint8_t *cube, uint8_t *planes, uint32_t L, hipStream_t stream) {
  const uint64_t n = (uint64_t)(L >> 5) * L * L;
  hipLaunchKernelGGL(cube_pack_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream, cube,
                     planes, L, (uint64_t)L * L * L / 2);
  return hipGetLastError();
}

hipError_t launch_unpack(const uint8_t *planes, uint8_t *cube, uint32_t L, hipStream_t stream) {
  const uint64_t n = (uint64_t)(L >> 5) * L * L;
  hipLaunchKernelGGL(cube_unpack_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream,
                     planes, cube, L, (uint64_t)L * L * L / 2);
  return hipGetLastError();
}

}  // namespace cube
}  // namespace potts
