// heatbath_packed.hip -- heat-bath half sweeps of a single lattice on its
// colour-split copy (the planes packed.hip sweeps; Sec. 7 names the heat bath
// as the other single-spin-flip update).
//
// The new value of a site does not depend on its current value, so a colour-c
// half sweep reads only plane c^1 (the neighbours) and writes plane c: N bytes
// per half sweep.  A work item is 16 packed bytes (16 sites of colour c) of R
// rows, walked downwards as in packed.hip, each passive row loaded once.
//
// The draw (contract: value v weighs D[n_max - n(v)], D[0] = 2^32, D[d] =
// thr[d-1]; the distinct neighbour values in order of first appearance among
// (up, down, left, right), then the others ascending; r = floor(w Z / 2^32)
// picks the first value whose cumulative weight exceeds r):
//   * which neighbour values are equal (six flags, four sites at a time with
//     byte-wise arithmetic) indexes a 64-entry table built on the host;
//   * the cumulative weights of the ranked neighbour values c_i are turned
//     into cuts on the word itself: r < c_i exactly when w < ceil(c_i 2^32 /
//     Z), so four 32-bit compares and byte selects pick among the neighbour
//     values;
//   * past them (r >= S, the neighbour values' total), the run of other
//     values, each of weight w0 = D[n_max], is indexed by j = floor((r - S) /
//     w0) (an FP32 estimate from above and one integer check), and the j-th
//     value held by no neighbour comes from a bit mask of the neighbour values
//     (q <= 16) or from the sorted neighbour values.
#include <hip/hip_runtime.h>

#include <string.h>

#include <algorithm>

#include "device.hpp"
#include "kernels.hpp"
#include "sweep_row.hpp"

namespace potts {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

using namespace row;

// Per byte of up/down/left/right: the six "differs" flags ab, ac, ad, bc, bd,
// cd at bits 7..2, bits 1..0 clear (byte << 2 is then the pattern's 16-byte
// table offset).  CMP 0: values below 16, 1: below 128, 2: any byte.
template <int CMP>
__device__ __forceinline__ uint32_t pair_pattern(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  uint32_t hi, lo;  // flags ab, ac, ad, bc at bits 7..4; bd, cd at bits 7..6
  if (CMP == 0) {
    hi = bfi(0xE0E0E0E0u, bfi(0xC0C0C0C0u, bfi(0x80808080u, (a ^ b) + 0x7F7F7F7Fu, (a ^ c) + 0x3F3F3F3Fu),
                              (a ^ d) + 0x1F1F1F1Fu),
             (b ^ c) + 0x0F0F0F0Fu);
    lo = bfi(0x80808080u, (b ^ d) + 0x7F7F7F7Fu, (c ^ d) + 0x3F3F3F3Fu);
  } else {
    auto f = [](uint32_t x) { return CMP == 1 ? x + 0x7F7F7F7Fu : (((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x); };
    hi = bfi(0xE0E0E0E0u, bfi(0xC0C0C0C0u, bfi(0x80808080u, f(a ^ b), f(a ^ c) >> 1), f(a ^ d) >> 2), f(b ^ c) >> 3);
    lo = bfi(0x80808080u, f(b ^ d), f(c ^ d) >> 1);
  }
  return bfi(0xF0F0F0F0u, hi, lo >> 4) & 0xFCFCFCFCu;
}

// dst.byte_J = (w <= t) ? src.byte_J : dst.byte_J: one v_cmp and one SDWA
// v_cndmask.  gfx950 needs two wait states between a VALU write of VCC and a
// VALU read of it, and one between an SDWA byte write and the next read of
// that register (TAIL: the last select of a byte, whose result compiled code
// reads next).
#define POTTS_HB_SEL(J, TAIL)                                                                      \
  asm("v_cmp_le_u32 vcc, %1, %2\n\ts_nop 1\n\tv_cndmask_b32_sdwa %0, %0, %3, vcc dst_sel:BYTE_" #J \
      " dst_unused:UNUSED_PRESERVE src0_sel:BYTE_" #J " src1_sel:BYTE_" #J TAIL                    \
      : "+v"(dst) : "v"(w), "v"(t), "v"(src) : "vcc")
template <int J, bool LAST = false>
__device__ __forceinline__ void select_byte(uint32_t &dst, uint32_t w, uint32_t t, uint32_t src) {
  if (LAST) {
    if (J == 0) POTTS_HB_SEL(0, "\n\ts_nop 0");
    else if (J == 1) POTTS_HB_SEL(1, "\n\ts_nop 0");
    else if (J == 2) POTTS_HB_SEL(2, "\n\ts_nop 0");
    else POTTS_HB_SEL(3, "\n\ts_nop 0");
  } else {
    if (J == 0) POTTS_HB_SEL(0, "");
    else if (J == 1) POTTS_HB_SEL(1, "");
    else if (J == 2) POTTS_HB_SEL(2, "");
    else POTTS_HB_SEL(3, "");
  }
}
#undef POTTS_HB_SEL

// dst.byte_J = (w <= t) ? src.byte_J : k.byte_0 (the first select of a byte
// also places the value no neighbour holds).
#define POTTS_HB_PLACE(J)                                                                          \
  asm("v_cmp_le_u32 vcc, %1, %2\n\ts_nop 1\n\tv_cndmask_b32_sdwa %0, %3, %4, vcc dst_sel:BYTE_" #J \
      " dst_unused:UNUSED_PRESERVE src0_sel:BYTE_0 src1_sel:BYTE_" #J                              \
      : "+v"(dst) : "v"(w), "v"(t), "v"(k), "v"(src) : "vcc")
template <int J>
__device__ __forceinline__ void place_select(uint32_t &dst, uint32_t w, uint32_t t, uint32_t k, uint32_t src) {
  if (J == 0) POTTS_HB_PLACE(0);
  else if (J == 1) POTTS_HB_PLACE(1);
  else if (J == 2) POTTS_HB_PLACE(2);
  else POTTS_HB_PLACE(3);
}
#undef POTTS_HB_PLACE

// float -> u32, truncating and saturating (v_cvt_u32_f32): the estimate below
// is huge when the draw lands on a neighbour value, and is not used then.
__device__ __forceinline__ uint32_t cvt_u32_sat(float f) {
  uint32_t r;
  asm("v_cvt_u32_f32 %0, %1" : "=v"(r) : "v"(f));
  return r;
}

// u32 -> float, rounded to nearest (one v_cvt_f32_u32; written out so that
// the pair below is not re-read as a 64-bit conversion)
__device__ __forceinline__ float cvt_f32(uint32_t x) {
  float r;
  asm("v_cvt_f32_u32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// The j-th value (from 0, ascending) that none of the byte-J values of up,
// dn, lf, rt holds, for values below 16: with m the set of neighbour values as
// a bit mask, k = j + |{v in m : v <= k}|, reached from k = j in four steps
// (each step before the last adds at least one of the at most four values).
// kk = k + 1 is carried, so |{v <= k}| = popcount of the low kk bits of m.
template <int J>
__device__ __forceinline__ uint32_t free_value16(uint32_t j, uint32_t up, uint32_t dn, uint32_t lf, uint32_t rt) {
  const uint32_t m = (1u << byte_of(up, J)) | (1u << byte_of(dn, J)) | (1u << byte_of(lf, J)) | (1u << byte_of(rt, J));
  const uint32_t j1 = j + 1u;
  uint32_t kk = j1 + __popc(__builtin_amdgcn_ubfe(m, 0u, j1));
  kk = j1 + __popc(__builtin_amdgcn_ubfe(m, 0u, kk));
  kk = j1 + __popc(__builtin_amdgcn_ubfe(m, 0u, kk));
  return j + __popc(__builtin_amdgcn_ubfe(m, 0u, kk));
}

// The j-th value (from 0, ascending) that none of a, b, c, d holds.
__device__ __forceinline__ uint32_t free_value(uint32_t j, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  auto order = [](uint32_t &x, uint32_t &y) {
    const uint32_t lo = min(x, y), hi = max(x, y);
    x = lo;
    y = hi;
  };
  order(a, b);
  order(c, d);
  order(a, c);
  order(b, d);
  order(b, c);
  uint32_t k = j;
  k += a <= k;
  k += b != a && b <= k;
  k += c != b && c <= k;
  k += d != c && d <= k;
  return k;
}

// The new value of byte J of a 4-site group: up/dn/lf/rt the neighbour dwords,
// pf their pattern bytes, w the site's word.  Written into byte J of out.
template <int J, int CMP, bool WIDE>
__device__ __forceinline__ void draw(uint32_t &out, uint32_t up, uint32_t dn, uint32_t lf, uint32_t rt, uint32_t pf,
                                     uint32_t w, const uint8_t *tab) {
  const uint32_t off = table_offset<J, 2>(pf);
  const u32x4 zs = *reinterpret_cast<const u32x4 *>(tab + HbTable::kZs + off);   // Z lo/hi, S lo/hi
  const uint2 wi = *reinterpret_cast<const uint2 *>(tab + HbTable::kWi + off);   // w0, 1/w0 rounded up (FP32)
  const uint64_t S = ((uint64_t)zs.w << 32) | zs.z;
  // X = floor(w Z / 2^32) - S (Z = zs.y 2^32 + zs.x < 2^41), modulo 2^64: when
  // the draw lands in the run of values no neighbour holds (r >= S) it is the
  // offset into that run, X < 2^40; otherwise a cut below picks a neighbour
  // value and what follows from X is overwritten.
  const uint64_t X = (uint64_t)w * zs.y + __umulhi(w, zs.x) - S;
  // j = floor(X / w0): the FP32 estimate lies in [X / w0, X / w0 + 2^-10) (the
  // reciprocal carries a 2^-19 upward bias against four roundings of 2^-24 and
  // X / w0 < 256), so it is exact or one too high
  const float xf = __builtin_fmaf(cvt_f32((uint32_t)(X >> 32)), 4294967296.0f, cvt_f32((uint32_t)X));
  const uint32_t je = cvt_u32_sat(xf * __uint_as_float(wi.y));
  const uint32_t j = je - (uint32_t)((uint64_t)je * wi.x > X);
  uint32_t k;
  if (CMP == 0) {
    k = free_value16<J>(j, up, dn, lf, rt);
  } else {
    k = free_value(j, byte_of(up, J), byte_of(dn, J), byte_of(lf, J), byte_of(rt, J));
  }
  if (!WIDE) {
    // narrow cuts: rank i wins when w <= cut_i (= ceil(c_i 2^32 / Z) - 1)
    const u32x4 cut = *reinterpret_cast<const u32x4 *>(tab + HbTable::kCut + off);
    place_select<J>(out, w, cut.w, k, rt);
    select_byte<J>(out, w, cut.z, lf);
    select_byte<J>(out, w, cut.y, dn);
    select_byte<J, true>(out, w, cut.x, up);
  } else {
    // wide cuts (some weights are 0): rank i wins when w < cut_i, cut_i <= 2^32
    const uint64_t *c64 = reinterpret_cast<const uint64_t *>(tab + HbTable::kCut64 + 2 * off);
    uint32_t v = k;
    if ((uint64_t)w < c64[3]) v = byte_of(rt, J);
    if ((uint64_t)w < c64[2]) v = byte_of(lf, J);
    if ((uint64_t)w < c64[1]) v = byte_of(dn, J);
    if ((uint64_t)w < c64[0]) v = byte_of(up, J);
    out = (out & ~(0xFFu << (8 * J))) | ((v & 0xFFu) << (8 * J));
  }
}

// Four sites (one packed dword, group g of an item row): words wa..wd.
template <int CMP, bool WIDE>
__device__ __forceinline__ uint32_t draw4(uint32_t up, uint32_t dn, uint32_t lf, uint32_t rt, uint32_t w0_,
                                          uint32_t w1_, uint32_t w2_, uint32_t w3_, const uint8_t *tab) {
  const uint32_t pf = pair_pattern<CMP>(up, dn, lf, rt);
  uint32_t out = 0;
  draw<0, CMP, WIDE>(out, up, dn, lf, rt, pf, w0_, tab);
  draw<1, CMP, WIDE>(out, up, dn, lf, rt, pf, w1_, tab);
  draw<2, CMP, WIDE>(out, up, dn, lf, rt, pf, w2_, tab);
  draw<3, CMP, WIDE>(out, up, dn, lf, rt, pf, w3_, tab);
  return out;
}

struct HbCarry {
  u32x4 u;  // passive row y-1
  u32x4 p;  // passive row y
};

// One item row: the 16 active sites at a_off (written), the passive row below
// at d_off, the passive dword beside the item at side_off (left of it when
// O == 0, right of it when O == 1).  ctr: Philox chunk of the item's first
// byte (a multiple of 8), h: the half sweep's Philox head.
template <int COLOUR, int O, int CMP, bool PRIV, bool WIDE>
__device__ __forceinline__ void hb_row(const PhiloxHead &h, __amdgpu_buffer_rsrc_t rs, const uint8_t *tab,
                                       uint8_t *hist, uint32_t lane_off, uint32_t a_off, uint32_t d_off,
                                       uint32_t side_off, uint32_t ctr, HbCarry &cy, uint32_t &nz) {
  const u32x4 dn = load16(rs, d_off);
  const uint32_t side = load4(rs, side_off);
  const uint32_t P[4] = {cy.p.x, cy.p.y, cy.p.z, cy.p.w};
  const uint32_t U[4] = {cy.u.x, cy.u.y, cy.u.z, cy.u.w};
  const uint32_t D[4] = {dn.x, dn.y, dn.z, dn.w};
  uint32_t out[4];
  const uint32_t x0 = h.a0 ^ ctr;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    // the other horizontal neighbour: the passive byte one site over
    const uint32_t x = O == 0 ? alignbyte(P[g], g == 0 ? side : P[g - 1], 3)
                              : alignbyte(g == 3 ? side : P[g + 1], P[g], 1);
    const uint32_t lf = O == 0 ? x : P[g];
    const uint32_t rt = O == 0 ? P[g] : x;
    // packed bytes 4g, 4g+1 use block 2g (words 0, 2), 4g+2, 4g+3 block 2g+1
    const Words b0 = philox_tail(x0 ^ (uint32_t)(2 * g), h);
    const Words b1 = philox_tail(x0 ^ (uint32_t)(2 * g + 1), h);
    out[g] = draw4<CMP, WIDE>(U[g], D[g], lf, rt, b0.w0, b0.w2, b1.w0, b1.w2, tab);
    if (COLOUR == 1) nz += __popc(diff_pattern<CMP>(out[g], U[g], D[g], lf, rt) & 0xF0F0F0F0u);
  }
  u32x4 o;
  o.x = out[0];
  o.y = out[1];
  o.z = out[2];
  o.w = out[3];
  store16(rs, a_off, o);
  if (PRIV) {
    count_active_private(hist, lane_off, out[0], out[1]);
    count_active_private(hist, lane_off, out[2], out[3]);
  } else {
    count_active_shared(reinterpret_cast<uint32_t *>(hist), out[0], out[1]);
    count_active_shared(reinterpret_cast<uint32_t *>(hist), out[2], out[3]);
  }
  cy.u = cy.p;
  cy.p = dn;
}

// The compiler's register choice (about 92 VGPRs, 5 waves per SIMD) measured
// faster than 6 or 8 waves per SIMD forced (1.81 against 1.91 and 1.94 ps per
// site update at L = 8192, q = 9: the forced forms spill inside the loop).
template <int COLOUR, int CMP, bool PRIV, bool WIDE>
__global__ __launch_bounds__(kBlock) void hb_packed_kernel(HbLaunch launch) {
  __shared__ __align__(16) uint8_t tab[HbTable::kBytes];
  constexpr uint32_t kHistWords = PRIV ? 64u * (CMP == 0 ? 16u : kPrivateHistMaxQ) : 256u;
  __shared__ __align__(16) uint32_t hist[kHistWords];
  __shared__ uint32_t partial[256];
  __shared__ unsigned long long esum;
  const StripParams &p = launch.p;
  const uint32_t bid = COLOUR == 1 ? gridDim.x - 1 - blockIdx.x : blockIdx.x;
  const uint32_t first = bid * kBlock + threadIdx.x;
  const uint32_t stride = gridDim.x * kBlock;
  const uint64_t t = p.t0 + launch.sweep;
  const PhiloxHead h = philox_head((uint32_t)t, (uint32_t)(t >> 32), (uint32_t)COLOUR + 4u, p.k0, p.k1);
  const uint32_t q = p.q;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = threadIdx.x >> 6;

  {
    const u32x4 *src = reinterpret_cast<const u32x4 *>(launch.table);
    u32x4 *dst = reinterpret_cast<u32x4 *>(tab);
    const uint32_t n = (WIDE ? HbTable::kBytes : HbTable::kCut64) / 16;
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) dst[i] = src[i];
  }
  const uint32_t nh = PRIV ? 64 * q : q;
  for (uint32_t i = threadIdx.x; i < nh; i += kBlock) hist[i] = 0;
  if (threadIdx.x == 0) esum = 0;
  if (p.stripes) {
    __shared__ unsigned long long fold_acc[COLOUR == 0 ? 257 : 1];
    if (COLOUR == 0 && bid == 0 && launch.sweep > 0) fold_stripes<kBlock>(p, t - 1, fold_acc);
  } else if (COLOUR == 1 && bid == 0) {
    unsigned long long *rec_next = p.ring + ((t + 1) & (p.cap - 1)) * (uint64_t)(q + 1);
    for (uint32_t i = threadIdx.x; i < q + 1; i += kBlock) rec_next[i] = 0;
  }
  __syncthreads();

  const __amdgpu_buffer_rsrc_t rs = lattice_rsrc(p.spins);
  uint8_t *hist_bytes = reinterpret_cast<uint8_t *>(hist);
  const uint32_t lane_off = lane * 4u;
  const uint32_t L = p.L;
  const uint32_t half = L >> 1;
  const uint32_t plane = half * L;
  const uint32_t a_base = COLOUR == 0 ? 0u : plane;
  const uint32_t p_base = COLOUR == 0 ? plane : 0u;
  const uint32_t rows = p.rows;
  uint32_t nz = 0, sites = 0;

  for (uint32_t item = first; item < p.nitems; item += stride) {
    const uint32_t rb = p.item_shift >= 0 ? item >> p.item_shift
                                          : (uint32_t)__umul64hi((uint64_t)item, p.item_magic);
    const uint32_t xi = item - rb * p.ipr;
    const uint32_t col = xi * 16u;
    const uint32_t left_col = col == 0 ? half - 4 : col - 4;
    const uint32_t right_col = col + 16 == half ? 0u : col + 16;
    const uint32_t r0 = rb * rows;
    const uint32_t rp = r0 == 0 ? L - 1 : r0 - 1;
    HbCarry cy;
    cy.u = load16(rs, p_base + rp * half + col);
    cy.p = load16(rs, p_base + r0 * half + col);
    uint32_t ctr = r0 * p.row_words + (col >> 1);
    constexpr bool kLeftFirst = COLOUR == 0;  // row parity 0: O = COLOUR
    for (uint32_t k = 0; k < rows; k += 2) {
      const uint32_t y = r0 + k;
      hb_row<COLOUR, COLOUR, CMP, PRIV, WIDE>(h, rs, tab, hist_bytes, lane_off, a_base + y * half + col,
                                               p_base + (y + 1) * half + col,
                                               p_base + y * half + (kLeftFirst ? left_col : right_col), ctr, cy, nz);
      ctr += p.row_words;
      const uint32_t yd = k + 2 == rows ? (r0 + rows == L ? 0u : r0 + rows) : y + 2;
      hb_row<COLOUR, COLOUR ^ 1, CMP, PRIV, WIDE>(h, rs, tab, hist_bytes, lane_off, a_base + (y + 1) * half + col,
                                                   p_base + yd * half + col,
                                                   p_base + (y + 1) * half + (kLeftFirst ? right_col : left_col),
                                                   ctr, cy, nz);
      ctr += p.row_words;
    }
    sites += 16 * rows;
  }

  if (COLOUR == 1) {
    const uint32_t e = wave_sum(4u * sites - nz);
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
  unsigned long long *rec = p.ring + (t & (p.cap - 1)) * (uint64_t)(q + 1);
  unsigned long long *dst =
      p.stripes ? p.stripes + ((t & 1) * p.nstripes + (bid & (p.nstripes - 1))) * (uint64_t)stripe_words(q) : rec;
  for (uint32_t v = threadIdx.x; v < q; v += kBlock) {
    const uint32_t s = PRIV ? partial[v] : hist[v];
    if (s) atomicAdd(&dst[1 + v], (unsigned long long)s);
  }
  if (COLOUR == 1 && threadIdx.x == 0 && esum) atomicAdd(&dst[0], esum);
}

template <int COLOUR, bool WIDE>
hipError_t launch_w(const HbLaunch &l, unsigned grid, uint32_t q, hipStream_t stream) {
  if (q <= 16)
    hipLaunchKernelGGL((hb_packed_kernel<COLOUR, 0, true, WIDE>), dim3(grid), dim3(kBlock), 0, stream, l);
  else if (q <= kPrivateHistMaxQ)
    hipLaunchKernelGGL((hb_packed_kernel<COLOUR, 1, true, WIDE>), dim3(grid), dim3(kBlock), 0, stream, l);
  else if (q <= 128)
    hipLaunchKernelGGL((hb_packed_kernel<COLOUR, 1, false, WIDE>), dim3(grid), dim3(kBlock), 0, stream, l);
  else
    hipLaunchKernelGGL((hb_packed_kernel<COLOUR, 2, false, WIDE>), dim3(grid), dim3(kBlock), 0, stream, l);
  return hipGetLastError();
}

}  // namespace

bool build_heatbath_table(const uint32_t thr[4], uint32_t q, HbTable *t) {
  memset(t->bytes, 0, sizeof(t->bytes));
  const bool wide = !thr[0] || !thr[1] || !thr[2] || !thr[3];
  uint32_t *cut = reinterpret_cast<uint32_t *>(t->bytes + HbTable::kCut);
  uint32_t *zs = reinterpret_cast<uint32_t *>(t->bytes + HbTable::kZs);
  uint32_t *wi = reinterpret_cast<uint32_t *>(t->bytes + HbTable::kWi);
  uint64_t *cut64 = reinterpret_cast<uint64_t *>(t->bytes + HbTable::kCut64);
  auto weight = [&](uint32_t gap) -> uint64_t { return gap == 0 ? (1ull << 32) : (uint64_t)thr[gap - 1]; };
  for (uint32_t pat = 0; pat < 64; ++pat) {
    const uint32_t eab = !(pat & 32u), eac = !(pat & 16u), ead = !(pat & 8u);
    const uint32_t ebc = !(pat & 4u), ebd = !(pat & 2u), ecd = !(pat & 1u);
    const uint32_t na = 1 + eab + eac + ead, nb = 1 + eab + ebc + ebd;
    const uint32_t nc = 1 + eac + ebc + ecd, nd = 1 + ead + ebd + ecd;
    const uint32_t nmax = std::max(std::max(na, nb), std::max(nc, nd));
    // b, c, d count where they appear first
    const bool fb = !eab, fc = !eac && !ebc, fd = !ead && !ebd && !ecd;
    const uint64_t wa = weight(nmax - na);
    const uint64_t wb = fb ? weight(nmax - nb) : 0;
    const uint64_t wc = fc ? weight(nmax - nc) : 0;
    const uint64_t wd = fd ? weight(nmax - nd) : 0;
    const uint32_t m = 1 + fb + fc + fd;
    const uint64_t w0 = nmax >= 1 && nmax <= 4 ? (uint64_t)thr[nmax - 1] : 0;
    const uint64_t S = wa + wb + wc + wd;
    uint64_t Z = S + (q > m ? (uint64_t)(q - m) * w0 : 0);
    if (Z == 0) Z = 1;  // a pattern no four values show (equality is transitive)
    const uint64_t c[4] = {wa, wa + wb, wa + wb + wc, S};
    for (int i = 0; i < 4; ++i) {
      // r = floor(w Z / 2^32) < c  <=>  w < ceil(c 2^32 / Z)
      const unsigned __int128 num = ((unsigned __int128)c[i] << 32) + (Z - 1);
      uint64_t T = (uint64_t)(num / Z);
      if (T > (1ull << 32)) T = 1ull << 32;
      cut64[pat * 4 + i] = T;
      cut[pat * 4 + i] = T == 0 ? 0u : (uint32_t)(T - 1);
    }
    zs[pat * 4 + 0] = (uint32_t)Z;
    zs[pat * 4 + 1] = (uint32_t)(Z >> 32);
    zs[pat * 4 + 2] = (uint32_t)S;
    zs[pat * 4 + 3] = (uint32_t)(S >> 32);
    // 1/w0 rounded up by 2^-19 relative, so the kernel's FP32 estimate of
    // floor(X / w0) is never below it
    const float inv = w0 ? (float)((1.0 + 0x1p-19) / (double)w0) : 0.0f;
    uint32_t inv_bits;
    memcpy(&inv_bits, &inv, 4);
    wi[pat * 4 + 0] = (uint32_t)w0;
    wi[pat * 4 + 1] = inv_bits;
  }
  return wide;
}

hipError_t launch_heatbath_packed(const HbLaunch &l, int colour, unsigned grid, bool wide, hipStream_t stream) {
  if (grid == 0) return hipSuccess;
  const uint32_t q = l.p.q;
  if (colour == 0) return wide ? launch_w<0, true>(l, grid, q, stream) : launch_w<0, false>(l, grid, q, stream);
  return wide ? launch_w<1, true>(l, grid, q, stream) : launch_w<1, false>(l, grid, q, stream);
}

}  // namespace potts
