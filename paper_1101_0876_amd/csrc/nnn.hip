// nnn.hip -- the square lattice with first and second neighbours (Sec. 7:
// with second-neighbour couplings the lattice splits into nine independent
// sub-lattices instead of two).  Contract:
//   - H = -sum_<ij> delta - j2 sum_<<ij>> delta over the four nearest and the
//     four diagonal neighbours (Eq. 1 extended);
//   - L x L periodic, L % 12 == 0; colour c = 3 (y mod 3) + (x mod 3), one
//     sweep = colours 0..8 in turn;
//   - table entry (d1 + 4) * 9 + (d2 + 4), d1/d2 = the drops in equal
//     nearest/diagonal neighbours from the current value to the proposal:
//     2^32 when d1 + j2 d2 <= 0, else min(floor(exp(-beta (d1 + j2 d2)) 2^32),
//     2^32 - 1); accept iff w_acc < entry;
//   - Philox block per (6-byte row segment, sweep, colour): counter (t_lo,
//     y L/6 + x/6, t_hi, 16 + colour); site x takes (w[2b], w[2b+1]),
//     b = (x/3) & 1 (a segment holds two sites of each colour); initial
//     conditions as on the nearest-neighbour lattice;
//   - records {e1, e2, hist[q]} per sweep: nearest and diagonal satisfied
//     bonds (2N each) and the populations.
//
// Kernels: up to L = 16380 one launch per row class (y mod 3) does the
// three colours of that class with the three rows around each active row in
// LDS (below).  Beyond that, a colour pass runs one thread per 6-byte segment
// of the rows of its colour: the segment's two active sites (x0 = 6m + cx and x0 + 3) and
// their neighbours are the six bytes x0-1 .. x0+4 of rows y-1, y, y+1, read
// as three dwords per row and shifted into place with v_alignbyte and v_perm
// (byte 0: the first site's view, byte 1: the second's); both sites are
// compared at once as flag patterns and written back with byte stores, so
// neighbouring threads never rewrite each other's bytes.  The row-class
// launches count the record of their sweep as they go (partial sums in
// striped slots, folded by a one-block kernel); after the per-colour passes
// it comes from one measurement kernel over the final lattice.
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/potts.h"
#include "device.hpp"
#include "sweep_row.hpp"

struct potts_nnn_state {
  int32_t L = 0, q = 0;
  uint64_t seed = 0;
  int64_t t = 0;
  uint8_t *spins = nullptr;
  hipStream_t stream = nullptr;
  unsigned long long *records = nullptr;  // ring of rec_cap slots of 2 + q
  int64_t rec_cap = 0;
  unsigned long long *scratch = nullptr;  // 2 + q words for measurements
  unsigned long long *stripes = nullptr;  // kStripes partial records of 2 + q words, kept zero between sweeps
  int32_t kernel = 0;  // 0 automatic, 1 row class in LDS, 2 segment per colour
  bool have_thr = false;
  double thr_beta = 0.0, thr_j2 = 0.0;
  uint64_t thr[81] = {};
};

namespace potts {
int record_error(int code, const std::string &msg);
}

namespace {

using potts::PhiloxHead;
using potts::row::diff_pattern;
using potts::row::alignbyte;
using potts::row::lattice_rsrc;
using potts::row::load4;
using potts::row::perm;
using potts::Words;
using potts::byte_of;
using potts::count_equal;
using potts::philox4x32_10;
using potts::philox_head;
using potts::philox_tail;
using potts::scale_to_q;
using potts::wave_sum;
using potts::zero_bytes;

constexpr int kBlock = 256;
constexpr int64_t kRingSlots = 4096;
// partial records in striped slots (workgroup number mod kStripes), so that
// no record word takes more than a few hundred atomics; a one-block kernel
// folds them into the ring slot
constexpr uint32_t kStripes = 32;

struct NnnLattice {
  uint8_t *spins;
  uint32_t L, q;
  uint32_t k0, k1;
};

struct NnnPass {
  NnnLattice g;
  uint32_t t_lo, t_hi;
  uint32_t colour;
  uint64_t thr[81];
};

__device__ __forceinline__ uint32_t alignb(uint32_t hi, uint32_t lo, uint32_t shift) {
  return __builtin_amdgcn_alignbyte(hi, lo, shift);
}

// Grid: x over the segments of a row, y over the rows of the pass's colour.
// The four neighbour groups are compared with the current values and the
// proposals as byte-wise "differs" flag patterns (bits 7..4 of every byte, the
// row kernels' diff_pattern, CMP by q); a site's counts are the popcounts of
// its pattern byte: d1 = n1(s) - n1(k) = diff1(k) - diff1(s).
// k: "differs from the proposal" flags, s: "differs from the current value"
// flags, at bits 7..4 of every byte (bits 3..0 garbage): per byte, the
// proposal's flags above and the current value's "equal" flags below, so
// that the popcount of byte j is 4 - n(k) + n(s) = d + 4 for its site.
__device__ __forceinline__ uint32_t count_flags(uint32_t k, uint32_t s) {
  return (k & 0xF0F0F0F0u) | ((~s >> 4) & 0x0F0F0F0Fu);
}

template <int CMP>
__global__ __launch_bounds__(kBlock) void nnn_pass_kernel(NnnPass p) {
  __shared__ uint64_t table[81];
  for (uint32_t i = threadIdx.x; i < 81; i += kBlock) table[i] = p.thr[i];
  __syncthreads();
  const uint32_t L = p.g.L, cpr = L >> 2, spr = L / 6;
  const uint32_t m = blockIdx.x * kBlock + threadIdx.x;
  if (m >= spr) return;
  const uint32_t cy = p.colour / 3, cx = p.colour - 3 * cy;
  const uint32_t y = 3 * blockIdx.y + cy;
  const uint32_t yu = y == 0 ? L - 1 : y - 1, yd = y + 1 == L ? 0 : y + 1;
  // the rows are the same for the whole workgroup: buffer resources in scalar
  // registers, 32-bit lane offsets
  const __amdgpu_buffer_rsrc_t row = lattice_rsrc(p.g.spins + (size_t)y * L);
  const __amdgpu_buffer_rsrc_t up = lattice_rsrc(p.g.spins + (size_t)yu * L);
  const __amdgpu_buffer_rsrc_t dn = lattice_rsrc(p.g.spins + (size_t)yd * L);
  // window: bytes x0-1 .. x0+4 (periodic), from three dwords starting at d0
  const uint32_t x0 = 6 * m + cx;
  const uint32_t w0 = x0 == 0 ? L - 1 : x0 - 1;
  const uint32_t d0 = w0 >> 2, sh = w0 & 3u;
  const uint32_t o0 = 4 * d0, o1 = 4 * (d0 + 1 == cpr ? 0 : d0 + 1), o2 = 4 * (d0 + 2 >= cpr ? d0 + 2 - cpr : d0 + 2);
  // per row: (centre, left, right) dwords whose byte 0 is the first site's
  // view (x0 + 0, -1, +1) and byte 1 the second site's (x0 + 3 + 0, -1, +1)
  auto views = [&](const __amdgpu_buffer_rsrc_t &r, uint32_t &c, uint32_t &l, uint32_t &rt) {
    const uint32_t a = load4(r, o0), b = load4(r, o1), d = load4(r, o2);
    const uint32_t lo = alignbyte(b, a, sh), hi = alignbyte(d, b, sh);  // window bytes 0..3, 4..7
    c = perm(hi, lo, 0x0C0C0401u);   // bytes 1, 4
    l = perm(hi, lo, 0x0C0C0300u);   // bytes 0, 3
    rt = perm(hi, lo, 0x0C0C0502u);  // bytes 2, 5
  };
  uint32_t cur, left, right, U, ul, ur, D, dl, dr;
  views(row, cur, left, right);
  views(up, U, ul, ur);
  views(dn, D, dl, dr);

  const PhiloxHead h = philox_head(p.t_lo, p.t_hi, 16u + p.colour, p.g.k0, p.g.k1);
  const Words w = philox_tail(h.a0 ^ (y * spr + m), h);  // segment x0 / 6 == m
  const uint32_t prop = scale_to_q(w.w0, p.g.q) | (scale_to_q(w.w2, p.g.q) << 8);
  const uint32_t s1 = diff_pattern<CMP>(cur, left, right, U, D), k1 = diff_pattern<CMP>(prop, left, right, U, D);
  const uint32_t s2 = diff_pattern<CMP>(cur, ul, ur, dl, dr), k2 = diff_pattern<CMP>(prop, ul, ur, dl, dr);
  const uint32_t x1 = x0 + 3;
  const uint32_t c1 = count_flags(k1, s1), c2 = count_flags(k2, s2);
#pragma unroll
  for (uint32_t i = 0; i < 2; ++i) {
    const uint32_t mk = 0xFFu << (8 * i);
    const uint32_t wacc = i == 0 ? w.w1 : w.w3;
    if ((uint64_t)wacc < table[__popc(c1 & mk) * 9 + __popc(c2 & mk)])
      __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(prop >> (8 * i)), row, i == 0 ? x0 : x1, 0, 0);
  }
}

// The three colours of one row class (y mod 3 == cy) in one launch: a
// workgroup per active row y holds rows y-1, y, y+1 in LDS (each padded with
// the periodic dword on both ends) and runs the sub-passes cx = 0, 1, 2 with a
// barrier between them (a site's neighbours in row y have the other residues
// mod 3, rows y +- 1 are not updated by this class), then writes row y back.
// Within a sub-pass a thread takes a 12-byte block of row y: its four sites
// x = 12k + cx + 3j (j = 0..3), the two Philox blocks of segments 2k and
// 2k + 1, and all four sites compared at once.  Lattices up to kRowsMaxL.
constexpr uint32_t kRowsMaxL = 16380;

// bytes R0..R3 of the five dwords d[0..4] (byte r = d[r/4].byte(r%4))
template <int R0, int R1, int R2, int R3>
__device__ __forceinline__ uint32_t gather4(const uint32_t d[5]) {
  constexpr uint32_t s01 = 0x0C0C0000u | (uint32_t)(R0 % 4) | ((uint32_t)(R1 / 4 == R0 / 4 ? R1 % 4 : 4 + R1 % 4) << 8);
  constexpr uint32_t s23 = 0x0C0C0000u | (uint32_t)(R2 % 4) | ((uint32_t)(R3 / 4 == R2 / 4 ? R3 % 4 : 4 + R3 % 4) << 8);
  const uint32_t lo = perm(d[R1 / 4], d[R0 / 4], s01);
  const uint32_t hi = perm(d[R3 / 4], d[R2 / 4], s23);
  return perm(hi, lo, 0x05040100u);
}

// left, centre and right views of the four sites for sub-pass CX: byte j of
// each is the byte at x - 1, x, x + 1 for site j (dword 0 starts at 12k - 4)
template <int CX>
__device__ __forceinline__ void row_views(const uint32_t d[5], uint32_t &l, uint32_t &c, uint32_t &r) {
  l = gather4<3 + CX, 6 + CX, 9 + CX, 12 + CX>(d);
  c = gather4<4 + CX, 7 + CX, 10 + CX, 13 + CX>(d);
  r = gather4<5 + CX, 8 + CX, 11 + CX, 14 + CX>(d);
}

// The record of a sweep is counted while the row-class launches run: a bond
// is counted when its later-coloured end is updated (its other end is final
// then, and the colours are updated in increasing order), from that site's
// final value; every site's final value is counted when it is updated.
// Which of a site's neighbours come earlier depends only on its row class cy
// and column class cx: left when cx >= 1, right when cx == 2, the row above
// (and its diagonals) when cy >= 1, the row below when cy == 2.  mask1 / mask2
// select those neighbours' flags (bits 7..4: left, right, up, down / up-left,
// up-right, down-left, down-right) in every byte.
struct RowRecord {
  uint32_t mask1, mask2;
  uint32_t e1, e2;      // this thread's satisfied nearest / diagonal bonds
  uint8_t *hist;        // PRIV: lane-private columns (value << 8 | lane * 4), else q shared bins
  uint32_t lane_off;
};

template <bool PRIV>
__device__ __forceinline__ void count_values(RowRecord &r, uint32_t v) {
#pragma unroll
  for (uint32_t b = 0; b < 4; ++b) {
    if (PRIV)
      atomicAdd(reinterpret_cast<uint32_t *>(r.hist + perm(v, r.lane_off, 0x0C0C0000u | ((4u + b) << 8))), 1u);
    else
      atomicAdd(reinterpret_cast<uint32_t *>(r.hist) + byte_of(v, b), 1u);
  }
}

template <int CMP, int CX, bool PRIV>
__device__ __forceinline__ void rows_subpass(const NnnPass &p, uint32_t y, uint32_t *ru, uint32_t *rc, uint32_t *rd,
                                             const uint64_t *table, RowRecord &rec) {
  {
    const uint32_t cy = p.colour;
    const uint32_t l_lo = CX >= 1, r_lo = CX == 2, u_lo = cy >= 1, d_lo = cy == 2;
    rec.mask1 = ((l_lo << 7) | (r_lo << 6) | (u_lo << 5) | (d_lo << 4)) * 0x01010101u;
    rec.mask2 = ((u_lo << 7) | (u_lo << 6) | (d_lo << 5) | (d_lo << 4)) * 0x01010101u;
  }
  const uint32_t L = p.g.L, nblk = L / 12, spr = L / 6;
  const PhiloxHead h = philox_head(p.t_lo, p.t_hi, 16u + 3u * p.colour + CX, p.g.k0, p.g.k1);
  uint8_t *rcb = reinterpret_cast<uint8_t *>(rc);
  for (uint32_t k = threadIdx.x; k < nblk; k += kBlock) {
    // padded dwords 3k .. 3k+4 hold x = 12k - 4 .. 12k + 15
    uint32_t du[5], dc[5], dd[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      du[i] = ru[3 * k + i];
      dc[i] = rc[3 * k + i];
      dd[i] = rd[3 * k + i];
    }
    uint32_t left, cur, right, ul, U, ur, dl, D, dr;
    row_views<CX>(dc, left, cur, right);
    row_views<CX>(du, ul, U, ur);
    row_views<CX>(dd, dl, D, dr);
    const uint32_t seg = y * spr + 2 * k;
    const Words a = philox_tail(h.a0 ^ seg, h);
    const Words b = philox_tail(h.a0 ^ (seg + 1), h);
    const uint32_t q = p.g.q;
    const uint32_t prop = scale_to_q(a.w0, q) | (scale_to_q(a.w2, q) << 8) | (scale_to_q(b.w0, q) << 16) |
                          (scale_to_q(b.w2, q) << 24);
    const uint32_t s1 = diff_pattern<CMP>(cur, left, right, U, D), k1 = diff_pattern<CMP>(prop, left, right, U, D);
    const uint32_t s2 = diff_pattern<CMP>(cur, ul, ur, dl, dr), k2 = diff_pattern<CMP>(prop, ul, ur, dl, dr);
    const uint32_t c1 = count_flags(k1, s1), c2 = count_flags(k2, s2);
    const uint32_t wacc[4] = {a.w1, a.w3, b.w1, b.w3};
    uint32_t sel = 0x03020100u;  // byte j from the proposal (4 + j) or the current value (j)
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      const uint32_t mk = 0xFFu << (8 * j);
      if ((uint64_t)wacc[j] < table[__popc(c1 & mk) * 9 + __popc(c2 & mk)]) {
        rcb[4 + 12 * k + CX + 3 * j] = (uint8_t)(prop >> (8 * j));
        sel |= 4u << (8 * j);
      }
    }
    // the final values' "differs" flags; equal earlier neighbours are bonds
    rec.e1 += __popc(rec.mask1 & ~perm(k1, s1, sel));
    rec.e2 += __popc(rec.mask2 & ~perm(k2, s2, sel));
    count_values<PRIV>(rec, perm(prop, cur, sel));
  }
}

// LDS row stride of the row-class kernel: the three rows are copied in
// chunks of 64 dwords to dwords 1 .. 64 * ceil(L/256) of their LDS rows, with
// the periodic dwords at 0 and L/4 + 1.
__host__ __device__ inline uint32_t rows_stride(uint32_t L) { return 64u * (((L >> 2) + 63u) >> 6) + 2u; }

// PRIV (q <= 16): populations in 16 lane-private LDS columns, else q shared
// bins.  The record is added into stripe blockIdx.x mod kStripes of stripes.
template <int CMP, bool PRIV>
__global__ __launch_bounds__(kBlock) void nnn_rows_kernel(NnnPass p, unsigned long long *stripes) {
  extern __shared__ uint32_t rows_lds[];
  __shared__ uint64_t table[81];
  __shared__ __align__(16) uint32_t hist[PRIV ? 64 * 16 : 256];
  __shared__ uint32_t part[256 + 2];
  for (uint32_t i = threadIdx.x; i < 81; i += kBlock) table[i] = p.thr[i];
  const uint32_t q = p.g.q;
  for (uint32_t i = threadIdx.x; i < (PRIV ? 64 * q : q); i += kBlock) hist[i] = 0;
  if (threadIdx.x < 2) part[256 + threadIdx.x] = 0;
  RowRecord rec{0u, 0u, 0u, 0u, reinterpret_cast<uint8_t *>(hist), (threadIdx.x & 63u) * 4u};
  const uint32_t L = p.g.L, cpr = L >> 2, W = rows_stride(L);
  const uint32_t y = 3 * blockIdx.x + p.colour;  // p.colour: the row class cy
  const uint32_t yu = y == 0 ? L - 1 : y - 1, yd = y + 1 == L ? 0 : y + 1;
  uint32_t *ru = rows_lds, *rc = rows_lds + W, *rd = rows_lds + 2 * W;
  // row resources that end with the row: the lanes of a chunk past its end
  // read zeros, which land in the slack of the LDS row
  const __amdgpu_buffer_rsrc_t grow = __builtin_amdgcn_make_buffer_rsrc(p.g.spins + (size_t)y * L, 0, (int)L, 0x00020000);
  const __amdgpu_buffer_rsrc_t gup = __builtin_amdgcn_make_buffer_rsrc(p.g.spins + (size_t)yu * L, 0, (int)L, 0x00020000);
  const __amdgpu_buffer_rsrc_t gdn = __builtin_amdgcn_make_buffer_rsrc(p.g.spins + (size_t)yd * L, 0, (int)L, 0x00020000);
  // straight from memory into LDS, 64 dwords per wave instruction, with no
  // register round trip and no wait before the barrier
  const uint32_t lane = threadIdx.x & 63u;
  typedef __attribute__((address_space(3))) void *lds_ptr;
  for (uint32_t c = threadIdx.x >> 6; c < (cpr + 63) >> 6; c += kBlock / 64) {
    const uint32_t off = 4 * (64 * c + lane);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(gup, (lds_ptr)(ru + 1 + 64 * c), 4, off, 0, 0, 0);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(grow, (lds_ptr)(rc + 1 + 64 * c), 4, off, 0, 0, 0);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(gdn, (lds_ptr)(rd + 1 + 64 * c), 4, off, 0, 0, 0);
  }
  __syncthreads();
  if (threadIdx.x == 0) {  // periodic padding
    ru[0] = ru[cpr];
    ru[cpr + 1] = ru[1];
    rc[0] = rc[cpr];
    rc[cpr + 1] = rc[1];
    rd[0] = rd[cpr];
    rd[cpr + 1] = rd[1];
  }
  __syncthreads();
  rows_subpass<CMP, 0, PRIV>(p, y, ru, rc, rd, table, rec);
  __syncthreads();
  // the padding dwords of row y mirror its ends: refresh them after each sub-pass
  if (threadIdx.x == 0) {
    rc[0] = rc[cpr];
    rc[cpr + 1] = rc[1];
  }
  __syncthreads();
  rows_subpass<CMP, 1, PRIV>(p, y, ru, rc, rd, table, rec);
  __syncthreads();
  if (threadIdx.x == 0) {
    rc[0] = rc[cpr];
    rc[cpr + 1] = rc[1];
  }
  __syncthreads();
  rows_subpass<CMP, 2, PRIV>(p, y, ru, rc, rd, table, rec);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < cpr; i += kBlock) __builtin_amdgcn_raw_buffer_store_b32(rc[i + 1], grow, 4 * i, 0, 0);
  // the workgroup's share of the record
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t e1 = wave_sum(rec.e1), e2 = wave_sum(rec.e2);
  if (lane == 0) {
    if (e1) atomicAdd(&part[256], e1);
    if (e2) atomicAdd(&part[257], e2);
  }
  if (PRIV) {
    for (uint32_t v = wave; v < q; v += kBlock / 64) {
      const uint32_t n = wave_sum(hist[v * 64u + lane]);
      if (lane == 0) part[v] = n;
    }
  }
  __syncthreads();
  unsigned long long *dst = stripes + (blockIdx.x % kStripes) * (uint64_t)(q + 2);
  for (uint32_t v = threadIdx.x; v < q; v += kBlock) {
    const uint32_t n = PRIV ? part[v] : hist[v];
    if (n) atomicAdd(&dst[2 + v], (unsigned long long)n);
  }
  if (threadIdx.x < 2 && part[256 + threadIdx.x])
    atomicAdd(&dst[threadIdx.x], (unsigned long long)part[256 + threadIdx.x]);
}

// e1 (right, down), e2 (down-right, down-left) and populations of the
// lattice, added to one of kStripes partial records (block number mod
// kStripes, so that no record word takes more than a few hundred atomics);
// nnn_fold_kernel then sums the stripes into the record and clears them.
// Grid: x over the chunks of a row, y strided over bands of kMeasureRows rows
// (a band's loads are issued together).  PRIV (q <= 64): populations counted
// in lane-private LDS columns (no two lanes share a counter); else q shared
// bins.
constexpr uint32_t kMeasureRows = 8;
constexpr uint32_t kPrivMaxQ = 64;
constexpr uint32_t kMeasureBlocks = 2048;

template <bool PRIV>
__global__ __launch_bounds__(kBlock) void nnn_measure_kernel(NnnLattice g, unsigned long long *stripes) {
  __shared__ __align__(16) uint32_t hist[PRIV ? 64 * kPrivMaxQ : 256];
  __shared__ uint32_t part[256 + 2];
  const uint32_t q = g.q, lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  for (uint32_t i = threadIdx.x; i < (PRIV ? 64 * q : q); i += kBlock) hist[i] = 0;
  if (threadIdx.x < 2) part[256 + threadIdx.x] = 0;
  __syncthreads();
  const uint32_t L = g.L, cpr = L >> 2;
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t nbands = (L + kMeasureRows - 1) / kMeasureRows;
  uint32_t e1 = 0, e2 = 0;
  if (j < cpr) {
    const uint32_t jl = j == 0 ? cpr - 1 : j - 1, jr = j + 1 == cpr ? 0 : j + 1;
    uint8_t *hb = reinterpret_cast<uint8_t *>(hist);
    for (uint32_t band = blockIdx.y; band < nbands; band += gridDim.y) {
      const uint32_t y0 = band * kMeasureRows;
      const uint32_t rows = L - y0 < kMeasureRows ? L - y0 : kMeasureRows;
      uint32_t c[kMeasureRows + 1], r[kMeasureRows + 1], l[kMeasureRows + 1];
#pragma unroll
      for (uint32_t k = 0; k <= kMeasureRows; ++k) {
        if (k <= rows) {
          const uint32_t y = y0 + k >= L ? y0 + k - L : y0 + k;
          const uint32_t *row = reinterpret_cast<const uint32_t *>(g.spins + (size_t)y * L);
          c[k] = row[j];
          r[k] = row[jr];
          l[k] = row[jl];
        }
      }
#pragma unroll
      for (uint32_t k = 0; k < kMeasureRows; ++k) {
        if (k < rows) {
          const uint32_t cur = c[k], D = c[k + 1];
          const uint32_t right = alignb(r[k], cur, 1);
          const uint32_t dr = alignb(r[k + 1], D, 1), dl = alignb(D, l[k + 1], 3);
          e1 += __popc(zero_bytes(cur ^ right)) + __popc(zero_bytes(cur ^ D));
          e2 += __popc(zero_bytes(cur ^ dr)) + __popc(zero_bytes(cur ^ dl));
          if (PRIV) {
#pragma unroll
            for (uint32_t b = 0; b < 4; ++b)
              atomicAdd(reinterpret_cast<uint32_t *>(
                            hb + __builtin_amdgcn_perm(cur, lane * 4u, 0x0C0C0000u | ((4u + b) << 8))),
                        1u);
          } else {
            for (uint32_t b = 0; b < 4; ++b) atomicAdd(&hist[byte_of(cur, b)], 1u);
          }
        }
      }
    }
  }
  e1 = wave_sum(e1);
  e2 = wave_sum(e2);
  if (lane == 0) {
    if (e1) atomicAdd(&part[256], e1);
    if (e2) atomicAdd(&part[257], e2);
  }
  __syncthreads();
  if (PRIV) {
    for (uint32_t v = wave; v < q; v += kBlock / 64) {
      const uint32_t n = wave_sum(hist[v * 64u + lane]);
      if (lane == 0) part[v] = n;
    }
    __syncthreads();
  }
  unsigned long long *dst = stripes + ((blockIdx.y * gridDim.x + blockIdx.x) % kStripes) * (uint64_t)(q + 2);
  for (uint32_t v = threadIdx.x; v < q; v += kBlock) {
    const uint32_t n = PRIV ? part[v] : hist[v];
    if (n) atomicAdd(&dst[2 + v], (unsigned long long)n);
  }
  if (threadIdx.x < 2 && part[256 + threadIdx.x])
    atomicAdd(&dst[threadIdx.x], (unsigned long long)part[256 + threadIdx.x]);
}

// rec[i] = sum over the stripes of word i, then the stripes are cleared; every
// (stripe, word) pair is loaded by its own thread
__global__ __launch_bounds__(kBlock) void nnn_fold_kernel(unsigned long long *stripes, uint32_t words,
                                                          unsigned long long *rec) {
  __shared__ unsigned long long acc[258];
  for (uint32_t i = threadIdx.x; i < words; i += kBlock) acc[i] = 0;
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < kStripes * words; k += kBlock) {
    const unsigned long long v = stripes[k];
    if (v) {
      atomicAdd(&acc[k % words], v);
      stripes[k] = 0;
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < words; i += kBlock) rec[i] = acc[i];
}

void launch_measure(const NnnLattice &g, unsigned long long *stripes, unsigned long long *rec,
                    hipStream_t stream) {
  const uint32_t bx = ((g.L >> 2) + kBlock - 1) / kBlock;
  const uint32_t nbands = (g.L + kMeasureRows - 1) / kMeasureRows;
  const uint32_t by = std::max<uint32_t>(1u, std::min<uint32_t>(nbands, kMeasureBlocks / bx));
  if (g.q <= kPrivMaxQ)
    hipLaunchKernelGGL(nnn_measure_kernel<true>, dim3(bx, by), dim3(kBlock), 0, stream, g, stripes);
  else
    hipLaunchKernelGGL(nnn_measure_kernel<false>, dim3(bx, by), dim3(kBlock), 0, stream, g, stripes);
  hipLaunchKernelGGL(nnn_fold_kernel, dim3(1), dim3(kBlock), 0, stream, stripes, g.q + 2, rec);
}

__global__ __launch_bounds__(kBlock) void nnn_init_kernel(NnnLattice g, int random) {
  const uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint32_t cpr = g.L >> 2;
  if (c >= (uint64_t)g.L * cpr) return;
  uint32_t out = 0;
  if (random) {
    const Words w = philox4x32_10(0u, (uint32_t)c, 0u, 2u, g.k0, g.k1);
    out = scale_to_q(w.w0, g.q) | (scale_to_q(w.w1, g.q) << 8) | (scale_to_q(w.w2, g.q) << 16) |
          (scale_to_q(w.w3, g.q) << 24);
  }
  reinterpret_cast<uint32_t *>(g.spins)[c] = out;
}

int fail(int code, const std::string &msg) { return potts::record_error(code, msg); }

#define NNN_TRY(call)                                                                                \
  do {                                                                                               \
    hipError_t e_ = (call);                                                                          \
    if (e_ != hipSuccess) return fail(POTTS_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

NnnLattice lattice_of(const potts_nnn_state *s) {
  NnnLattice g;
  g.spins = s->spins;
  g.L = (uint32_t)s->L;
  g.q = (uint32_t)s->q;
  g.k0 = (uint32_t)s->seed;
  g.k1 = (uint32_t)(s->seed >> 32);
  return g;
}

void release(potts_nnn_state *s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->spins) (void)hipFree(s->spins);
  if (s->records) (void)hipFree(s->records);
  if (s->scratch) (void)hipFree(s->scratch);
  if (s->stripes) (void)hipFree(s->stripes);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

int table81(double beta, double j2, uint64_t thr[81]) {
  if (!thr) return fail(POTTS_EINVAL, "thr is NULL");
  if (!(beta >= 0.0) || !isfinite(beta)) return fail(POTTS_EINVAL, "beta must be finite and >= 0");
  if (!isfinite(j2)) return fail(POTTS_EINVAL, "j2 must be finite");
  for (int d1 = -4; d1 <= 4; ++d1)
    for (int d2 = -4; d2 <= 4; ++d2) {
      const double de = (double)d1 + j2 * (double)d2;
      uint64_t v = 1ull << 32;
      if (de > 0.0) {
        const double scaled = floor(ldexp(exp(-beta * de), 32));
        v = scaled >= 4294967295.0 ? 4294967295ull : (uint64_t)scaled;
      }
      thr[(d1 + 4) * 9 + (d2 + 4)] = v;
    }
  return POTTS_OK;
}

int run(potts_nnn_state *s, const uint64_t thr[81], int64_t nsweeps) {
  if (!s) return fail(POTTS_EINVAL, "state is NULL");
  if (nsweeps < 0) return fail(POTTS_EINVAL, "nsweeps must be >= 0");
  if (nsweeps > INT64_MAX - s->t) return fail(POTTS_ERANGE, "sweep counter overflow");
  for (int i = 0; i < 81; ++i)
    if (thr[i] > (1ull << 32)) return fail(POTTS_EINVAL, "table entries must be <= 2^32");
  if (nsweeps == 0) return POTTS_OK;
  const int64_t rl = s->q + 2;
  NnnPass p{};
  p.g = lattice_of(s);
  for (int i = 0; i < 81; ++i) p.thr[i] = thr[i];
  const uint32_t L = (uint32_t)s->L;
  const dim3 pass_grid((L / 6 + kBlock - 1) / kBlock, L / 3);
  const bool rows = s->kernel == 1 || (s->kernel == 0 && L <= kRowsMaxL);
  const size_t rows_lds = (size_t)3 * rows_stride(L) * 4;
  for (int64_t k = 0; k < nsweeps; ++k) {
    const int64_t t = s->t + k;
    p.t_lo = (uint32_t)(uint64_t)t;
    p.t_hi = (uint32_t)((uint64_t)t >> 32);
    for (uint32_t c = 0; rows && c < 3; ++c) {
      p.colour = c;  // the row class
      if (s->q <= 16)
        hipLaunchKernelGGL((nnn_rows_kernel<0, true>), dim3(L / 3), dim3(kBlock), rows_lds, s->stream, p, s->stripes);
      else if (s->q <= 128)
        hipLaunchKernelGGL((nnn_rows_kernel<1, false>), dim3(L / 3), dim3(kBlock), rows_lds, s->stream, p, s->stripes);
      else
        hipLaunchKernelGGL((nnn_rows_kernel<2, false>), dim3(L / 3), dim3(kBlock), rows_lds, s->stream, p, s->stripes);
    }
    for (uint32_t c = 0; !rows && c < 9; ++c) {
      p.colour = c;
      if (s->q <= 16)
        hipLaunchKernelGGL(nnn_pass_kernel<0>, pass_grid, dim3(kBlock), 0, s->stream, p);
      else if (s->q <= 128)
        hipLaunchKernelGGL(nnn_pass_kernel<1>, pass_grid, dim3(kBlock), 0, s->stream, p);
      else
        hipLaunchKernelGGL(nnn_pass_kernel<2>, pass_grid, dim3(kBlock), 0, s->stream, p);
    }
    unsigned long long *rec = s->records + (t & (s->rec_cap - 1)) * rl;
    if (rows)  // the row-class launches counted the record into the stripes
      hipLaunchKernelGGL(nnn_fold_kernel, dim3(1), dim3(kBlock), 0, s->stream, s->stripes, (uint32_t)rl, rec);
    else
      launch_measure(p.g, s->stripes, rec, s->stream);
    NNN_TRY(hipGetLastError());
  }
  s->t += nsweeps;
  return POTTS_OK;
}

}  // namespace

extern "C" {

int potts_nnn_init(int32_t L, int32_t q, uint64_t seed, potts_start start, potts_nnn_state **out) {
  if (!out) return fail(POTTS_EINVAL, "out is NULL");
  *out = nullptr;
  if (L < 12 || L % 12 || q < 2 || q > POTTS_QMAX || (start != POTTS_ORDERED && start != POTTS_RANDOM))
    return fail(POTTS_EINVAL, "need L >= 12, L % 12 == 0, 2 <= q <= 256 and a valid start");
  if ((uint64_t)L * L / 4 >= (1ull << 32)) return fail(POTTS_ERANGE, "L*L/4 must be below 2^32");
  potts_nnn_state *s = new (std::nothrow) potts_nnn_state();
  if (!s) return fail(POTTS_ENOMEM, "host allocation failed");
  s->L = L;
  s->q = q;
  s->seed = seed;
  s->rec_cap = kRingSlots;
  if (hipStreamCreate(&s->stream) != hipSuccess || hipMalloc(&s->spins, (size_t)L * L) != hipSuccess ||
      hipMalloc(&s->records, (size_t)kRingSlots * (q + 2) * 8) != hipSuccess ||
      hipMalloc(&s->scratch, (size_t)(q + 2) * 8) != hipSuccess ||
      hipMalloc(&s->stripes, (size_t)kStripes * (q + 2) * 8) != hipSuccess) {
    (void)hipGetLastError();
    release(s);
    return fail(POTTS_ENOMEM, "device allocation failed");
  }
  const NnnLattice g = lattice_of(s);
  const uint64_t chunks = (uint64_t)L * (L >> 2);
  hipLaunchKernelGGL(nnn_init_kernel, dim3((unsigned)((chunks + kBlock - 1) / kBlock)), dim3(kBlock), 0, s->stream,
                     g, start == POTTS_RANDOM ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemsetAsync(s->stripes, 0, (size_t)kStripes * (q + 2) * 8, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    release(s);
    return fail(POTTS_EDEVICE, std::string("nnn_init_kernel: ") + hipGetErrorString(e));
  }
  *out = s;
  return POTTS_OK;
}

int potts_nnn_table(double beta, double j2, uint64_t thr[81]) { return table81(beta, j2, thr); }

int potts_nnn_sweep(potts_nnn_state *s, double beta, double j2, int64_t nsweeps) {
  if (!s) return fail(POTTS_EINVAL, "state is NULL");
  if (!s->have_thr || s->thr_beta != beta || s->thr_j2 != j2) {
    uint64_t thr[81];
    const int rc = table81(beta, j2, thr);
    if (rc) return rc;
    std::copy(thr, thr + 81, s->thr);
    s->thr_beta = beta;
    s->thr_j2 = j2;
    s->have_thr = true;
  }
  return run(s, s->thr, nsweeps);
}

int potts_nnn_sweep_thr(potts_nnn_state *s, const uint64_t thr[81], int64_t nsweeps) {
  if (!thr) return fail(POTTS_EINVAL, "thr is NULL");
  return run(s, thr, nsweeps);
}

int potts_nnn_records(potts_nnn_state *s, int64_t t0, int64_t n, int64_t *out) {
  if (!s || (!out && n > 0)) return fail(POTTS_EINVAL, "NULL argument");
  if (n < 0 || t0 < 0) return fail(POTTS_EINVAL, "negative record index or count");
  const int64_t oldest = s->t - s->rec_cap + 1;
  if (t0 < (oldest > 0 ? oldest : 0) || t0 + n > s->t) return fail(POTTS_ERANGE, "requested records are not in the ring");
  const int64_t rl = s->q + 2;
  for (int64_t done = 0; done < n;) {
    const int64_t slot = (t0 + done) & (s->rec_cap - 1);
    const int64_t run_n = std::min<int64_t>(n - done, s->rec_cap - slot);
    NNN_TRY(hipMemcpyAsync(out + done * rl, s->records + slot * rl, (size_t)(run_n * rl) * 8,
                           hipMemcpyDeviceToHost, s->stream));
    done += run_n;
  }
  NNN_TRY(hipStreamSynchronize(s->stream));
  return POTTS_OK;
}

int potts_nnn_observables(potts_nnn_state *s, potts_nnn_obs *out) {
  if (!s || !out) return fail(POTTS_EINVAL, "NULL argument");
  const int64_t rl = s->q + 2;
  launch_measure(lattice_of(s), s->stripes, s->scratch, s->stream);
  NNN_TRY(hipGetLastError());
  std::vector<int64_t> rec((size_t)rl);
  NNN_TRY(hipMemcpyAsync(rec.data(), s->scratch, (size_t)rl * 8, hipMemcpyDeviceToHost, s->stream));
  NNN_TRY(hipStreamSynchronize(s->stream));
  out->t = s->t;
  out->e1 = rec[0];
  out->e2 = rec[1];
  out->q = s->q;
  out->L = s->L;
  out->nmax = 0;
  for (int v = 0; v < POTTS_QMAX; ++v) out->hist[v] = v < s->q ? rec[2 + v] : 0;
  for (int v = 0; v < s->q; ++v) out->nmax = rec[2 + v] > out->nmax ? rec[2 + v] : out->nmax;
  return POTTS_OK;
}

int potts_nnn_get_spins(potts_nnn_state *s, uint8_t *host_out) {
  if (!s || !host_out) return fail(POTTS_EINVAL, "NULL argument");
  NNN_TRY(hipMemcpyAsync(host_out, s->spins, (size_t)s->L * s->L, hipMemcpyDeviceToHost, s->stream));
  NNN_TRY(hipStreamSynchronize(s->stream));
  return POTTS_OK;
}

int potts_nnn_tune(potts_nnn_state *s, int32_t kernel) {
  if (!s) return fail(POTTS_EINVAL, "state is NULL");
  if (kernel < 0 || kernel > 2) return fail(POTTS_EINVAL, "kernel must be 0, 1 or 2");
  if (kernel == 1 && (uint32_t)s->L > kRowsMaxL) return fail(POTTS_EINVAL, "the row-class kernel needs L <= 16380");
  s->kernel = kernel;
  return POTTS_OK;
}

int64_t potts_nnn_time(const potts_nnn_state *s) { return s ? s->t : -1; }

void *potts_nnn_stream(const potts_nnn_state *s) { return s ? (void *)s->stream : nullptr; }

void potts_nnn_free(potts_nnn_state *s) { release(s); }

}  // extern "C"
