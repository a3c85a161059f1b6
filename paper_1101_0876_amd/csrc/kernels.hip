// kernels.hip -- general-shape HIP kernels (gfx950) and their launchers: the
// 4-byte-chunk half sweep used when L % 16 != 0 (the main path for L % 16 == 0
// is in strip.hip), the initial condition, the standalone measurement of the
// energy and populations, and a fill kernel.
//
// Chunk kernel: one thread per 4-byte row chunk (two active sites, one Philox
// block).  It reads its dword, the dwords above and below and the two side
// dwords, updates the two sites of the active colour and writes the dword
// back.  Sites of one colour only have neighbours of the other colour (Sec. 3)
// and the other colour's bytes are written back unchanged, so the update runs
// in place without races.  The colour-1 pass also reduces the sweep's energy
// and populations (every site is final then; every bond joins the colours).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "kernels.hpp"

namespace potts {
namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// General path for L % 16 != 0: one thread per 4-byte chunk (two active
// sites, one Philox block), grid-stride, shared-bin histogram.
__device__ __forceinline__ uint32_t pick_threshold(const Thresholds &thr, int d) {
  return d == 1 ? thr.v[0] : d == 2 ? thr.v[1] : d == 3 ? thr.v[2] : thr.v[3];
}

template <int COLOUR>
__global__ __launch_bounds__(kBlock) void sweep4_kernel(SweepParams p) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t esum;
  for (uint32_t v = threadIdx.x; v < p.q; v += kBlock) hist[v] = 0;
  if (threadIdx.x == 0) esum = 0;
  if (COLOUR == 1 && blockIdx.x == 0 && p.rec_clear) {
    for (uint32_t i = threadIdx.x; i < p.q + 1; i += kBlock) p.rec_clear[i] = 0;
  }
  __syncthreads();

  const uint32_t cpr = p.L >> 2;
  uint32_t e = 0;
  for (uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x; g < p.nchunks;
       g += (uint64_t)gridDim.x * kBlock) {
    const uint32_t y = (uint32_t)(g / cpr);
    const uint32_t j = (uint32_t)(g - (uint64_t)y * cpr);
    const uint32_t yu = y == 0 ? p.L - 1 : y - 1;
    const uint32_t yd = y + 1 == p.L ? 0 : y + 1;
    uint32_t *row = reinterpret_cast<uint32_t *>(p.spins + (size_t)y * p.L);
    const uint32_t *rowu = reinterpret_cast<const uint32_t *>(p.spins + (size_t)yu * p.L);
    const uint32_t *rowd = reinterpret_cast<const uint32_t *>(p.spins + (size_t)yd * p.L);
    const uint32_t cur = row[j];
    const uint32_t up = rowu[j];
    const uint32_t dn = rowd[j];
    const uint32_t lf = row[j == 0 ? cpr - 1 : j - 1];
    const uint32_t rt = row[j + 1 == cpr ? 0 : j + 1];
    const uint32_t left = (cur << 8) | (lf >> 24);   // byte i: spin at x-1
    const uint32_t right = (cur >> 8) | (rt << 24);  // byte i: spin at x+1

    const Words w = philox4x32_10(p.t_lo, (uint32_t)g, p.t_hi, (uint32_t)COLOUR, p.k0, p.k1);
    const uint32_t o = (COLOUR + y) & 1u;  // byte offset of the first active site
    const uint32_t ka = scale_to_q(w.w0, p.q);
    const uint32_t kb = scale_to_q(w.w2, p.q);
    const uint32_t prop = (ka << (8 * o)) | (kb << (8 * (o + 2)));
    const uint32_t n_cur = count_equal(cur, up, dn, left, right);
    const uint32_t n_new = count_equal(prop, up, dn, left, right);

    const uint32_t sa = byte_of(cur, o), sb = byte_of(cur, o + 2);
    const uint32_t nsa = byte_of(n_cur, o), nka = byte_of(n_new, o);
    const uint32_t nsb = byte_of(n_cur, o + 2), nkb = byte_of(n_new, o + 2);
    const int da = (int)nsa - (int)nka;
    const int db = (int)nsb - (int)nkb;
    const bool acc_a = da <= 0 || w.w1 < pick_threshold(p.thr, da);
    const bool acc_b = db <= 0 || w.w3 < pick_threshold(p.thr, db);
    const uint32_t na = acc_a ? ka : sa;
    const uint32_t nb = acc_b ? kb : sb;
    const uint32_t keep = ~((0xFFu << (8 * o)) | (0xFFu << (8 * (o + 2))));
    const uint32_t out = (cur & keep) | (na << (8 * o)) | (nb << (8 * (o + 2)));
    row[j] = out;
    if (COLOUR == 1) {
      for (uint32_t b = 0; b < 4; ++b) atomicAdd(&hist[byte_of(out, b)], 1u);
      e += (acc_a ? nka : nsa) + (acc_b ? nkb : nsb);
    }
  }
  if (COLOUR == 1) {
    e = wave_sum(e);
    if ((threadIdx.x & 63) == 0 && e) atomicAdd(&esum, e);
    __syncthreads();
    for (uint32_t v = threadIdx.x; v < p.q; v += kBlock) {
      const uint32_t c = hist[v];
      if (c) atomicAdd(&p.rec[1 + v], (unsigned long long)c);
    }
    if (threadIdx.x == 0 && esum) atomicAdd(&p.rec[0], (unsigned long long)esum);
  }
}

// ---------------------------------------------------------------------------
// Heat-bath update (Sec. 7 names other single-spin-flip algorithms as the
// extension of the Metropolis update): the new value k is drawn with weight
// exp(beta n(k)), n(k) = neighbours equal to k, whatever the current value.
// Weights relative to the best neighbour count n_max: value v weighs
// D[n_max - n(v)] with D[0] = 2^32 and D[d] = thr[d-1].  Ranking: the distinct
// neighbour values in order of first appearance among (up, down, left,
// right), then the other values ascending; r = floor(w Z / 2^32) picks the
// first value whose cumulative weight exceeds r.  Non-neighbour values all
// weigh D[n_max], so that run is indexed with one division and the j-th
// value outside the (at most four) neighbour values comes from one pass over
// those values in ascending order.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(uint8_t *p) {
  return __builtin_amdgcn_make_buffer_rsrc(p, 0, (int)0xFFFFFFFFu, 0x00020000);
}

// Everything of the draw that depends only on which of the four neighbours
// are equal comes from a 64-entry LDS table indexed by the six "differs"
// flags (ab, ac, ad, bc, bd, cd; a = up, b = down, c = left, d = right),
// built per workgroup from the thresholds: the cumulative weights of the
// ranked neighbour values (a, then b, c, d where they appear first; a value
// seen before weighs 0 there), S (their total), Z = S + (q - m) w0 (m distinct
// neighbour values, w0 = D[n_max] the weight of each other value) and the FP32
// reciprocal of w0.  Field-major (one array of 64 per field): lanes reading
// different entries meet in a bank only when the entry numbers agree in
// their low bits, where 64-byte entries put every other entry in one bank.
enum HbField { kSa, kSab, kSabc, kS, kZ, kW0Inv, kHbFields };

__device__ void fill_heatbath_entry(uint64_t (*tab)[64], uint32_t pat, uint32_t q, const Thresholds &thr,
                                    const double *inv) {
  const uint32_t eab = !(pat & 32u), eac = !(pat & 16u), ead = !(pat & 8u);
  const uint32_t ebc = !(pat & 4u), ebd = !(pat & 2u), ecd = !(pat & 1u);
  const uint32_t na = 1 + eab + eac + ead, nb = 1 + eab + ebc + ebd;
  const uint32_t nc = 1 + eac + ebc + ecd, nd = 1 + ead + ebd + ecd;
  const uint32_t nmax = max(max(na, nb), max(nc, nd));
  const bool fb = !eab, fc = !eac && !ebc, fd = !ead && !ebd && !ecd;
  auto weight = [&](uint32_t gap) -> uint64_t { return gap == 0 ? (1ull << 32) : (uint64_t)thr.v[gap - 1]; };
  const uint64_t wa = weight(nmax - na);
  const uint64_t wb = fb ? weight(nmax - nb) : 0;
  const uint64_t wc = fc ? weight(nmax - nc) : 0;
  const uint64_t wd = fd ? weight(nmax - nd) : 0;
  const uint32_t m = 1 + fb + fc + fd;
  const uint32_t w0 = thr.v[nmax - 1];
  const uint64_t s = wa + wb + wc + wd;
  tab[kSa][pat] = wa;
  tab[kSab][pat] = wa + wb;
  tab[kSabc][pat] = wa + wb + wc;
  tab[kS][pat] = s;
  // patterns no four values can show (equality is transitive) are never
  // looked up; their entries are whatever the formulas give
  tab[kZ][pat] = s + (uint64_t)(q - m) * w0;
  tab[kW0Inv][pat] = w0 | (uint64_t)__float_as_uint((float)inv[nmax - 1]) << 32;
}

// Per byte of up/down/left/right: the six "differs" flags at bits 7..2 (ab,
// ac, ad, bc, bd, cd), bits 1..0 clear.  CMP as in the row kernels: 0 for
// values below 16 (x + 0x7F/0x3F/0x1F/0x0F sets exactly bit 7/6/5/4 when
// x != 0), 1 below 128 (x + 0x7F flags bit 7), 2 for any byte (exact test).
template <int CMP>
__device__ __forceinline__ uint32_t pair_flags(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  auto bfi = [](uint32_t mask, uint32_t x, uint32_t y) { return (x & mask) | (y & ~mask); };
  uint32_t hi, lo;  // flags ab, ac, ad, bc at bits 7..4; bd, cd at bits 7..6
  if (CMP == 0) {
    hi = bfi(0xE0E0E0E0u, bfi(0xC0C0C0C0u, bfi(0x80808080u, (a ^ b) + 0x7F7F7F7Fu, (a ^ c) + 0x3F3F3F3Fu),
                              (a ^ d) + 0x1F1F1F1Fu),
             (b ^ c) + 0x0F0F0F0Fu);
    lo = bfi(0x80808080u, (b ^ d) + 0x7F7F7F7Fu, (c ^ d) + 0x3F3F3F3Fu);
  } else {
    auto f = [](uint32_t x) {
      return CMP == 1 ? x + 0x7F7F7F7Fu : (((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x);
    };
    hi = bfi(0xE0E0E0E0u, bfi(0xC0C0C0C0u, bfi(0x80808080u, f(a ^ b), f(a ^ c) >> 1), f(a ^ d) >> 2),
             f(b ^ c) >> 3);
    lo = bfi(0x80808080u, f(b ^ d), f(c ^ d) >> 1);
  }
  return bfi(0xF0F0F0F0u, hi, lo >> 4) & 0xFCFCFCFCu;
}

// One draw from the table entries of the site's pattern.
__device__ __forceinline__ uint32_t heatbath_draw(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t w,
                                                  const uint64_t (*tab)[64], uint32_t pat) {
  const uint64_t sa = tab[kSa][pat], sab = tab[kSab][pat];
  const uint64_t sabc = tab[kSabc][pat], S = tab[kS][pat];
  const uint64_t Z = tab[kZ][pat];  // < 2^41
  const uint64_t wi = tab[kW0Inv][pat];
  const uint32_t w0 = (uint32_t)wi;
  const float inv = __uint_as_float((uint32_t)(wi >> 32));
  // r = floor(w Z / 2^32), exactly, from the two halves of Z
  const uint64_t r = (uint64_t)w * (Z >> 32) + (((uint64_t)w * (Z & 0xFFFFFFFFull)) >> 32);
  // past the neighbour values: j = floor(X / w0) for X = r - S < (q - m) w0
  // (so w0 > 0 and j < 256).  X in FP32 (two conversions and one fma) times
  // the FP32 reciprocal is within 1e-6 relative, 3e-4 absolute, of X / w0,
  // so its floor is j - 1, j or j + 1; one integer check each way, taken from
  // the estimate, makes it exact.  Computed for every lane (no divergent
  // branch); lanes that stopped earlier discard it.
  const uint64_t X = r >= S ? r - S : 0;
  const float xf = __builtin_fmaf((float)(uint32_t)(X >> 32), 4294967296.0f, (float)(uint32_t)X);
  uint32_t j = (uint32_t)(xf * inv);
  const uint64_t jw = (uint64_t)j * w0;
  j = j - (uint32_t)(jw > X) + (uint32_t)(jw + w0 <= X);
  // the j-th value that no neighbour holds: with the neighbour values in
  // ascending order, each one at or below the running candidate that is not a
  // repeat of the one before moves it up by one
  uint32_t e[4] = {a, b, c, d};
  auto order = [](uint32_t &x, uint32_t &y) {
    const uint32_t lo = min(x, y), hi = max(x, y);
    x = lo;
    y = hi;
  };
  order(e[0], e[1]);
  order(e[2], e[3]);
  order(e[0], e[2]);
  order(e[1], e[3]);
  order(e[1], e[2]);
  uint32_t k = j;
  k += e[0] <= k;
  k += e[1] != e[0] && e[1] <= k;
  k += e[2] != e[1] && e[2] <= k;
  k += e[3] != e[2] && e[3] <= k;
  return r < sa ? a : r < sab ? b : r < sabc ? c : r < S ? d : k;
}

// Grid: x over the chunks of a row, y strided over the rows (no division per
// chunk); the Philox head of the half sweep is the same for every lane.
// Populations (colour 1) in q shared LDS bins: a chunk whose four bytes are
// equal adds 4 with one atomic.  (Lane-private columns, value * 64 + lane,
// were far slower here: the adds of one instruction to a shared bin are
// cheaper than 64 adds to distinct addresses.)
template <int COLOUR, int CMP>
__global__ __launch_bounds__(kBlock) void heatbath4_kernel(SweepParams p) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t esum;
  __shared__ uint64_t table[kHbFields][64];
  const uint32_t lane = threadIdx.x & 63u;
  for (uint32_t v = threadIdx.x; v < p.q; v += kBlock) hist[v] = 0;
  if (threadIdx.x == 0) esum = 0;
  if (threadIdx.x < 64) fill_heatbath_entry(table, threadIdx.x, p.q, p.thr, p.inv_thr);
  if (COLOUR == 1 && blockIdx.x == 0 && blockIdx.y == 0 && p.rec_clear) {
    for (uint32_t i = threadIdx.x; i < p.q + 1; i += kBlock) p.rec_clear[i] = 0;
  }
  __syncthreads();

  const uint32_t L = p.L, cpr = L >> 2;
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  const PhiloxHead h = philox_head(p.t_lo, p.t_hi, (uint32_t)COLOUR + 4u, p.k0, p.k1);
  uint32_t e = 0;
  if (j < cpr) {
    const uint32_t jl = j == 0 ? cpr - 1 : j - 1, jr = j + 1 == cpr ? 0 : j + 1;
    const uint32_t oj = 4 * j, ol = 4 * jl, orr = 4 * jr;
    for (uint32_t y = blockIdx.y; y < L; y += gridDim.y) {
      const uint32_t yu = y == 0 ? L - 1 : y - 1;
      const uint32_t yd = y + 1 == L ? 0 : y + 1;
      // the rows are the same for the whole workgroup: buffer resources in
      // scalar registers, 32-bit lane offsets
      const __amdgpu_buffer_rsrc_t row = row_rsrc(p.spins + (size_t)y * L);
      const uint32_t up = __builtin_amdgcn_raw_buffer_load_b32(row_rsrc(p.spins + (size_t)yu * L), oj, 0, 0);
      const uint32_t dn = __builtin_amdgcn_raw_buffer_load_b32(row_rsrc(p.spins + (size_t)yd * L), oj, 0, 0);
      const uint32_t cur = __builtin_amdgcn_raw_buffer_load_b32(row, oj, 0, 0);
      const uint32_t left =  // byte i: spin at x-1
          __builtin_amdgcn_alignbyte(cur, __builtin_amdgcn_raw_buffer_load_b32(row, ol, 0, 0), 3);
      const uint32_t right =  // byte i: spin at x+1
          __builtin_amdgcn_alignbyte(__builtin_amdgcn_raw_buffer_load_b32(row, orr, 0, 0), cur, 1);

      const Words w = philox_tail(h.a0 ^ (y * cpr + j), h);
      const uint32_t o = (COLOUR + y) & 1u;  // byte of the first active site; the second is o + 2
      const uint32_t pat = pair_flags<CMP>(up, dn, left, right);
      uint32_t out = cur;
#pragma unroll
      for (uint32_t s = 0; s < 2; ++s) {
        const uint32_t i = o + 2 * s;
        const uint32_t a = byte_of(up, i), b = byte_of(dn, i), c = byte_of(left, i), d = byte_of(right, i);
        const uint32_t k = heatbath_draw(a, b, c, d, s == 0 ? w.w0 : w.w2, table, byte_of(pat, i) >> 2);
        out = (out & ~(0xFFu << (8 * i))) | (k << (8 * i));
        if (COLOUR == 1) e += (k == a) + (k == b) + (k == c) + (k == d);
      }
      __builtin_amdgcn_raw_buffer_store_b32(out, row, oj, 0, 0);
      if (COLOUR == 1) {
        const uint32_t v0 = out & 0xFFu;
        const bool same = out == v0 * 0x01010101u;
        atomicAdd(&hist[v0], same ? 4u : 1u);
        if (!same)
          for (uint32_t bb = 1; bb < 4; ++bb) atomicAdd(&hist[byte_of(out, bb)], 1u);
      }
    }
  }
  if (COLOUR == 1) {
    e = wave_sum(e);
    if (lane == 0 && e) atomicAdd(&esum, e);
    __syncthreads();
    for (uint32_t v = threadIdx.x; v < p.q; v += kBlock) {
      const uint32_t cnt = hist[v];
      if (cnt) atomicAdd(&p.rec[1 + v], (unsigned long long)cnt);
    }
    if (threadIdx.x == 0 && esum) atomicAdd(&p.rec[0], (unsigned long long)esum);
  }
}

__global__ __launch_bounds__(kBlock) void init_kernel(InitParams p) {
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= p.nchunks) return;
  uint32_t out = 0;
  if (p.random) {
    const Words w = philox4x32_10(0u, (uint32_t)g, 0u, 2u, p.k0, p.k1);
    out = scale_to_q(w.w0, p.q) | (scale_to_q(w.w1, p.q) << 8) | (scale_to_q(w.w2, p.q) << 16) |
          (scale_to_q(w.w3, p.q) << 24);
  }
  reinterpret_cast<uint32_t *>(p.spins)[g] = out;
}

// Standalone measurement of e_sat and the populations (no sweep); shares no
// code with the fused reductions of the sweep kernels.
__global__ __launch_bounds__(kBlock) void measure_kernel(MeasureParams p) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t esum;
  for (uint32_t v = threadIdx.x; v < p.q; v += kBlock) hist[v] = 0;
  if (threadIdx.x == 0) esum = 0;
  __syncthreads();
  const uint32_t cpr = p.L >> 2;
  uint32_t e = 0;
  for (uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x; g < p.nchunks;
       g += (uint64_t)gridDim.x * kBlock) {
    const uint32_t y = (uint32_t)(g / cpr);
    const uint32_t j = (uint32_t)(g - (uint64_t)y * cpr);
    const uint32_t yd = y + 1 == p.L ? 0 : y + 1;
    const uint32_t *row = reinterpret_cast<const uint32_t *>(p.spins + (size_t)y * p.L);
    const uint32_t *rowd = reinterpret_cast<const uint32_t *>(p.spins + (size_t)yd * p.L);
    const uint32_t cur = row[j];
    const uint32_t dn = rowd[j];
    const uint32_t rt = row[j + 1 == cpr ? 0 : j + 1];
    const uint32_t right = (cur >> 8) | (rt << 24);
    e += __popc(zero_bytes(cur ^ right)) + __popc(zero_bytes(cur ^ dn));
    for (uint32_t i = 0; i < 4; ++i) atomicAdd(&hist[byte_of(cur, i)], 1u);
  }
  e = wave_sum(e);
  if ((threadIdx.x & 63) == 0 && e) atomicAdd(&esum, e);
  __syncthreads();
  for (uint32_t v = threadIdx.x; v < p.q; v += kBlock) {
    const uint32_t c = hist[v];
    if (c) atomicAdd(&p.out[1 + v], (unsigned long long)c);
  }
  if (threadIdx.x == 0 && esum) atomicAdd(&p.out[0], (unsigned long long)esum);
}

__global__ void fill_u64_kernel(unsigned long long *p, uint64_t n, unsigned long long value) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

inline unsigned grid_for(uint64_t items) { return (unsigned)((items + kBlock - 1) / kBlock); }

// persistent grid: enough workgroups to fill the chip, never more than the work
inline unsigned persistent_grid(uint64_t items, unsigned max_groups) {
  const uint64_t need = (items + kBlock - 1) / kBlock;
  return (unsigned)(need < max_groups ? (need ? need : 1) : max_groups);
}

}  // namespace

hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long value,
                           hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(n)), dim3(kBlock), 0, stream, p, n, value);
  return hipGetLastError();
}

hipError_t launch_init(const InitParams &p, hipStream_t stream) {
  hipLaunchKernelGGL(init_kernel, dim3(grid_for(p.nchunks)), dim3(kBlock), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_half_sweep(const SweepParams &p, int colour, hipStream_t stream) {
  const unsigned grid = persistent_grid(p.nchunks, 4096);
  if (colour == 0)
    hipLaunchKernelGGL(sweep4_kernel<0>, dim3(grid), dim3(kBlock), 0, stream, p);
  else
    hipLaunchKernelGGL(sweep4_kernel<1>, dim3(grid), dim3(kBlock), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_heatbath(const SweepParams &p, int colour, hipStream_t stream) {
  SweepParams h = p;
  for (int d = 0; d < 4; ++d) h.inv_thr[d] = h.thr.v[d] ? 1.0 / (double)h.thr.v[d] : 0.0;
  const uint32_t bx = ((p.L >> 2) + kBlock - 1) / kBlock;
  const uint32_t by = std::max<uint32_t>(1u, std::min<uint32_t>(p.L, 4096u / bx));
  const dim3 grid(bx, by);
  const int cmp = p.q <= 16 ? 0 : p.q <= 128 ? 1 : 2;
  if (colour == 0) {
    if (cmp == 0) hipLaunchKernelGGL((heatbath4_kernel<0, 0>), grid, dim3(kBlock), 0, stream, h);
    else if (cmp == 1) hipLaunchKernelGGL((heatbath4_kernel<0, 1>), grid, dim3(kBlock), 0, stream, h);
    else hipLaunchKernelGGL((heatbath4_kernel<0, 2>), grid, dim3(kBlock), 0, stream, h);
  } else {
    if (cmp == 0) hipLaunchKernelGGL((heatbath4_kernel<1, 0>), grid, dim3(kBlock), 0, stream, h);
    else if (cmp == 1) hipLaunchKernelGGL((heatbath4_kernel<1, 1>), grid, dim3(kBlock), 0, stream, h);
    else hipLaunchKernelGGL((heatbath4_kernel<1, 2>), grid, dim3(kBlock), 0, stream, h);
  }
  return hipGetLastError();
}

hipError_t launch_measure(const MeasureParams &p, hipStream_t stream) {
  const unsigned grid = persistent_grid(p.nchunks, 4096);
  hipLaunchKernelGGL(measure_kernel, dim3(grid), dim3(kBlock), 0, stream, p);
  return hipGetLastError();
}

}  // namespace potts
