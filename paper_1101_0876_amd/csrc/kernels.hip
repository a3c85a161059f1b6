// kernels.hip -- HIP kernels (gfx950) for the checkerboard Metropolis sweep of
// the 2D q-state Potts model, and their host-side launchers.
//
// Layout: uint8 spins, row-major, L % 4 == 0.  One kernel launch updates one
// colour (sites with (x+y) & 1 == colour).  Sites of one colour only have
// neighbours of the other colour (Sec. 3), and every write puts the other
// colour's bytes back unchanged, so the update runs in place without races.
//
// Work item of the main kernel: 16 consecutive bytes of one row (L % 16 == 0),
// i.e. 8 sites of the active colour, updated with four Philox4x32-10 blocks
// (one per 4-byte chunk).  The active and passive bytes are gathered into
// packed dwords with v_perm, and the four neighbour comparisons of four sites
// run at once as byte-wise SWAR: each comparison leaves a "differs" flag in a
// distinct high bit of every byte (bits 7..4), so a site's byte holds the
// pattern of its four neighbours.  The pair (pattern for the current spin,
// pattern for the proposal) indexes a 256-entry LDS table that holds the
// acceptance threshold of that energy change (2^32 when dE <= 0), so each site
// needs one table read and one 64-bit compare.  Accepted bytes are merged back
// with v_perm.  Items cover the lattice with a grid-stride loop over a
// persistent grid.
//
// Fused reductions (Sec. 3.4, Sec. 7): the colour-1 pass sees every site's
// final value for the sweep, so it alone builds the population histogram
// (lane-private LDS counters, no conflicts) and the satisfied-bond count
// (sum over colour-1 sites of equal neighbours; every bond joins the two
// colours).  Each workgroup adds its totals to the sweep's record with one
// 64-bit atomic per bin.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"

namespace potts {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ uint32_t bfi(uint32_t mask, uint32_t a, uint32_t b) {
  return (a & mask) | (b & ~mask);
}

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

__device__ __forceinline__ uint32_t alignbyte(uint32_t hi, uint32_t lo, uint32_t shift) {
  return __builtin_amdgcn_alignbyte(hi, lo, shift);
}

// Byte-wise "differs" flags of v against the four neighbour dwords, packed as
// bit 7 (a), bit 6 (b), bit 5 (c), bit 4 (d) of every byte; bits 3..0 are
// garbage.  CMP selects the arithmetic by the largest spin value:
//   0: q <= 16  -- x = a^v < 16, so (x + 0x7F), (x + 0x3F), (x + 0x1F),
//                  (x + 0x0F) put the x != 0 flag exactly at bits 7, 6, 5, 4
//   1: q <= 128 -- x < 128: (x + 0x7F) flags bit 7, shifted into place
//   2: q <= 256 -- exact zero-byte test
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
    uint32_t f[4];
    const uint32_t nb[4] = {a, b, c, d};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t x = nb[i] ^ v;
      if (CMP == 1) {
        f[i] = x + 0x7F7F7F7Fu;
      } else {
        f[i] = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;
      }
    }
    return bfi(0xE0E0E0E0u, bfi(0xC0C0C0C0u, bfi(0x80808080u, f[0], f[1] >> 1), f[2] >> 2), f[3] >> 3);
  }
}

// acceptance table: entry (k_pattern << 4 | s_pattern) = 2^32 if dE <= 0, else
// thr[dE-1], with dE = popcount(k_pattern) - popcount(s_pattern)
__device__ __forceinline__ void fill_accept_table(uint64_t *table, const Thresholds &thr) {
  for (uint32_t i = threadIdx.x; i < 256; i += kBlock) {
    const int de = __popc(i >> 4) - __popc(i & 15u);
    table[i] = de <= 0 ? (1ull << 32) : (uint64_t)(de == 1 ? thr.v[0] : de == 2 ? thr.v[1] : de == 3 ? thr.v[2] : thr.v[3]);
  }
}

// Row of item i (items_per_row = L/16): shift when a power of two, else a
// 64-bit multiply-high by ceil(2^64 / items_per_row).
__device__ __forceinline__ uint32_t row_of(uint32_t i, const Sweep16Params &p) {
  if (p.row_shift >= 0) return i >> p.row_shift;
  return (uint32_t)__umul64hi((uint64_t)i, p.row_magic);
}

template <int COLOUR, int CMP, bool PRIVATE_HIST>
__global__ __launch_bounds__(kBlock) void sweep16_kernel(Sweep16Params p) {
  extern __shared__ uint32_t lds[];
  uint64_t *table = reinterpret_cast<uint64_t *>(lds);  // 256 x u64
  uint32_t *hist = lds + 512;                             // per wave q x 64 lanes, or q shared
  uint32_t *partial = hist + (PRIVATE_HIST ? kWaves * 64 * p.q : p.q);  // kWaves x q, + esum
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = threadIdx.x >> 6;

  fill_accept_table(table, p.thr);
  if (COLOUR == 1) {
    const uint32_t nh = PRIVATE_HIST ? kWaves * 64 * p.q : p.q;
    for (uint32_t i = threadIdx.x; i < nh; i += kBlock) hist[i] = 0;
    if (blockIdx.x == 0 && p.rec_clear)
      for (uint32_t i = threadIdx.x; i < p.q + 1; i += kBlock) p.rec_clear[i] = 0;
  }
  __syncthreads();

  const uint32_t L = p.L;
  const uint32_t ipr = L >> 4;
  const uint32_t q = p.q;
  // byte 0: this lane's column in the private histogram, in bytes
  const uint32_t lane_off = lane * 4u;
  uint32_t *my_hist = hist + (PRIVATE_HIST ? wave * 64u * q : 0u);
  uint32_t nz_sum = 0, sites = 0;

  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < p.nitems; i += gridDim.x * kBlock) {
    const uint32_t y = row_of(i, p);
    const uint32_t xi = i - y * ipr;
    const uint32_t yu = y == 0 ? L - 1 : y - 1;
    const uint32_t yd = y + 1 == L ? 0 : y + 1;
    uint8_t *row = p.spins + (size_t)y * L;
    const uint4 c = *reinterpret_cast<const uint4 *>(row + xi * 16u);
    const uint4 u = *reinterpret_cast<const uint4 *>(p.spins + (size_t)yu * L + xi * 16u);
    const uint4 d = *reinterpret_cast<const uint4 *>(p.spins + (size_t)yd * L + xi * 16u);
    const uint32_t lf = *reinterpret_cast<const uint32_t *>(row + (xi == 0 ? L - 4 : xi * 16u - 4));
    const uint32_t rt = *reinterpret_cast<const uint32_t *>(row + (xi + 1 == ipr ? 0 : xi * 16u + 16));

    // o = byte offset of the active sites inside each dword
    const uint32_t o = (COLOUR + y) & 1u;
    const uint32_t sel_a = 0x06040200u + o * 0x01010101u;  // active bytes of (lo, hi) dwords
    const uint32_t sel_p = 0x07050301u - o * 0x01010101u;  // passive bytes
    const uint32_t s_lo = perm(c.y, c.x, sel_a), s_hi = perm(c.w, c.z, sel_a);
    const uint32_t p_lo = perm(c.y, c.x, sel_p), p_hi = perm(c.w, c.z, sel_p);
    const uint32_t u_lo = perm(u.y, u.x, sel_a), u_hi = perm(u.w, u.z, sel_a);
    const uint32_t d_lo = perm(d.y, d.x, sel_a), d_hi = perm(d.w, d.z, sel_a);
    // horizontal neighbours: one is the passive byte at the same packed index,
    // the other the passive byte one site over (left when o == 0, right when o == 1)
    const uint32_t x_lo = o ? alignbyte(p_hi, p_lo, 1) : alignbyte(p_lo, lf, 3);
    const uint32_t x_hi = o ? alignbyte(rt, p_hi, 1) : alignbyte(p_hi, p_lo, 3);

    // Philox: block m serves dword m; its (w0,w1) the site at byte o, (w2,w3) at byte o+2
    const uint32_t ctr = i * 4u;
    const Words b0 = philox4x32_10(ctr + 0, p.t_lo, p.t_hi, (uint32_t)COLOUR, p.k0, p.k1);
    const Words b1 = philox4x32_10(ctr + 1, p.t_lo, p.t_hi, (uint32_t)COLOUR, p.k0, p.k1);
    const Words b2 = philox4x32_10(ctr + 2, p.t_lo, p.t_hi, (uint32_t)COLOUR, p.k0, p.k1);
    const Words b3 = philox4x32_10(ctr + 3, p.t_lo, p.t_hi, (uint32_t)COLOUR, p.k0, p.k1);
    const uint32_t k_lo = scale_to_q(b0.w0, q) | (scale_to_q(b0.w2, q) << 8) |
                          (scale_to_q(b1.w0, q) << 16) | (scale_to_q(b1.w2, q) << 24);
    const uint32_t k_hi = scale_to_q(b2.w0, q) | (scale_to_q(b2.w2, q) << 8) |
                          (scale_to_q(b3.w0, q) << 16) | (scale_to_q(b3.w2, q) << 24);
    const uint32_t acc_w[8] = {b0.w1, b0.w3, b1.w1, b1.w3, b2.w1, b2.w3, b3.w1, b3.w3};

    const uint32_t ps_lo = diff_pattern<CMP>(s_lo, u_lo, d_lo, p_lo, x_lo);
    const uint32_t ps_hi = diff_pattern<CMP>(s_hi, u_hi, d_hi, p_hi, x_hi);
    const uint32_t pk_lo = diff_pattern<CMP>(k_lo, u_lo, d_lo, p_lo, x_lo);
    const uint32_t pk_hi = diff_pattern<CMP>(k_hi, u_hi, d_hi, p_hi, x_hi);
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
    const uint32_t ns_lo = perm(k_lo, s_lo, sel_lo);
    const uint32_t ns_hi = perm(k_hi, s_hi, sel_hi);
    // interleave new active bytes with the unchanged passive ones
    const uint32_t sel_w0 = o ? 0x05010400u : 0x01050004u;
    const uint32_t sel_w1 = o ? 0x07030602u : 0x03070206u;
    uint4 out;
    out.x = perm(ns_lo, p_lo, sel_w0);
    out.y = perm(ns_lo, p_lo, sel_w1);
    out.z = perm(ns_hi, p_hi, sel_w0);
    out.w = perm(ns_hi, p_hi, sel_w1);
    *reinterpret_cast<uint4 *>(row + xi * 16u) = out;

    if (COLOUR == 1) {
      // differing neighbours of the new spins, 8 sites
      nz_sum += __popc(perm(pk_lo, ps_lo, sel_lo) & 0xF0F0F0F0u) +
                __popc(perm(pk_hi, ps_hi, sel_hi) & 0xF0F0F0F0u);
      sites += 8;
      const uint32_t words[4] = {out.x, out.y, out.z, out.w};
#pragma unroll
      for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          if (PRIVATE_HIST) {
            // byte address (value << 8) | lane*4 built by one v_perm
            const uint32_t addr = perm(words[m], lane_off, 0x0C0C0000u | ((4u + b) << 8));
            atomicAdd(reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(my_hist) + addr), 1u);
          } else {
            atomicAdd(&my_hist[(words[m] >> (8 * b)) & 0xFFu], 1u);
          }
        }
      }
    }
  }

  if (COLOUR == 1) {
    uint32_t *esum = partial + kWaves * q;
    if (threadIdx.x == 0) *esum = 0;
    __syncthreads();
    const uint32_t e = wave_sum(4u * sites - nz_sum);
    if (lane == 0 && e) atomicAdd(esum, e);
    if (PRIVATE_HIST) {
      for (uint32_t v = 0; v < q; ++v) {
        const uint32_t s = wave_sum(my_hist[v * 64u + lane]);
        if (lane == 0) partial[wave * q + v] = s;
      }
    }
    __syncthreads();
    for (uint32_t v = threadIdx.x; v < q; v += kBlock) {
      uint32_t s = 0;
      if (PRIVATE_HIST) {
        for (int w = 0; w < kWaves; ++w) s += partial[w * q + v];
      } else {
        s = hist[v];
      }
      if (s) atomicAdd(&p.rec[1 + v], (unsigned long long)s);
    }
    if (threadIdx.x == 0 && *esum) atomicAdd(&p.rec[0], (unsigned long long)*esum);
  }
}

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

    const Words w = philox4x32_10((uint32_t)g, p.t_lo, p.t_hi, (uint32_t)COLOUR, p.k0, p.k1);
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

__global__ __launch_bounds__(kBlock) void init_kernel(InitParams p) {
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= p.nchunks) return;
  uint32_t out = 0;
  if (p.random) {
    const Words w = philox4x32_10((uint32_t)g, 0u, 0u, 2u, p.k0, p.k1);
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

template <int COLOUR, int CMP, bool PRIV>
hipError_t launch16_t(const Sweep16Params &p, unsigned grid, size_t lds, hipStream_t stream) {
  hipLaunchKernelGGL((sweep16_kernel<COLOUR, CMP, PRIV>), dim3(grid), dim3(kBlock), lds, stream, p);
  return hipGetLastError();
}

template <int COLOUR>
hipError_t launch16_c(const Sweep16Params &p, unsigned grid, size_t lds, hipStream_t stream) {
  const bool priv = p.q <= kPrivateHistMaxQ;
  if (p.q <= 16) return priv ? launch16_t<COLOUR, 0, true>(p, grid, lds, stream)
                             : launch16_t<COLOUR, 0, false>(p, grid, lds, stream);
  if (p.q <= 128) return priv ? launch16_t<COLOUR, 1, true>(p, grid, lds, stream)
                              : launch16_t<COLOUR, 1, false>(p, grid, lds, stream);
  return launch16_t<COLOUR, 2, false>(p, grid, lds, stream);
}

}  // namespace

size_t sweep16_lds_bytes(uint32_t q, int colour) {
  if (colour == 0) return 256 * 8;  // acceptance table only
  const bool priv = q <= kPrivateHistMaxQ;
  const size_t hist_words = priv ? (size_t)kWaves * 64 * q : q;
  return 256 * 8 + hist_words * 4 + ((size_t)kWaves * q + 1) * 4;
}

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

hipError_t launch_half_sweep16(const Sweep16Params &p, int colour, unsigned max_groups,
                               hipStream_t stream) {
  const unsigned grid = persistent_grid(p.nitems, max_groups);
  const size_t lds = sweep16_lds_bytes(p.q, colour);
  return colour == 0 ? launch16_c<0>(p, grid, lds, stream) : launch16_c<1>(p, grid, lds, stream);
}

hipError_t launch_measure(const MeasureParams &p, hipStream_t stream) {
  const unsigned grid = persistent_grid(p.nchunks, 4096);
  hipLaunchKernelGGL(measure_kernel, dim3(grid), dim3(kBlock), 0, stream, p);
  return hipGetLastError();
}

}  // namespace potts
