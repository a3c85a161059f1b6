// tiles.hip -- several Metropolis sweeps per launch on LDS tiles whose halos
// are recomputed (temporal blocking).
//
// A workgroup owns a tile of ty rows x tx bytes of the row-major lattice.  It
// copies the tile and a halo around it (h rows above and below, 16 bytes
// left and right) from `src` into LDS, runs up to h/2 sweeps there, and writes
// the tile's interior to `dst` (a second buffer: other workgroups still read
// their halos from `src`).  Because every site's random words are a function
// of (seed, site, sweep) alone (Sec. 3.2's independent streams, here
// counter-based), a workgroup can recompute its neighbours' updates exactly:
// a half sweep updates every site with its four neighbours in LDS, and a site
// is exact after k half sweeps if it lies at least k sites inside the copied
// region.  After s sweeps (2s half sweeps) everything at distance >= 2s is
// exact, which covers the interior and, for the energy, its neighbours.  So
// one launch replaces 2s launches of the streaming kernels, at the price of
// updating the halo too: what pays on lattices whose half sweep is too short
// to hide a kernel boundary (L up to a few thousand).
//
// LDS row layout (pitch tx + 64): 16 bytes of padding, the 16-byte left halo,
// the interior, the 16-byte right halo, 16 bytes of padding.  Items are the
// 16-byte row pieces of sweep_row.hpp (8 active sites); the items next to the
// padding take a garbage side dword, which only spoils the outermost sites,
// as the distance argument allows.  Rows 0 and last are never updated.
//
// Records: the colour-1 pass of sweep s counts the final values of the
// interior's sites and the differing neighbours of its colour-1 sites; the
// workgroup adds them into partial-record set s (striped by workgroup), and
// fold_sets_kernel turns set s into the ring slot of sweep t0 + s.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"
#include "sweep_row.hpp"

namespace potts {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

using namespace row;

__device__ __forceinline__ u32x4 lds16(const uint8_t *p) { return *reinterpret_cast<const u32x4 *>(p); }
__device__ __forceinline__ uint32_t lds4(const uint8_t *p) { return *reinterpret_cast<const uint32_t *>(p); }

// One 16-byte item at LDS row r, item column k (bytes 16 + 16k of the row).
// Returns the differing-neighbour count of its colour-1 sites (colour 1 only,
// and only when COUNT: the item is in the interior).
template <int COLOUR, int O, int CMP, bool PRIV, bool WIDE>
__device__ __forceinline__ uint32_t tile_item(uint8_t *tile, uint32_t pitch, uint32_t r, uint32_t k,
                                              uint32_t chunk, bool count, const PhiloxHead &h, uint32_t q,
                                              const uint8_t *table, uint8_t *hist, uint32_t lane_off) {
  uint8_t *cur_p = tile + r * pitch + 16u + 16u * k;
  const u32x4 cur = lds16(cur_p);
  const u32x4 up = lds16(cur_p - pitch);
  const u32x4 dn = lds16(cur_p + pitch);
  const uint32_t side = O == 0 ? lds4(cur_p - 4) : lds4(cur_p + 16);
  const Row8 o = update8<COLOUR, O, CMP, WIDE>(
      perm(cur.y, cur.x, kSel<O>), perm(cur.w, cur.z, kSel<O>), perm(cur.y, cur.x, kSel<O ^ 1>),
      perm(cur.w, cur.z, kSel<O ^ 1>), perm(up.y, up.x, kSel<O>), perm(up.w, up.z, kSel<O>),
      perm(dn.y, dn.x, kSel<O>), perm(dn.w, dn.z, kSel<O>), side, chunk, h, q, table);
  *reinterpret_cast<u32x4 *>(cur_p) = o.out;
  if (COLOUR == 1 && count) {
    if (PRIV)
      count_row_private(hist, lane_off, o.out);
    else
      count_row_shared(reinterpret_cast<uint32_t *>(hist), o.out);
    return __popc(o.nz_lo & 0xF0F0F0F0u) + __popc(o.nz_hi & 0xF0F0F0F0u);
  }
  return 0;
}

// One half sweep over every updatable item of the tile (LDS rows 1 .. rows-2,
// all item columns); rows of one parity first, so a wave mostly sees one O.
template <int COLOUR, int CMP, bool PRIV, bool WIDE>
__device__ __forceinline__ uint32_t tile_half(uint8_t *tile, const TileParams &p, uint32_t y0, uint32_t x0,
                                              uint64_t t, const uint8_t *table, uint8_t *hist,
                                              uint32_t lane_off) {
  const PhiloxHead h = philox_head((uint32_t)t, (uint32_t)(t >> 32), (uint32_t)COLOUR, p.k0, p.k1);
  const uint32_t L = p.L;
  const uint32_t pitch = p.tx + 64u;
  const uint32_t chunks = (p.tx + 32u) >> 4;
  const uint32_t rows = p.ty + 2u * p.halo;
  const uint32_t per_parity = ((rows - 2u) >> 1) * chunks;  // rows - 2 is even
  const uint32_t row_words = L >> 2;
  uint32_t nz = 0;
  for (uint32_t i = threadIdx.x; i < 2u * per_parity; i += kBlock) {
    const uint32_t par = i >= per_parity;  // 0: odd LDS rows, 1: even ones
    const uint32_t j = i - par * per_parity;
    const uint32_t rr = j / chunks;
    const uint32_t k = j - rr * chunks;
    const uint32_t r = 2u * rr + 1u + par;
    // global row and byte column of the item (y0, x0, halo, tx even; L % 16 == 0)
    uint32_t gy = y0 + r + L - p.halo;
    gy = gy >= L ? gy - L : gy;
    gy = gy >= L ? gy - L : gy;
    uint32_t gx = x0 + 16u * k + L - 16u;
    gx = gx >= L ? gx - L : gx;
    gx = gx >= L ? gx - L : gx;
    const uint32_t chunk = gy * row_words + (gx >> 2);
    const bool count = r >= p.halo && r < p.halo + p.ty && k >= 1u && k <= (p.tx >> 4);
    // site parity: (gx + gy) & 1 with gx even, and gy & 1 == r & 1
    if (((COLOUR + r) & 1u) == 0)
      nz += tile_item<COLOUR, 0, CMP, PRIV, WIDE>(tile, pitch, r, k, chunk, count, h, p.q, table, hist, lane_off);
    else
      nz += tile_item<COLOUR, 1, CMP, PRIV, WIDE>(tile, pitch, r, k, chunk, count, h, p.q, table, hist, lane_off);
  }
  return nz;
}

template <int CMP, bool PRIV, bool WIDE>
__global__ __launch_bounds__(kBlock) void tile_kernel(TileParams p) {
  __shared__ __align__(16) uint32_t table_words[512];
  constexpr uint32_t kHistWords = PRIV ? 64u * (CMP == 0 ? 16u : kPrivateHistMaxQ) : 256u;
  __shared__ __align__(16) uint32_t hist[kHistWords];
  __shared__ uint32_t partial[256 + kWaves];
  extern __shared__ __align__(16) uint32_t lds[];
  uint8_t *tile = reinterpret_cast<uint8_t *>(lds);
  uint8_t *table = reinterpret_cast<uint8_t *>(table_words);
  uint8_t *hb = reinterpret_cast<uint8_t *>(hist);
  const uint32_t L = p.L, q = p.q;
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t lane_off = lane * 4u;
  const uint32_t pitch = p.tx + 64u;
  const uint32_t chunks = (p.tx + 32u) >> 4;
  const uint32_t rows = p.ty + 2u * p.halo;
  const uint32_t tyi = blockIdx.x / p.tiles_x;
  const uint32_t txi = blockIdx.x - tyi * p.tiles_x;
  const uint32_t y0 = tyi * p.ty, x0 = txi * p.tx;

  fill_accept_table<WIDE>(table, p.thr);
  for (uint32_t i = threadIdx.x; i < rows * chunks; i += kBlock) {
    const uint32_t r = i / chunks, k = i - r * chunks;
    uint32_t gy = y0 + r + L - p.halo;
    gy = gy >= L ? gy - L : gy;
    gy = gy >= L ? gy - L : gy;
    uint32_t gx = x0 + 16u * k + L - 16u;
    gx = gx >= L ? gx - L : gx;
    gx = gx >= L ? gx - L : gx;
    *reinterpret_cast<u32x4 *>(tile + r * pitch + 16u + 16u * k) =
        *reinterpret_cast<const u32x4 *>(p.src + (size_t)gy * L + gx);
  }
  // the padding: defined values (they only feed sites that end up spoiled)
  for (uint32_t r = threadIdx.x; r < rows; r += kBlock) {
    *reinterpret_cast<u32x4 *>(tile + r * pitch) = u32x4{0u, 0u, 0u, 0u};
    *reinterpret_cast<u32x4 *>(tile + r * pitch + pitch - 16u) = u32x4{0u, 0u, 0u, 0u};
  }
  const uint32_t nh = PRIV ? 64u * q : q;
  const uint32_t sw = stripe_words(q);
  // colour-1 sites of the interior: 4 bonds each
  const unsigned long long bonds = 2ull * p.tx * p.ty;
  for (uint32_t s = 0; s < p.nsweeps; ++s) {
    const uint64_t t = p.t0 + s;
    for (uint32_t i = threadIdx.x; i < nh; i += kBlock) hist[i] = 0;
    __syncthreads();
    tile_half<0, CMP, PRIV, WIDE>(tile, p, y0, x0, t, table, hb, lane_off);
    __syncthreads();
    const uint32_t nz = tile_half<1, CMP, PRIV, WIDE>(tile, p, y0, x0, t, table, hb, lane_off);
    const uint32_t nz_w = wave_sum(nz);
    __syncthreads();
    if (PRIV) {
      for (uint32_t v = wave; v < q; v += kWaves) {
        const uint32_t c = wave_sum(hist[v * 64u + lane]);
        if (lane == 0) partial[v] = c;
      }
    } else {
      for (uint32_t v = threadIdx.x; v < q; v += kBlock) partial[v] = hist[v];
    }
    if (lane == 0) partial[q + wave] = nz_w;
    __syncthreads();
    unsigned long long *dst =
        p.stripes + ((uint64_t)s * p.nstripes + (blockIdx.x & (p.nstripes - 1))) * (uint64_t)sw;
    for (uint32_t v = threadIdx.x; v < q; v += kBlock)
      if (partial[v]) atomicAdd(&dst[1 + v], (unsigned long long)partial[v]);
    if (threadIdx.x == 0) {
      unsigned long long nzt = 0;
      for (int w = 0; w < kWaves; ++w) nzt += partial[q + w];
      atomicAdd(&dst[0], bonds - nzt);
    }
  }
  __syncthreads();
  // the interior (LDS rows halo .. halo+ty-1, bytes 32 .. 32+tx-1) to dst
  const uint32_t ichunks = p.tx >> 4;
  for (uint32_t i = threadIdx.x; i < p.ty * ichunks; i += kBlock) {
    const uint32_t r = i / ichunks, k = i - r * ichunks;
    *reinterpret_cast<u32x4 *>(p.dst + (size_t)(y0 + r) * L + x0 + 16u * k) =
        lds16(tile + (p.halo + r) * pitch + 32u + 16u * k);
  }
}

// Set s of the partial records (nstripes stripes) summed into ring slot
// t0 + s, then cleared; one workgroup per set.
__global__ __launch_bounds__(kBlock) void fold_sets_kernel(TileParams p, unsigned long long *ring, uint64_t cap) {
  __shared__ unsigned long long acc[257];
  const uint32_t s = blockIdx.x;
  const uint32_t n = p.q + 1, sw = stripe_words(p.q), total = p.nstripes * n;
  unsigned long long *set = p.stripes + (uint64_t)s * p.nstripes * sw;
  unsigned long long *slot = ring + ((p.t0 + s) & (cap - 1)) * (uint64_t)n;
  for (uint32_t i = threadIdx.x; i < n; i += kBlock) acc[i] = 0;
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < total; k += kBlock) {
    const uint32_t st = k / n, i = k - st * n;
    const unsigned long long v = set[st * sw + i];
    if (v) {
      atomicAdd(&acc[i], v);
      set[st * sw + i] = 0;
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n; i += kBlock) slot[i] = acc[i];
}

template <int CMP, bool PRIV, bool WIDE>
hipError_t launch_t(const TileParams &p, unsigned grid, size_t lds, hipStream_t stream) {
  hipLaunchKernelGGL((tile_kernel<CMP, PRIV, WIDE>), dim3(grid), dim3(kBlock), lds, stream, p);
  return hipGetLastError();
}

template <bool WIDE>
hipError_t launch_w(const TileParams &p, unsigned grid, size_t lds, hipStream_t stream) {
  if (p.q <= 16) return launch_t<0, true, WIDE>(p, grid, lds, stream);
  if (p.q <= kPrivateHistMaxQ) return launch_t<1, true, WIDE>(p, grid, lds, stream);
  if (p.q <= 128) return launch_t<1, false, WIDE>(p, grid, lds, stream);
  return launch_t<2, false, WIDE>(p, grid, lds, stream);
}

}  // namespace

size_t tile_lds_bytes(uint32_t tx, uint32_t ty, uint32_t halo) {
  return (size_t)(ty + 2u * halo) * (tx + 64u);
}

bool tile_shape_ok(uint32_t L, uint32_t tx, uint32_t ty, uint32_t halo) {
  return L % 16 == 0 && tx >= 16 && tx % 16 == 0 && L % tx == 0 && ty >= 2 && ty % 2 == 0 && L % ty == 0 &&
         halo >= 2 && halo % 2 == 0 && halo <= kTileMaxHalo && halo <= L &&
         tile_lds_bytes(tx, ty, halo) <= kTileMaxLds;
}

hipError_t launch_tiles(const TileParams &p, hipStream_t stream) {
  if (p.nsweeps == 0) return hipSuccess;
  if (!tile_shape_ok(p.L, p.tx, p.ty, p.halo) || 2u * p.nsweeps > p.halo || p.nsweeps > kTileMaxSweeps)
    return hipErrorInvalidValue;
  const unsigned grid = (p.L / p.tx) * (p.L / p.ty);
  const size_t lds = tile_lds_bytes(p.tx, p.ty, p.halo);
  const bool wide = !p.thr.v[0] || !p.thr.v[1] || !p.thr.v[2] || !p.thr.v[3];
  return wide ? launch_w<true>(p, grid, lds, stream) : launch_w<false>(p, grid, lds, stream);
}

hipError_t launch_fold_sets(const TileParams &p, unsigned long long *ring, uint64_t cap, hipStream_t stream) {
  if (p.nsweeps == 0) return hipSuccess;
  hipLaunchKernelGGL(fold_sets_kernel, dim3(p.nsweeps), dim3(kBlock), 0, stream, p, ring, cap);
  return hipGetLastError();
}

}  // namespace potts
