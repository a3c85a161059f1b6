// cubic.hip -- the Potts model on the simple-cubic lattice (Sec. 7: the
// checkerboard update carries over to three dimensions, with its two
// independent sub-lattices).  The 2D contract lifted to L x L x L: site
// (x, y, z) at byte (z L + y) L + x, colour (x + y + z) & 1, six neighbours
// (dE in -6..6, a six-entry threshold table), Philox counter (t_lo, chunk,
// t_hi, colour + 8), random start on counter word 3 = 10.  Records, rings and
// statistics are those of the 2D library with N = L^3 and 3N bonds.
//
// Two half-sweep kernels give identical results:
//   - colour-split (cubic_packed.hip, L % 32 == 0): the state keeps a copy of
//     the cube split into its two colour planes and sweeps there; the
//     row-major copy is rebuilt only when it is read;
//   - chunk (here, any L): one thread per 4-byte row chunk (two active sites,
//     one Philox block) on the row-major cube; the six neighbour dwords are
//     the row's own (shifted by one byte for x-1 and x+1), the same dword of
//     rows y-1 and y+1, and of planes z-1 and z+1.
// The colour-1 pass reduces the sweep's energy; populations come from both.
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/potts.h"
#include "cubic.hpp"
#include "device.hpp"
#include "kernels.hpp"

struct potts3d_state {
  int32_t L = 0, q = 0;
  uint64_t seed = 0;
  int64_t t = 0;
  uint8_t *spins = nullptr;   // row-major cube
  uint8_t *planes = nullptr;  // colour-split copy (L % 32 == 0)
  bool spins_valid = true;    // spins holds the current configuration
  bool planes_valid = false;  // planes holds it
  int32_t kernel = 0;         // 0 automatic, 1 colour-split, 2 chunk
  int32_t rows = 0;           // colour-split walk length (0 automatic)
  hipStream_t stream = nullptr;
  unsigned long long *records = nullptr;  // ring of rec_cap slots of 1+q
  int64_t rec_cap = 0;
  unsigned long long *scratch = nullptr;  // 1+q words for measurements
  double *stats_out = nullptr;
  bool have_thr = false;
  double thr_beta = 0.0;
  uint32_t thr[6] = {0, 0, 0, 0, 0, 0};
};

namespace potts {
int record_error(int code, const std::string &msg);
}

namespace {

using potts::Words;
using potts::byte_of;
using potts::philox4x32_10;
using potts::scale_to_q;
using potts::wave_sum;
using potts::zero_bytes;

constexpr int kBlock = 256;
constexpr int64_t kRingSlots = 4096;

struct Cube {
  uint8_t *spins;
  uint32_t L, q;
  uint64_t nchunks;  // L^3 / 4
  uint32_t k0, k1;
};

struct CubeSweep {
  Cube c;
  uint32_t t_lo, t_hi;
  uint32_t thr[6];
  unsigned long long *rec;        // this sweep's record (colour 1 adds to it)
  unsigned long long *rec_clear;  // the next sweep's record, zeroed by colour 1, or null
};

// per-byte count (0..6) of the six neighbour dwords equal to v
__device__ __forceinline__ uint32_t count_equal6(uint32_t v, const uint32_t nb[6]) {
  uint32_t n = 0;
#pragma unroll
  for (int i = 0; i < 6; ++i) n += zero_bytes(v ^ nb[i]) >> 7;
  return n;
}

__device__ __forceinline__ uint32_t pick6(const uint32_t thr[6], int d) {
  uint32_t t = thr[0];
#pragma unroll
  for (int i = 1; i < 6; ++i) t = d == i + 1 ? thr[i] : t;
  return t;
}

template <int COLOUR>
__global__ __launch_bounds__(kBlock) void cube_sweep_kernel(CubeSweep p) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t esum;
  const Cube &c = p.c;
  for (uint32_t v = threadIdx.x; v < c.q; v += kBlock) hist[v] = 0;
  if (threadIdx.x == 0) esum = 0;
  if (COLOUR == 1 && blockIdx.x == 0 && p.rec_clear)
    for (uint32_t i = threadIdx.x; i < c.q + 1; i += kBlock) p.rec_clear[i] = 0;
  __syncthreads();

  const uint32_t L = c.L, cpr = L >> 2;
  const size_t plane = (size_t)L * L;
  uint32_t e = 0;
  for (uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x; g < c.nchunks;
       g += (uint64_t)gridDim.x * kBlock) {
    const uint64_t r = g / cpr;  // row index z L + y
    const uint32_t j = (uint32_t)(g - r * cpr);
    const uint32_t z = (uint32_t)(r / L), y = (uint32_t)(r - (uint64_t)z * L);
    const uint32_t yu = y == 0 ? L - 1 : y - 1, yd = y + 1 == L ? 0 : y + 1;
    const uint32_t zb = z == 0 ? L - 1 : z - 1, zf = z + 1 == L ? 0 : z + 1;
    uint32_t *row = reinterpret_cast<uint32_t *>(c.spins + (size_t)z * plane + (size_t)y * L);
    auto dword = [&](uint32_t zz, uint32_t yy) {
      return reinterpret_cast<const uint32_t *>(c.spins + (size_t)zz * plane + (size_t)yy * L)[j];
    };
    const uint32_t cur = row[j];
    const uint32_t lf = row[j == 0 ? cpr - 1 : j - 1];
    const uint32_t rt = row[j + 1 == cpr ? 0 : j + 1];
    const uint32_t nb[6] = {(cur >> 8) | (rt << 24),  // byte i: x+1
                            (cur << 8) | (lf >> 24),  // byte i: x-1
                            dword(z, yd), dword(z, yu), dword(zf, y), dword(zb, y)};

    const Words w = philox4x32_10(p.t_lo, (uint32_t)g, p.t_hi, (uint32_t)COLOUR + 8u, c.k0, c.k1);
    const uint32_t o = (COLOUR + y + z) & 1u;  // byte of the first active site
    const uint32_t ka = scale_to_q(w.w0, c.q), kb = scale_to_q(w.w2, c.q);
    const uint32_t prop = (ka << (8 * o)) | (kb << (8 * (o + 2)));
    const uint32_t n_cur = count_equal6(cur, nb), n_new = count_equal6(prop, nb);
    const int da = (int)byte_of(n_cur, o) - (int)byte_of(n_new, o);
    const int db = (int)byte_of(n_cur, o + 2) - (int)byte_of(n_new, o + 2);
    const bool acc_a = da <= 0 || w.w1 < pick6(p.thr, da);
    const bool acc_b = db <= 0 || w.w3 < pick6(p.thr, db);
    const uint32_t na = acc_a ? ka : byte_of(cur, o);
    const uint32_t nbv = acc_b ? kb : byte_of(cur, o + 2);
    const uint32_t keep = ~((0xFFu << (8 * o)) | (0xFFu << (8 * (o + 2))));
    const uint32_t out = (cur & keep) | (na << (8 * o)) | (nbv << (8 * (o + 2)));
    row[j] = out;
    if (COLOUR == 1) {
      for (uint32_t b = 0; b < 4; ++b) atomicAdd(&hist[byte_of(out, b)], 1u);
      e += (acc_a ? byte_of(n_new, o) : byte_of(n_cur, o)) + (acc_b ? byte_of(n_new, o + 2) : byte_of(n_cur, o + 2));
    }
  }
  if (COLOUR == 1) {
    e = wave_sum(e);
    if ((threadIdx.x & 63) == 0 && e) atomicAdd(&esum, e);
    __syncthreads();
    for (uint32_t v = threadIdx.x; v < c.q; v += kBlock) {
      const uint32_t n = hist[v];
      if (n) atomicAdd(&p.rec[1 + v], (unsigned long long)n);
    }
    if (threadIdx.x == 0 && esum) atomicAdd(&p.rec[0], (unsigned long long)esum);
  }
}

__global__ __launch_bounds__(kBlock) void cube_init_kernel(Cube c, int random) {
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= c.nchunks) return;
  uint32_t out = 0;
  if (random) {
    const Words w = philox4x32_10(0u, (uint32_t)g, 0u, 10u, c.k0, c.k1);
    out = scale_to_q(w.w0, c.q) | (scale_to_q(w.w1, c.q) << 8) | (scale_to_q(w.w2, c.q) << 16) |
          (scale_to_q(w.w3, c.q) << 24);
  }
  reinterpret_cast<uint32_t *>(c.spins)[g] = out;
}

// e_sat (3N bonds, through +x, +y, +z) and populations; out must start zeroed
__global__ __launch_bounds__(kBlock) void cube_measure_kernel(Cube c, unsigned long long *out) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t esum;
  for (uint32_t v = threadIdx.x; v < c.q; v += kBlock) hist[v] = 0;
  if (threadIdx.x == 0) esum = 0;
  __syncthreads();
  const uint32_t L = c.L, cpr = L >> 2;
  const size_t plane = (size_t)L * L;
  uint32_t e = 0;
  for (uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x; g < c.nchunks;
       g += (uint64_t)gridDim.x * kBlock) {
    const uint64_t r = g / cpr;
    const uint32_t j = (uint32_t)(g - r * cpr);
    const uint32_t z = (uint32_t)(r / L), y = (uint32_t)(r - (uint64_t)z * L);
    const uint32_t yd = y + 1 == L ? 0 : y + 1, zf = z + 1 == L ? 0 : z + 1;
    const uint32_t *row = reinterpret_cast<const uint32_t *>(c.spins + (size_t)z * plane + (size_t)y * L);
    const uint32_t cur = row[j];
    const uint32_t rt = row[j + 1 == cpr ? 0 : j + 1];
    const uint32_t right = (cur >> 8) | (rt << 24);
    const uint32_t dn = reinterpret_cast<const uint32_t *>(c.spins + (size_t)z * plane + (size_t)yd * L)[j];
    const uint32_t fw = reinterpret_cast<const uint32_t *>(c.spins + (size_t)zf * plane + (size_t)y * L)[j];
    e += __popc(zero_bytes(cur ^ right)) + __popc(zero_bytes(cur ^ dn)) + __popc(zero_bytes(cur ^ fw));
    for (uint32_t i = 0; i < 4; ++i) atomicAdd(&hist[byte_of(cur, i)], 1u);
  }
  e = wave_sum(e);
  if ((threadIdx.x & 63) == 0 && e) atomicAdd(&esum, e);
  __syncthreads();
  for (uint32_t v = threadIdx.x; v < c.q; v += kBlock) {
    const uint32_t n = hist[v];
    if (n) atomicAdd(&out[1 + v], (unsigned long long)n);
  }
  if (threadIdx.x == 0 && esum) atomicAdd(&out[0], (unsigned long long)esum);
}

unsigned grid_of(uint64_t items, unsigned cap) {
  const uint64_t need = (items + kBlock - 1) / kBlock;
  return (unsigned)(need < cap ? (need ? need : 1) : cap);
}

int fail(int code, const std::string &msg) { return potts::record_error(code, msg); }

#define HIP_TRY3(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) return fail(POTTS_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

Cube cube_of(const potts3d_state *s) {
  Cube c;
  c.spins = s->spins;
  c.L = (uint32_t)s->L;
  c.q = (uint32_t)s->q;
  c.nchunks = (uint64_t)s->L * s->L * s->L / 4;
  c.k0 = (uint32_t)s->seed;
  c.k1 = (uint32_t)(s->seed >> 32);
  return c;
}

void release(potts3d_state *s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->spins) (void)hipFree(s->spins);
  if (s->planes) (void)hipFree(s->planes);
  if (s->records) (void)hipFree(s->records);
  if (s->scratch) (void)hipFree(s->scratch);
  if (s->stats_out) (void)hipFree(s->stats_out);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

bool packed_ok(const potts3d_state *s) { return s->L % 32 == 0; }

bool use_packed(const potts3d_state *s) { return s->kernel == 1 || (s->kernel == 0 && packed_ok(s)); }

// longest walk that still leaves >= 2048 workgroups to spread over the chip
uint32_t packed_rows(const potts3d_state *s) {
  if (s->rows) return (uint32_t)s->rows;
  const uint64_t L = (uint64_t)s->L, ipr = L / 32;
  for (uint32_t R : {32u, 16u, 8u, 4u})
    if (ipr * L * (L / R) >= 2048ull * kBlock) return R;
  return 2;
}

// make the row-major cube current
int sync_spins(potts3d_state *s) {
  if (s->spins_valid) return POTTS_OK;
  HIP_TRY3(potts::cube::launch_unpack(s->planes, s->spins, (uint32_t)s->L, s->stream));
  s->spins_valid = true;
  return POTTS_OK;
}

// make the colour-split copy current (allocated on first use)
int sync_planes(potts3d_state *s) {
  if (s->planes_valid) return POTTS_OK;
  if (!s->planes && hipMalloc(&s->planes, (size_t)s->L * s->L * s->L) != hipSuccess) {
    (void)hipGetLastError();
    s->planes = nullptr;
    return fail(POTTS_ENOMEM, "device allocation of the colour planes failed");
  }
  HIP_TRY3(potts::cube::launch_pack(s->spins, s->planes, (uint32_t)s->L, s->stream));
  s->planes_valid = true;
  return POTTS_OK;
}

int run(potts3d_state *s, const uint32_t thr[6], int64_t nsweeps) {
  if (!s) return fail(POTTS_EINVAL, "state is NULL");
  if (nsweeps < 0) return fail(POTTS_EINVAL, "nsweeps must be >= 0");
  if (nsweeps > INT64_MAX - s->t) return fail(POTTS_ERANGE, "sweep counter overflow");
  if (nsweeps == 0) return POTTS_OK;
  const int64_t rl = s->q + 1;
  const bool packed = use_packed(s);
  const int rc = packed ? sync_planes(s) : sync_spins(s);
  if (rc) return rc;
  // the first sweep's slot; each colour-1 launch clears the next one
  const int64_t slot = s->t & (s->rec_cap - 1);
  HIP_TRY3(hipMemsetAsync(s->records + slot * rl, 0, (size_t)rl * 8, s->stream));
  if (packed) {
    potts::cube::CubeLaunch l{};
    l.planes = s->planes;
    l.plane_bytes = (uint64_t)s->L * s->L * s->L / 2;
    l.L = (uint32_t)s->L;
    l.q = (uint32_t)s->q;
    l.ipr = l.L / 32;
    l.rows = packed_rows(s);
    l.nitems = l.ipr * l.L * (l.L / l.rows);
    l.k0 = (uint32_t)s->seed;
    l.k1 = (uint32_t)(s->seed >> 32);
    for (int i = 0; i < 6; ++i) l.thr.v[i] = thr[i];
    const unsigned grid = potts::cube::packed_grid(l);
    for (int64_t k = 0; k < nsweeps; ++k) {
      const int64_t t = s->t + k;
      l.t_lo = (uint32_t)(uint64_t)t;
      l.t_hi = (uint32_t)((uint64_t)t >> 32);
      l.rec = s->records + (t & (s->rec_cap - 1)) * rl;
      l.rec_clear = nullptr;
      HIP_TRY3(potts::cube::launch_packed(l, 0, grid, s->stream));
      l.rec_clear = s->records + ((t + 1) & (s->rec_cap - 1)) * rl;
      HIP_TRY3(potts::cube::launch_packed(l, 1, grid, s->stream));
    }
    s->spins_valid = false;
  } else {
    CubeSweep p{};
    p.c = cube_of(s);
    for (int i = 0; i < 6; ++i) p.thr[i] = thr[i];
    const unsigned grid = grid_of(p.c.nchunks, 4096);
    for (int64_t k = 0; k < nsweeps; ++k) {
      const int64_t t = s->t + k;
      p.t_lo = (uint32_t)(uint64_t)t;
      p.t_hi = (uint32_t)((uint64_t)t >> 32);
      p.rec = s->records + (t & (s->rec_cap - 1)) * rl;
      p.rec_clear = nullptr;
      hipLaunchKernelGGL(cube_sweep_kernel<0>, dim3(grid), dim3(kBlock), 0, s->stream, p);
      p.rec_clear = s->records + ((t + 1) & (s->rec_cap - 1)) * rl;
      hipLaunchKernelGGL(cube_sweep_kernel<1>, dim3(grid), dim3(kBlock), 0, s->stream, p);
      HIP_TRY3(hipGetLastError());
    }
    s->planes_valid = false;
  }
  s->t += nsweeps;
  return POTTS_OK;
}

int table6(double beta, uint32_t thr[6]) {
  if (!thr) return fail(POTTS_EINVAL, "thr is NULL");
  if (!(beta >= 0.0) || !isfinite(beta)) return fail(POTTS_EINVAL, "beta must be finite and >= 0");
  for (int d = 1; d <= 6; ++d) {
    const double scaled = floor(ldexp(exp(-beta * (double)d), 32));
    thr[d - 1] = scaled >= 4294967295.0 ? 4294967295u : (uint32_t)scaled;
  }
  return POTTS_OK;
}

int window(const potts3d_state *s, int64_t t0, int64_t n, int64_t *slot0) {
  if (n < 0 || t0 < 0) return fail(POTTS_EINVAL, "negative record index or count");
  const int64_t oldest = s->t - s->rec_cap + 1;
  if (t0 < (oldest > 0 ? oldest : 0) || t0 + n > s->t)
    return fail(POTTS_ERANGE, "requested records are not in the ring");
  *slot0 = t0 & (s->rec_cap - 1);
  return POTTS_OK;
}

}  // namespace

extern "C" {

int potts3d_init(int32_t L, int32_t q, uint64_t seed, potts_start start, potts3d_state **out) {
  if (!out) return fail(POTTS_EINVAL, "out is NULL");
  *out = nullptr;
  if (L < 4 || L % 4 || q < 2 || q > POTTS_QMAX || (start != POTTS_ORDERED && start != POTTS_RANDOM))
    return fail(POTTS_EINVAL, "need L >= 4, L % 4 == 0, 2 <= q <= 256 and a valid start");
  if ((uint64_t)L * L * L / 4 >= (1ull << 32)) return fail(POTTS_ERANGE, "L^3/4 must be below 2^32");
  potts3d_state *s = new (std::nothrow) potts3d_state();
  if (!s) return fail(POTTS_ENOMEM, "host allocation failed");
  s->L = L;
  s->q = q;
  s->seed = seed;
  s->rec_cap = kRingSlots;
  const size_t n = (size_t)L * L * L;
  if (hipStreamCreate(&s->stream) != hipSuccess || hipMalloc(&s->spins, n) != hipSuccess ||
      hipMalloc(&s->records, (size_t)kRingSlots * (q + 1) * 8) != hipSuccess ||
      hipMalloc(&s->scratch, (size_t)(q + 1) * 8) != hipSuccess || hipMalloc(&s->stats_out, 8 * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    release(s);
    return fail(POTTS_ENOMEM, "device allocation failed");
  }
  const Cube c = cube_of(s);
  hipLaunchKernelGGL(cube_init_kernel, dim3((unsigned)((c.nchunks + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s->stream, c, start == POTTS_RANDOM ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    release(s);
    return fail(POTTS_EDEVICE, std::string("cube_init_kernel: ") + hipGetErrorString(e));
  }
  *out = s;
  return POTTS_OK;
}

int potts3d_threshold_table(double beta, uint32_t thr[6]) { return table6(beta, thr); }

int potts3d_sweep(potts3d_state *s, double beta, int64_t nsweeps) {
  if (!s) return fail(POTTS_EINVAL, "state is NULL");
  if (!s->have_thr || s->thr_beta != beta) {
    uint32_t thr[6];
    const int rc = table6(beta, thr);
    if (rc) return rc;
    for (int i = 0; i < 6; ++i) s->thr[i] = thr[i];
    s->thr_beta = beta;
    s->have_thr = true;
  }
  return run(s, s->thr, nsweeps);
}

int potts3d_sweep_thr(potts3d_state *s, const uint32_t thr[6], int64_t nsweeps) {
  if (!thr) return fail(POTTS_EINVAL, "thr is NULL");
  return run(s, thr, nsweeps);
}

int potts3d_records(potts3d_state *s, int64_t t0, int64_t n, int64_t *out) {
  if (!s || (!out && n > 0)) return fail(POTTS_EINVAL, "NULL argument");
  int64_t slot0 = 0;
  const int rc = window(s, t0, n, &slot0);
  if (rc) return rc;
  const int64_t rl = s->q + 1;
  for (int64_t done = 0; done < n;) {
    const int64_t slot = (slot0 + done) & (s->rec_cap - 1);
    const int64_t run_n = std::min<int64_t>(n - done, s->rec_cap - slot);
    HIP_TRY3(hipMemcpyAsync(out + done * rl, s->records + slot * rl, (size_t)(run_n * rl) * 8,
                            hipMemcpyDeviceToHost, s->stream));
    done += run_n;
  }
  HIP_TRY3(hipStreamSynchronize(s->stream));
  return POTTS_OK;
}

int potts3d_observables(potts3d_state *s, potts_obs *out) {
  if (!s || !out) return fail(POTTS_EINVAL, "NULL argument");
  const int64_t rl = s->q + 1;
  const int rc = sync_spins(s);
  if (rc) return rc;
  HIP_TRY3(hipMemsetAsync(s->scratch, 0, (size_t)rl * 8, s->stream));
  const Cube c = cube_of(s);
  hipLaunchKernelGGL(cube_measure_kernel, dim3(grid_of(c.nchunks, 4096)), dim3(kBlock), 0, s->stream, c, s->scratch);
  HIP_TRY3(hipGetLastError());
  std::vector<int64_t> rec((size_t)rl);
  HIP_TRY3(hipMemcpyAsync(rec.data(), s->scratch, (size_t)rl * 8, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY3(hipStreamSynchronize(s->stream));
  out->t = s->t;
  out->e_sat = rec[0];
  out->q = s->q;
  out->L = s->L;
  out->nmax = 0;
  for (int v = 0; v < POTTS_QMAX; ++v) out->hist[v] = v < s->q ? rec[1 + v] : 0;
  for (int v = 0; v < s->q; ++v) out->nmax = rec[1 + v] > out->nmax ? rec[1 + v] : out->nmax;
  return POTTS_OK;
}

int potts3d_stats(potts3d_state *s, int64_t t0, int64_t n, double beta, potts_summary *out) {
  if (!s || !out) return fail(POTTS_EINVAL, "NULL argument");
  if (n < 1 || n > (1ll << 24)) return fail(POTTS_EINVAL, "window must hold 1 .. 2^24 records");
  if (!(beta >= 0.0) || !isfinite(beta)) return fail(POTTS_EINVAL, "beta must be finite and >= 0");
  int64_t slot0 = 0;
  const int rc = window(s, t0, n, &slot0);
  if (rc) return rc;
  potts::StatsParams p{};
  p.ring = s->records;
  p.cap = s->rec_cap;
  p.slot0 = slot0;
  p.n = n;
  p.q = (uint32_t)s->q;
  p.N = (uint64_t)s->L * s->L * s->L;
  p.beta = beta;
  p.out = s->stats_out;
  HIP_TRY3(potts::launch_stats(p, s->stream));
  double v[5];
  HIP_TRY3(hipMemcpyAsync(v, s->stats_out, sizeof(v), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY3(hipStreamSynchronize(s->stream));
  out->n = n;
  out->e = v[0];
  out->C = v[1];
  out->V_L = v[2];
  out->m = v[3];
  out->chi = v[4];
  return POTTS_OK;
}

int potts3d_get_spins(potts3d_state *s, uint8_t *host_out) {
  if (!s || !host_out) return fail(POTTS_EINVAL, "NULL argument");
  const int rc = sync_spins(s);
  if (rc) return rc;
  HIP_TRY3(hipMemcpyAsync(host_out, s->spins, (size_t)s->L * s->L * s->L, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY3(hipStreamSynchronize(s->stream));
  return POTTS_OK;
}

int potts3d_tune(potts3d_state *s, int32_t kernel, int32_t rows) {
  if (!s) return fail(POTTS_EINVAL, "state is NULL");
  if (kernel < 0 || kernel > 2) return fail(POTTS_EINVAL, "kernel must be 0 (automatic), 1 or 2");
  if (kernel == 1 && !packed_ok(s)) return fail(POTTS_EINVAL, "the colour-split kernel needs L % 32 == 0");
  if (rows < 0 || rows % 2 || (rows && (rows > s->L || s->L % rows)))
    return fail(POTTS_EINVAL, "rows must be 0 or an even divisor of L");
  s->kernel = kernel;
  s->rows = rows;
  return POTTS_OK;
}

int64_t potts3d_time(const potts3d_state *s) { return s ? s->t : -1; }

void *potts3d_stream(const potts3d_state *s) { return s ? (void *)s->stream : nullptr; }

void potts3d_free(potts3d_state *s) { release(s); }

}  // extern "C"
