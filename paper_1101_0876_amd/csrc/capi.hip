// capi.hip -- the C ABI declared in include/potts.h: state lifetime, the
// per-temperature threshold table, sweep launches, records and checkpoints.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "../../include/potts.h"
#include "drawn.hpp"
#include "band.hpp"
#include "kernels.hpp"

struct potts_state {
  int32_t L = 0, q = 0;
  uint64_t seed = 0;
  int64_t t = 0;              // sweeps done
  int64_t rec_from = 0;       // first sweep index whose record is still valid
  uint8_t *spins = nullptr;   // current lattice
  uint8_t *spins2 = nullptr;  // second buffer
  bool owns_spins = true;
  hipStream_t stream = nullptr;
  bool owns_stream = false;
  unsigned long long *records = nullptr;  // ring of rec_cap slots of (1+q)
  int64_t rec_cap = 0;
  unsigned long long *scratch = nullptr;  // 1+q int64 for measurements
  unsigned long long *stripes = nullptr;  // partial records of the strip kernel (2 sets)
  double *stats_out = nullptr;            // 5 doubles
  bool have_thr = false;
  double thr_beta = 0.0;
  uint32_t thr[4] = {0, 0, 0, 0};
  int kernel = 0;          // 0 automatic, 1 strip, 2 chunk, 3 LDS-resident, 4 colour-split, 5 tiles, 6 LDS-resident with pre-drawn words, 7 LDS bands
  uint32_t rows = 0;       // strip rows per work item, 0 = automatic
  unsigned max_groups = 0; // persistent grid size, 0 = automatic
  uint32_t wpe = 0;        // colour-split kernel: waves per SIMD asked of the compiler (0 = its choice)
  // The colour-split kernel works on a copy of the lattice in spins2 split
  // into its two colour planes; the row-major lattice in spins is rebuilt
  // only when something reads it, and the copy only when it is stale.
  bool spins_valid = true;    // spins holds the current configuration
  bool planes_valid = false;  // spins2 holds it, colour-split
  // heat-bath draw table of the colour-split kernel (device copy, and the host
  // copy it was uploaded from, valid for hb_thr and q)
  potts::HbTable *hb_dev = nullptr;
  potts::HbTable *hb_host = nullptr;
  uint32_t hb_thr[4] = {0, 0, 0, 0};
  bool hb_valid = false, hb_wide = false;
  // graph replay of colour-split sweeps: graph_sweeps sweeps per captured
  // graph (0 = off); the graph's kernels read g_desc, written once per call
  int32_t graph_sweeps = 0;
  potts::StripParams *g_desc = nullptr;  // device, one descriptor
  potts::StripTile *g_tiles = nullptr;   // device, the lattice's tiles
  size_t g_ntiles = 0;
  hipGraph_t g_graph = nullptr;
  hipGraphExec_t g_exec = nullptr;
  uint32_t g_rows = 0, g_wpe = 0;        // what the graph was captured for
  int32_t g_K = 0;
  bool g_wide = false;
  // several sweeps per launch on LDS tiles (tiles.hip): the shape asked for
  // (0 = automatic) and the partial records of a launch's sweeps
  uint32_t tile_tx = 0, tile_ty = 0, tile_sweeps = 0;
  unsigned long long *tstripes = nullptr;
  // pre-drawn random words of a chunk of sweeps (drawn.hpp), allocated on first use
  uint32_t *drawn = nullptr;
  // persistent sweeps on LDS bands (band.hip): the shape asked for (0 =
  // automatic), the edge-row exchange buffer, the flags with their epoch, the
  // partial records of a launch and the host-visible error word
  uint32_t band_rows = 0, band_block = 0;
  uint32_t band_auto_rows = 0, band_auto_block = 0;  // the automatic shape, once found
  bool band_auto_tried = false;
  uint8_t *bxbuf = nullptr;
  size_t bxbytes = 0;
  uint32_t *bflags = nullptr;
  size_t bflag_words = 0;
  uint32_t bepoch = 0;
  unsigned long long *bstripes = nullptr;
  uint32_t *berr = nullptr;
  uint64_t bclock_khz = 0;  // rate of the kernel's wall clock
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

}  // namespace

namespace potts {
int record_error(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}
}  // namespace potts

namespace {

int hip_fail(hipError_t e, const char *what) {
  return fail(POTTS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                                  \
  do {                                                 \
    hipError_t hip_err_ = (call);                      \
    if (hip_err_ != hipSuccess) return hip_fail(hip_err_, #call); \
  } while (0)

// Makes the row-major lattice current (queued on the state's stream).
int sync_spins(potts_state *s) {
  if (s->spins_valid) return POTTS_OK;
  HIP_TRY(potts::launch_unpack(s->spins2, s->spins, (uint32_t)s->L, s->stream));
  s->spins_valid = true;
  return POTTS_OK;
}

// The ring holds a power-of-two number of slots (>= the capacity asked for),
// so kernels find a sweep's slot with a mask.
// partial records per set of the strip kernel's single-lattice launches
constexpr uint32_t kStripes = 32;

int64_t ring_slots(int64_t capacity) {
  int64_t n = 2;
  while (n < capacity) n <<= 1;
  return n;
}

bool valid_shape(int32_t L, int32_t q) { return L >= 4 && L % 4 == 0 && q >= 2 && q <= POTTS_QMAX; }

uint64_t n_sites(const potts_state *s) { return (uint64_t)s->L * (uint64_t)s->L; }

void release(potts_state *s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->owns_spins) {
    if (s->spins) (void)hipFree(s->spins);
    if (s->spins2) (void)hipFree(s->spins2);
  }
  if (s->records) (void)hipFree(s->records);
  if (s->scratch) (void)hipFree(s->scratch);
  if (s->stripes) (void)hipFree(s->stripes);
  if (s->stats_out) (void)hipFree(s->stats_out);
  if (s->g_exec) (void)hipGraphExecDestroy(s->g_exec);
  if (s->g_graph) (void)hipGraphDestroy(s->g_graph);
  if (s->g_desc) (void)hipFree(s->g_desc);
  if (s->g_tiles) (void)hipFree(s->g_tiles);
  if (s->hb_dev) (void)hipFree(s->hb_dev);
  if (s->tstripes) (void)hipFree(s->tstripes);
  if (s->drawn) (void)hipFree(s->drawn);
  if (s->bxbuf) (void)hipFree(s->bxbuf);
  if (s->bflags) (void)hipFree(s->bflags);
  if (s->bstripes) (void)hipFree(s->bstripes);
  if (s->berr) (void)hipHostFree(s->berr);
  if (s->hb_host) (void)hipHostFree(s->hb_host);
  if (s->owns_stream && s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

int write_initial(potts_state *s, potts_start start) {
  potts::InitParams p{};
  p.spins = s->spins;
  p.L = (uint32_t)s->L;
  p.q = (uint32_t)s->q;
  p.nchunks = n_sites(s) / 4;
  p.k0 = (uint32_t)s->seed;
  p.k1 = (uint32_t)(s->seed >> 32);
  p.random = start == POTTS_RANDOM;
  HIP_TRY(potts::launch_init(p, s->stream));
  return POTTS_OK;
}

int create(int32_t L, int32_t q, uint64_t seed, potts_start start, void *dev_spins, void *dev_spins2,
           size_t bytes, void *stream, bool external, int64_t rec_cap, potts_state **out) {
  if (!out) return fail(POTTS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!valid_shape(L, q)) return fail(POTTS_EINVAL, "need L >= 4, L % 4 == 0, 2 <= q <= 256");
  if (start != POTTS_ORDERED && start != POTTS_RANDOM) return fail(POTTS_EINVAL, "bad start");
  if ((uint64_t)L * (uint64_t)L / 4 >= (1ull << 32))
    return fail(POTTS_ERANGE, "L*L/4 must be below 2^32 (Philox counter word)");
  if (rec_cap == 0) rec_cap = 4096;
  if (rec_cap < 2 || rec_cap > (1ll << 40)) return fail(POTTS_EINVAL, "records_capacity must be in 2 .. 2^40");
  rec_cap = ring_slots(rec_cap);
  const size_t nbytes = (size_t)L * (size_t)L;
  // caller buffers: both or neither (neither = library-owned buffers on the caller's stream)
  const bool ext_buffers = external && (dev_spins || dev_spins2);
  if (ext_buffers && (!dev_spins || !dev_spins2 || bytes < nbytes))
    return fail(POTTS_EINVAL, "give both buffers (each at least L*L bytes) or neither");
  potts_state *s = new (std::nothrow) potts_state();
  if (!s) return fail(POTTS_ENOMEM, "host allocation failed");
  s->L = L;
  s->q = q;
  s->seed = seed;
  if (external) {
    s->stream = (hipStream_t)stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      release(s);
      return hip_fail(e, "hipStreamCreateWithFlags");
    }
    s->owns_stream = true;
  }
  if (ext_buffers) {
    s->owns_spins = false;
    s->spins = (uint8_t *)dev_spins;
    s->spins2 = (uint8_t *)dev_spins2;
  } else {
    if (hipMalloc(&s->spins, nbytes) != hipSuccess || hipMalloc(&s->spins2, nbytes) != hipSuccess) {
      (void)hipGetLastError();
      release(s);
      return fail(POTTS_ENOMEM, "hipMalloc of the lattice failed");
    }
  }
  s->rec_cap = rec_cap;
  const size_t rec_bytes = (size_t)rec_cap * (size_t)(q + 1) * sizeof(unsigned long long);
  const uint64_t stripe_total = 2ull * kStripes * potts::stripe_words((uint32_t)q);
  if (hipMalloc(&s->records, rec_bytes) != hipSuccess ||
      hipMalloc(&s->scratch, (size_t)(q + 1) * sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&s->stats_out, 8 * sizeof(double)) != hipSuccess ||
      hipMalloc(&s->stripes, stripe_total * sizeof(unsigned long long)) != hipSuccess) {
    (void)hipGetLastError();
    release(s);
    return fail(POTTS_ENOMEM, "hipMalloc of the record ring failed");
  }
  int rc = write_initial(s, start);
  if (rc == POTTS_OK) {
    hipError_t e = potts::launch_fill_u64(s->stripes, stripe_total, 0ull, s->stream);
    if (e != hipSuccess) rc = hip_fail(e, "launch_fill_u64");
  }
  if (rc == POTTS_OK) {
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
  }
  if (rc != POTTS_OK) {
    release(s);
    return rc;
  }
  *out = s;
  return POTTS_OK;
}

int build_table(double beta, uint32_t thr[4]);

}  // namespace

namespace potts {
int build_threshold_table(double beta, uint32_t thr[4]) { return build_table(beta, thr); }
}  // namespace potts

namespace {

int build_table(double beta, uint32_t thr[4]) {
  if (!(beta >= 0.0) || !isfinite(beta)) return fail(POTTS_EINVAL, "beta must be finite and >= 0");
  for (int d = 1; d <= 4; ++d) {
    const double scaled = floor(exp(-beta * d) * 4294967296.0);
    thr[d - 1] = scaled >= 4294967295.0 ? 4294967295u : (uint32_t)scaled;
  }
  return POTTS_OK;
}

// the strip kernel addresses the lattice with 32-bit buffer offsets, whose
// range check leaves the last bytes of a 4 GiB buffer out: L * L < 2^32
bool strip_ok(const potts_state *s) { return s->L % 16 == 0 && s->L <= 65520; }

bool resident_ok(const potts_state *s) { return potts::resident_fits((uint32_t)s->L, (uint32_t)s->q); }

// single lattices of at most 512 eight-byte items (L <= 64): the resident
// kernel with its words drawn beforehand by the whole GPU, the automatic
// choice (the plain method, L = 64, q = 9, 1000 sweeps: 2.40 ms per run with
// the words drawn in the resident kernel itself)
bool drawn_ok(const potts_state *s) { return potts::drawn_fits((uint32_t)s->L, (uint32_t)s->q); }

bool use_drawn(const potts_state *s) { return drawn_ok(s) && (s->kernel == 6 || s->kernel == 0); }

bool use_resident(const potts_state *s) {
  return resident_ok(s) && (s->kernel == 3 || s->kernel == 6 || s->kernel == 0);
}

// the colour-split copy needs 16-byte groups of packed bytes: L % 32 == 0
bool packed_ok(const potts_state *s) { return strip_ok(s) && s->L % 32 == 0; }

bool auto_tiles(const potts_state *s);

bool use_packed(const potts_state *s) {
  return packed_ok(s) && (s->kernel == 4 || (s->kernel == 0 && !auto_tiles(s)));
}

bool use_strip(const potts_state *s) { return strip_ok(s) && (s->kernel == 1 || s->kernel == 0); }

// The tile shape (interior tx bytes x ty rows, sweeps per launch) of the
// multi-sweep tile kernel: the one asked for, else about 256-512 tiles per
// lattice (tx the largest of 256 .. 16 bytes up to L/8 dividing L, ty 16 rows
// up to L = 1024 and 32 above, or the largest even divisor below), 4 sweeps
// per launch.  Measured on MI355X (q = 6, ps per site update): L = 512 64x16
// 16.9 (128x16 21.6, 256x32 32.6), L = 1024 128x16 6.1 (64x16 6.4, 256x32
// 8.3), L = 2048 256x32 2.67 (256x64 with 8 sweeps 3.05, 128x16 3.64).
bool tile_shape(const potts_state *s, uint32_t *tx, uint32_t *ty, uint32_t *sweeps) {
  const uint32_t L = (uint32_t)s->L;
  *sweeps = s->tile_sweeps ? s->tile_sweeps : 4u;
  *tx = s->tile_tx;
  *ty = s->tile_ty;
  for (uint32_t c = 256; !*tx && c >= 16; c /= 2)
    if (L % c == 0 && (c * 8 <= L || c == 16)) *tx = c;
  for (uint32_t c = L <= 1024 ? 16u : 32u; !*ty && c >= 2; c /= 2)
    if (L % c == 0) *ty = c;
  return *tx && *ty && potts::tile_shape_ok(L, *tx, *ty, 2u * *sweeps);
}

bool tiles_ok(const potts_state *s) {
  uint32_t tx, ty, n;
  return s->L % 16 == 0 && s->L <= 65520 && tile_shape(s, &tx, &ty, &n);
}

// the automatic choice for lattices too large for one workgroup's LDS and too
// small for a half sweep to hide a kernel boundary: the colour-split kernel
// runs L = 512 / 1024 / 2048 at 48.7 / 12.2 / 3.47 ps per site update, the
// tiles at 16.9 / 6.1 / 2.67; from L = 4096 (1.64 against 1.86) the halo work
// costs more than the launches it saves
bool auto_tiles(const potts_state *s) { return s->L > 256 && s->L <= 2048 && tiles_ok(s); }

bool use_tiles(const potts_state *s) {
  return tiles_ok(s) && (s->kernel == 5 || (s->kernel == 0 && !use_resident(s) && auto_tiles(s)));
}

bool wide_table(const uint32_t thr[4]) { return !thr[0] || !thr[1] || !thr[2] || !thr[3]; }

// Lanes per band workgroup: the fewest of 256 / 512 / 1024 that give every
// item of a half sweep its own lane, else 1024.
uint32_t band_block_for(uint32_t L, uint32_t rows) {
  const uint64_t items = (uint64_t)rows * (L / 32);
  return items <= 256 ? 256u : items <= 512 ? 512u : 1024u;
}

// The band shape (rows per band, lanes per workgroup): the one asked for, or
// the first of 8, 16, 4, 32, 2 rows whose grid of L / rows workgroups can be
// resident at once.
bool band_shape(potts_state *s, uint32_t *rows, uint32_t *block) {
  const uint32_t L = (uint32_t)s->L;
  if (s->band_rows) {
    *rows = s->band_rows;
    *block = s->band_block ? s->band_block : band_block_for(L, *rows);
    bool fits = false;
    if (potts::band_resident(L, (uint32_t)s->q, *rows, *block, &fits) != hipSuccess) {
      (void)hipGetLastError();  // not left for a later launch check to report
      return false;
    }
    return fits;
  }
  if (!s->band_auto_tried) {
    s->band_auto_tried = true;
    static const uint32_t cand[] = {8, 16, 4, 32, 2};
    for (uint32_t r : cand) {
      bool fits = false;
      const uint32_t blk = band_block_for(L, r);
      if (potts::band_resident(L, (uint32_t)s->q, r, blk, &fits) != hipSuccess) {
        (void)hipGetLastError();
        return false;
      }
      if (fits) {
        s->band_auto_rows = r;
        s->band_auto_block = blk;
        break;
      }
    }
  }
  *rows = s->band_auto_rows;
  *block = s->band_auto_block;
  return *rows != 0;
}

bool band_ok(potts_state *s) {
  uint32_t rows, block;
  return s->L % 32 == 0 && s->L <= 16384 && band_shape(s, &rows, &block);
}

// The automatic choice for L = 2048 .. 4096: measured on MI355X (q = 6, ps
// per site update), L = 2048 2.06 (8-row bands of 512 lanes; the tile kernel
// 2.68), L = 4096 1.08 (16-row bands of 1024 lanes; the colour-split kernel
// 1.64).  At L = 1024 the tile kernel stays ahead (6.1 against 9.1: a half
// sweep there is shorter than the exchange of edge rows), and from L = 8192
// no band of whole rows whose grid the GPU holds at once fits in LDS.
bool auto_band(potts_state *s) { return s->L >= 2048 && s->L <= 4096 && band_ok(s); }

bool use_band(potts_state *s) { return s->kernel == 7 ? band_ok(s) : s->kernel == 0 && auto_band(s); }

}  // namespace

namespace potts {

// Items of `rows` rows and ipr items per row band over nrows rows, with the
// division item -> row band as a shift or a multiply.
void set_items(StripParams &p, uint32_t ipr, uint32_t nrows, uint32_t rows) {
  p.ipr = ipr;
  p.rows = rows;
  p.nitems = (nrows / rows) * ipr;
  p.item_shift = -1;
  p.item_magic = 0;
  if ((ipr & (ipr - 1)) == 0) {
    p.item_shift = 0;
    while ((1u << p.item_shift) < ipr) ++p.item_shift;
  } else {
    // ceil(2^64 / ipr); ipr >= 3 here
    p.item_magic = (uint64_t)(((unsigned __int128)1 << 64) / ipr) + 1;
  }
}

// Fills the per-lattice descriptor of the strip kernel (not t0/nsweeps/ring).
void fill_strip_params(StripParams &p, uint8_t *spins, uint32_t L, uint32_t q, uint64_t seed,
                       const uint32_t thr[4], uint32_t rows) {
  p.spins = spins;
  p.L = L;
  p.q = q;
  set_items(p, L / 16, L, rows);
  p.nrows = L;
  p.first_row = 0;
  p.up_row = L - 1;
  p.down_row = 0;
  p.ctr0 = 0;
  p.stripes = nullptr;
  p.nstripes = 0;
  p.row_words = L / 4;
  p.k0 = (uint32_t)seed;
  p.k1 = (uint32_t)(seed >> 32);
  for (int i = 0; i < 4; ++i) p.thr.v[i] = thr[i];
}

void fill_slab_params(StripParams &p, uint8_t *slab, uint32_t L, uint32_t h, uint32_t y0, uint32_t q,
                      uint64_t seed, const uint32_t thr[4], uint32_t rows) {
  fill_strip_params(p, slab, L, q, seed, thr, rows);
  set_items(p, L / 16, h, rows);
  p.nrows = h;
  p.first_row = 1;
  p.up_row = 0;
  p.down_row = h + 1;
  p.ctr0 = y0 * (L / 4);
}

uint32_t auto_strip_rows(uint32_t L, uint32_t nrows, uint64_t want) {
  const uint32_t ipr = L / 16;
  for (uint32_t r = 32; r > 2; r /= 2)
    if (nrows % r == 0 && (uint64_t)(nrows / r) * ipr >= want) return r;
  return 2;
}

}  // namespace potts

namespace {

using potts::fill_strip_params;

// Sweeps whose records the resident kernel writes whole: no slot clearing.
int run_resident(potts_state *s, const uint32_t thr[4], int64_t nsweeps) {
  potts::ResidentLaunch p{};
  p.jobs = nullptr;
  potts::ResidentJob &j = p.single;
  j.spins = s->spins;
  j.L = (uint32_t)s->L;
  j.q = (uint32_t)s->q;
  j.k0 = (uint32_t)s->seed;
  j.k1 = (uint32_t)(s->seed >> 32);
  for (int i = 0; i < 4; ++i) j.thr.v[i] = thr[i];
  j.ring = s->records;
  j.cap = (uint64_t)s->rec_cap;
  const int64_t chunk = 4096;  // bounds one launch's duration
  for (int64_t done = 0; done < nsweeps; done += chunk) {
    j.t0 = (uint64_t)(s->t + done);
    j.nsweeps = (uint32_t)std::min<int64_t>(chunk, nsweeps - done);
    HIP_TRY(potts::launch_resident(p, 1, j.L, j.q, wide_table(thr), s->stream));
  }
  s->t += nsweeps;
  return POTTS_OK;
}

// The same with the random words drawn first by a generator kernel over the
// whole GPU, kDrawnChunk sweeps at a time.
int run_drawn(potts_state *s, const uint32_t thr[4], int64_t nsweeps) {
  if (!s->drawn) {
    if (hipMalloc(&s->drawn, potts::drawn_words_bytes((uint32_t)s->L)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(POTTS_ENOMEM, "allocation of the pre-drawn words failed");
    }
  }
  potts::ResidentJob j{};
  j.spins = s->spins;
  j.L = (uint32_t)s->L;
  j.q = (uint32_t)s->q;
  j.k0 = (uint32_t)s->seed;
  j.k1 = (uint32_t)(s->seed >> 32);
  for (int i = 0; i < 4; ++i) j.thr.v[i] = thr[i];
  j.ring = s->records;
  j.cap = (uint64_t)s->rec_cap;
  const bool wide = wide_table(thr);
  for (int64_t done = 0; done < nsweeps; done += potts::kDrawnChunk) {
    j.t0 = (uint64_t)(s->t + done);
    j.nsweeps = (uint32_t)std::min<int64_t>(potts::kDrawnChunk, nsweeps - done);
    HIP_TRY(potts::launch_draw_words(j, s->drawn, s->stream));
    HIP_TRY(potts::launch_resident_drawn(j, s->drawn, wide, s->stream));
  }
  s->t += nsweeps;
  return POTTS_OK;
}

// rows per strip item: 32 when that still gives 2048 x 256 items (eight
// workgroups of 256 lanes per CU; L >= 32768), else 16.  Shorter strips on
// smaller lattices cost more than they gain: measured on MI355X (q = 6),
// 16-row strips run L = 4096 / 8192 / 16384 at 2.45 / 1.22 / 0.88 ps per
// site update, against 5.14 / 1.48 / 0.89 with the 2-, 8- and 32-row strips
// that a fixed item count would pick.
uint32_t strip_rows(const potts_state *s) {
  if (s->rows) return s->rows;
  const uint32_t L = (uint32_t)s->L;
  if (L % 32 == 0 && (uint64_t)(L / 32) * (L / 16) >= 2048ull * 256ull) return 32;
  return 16;
}

// rows per item of the colour-split kernel (32 sites per item row): the
// tallest of 32, 16, 8 that still gives 2^20 items (4096 workgroups), else 4.
// Measured on MI355X (q = 6): L = 4096 / 8192 / 16384 / 32768 run at
// 1.69 / 0.95 / 0.82 / 0.85 ps per site update with 4 / 4 / 8 / 32 rows.  Up to
// L = 4096 a sweep is bound by launch and per-workgroup overheads, and the
// shortest walk (most workgroups) wins: q = 9, L = 1024 / 2048 / 4096 take
// 12.8 / 14.3 / 27.4 us per sweep with 2 rows, 17.3 / 18.5 / 29.0 with 4.
uint32_t packed_rows(const potts_state *s) {
  if (s->rows) return s->rows;
  const uint32_t L = (uint32_t)s->L;
  for (uint32_t r = 32; r >= 8; r /= 2)
    if (L % r == 0 && (uint64_t)(L / r) * (L / 32) >= (1ull << 20)) return r;
  return L <= 4096 ? 2 : 4;
}

void drop_graph(potts_state *s) {
  if (s->g_exec) (void)hipGraphExecDestroy(s->g_exec);
  if (s->g_graph) (void)hipGraphDestroy(s->g_graph);
  s->g_exec = nullptr;
  s->g_graph = nullptr;
}

// Captures K colour-split sweeps of the lattice (tiled launches reading the
// device descriptor g_desc, then the fold-and-advance node) into a graph.
int capture_graph(potts_state *s, const potts::StripParams &p, int32_t K, bool wide) {
  drop_graph(s);
  const size_t ntiles = (p.nitems + 255) / 256;
  if (!s->g_desc && hipMalloc(&s->g_desc, sizeof(potts::StripParams)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(POTTS_ENOMEM, "allocation of the graph descriptor failed");
  }
  if (ntiles > s->g_ntiles) {
    if (s->g_tiles) (void)hipFree(s->g_tiles);
    s->g_tiles = nullptr;
    s->g_ntiles = 0;
    if (hipMalloc(&s->g_tiles, ntiles * sizeof(potts::StripTile)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(POTTS_ENOMEM, "allocation of the graph tiles failed");
    }
    s->g_ntiles = ntiles;
  }
  std::vector<potts::StripTile> tiles;
  for (uint32_t first = 0; first < p.nitems; first += 256)
    tiles.push_back(potts::StripTile{0, first, std::min<uint32_t>(256, p.nitems - first), first == 0 ? 1u : 0u});
  HIP_TRY(hipMemcpyAsync(s->g_tiles, tiles.data(), tiles.size() * sizeof(tiles[0]), hipMemcpyHostToDevice,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));  // the host tiles go away next
  HIP_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
  potts::StripLaunch l{};
  l.jobs = s->g_desc;
  l.tiles = s->g_tiles;
  potts::TileShape shape;
  shape.wpe = s->wpe;
  if (!potts::shape_ok(shape, p.q)) shape.wpe = 0;
  hipError_t e = hipSuccess;
  for (int32_t j = 0; j < K && e == hipSuccess; ++j) {
    l.sweep = (uint32_t)j;
    e = potts::launch_packed_tiled(l, 0, (unsigned)tiles.size(), shape, p.q, wide, s->stream);
    if (e == hipSuccess) e = potts::launch_packed_tiled(l, 1, (unsigned)tiles.size(), shape, p.q, wide, s->stream);
  }
  if (e == hipSuccess) e = potts::launch_fold_advance(s->g_desc, (uint32_t)K, s->stream);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(s->stream, &g);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&s->g_exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    s->g_exec = nullptr;
    return hip_fail(e, "capture of the sweep graph");
  }
  s->g_graph = g;
  s->g_rows = p.rows;
  s->g_K = K;
  s->g_wide = wide;
  s->g_wpe = s->wpe;
  return POTTS_OK;
}

// Sweeps on the colour-split copy in the second buffer (packed.hip): pack,
// sweep, unpack; records as the strip path (striped partial records).
int run_packed(potts_state *s, const uint32_t thr[4], int64_t nsweeps) {
  const uint32_t L = (uint32_t)s->L;
  if (!s->planes_valid) {
    HIP_TRY(potts::launch_pack(s->spins, s->spins2, L, s->stream));
    s->planes_valid = true;
  }
  s->spins_valid = false;
  potts::StripLaunch l{};
  potts::StripParams &p = l.single;
  const uint32_t rows = packed_rows(s);
  fill_strip_params(p, s->spins2, L, (uint32_t)s->q, s->seed, thr, rows);
  potts::set_items(p, L / 32, L, rows);
  p.ring = s->records;
  p.cap = (uint64_t)s->rec_cap;
  p.stripes = s->stripes;
  p.nstripes = kStripes;
  const unsigned groups = s->max_groups ? s->max_groups : 8192u;
  const uint64_t need = ((uint64_t)p.nitems + 255) / 256;
  const unsigned grid = (unsigned)(need < groups ? need : groups);
  const bool wide = wide_table(thr);
  // whole graphs of graph_sweeps sweeps first (one workgroup per tile, as the
  // grid-stride launch when the item count fits the grid), the rest direct
  int64_t done = 0;
  const int32_t K = s->graph_sweeps;
  if (K > 0 && nsweeps >= K && need <= groups) {
    if (!s->g_exec || s->g_K != K || s->g_rows != rows || s->g_wide != wide || s->g_wpe != s->wpe) {
      const int rc = capture_graph(s, p, K, wide);
      if (rc) return rc;
    }
    potts::StripParams d = p;
    d.t0 = (uint64_t)s->t;
    d.nsweeps = (uint64_t)K;
    HIP_TRY(potts::launch_set_desc(s->g_desc, d, s->stream));
    for (; done + K <= nsweeps; done += K) HIP_TRY(hipGraphLaunch(s->g_exec, s->stream));
  }
  const int64_t seg = 1ll << 30;
  for (int64_t base = done; base < nsweeps; base += seg) {
    const int64_t count = std::min<int64_t>(seg, nsweeps - base);
    p.t0 = (uint64_t)(s->t + base);
    p.nsweeps = (uint64_t)count;
    for (int64_t j = 0; j < count; ++j) {
      l.sweep = (uint32_t)j;
      HIP_TRY(potts::launch_packed_single(l, 0, grid, l.single.q, wide, s->wpe, s->stream));
      HIP_TRY(potts::launch_packed_single(l, 1, grid, l.single.q, wide, s->wpe, s->stream));
    }
    HIP_TRY(potts::launch_fold_stripes(p, p.t0 + (uint64_t)count - 1, s->stream));
  }
  s->t += nsweeps;
  if (!s->owns_spins) {
    // caller-owned buffers: the row-major lattice is current after every call,
    // and the next call packs it again, so writes between calls are seen
    HIP_TRY(potts::launch_unpack(s->spins2, s->spins, L, s->stream));
    s->spins_valid = true;
    s->planes_valid = false;
  }
  return POTTS_OK;
}

// Sweeps on LDS tiles, several per launch (tiles.hip), ping-ponging the
// row-major lattice between the state's two buffers; each launch's records
// are folded into their ring slots right after it.
int run_tiles(potts_state *s, const uint32_t thr[4], int64_t nsweeps) {
  uint32_t tx, ty, per;
  if (!tile_shape(s, &tx, &ty, &per)) return fail(POTTS_EINVAL, "no tile shape for this lattice");
  const uint32_t sw = potts::stripe_words((uint32_t)s->q);
  const uint64_t words = (uint64_t)potts::kTileMaxSweeps * kStripes * sw;
  if (!s->tstripes) {
    if (hipMalloc(&s->tstripes, words * sizeof(unsigned long long)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(POTTS_ENOMEM, "allocation of the tile partial records failed");
    }
    HIP_TRY(potts::launch_fill_u64(s->tstripes, words, 0ull, s->stream));
  }
  s->planes_valid = false;  // the second buffer now holds row-major lattices
  potts::TileParams p{};
  p.L = (uint32_t)s->L;
  p.q = (uint32_t)s->q;
  p.k0 = (uint32_t)s->seed;
  p.k1 = (uint32_t)(s->seed >> 32);
  for (int i = 0; i < 4; ++i) p.thr.v[i] = thr[i];
  p.tx = tx;
  p.ty = ty;
  p.halo = 2u * per;
  p.tiles_x = p.L / tx;
  p.stripes = s->tstripes;
  p.nstripes = kStripes;
  uint8_t *cur = s->spins, *other = s->spins2;
  for (int64_t done = 0; done < nsweeps; done += per) {
    p.nsweeps = (uint32_t)std::min<int64_t>(per, nsweeps - done);
    p.t0 = (uint64_t)(s->t + done);
    p.src = cur;
    p.dst = other;
    HIP_TRY(potts::launch_tiles(p, s->stream));
    HIP_TRY(potts::launch_fold_sets(p, s->records, (uint64_t)s->rec_cap, s->stream));
    std::swap(cur, other);
  }
  if (cur != s->spins) {
    if (s->owns_spins) {
      std::swap(s->spins, s->spins2);  // library-owned: the buffers trade roles
    } else {
      // the caller's buffer holds the lattice after every call
      HIP_TRY(hipMemcpyAsync(s->spins, cur, (size_t)n_sites(s), hipMemcpyDeviceToDevice, s->stream));
    }
  }
  s->t += nsweeps;
  return POTTS_OK;
}

// A neighbour wait of the band kernel that outlived its bound (possible only
// if its grid was not resident at once) leaves the error word set; the next
// call that sweeps or reads results reports it, and the flags start over.
int band_check(potts_state *s) {
  if (!s->berr || !__atomic_load_n(s->berr, __ATOMIC_ACQUIRE)) return POTTS_OK;
  __atomic_store_n(s->berr, 0u, __ATOMIC_RELEASE);
  if (s->bflags) HIP_TRY(potts::launch_fill_u64(reinterpret_cast<unsigned long long *>(s->bflags),
                                                (s->bflag_words + 1) / 2, 0ull, s->stream));
  s->bepoch = 0;
  return fail(POTTS_EDEVICE, "band sweeps: a wait on a neighbouring band outlived its bound; "
                             "the sweeps since the last successful read are invalid");
}

// Sweeps on LDS bands (band.hip), up to kBandMaxSweeps per cooperative
// launch, each launch's records folded into their ring slots right after it.
int run_band(potts_state *s, const uint32_t thr[4], int64_t nsweeps) {
  uint32_t rows, block;
  if (!band_shape(s, &rows, &block)) return fail(POTTS_EINVAL, "no band shape fits this lattice");
  const uint32_t L = (uint32_t)s->L, q = (uint32_t)s->q;
  const uint32_t bands = L / rows, parts = potts::band_parts(L);
  const size_t xbytes = (size_t)2 * bands * L;  // [plane][band][top, bottom][L/2]
  const size_t fwords = (size_t)bands * parts;
  if (xbytes > s->bxbytes) {
    if (s->bxbuf) (void)hipFree(s->bxbuf);
    s->bxbuf = nullptr;
    s->bxbytes = 0;
    if (hipMalloc(&s->bxbuf, xbytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(POTTS_ENOMEM, "allocation of the band exchange buffer failed");
    }
    s->bxbytes = xbytes;
  }
  if (fwords != s->bflag_words) {
    if (s->bflags) (void)hipFree(s->bflags);
    s->bflags = nullptr;
    s->bflag_words = 0;
    if (hipMalloc(&s->bflags, (fwords + 1) / 2 * 8) != hipSuccess) {
      (void)hipGetLastError();
      return fail(POTTS_ENOMEM, "allocation of the band flags failed");
    }
    HIP_TRY(potts::launch_fill_u64(reinterpret_cast<unsigned long long *>(s->bflags), (fwords + 1) / 2, 0ull,
                                   s->stream));
    s->bflag_words = fwords;
    s->bepoch = 0;
  }
  const uint32_t sw = potts::stripe_words(q);
  if (!s->bstripes) {
    const uint64_t words = (uint64_t)potts::kBandMaxSweeps * kStripes * sw;
    if (hipMalloc(&s->bstripes, words * sizeof(unsigned long long)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(POTTS_ENOMEM, "allocation of the band partial records failed");
    }
    HIP_TRY(potts::launch_fill_u64(s->bstripes, words, 0ull, s->stream));
  }
  if (!s->berr) {
    if (hipHostMalloc(reinterpret_cast<void **>(&s->berr), sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      s->berr = nullptr;
      return fail(POTTS_ENOMEM, "allocation of the band error word failed");
    }
    __atomic_store_n(s->berr, 0u, __ATOMIC_RELEASE);
  }
  if (!s->bclock_khz) {
    int dev = 0, khz = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    s->bclock_khz = (uint64_t)(khz > 0 ? khz : 100000);
  }
  // the bound on one neighbour wait: 0.25 s, or POTTS_BAND_WAIT_US
  // microseconds (a short bound makes the failure path testable)
  uint64_t wait_us = 250000;
  if (const char *w = getenv("POTTS_BAND_WAIT_US")) {
    char *end = nullptr;
    const unsigned long long v = strtoull(w, &end, 10);
    if (end != w && v > 0 && v <= 10000000ull) wait_us = v;
  }
  if (!s->planes_valid) {
    HIP_TRY(potts::launch_pack(s->spins, s->spins2, L, s->stream));
    s->planes_valid = true;
  }
  s->spins_valid = false;
  potts::BandParams p{};
  p.planes = s->spins2;
  p.xbuf = s->bxbuf;
  p.flags = s->bflags;
  p.err = s->berr;
  p.stripes = s->bstripes;
  p.nstripes = kStripes;
  p.L = L;
  p.q = q;
  p.rows = rows;
  p.bands = bands;
  p.parts = parts;
  p.prow_magic = (uint32_t)(((1ull << 32) + L / 32 - 1) / (L / 32));
  p.k0 = (uint32_t)s->seed;
  p.k1 = (uint32_t)(s->seed >> 32);
  for (int i = 0; i < 4; ++i) p.thr.v[i] = thr[i];
  p.wait_ticks = s->bclock_khz * wait_us / 1000u;
  potts::TileParams f{};
  f.q = q;
  f.stripes = s->bstripes;
  f.nstripes = kStripes;
  // one launch's records fold into distinct ring slots
  const int64_t kmax = std::min<int64_t>(potts::kBandMaxSweeps, s->rec_cap);
  for (int64_t done = 0; done < nsweeps;) {
    const int64_t K = std::min<int64_t>(kmax, nsweeps - done);
    p.t0 = (uint64_t)(s->t + done);
    p.nsweeps = (uint32_t)K;
    p.epoch = s->bepoch;
    HIP_TRY(potts::launch_band(p, block, s->stream));
    s->bepoch += 2u * (uint32_t)K;
    f.t0 = p.t0;
    f.nsweeps = (uint32_t)K;
    HIP_TRY(potts::launch_fold_sets(f, s->records, (uint64_t)s->rec_cap, s->stream));
    done += K;
  }
  s->t += nsweeps;
  if (!s->owns_spins) {
    HIP_TRY(potts::launch_unpack(s->spins2, s->spins, L, s->stream));
    s->spins_valid = true;
    s->planes_valid = false;
  }
  return POTTS_OK;
}

int run_sweeps(potts_state *s, const uint32_t thr[4], int64_t nsweeps) {
  if (!s) return fail(POTTS_EINVAL, "state is NULL");
  if (nsweeps < 0) return fail(POTTS_EINVAL, "nsweeps must be >= 0");
  if (nsweeps > INT64_MAX - s->t) return fail(POTTS_ERANGE, "sweep counter overflow");
  {
    const int rc = band_check(s);
    if (rc) return rc;
  }
  if (nsweeps == 0) return POTTS_OK;
  const bool band = use_band(s);
  if (band) return run_band(s, thr, nsweeps);
  if (use_resident(s) || !use_packed(s)) {
    // every other kernel sweeps the row-major lattice (the LDS-resident one
    // too, although the lattice may have a colour-split copy from heat-bath
    // sweeps)
    const int rc = sync_spins(s);
    if (rc) return rc;
    s->planes_valid = false;
  }
  if (use_drawn(s)) return run_drawn(s, thr, nsweeps);
  if (use_resident(s)) return run_resident(s, thr, nsweeps);
  if (use_tiles(s)) return run_tiles(s, thr, nsweeps);
  const int64_t rl = s->q + 1;
  HIP_TRY(potts::launch_fill_u64(s->records + (s->t % s->rec_cap) * rl, (uint64_t)rl, 0ull, s->stream));
  if (use_packed(s)) return run_packed(s, thr, nsweeps);
  if (use_strip(s)) {
    potts::StripLaunch l{};
    potts::StripParams &p = l.single;
    fill_strip_params(p, s->spins, (uint32_t)s->L, (uint32_t)s->q, s->seed, thr, strip_rows(s));
    p.t0 = (uint64_t)s->t;
    p.nsweeps = (uint64_t)nsweeps;
    p.ring = s->records;
    p.cap = (uint64_t)s->rec_cap;
    p.stripes = s->stripes;
    p.nstripes = kStripes;
    const unsigned groups = s->max_groups ? s->max_groups : 8192u;
    const uint64_t need = ((uint64_t)p.nitems + 255) / 256;
    const unsigned grid = (unsigned)(need < groups ? need : groups);
    const bool wide = wide_table(thr);
    // segments of at most 2^30 sweeps keep the launch's sweep index in 32 bits
    const int64_t seg = 1ll << 30;
    for (int64_t base = 0; base < nsweeps; base += seg) {
      const int64_t count = std::min<int64_t>(seg, nsweeps - base);
      p.t0 = (uint64_t)(s->t + base);
      for (int64_t j = 0; j < count; ++j) {
        l.sweep = (uint32_t)j;
        HIP_TRY(potts::launch_strip(l, 0, grid, p.q, wide, s->stream));
        HIP_TRY(potts::launch_strip(l, 1, grid, p.q, wide, s->stream));
      }
      // the segment's last sweep: no later colour-0 launch folds its records
      HIP_TRY(potts::launch_fold_stripes(p, p.t0 + (uint64_t)count - 1, s->stream));
    }
  } else {
    potts::SweepParams p{};
    p.spins = s->spins;
    p.L = (uint32_t)s->L;
    p.q = (uint32_t)s->q;
    p.nchunks = n_sites(s) / 4;
    p.k0 = (uint32_t)s->seed;
    p.k1 = (uint32_t)(s->seed >> 32);
    for (int i = 0; i < 4; ++i) p.thr.v[i] = thr[i];
    for (int64_t j = 0; j < nsweeps; ++j) {
      const int64_t t = s->t + j;
      p.t_lo = (uint32_t)(uint64_t)t;
      p.t_hi = (uint32_t)((uint64_t)t >> 32);
      p.rec = s->records + (t % s->rec_cap) * rl;
      p.rec_clear = nullptr;
      HIP_TRY(potts::launch_half_sweep(p, 0, s->stream));
      p.rec_clear = s->records + ((t + 1) % s->rec_cap) * rl;
      HIP_TRY(potts::launch_half_sweep(p, 1, s->stream));
    }
  }
  s->t += nsweeps;
  return POTTS_OK;
}

// Heat-bath sweeps on the colour-split copy (heatbath_packed.hip): the draw
// table is rebuilt and uploaded when the thresholds change; records through
// the striped partial records, as the Metropolis colour-split path.
int run_heatbath_packed(potts_state *s, const uint32_t thr[4], int64_t nsweeps) {
  const uint32_t L = (uint32_t)s->L;
  if (!s->hb_dev) {
    if (hipMalloc(&s->hb_dev, sizeof(potts::HbTable)) != hipSuccess ||
        hipHostMalloc(&s->hb_host, sizeof(potts::HbTable), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return fail(POTTS_ENOMEM, "allocation of the heat-bath table failed");
    }
  }
  if (!s->hb_valid || memcmp(s->hb_thr, thr, sizeof(s->hb_thr)) != 0) {
    // the previous upload from the host copy may still be queued
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->hb_wide = potts::build_heatbath_table(thr, (uint32_t)s->q, s->hb_host);
    HIP_TRY(hipMemcpyAsync(s->hb_dev, s->hb_host, sizeof(potts::HbTable), hipMemcpyHostToDevice, s->stream));
    memcpy(s->hb_thr, thr, sizeof(s->hb_thr));
    s->hb_valid = true;
  }
  if (!s->planes_valid) {
    HIP_TRY(potts::launch_pack(s->spins, s->spins2, L, s->stream));
    s->planes_valid = true;
  }
  s->spins_valid = false;
  potts::HbLaunch l{};
  potts::StripParams &p = l.p;
  const uint32_t rows = packed_rows(s);
  fill_strip_params(p, s->spins2, L, (uint32_t)s->q, s->seed, thr, rows);
  potts::set_items(p, L / 32, L, rows);
  p.ring = s->records;
  p.cap = (uint64_t)s->rec_cap;
  p.stripes = s->stripes;
  p.nstripes = kStripes;
  l.table = s->hb_dev;
  const unsigned groups = s->max_groups ? s->max_groups : 8192u;
  const uint64_t need = ((uint64_t)p.nitems + 255) / 256;
  const unsigned grid = (unsigned)(need < groups ? need : groups);
  const int64_t seg = 1ll << 30;
  for (int64_t base = 0; base < nsweeps; base += seg) {
    const int64_t count = std::min<int64_t>(seg, nsweeps - base);
    p.t0 = (uint64_t)(s->t + base);
    p.nsweeps = (uint64_t)count;
    for (int64_t j = 0; j < count; ++j) {
      l.sweep = (uint32_t)j;
      HIP_TRY(potts::launch_heatbath_packed(l, 0, grid, s->hb_wide, s->stream));
      HIP_TRY(potts::launch_heatbath_packed(l, 1, grid, s->hb_wide, s->stream));
    }
    HIP_TRY(potts::launch_fold_stripes(p, p.t0 + (uint64_t)count - 1, s->stream));
  }
  s->t += nsweeps;
  if (!s->owns_spins) {
    HIP_TRY(potts::launch_unpack(s->spins2, s->spins, L, s->stream));
    s->spins_valid = true;
    s->planes_valid = false;
  }
  return POTTS_OK;
}

// Heat-bath sweeps: on the colour-split copy where the lattice has one (L % 32
// == 0, kernel 0 or 4), else one thread per 4-byte chunk (kernels.hip); the
// sweep counter and records are shared with the Metropolis sweeps.
int run_heatbath(potts_state *s, const uint32_t thr[4], int64_t nsweeps) {
  if (!s) return fail(POTTS_EINVAL, "state is NULL");
  if (nsweeps < 0) return fail(POTTS_EINVAL, "nsweeps must be >= 0");
  if (nsweeps > INT64_MAX - s->t) return fail(POTTS_ERANGE, "sweep counter overflow");
  if (nsweeps == 0) return POTTS_OK;
  if (packed_ok(s) && (s->kernel == 0 || s->kernel == 4 || s->kernel == 7)) {
    const int64_t rl = s->q + 1;
    HIP_TRY(potts::launch_fill_u64(s->records + (s->t % s->rec_cap) * rl, (uint64_t)rl, 0ull, s->stream));
    return run_heatbath_packed(s, thr, nsweeps);
  }
  {
    const int rc = sync_spins(s);
    if (rc) return rc;
    s->planes_valid = false;
  }
  const int64_t rl = s->q + 1;
  HIP_TRY(potts::launch_fill_u64(s->records + (s->t % s->rec_cap) * rl, (uint64_t)rl, 0ull, s->stream));
  potts::SweepParams p{};
  p.spins = s->spins;
  p.L = (uint32_t)s->L;
  p.q = (uint32_t)s->q;
  p.nchunks = n_sites(s) / 4;
  p.k0 = (uint32_t)s->seed;
  p.k1 = (uint32_t)(s->seed >> 32);
  for (int i = 0; i < 4; ++i) p.thr.v[i] = thr[i];
  for (int64_t j = 0; j < nsweeps; ++j) {
    const int64_t t = s->t + j;
    p.t_lo = (uint32_t)(uint64_t)t;
    p.t_hi = (uint32_t)((uint64_t)t >> 32);
    p.rec = s->records + (t % s->rec_cap) * rl;
    p.rec_clear = nullptr;
    HIP_TRY(potts::launch_heatbath(p, 0, s->stream));
    p.rec_clear = s->records + ((t + 1) % s->rec_cap) * rl;
    HIP_TRY(potts::launch_heatbath(p, 1, s->stream));
  }
  s->t += nsweeps;
  return POTTS_OK;
}

// Validates [t0, t0+n) against the ring; returns the first slot.
int ring_window(const potts_state *s, int64_t t0, int64_t n, int64_t *slot0) {
  if (n < 0 || t0 < 0) return fail(POTTS_EINVAL, "negative record index or count");
  // the last sweep cleared the slot of the next one, so cap - 1 records survive
  const int64_t oldest = s->t - s->rec_cap + 1;
  const int64_t first = oldest > s->rec_from ? oldest : s->rec_from;
  if (t0 < first || t0 + n > s->t)
    return fail(POTTS_ERANGE, "requested records are not in the ring (kept: sweeps " +
                                  std::to_string(first) + " .. " + std::to_string(s->t - 1) + ")");
  *slot0 = t0 % s->rec_cap;
  return POTTS_OK;
}

int copy_records(potts_state *s, int64_t t0, int64_t n, int64_t *out) {
  int64_t slot0 = 0;
  int rc = ring_window(s, t0, n, &slot0);
  if (rc) return rc;
  const int64_t rl = s->q + 1;
  int64_t done = 0;
  while (done < n) {
    const int64_t slot = (slot0 + done) % s->rec_cap;
    const int64_t run = std::min<int64_t>(n - done, s->rec_cap - slot);
    HIP_TRY(hipMemcpyAsync(out + done * rl, s->records + slot * rl, (size_t)(run * rl) * 8,
                           hipMemcpyDeviceToHost, s->stream));
    done += run;
  }
  HIP_TRY(hipStreamSynchronize(s->stream));
  return band_check(s);
}

void fill_obs(const potts_state *s, const int64_t *rec, potts_obs *out) {
  memset(out, 0, sizeof(*out));
  out->t = s->t;
  out->q = s->q;
  out->L = s->L;
  out->e_sat = rec[0];
  for (int v = 0; v < s->q; ++v) {
    out->hist[v] = rec[1 + v];
    if (rec[1 + v] > out->nmax) out->nmax = rec[1 + v];
  }
}

const uint32_t kMagic[2] = {0x54544f50u, 0x314b4353u};  // "POTTSCK1"

}  // namespace

extern "C" {

int potts_init(int32_t L, int32_t q, uint64_t seed, potts_start start, potts_state **out) {
  return create(L, q, seed, start, nullptr, nullptr, 0, nullptr, false, 0, out);
}

int potts_init_ex(int32_t L, int32_t q, uint64_t seed, potts_start start, void *dev_spins,
                  void *dev_spins2, size_t bytes, void *hip_stream, int64_t records_capacity,
                  potts_state **out) {
  return create(L, q, seed, start, dev_spins, dev_spins2, bytes, hip_stream, true, records_capacity,
                out);
}

int potts_threshold_table(double beta, uint32_t thr[4]) {
  if (!thr) return fail(POTTS_EINVAL, "thr is NULL");
  return build_table(beta, thr);
}

int potts_sweep(potts_state *s, double beta, int64_t nsweeps) {
  if (!s) return fail(POTTS_EINVAL, "state is NULL");
  if (!s->have_thr || s->thr_beta != beta) {
    uint32_t thr[4];
    int rc = build_table(beta, thr);
    if (rc) return rc;
    memcpy(s->thr, thr, sizeof(thr));
    s->thr_beta = beta;
    s->have_thr = true;
  }
  return run_sweeps(s, s->thr, nsweeps);
}

int potts_sweep_heatbath(potts_state *s, double beta, int64_t nsweeps) {
  if (!s) return fail(POTTS_EINVAL, "state is NULL");
  uint32_t thr[4];
  int rc = build_table(beta, thr);
  if (rc) return rc;
  return run_heatbath(s, thr, nsweeps);
}

int potts_sweep_heatbath_thr(potts_state *s, const uint32_t thr[4], int64_t nsweeps) {
  if (!thr) return fail(POTTS_EINVAL, "thr is NULL");
  return run_heatbath(s, thr, nsweeps);
}

int potts_sweep_thr(potts_state *s, const uint32_t thr[4], int64_t nsweeps) {
  if (!thr) return fail(POTTS_EINVAL, "thr is NULL");
  return run_sweeps(s, thr, nsweeps);
}

int potts_slab_half_sweep(uint8_t *dev_slab, int32_t L, int32_t h, int64_t y0, int32_t q, uint64_t seed,
                          int64_t t, int32_t colour, const uint32_t thr[4], int64_t *dev_ring,
                          int64_t ring_slots, void *hip_stream) {
  if (!dev_slab || !thr) return fail(POTTS_EINVAL, "dev_slab or thr is NULL");
  if (L < 16 || L % 16 || L > 65536 || q < 2 || q > POTTS_QMAX)
    return fail(POTTS_EINVAL, "need L % 16 == 0, 16 <= L <= 65536, 2 <= q <= 256");
  if (h < 2 || h % 2 || y0 < 0 || y0 % 2 || y0 + h > L)
    return fail(POTTS_EINVAL, "need h even >= 2, y0 even >= 0 and y0 + h <= L");
  if ((uint64_t)(h + 2) * (uint64_t)L >= (1ull << 32)) return fail(POTTS_EINVAL, "the slab must stay below 4 GiB");
  if (colour != 0 && colour != 1) return fail(POTTS_EINVAL, "colour must be 0 or 1");
  if (t < 0) return fail(POTTS_EINVAL, "t must be >= 0");
  if (!dev_ring || ring_slots < 2 || (ring_slots & (ring_slots - 1)))
    return fail(POTTS_EINVAL, "need dev_ring with a power-of-two ring_slots >= 2");
  potts::StripLaunch l{};
  potts::StripParams &p = l.single;
  const uint32_t rows = potts::auto_strip_rows((uint32_t)L, (uint32_t)h, 2048ull * 256ull);
  potts::fill_slab_params(p, dev_slab, (uint32_t)L, (uint32_t)h, (uint32_t)y0, (uint32_t)q, seed, thr, rows);
  p.t0 = (uint64_t)t;
  p.nsweeps = 1;
  p.ring = reinterpret_cast<unsigned long long *>(dev_ring);
  p.cap = (uint64_t)ring_slots;
  l.sweep = 0;
  const uint64_t need = ((uint64_t)p.nitems + 255) / 256;
  const unsigned grid = (unsigned)(need < 8192 ? need : 8192);
  HIP_TRY(potts::launch_strip(l, colour, grid, p.q, wide_table(thr), static_cast<hipStream_t>(hip_stream)));
  return POTTS_OK;
}

int potts_tune_tiles(potts_state *s, int32_t tx, int32_t ty, int32_t sweeps) {
  if (!s) return fail(POTTS_EINVAL, "state is NULL");
  if (tx < 0 || ty < 0 || sweeps < 0 || sweeps > (int32_t)potts::kTileMaxSweeps)
    return fail(POTTS_EINVAL, "tx, ty >= 0 and sweeps in 0 .. 8");
  const uint32_t old_tx = s->tile_tx, old_ty = s->tile_ty, old_n = s->tile_sweeps;
  s->tile_tx = (uint32_t)tx;
  s->tile_ty = (uint32_t)ty;
  s->tile_sweeps = (uint32_t)sweeps;
  uint32_t a, b, c;
  if ((tx || ty || sweeps) && !tile_shape(s, &a, &b, &c)) {
    s->tile_tx = old_tx;
    s->tile_ty = old_ty;
    s->tile_sweeps = old_n;
    return fail(POTTS_EINVAL, "tile shape: tx % 16 == 0 and ty even dividing L, LDS of one tile within 44 KiB");
  }
  return POTTS_OK;
}

int potts_tune_band(potts_state *s, int32_t rows, int32_t block) {
  if (!s) return fail(POTTS_EINVAL, "state is NULL");
  if (rows < 0 || block < 0 || (!rows && block)) return fail(POTTS_EINVAL, "rows and block >= 0, block only with rows");
  const uint32_t old_rows = s->band_rows, old_block = s->band_block;
  s->band_rows = (uint32_t)rows;
  s->band_block = (uint32_t)block;
  uint32_t r, b;
  if (rows && !band_shape(s, &r, &b)) {
    (void)hipGetLastError();
    s->band_rows = old_rows;
    s->band_block = old_block;
    return fail(POTTS_EINVAL, "band shape: rows even dividing L, block 256 / 512 / 1024 >= L / 16, "
                              "LDS of one band within 136 KiB, grid resident at once");
  }
  return POTTS_OK;
}

int potts_tune_graph(potts_state *s, int32_t sweeps) {
  if (!s) return fail(POTTS_EINVAL, "state is NULL");
  if (sweeps < 0 || sweeps > 4096) return fail(POTTS_EINVAL, "sweeps per graph must be 0 .. 4096");
  s->graph_sweeps = sweeps;
  return POTTS_OK;
}

int potts_tune_occupancy(potts_state *s, int32_t waves_per_simd) {
  if (!s) return fail(POTTS_EINVAL, "state is NULL");
  if (waves_per_simd != 0 && waves_per_simd != 8) return fail(POTTS_EINVAL, "waves_per_simd must be 0 or 8");
  s->wpe = (uint32_t)waves_per_simd;
  return POTTS_OK;
}

int potts_slab_records(const int64_t *dev_rings, int32_t nslabs, int64_t ring_slots, int32_t q, int64_t t0,
                       int64_t n, int64_t *dev_out, void *hip_stream) {
  if (!dev_rings || (!dev_out && n > 0)) return fail(POTTS_EINVAL, "dev_rings or dev_out is NULL");
  if (nslabs < 1 || q < 2 || q > POTTS_QMAX) return fail(POTTS_EINVAL, "need nslabs >= 1 and 2 <= q <= 256");
  if (ring_slots < 2 || (ring_slots & (ring_slots - 1)))
    return fail(POTTS_EINVAL, "ring_slots must be a power of two >= 2");
  if (t0 < 0 || n < 0 || n > ring_slots) return fail(POTTS_EINVAL, "need t0 >= 0 and 0 <= n <= ring_slots");
  HIP_TRY(potts::launch_slab_fold(reinterpret_cast<const unsigned long long *>(dev_rings), (uint32_t)nslabs,
                                  (uint64_t)ring_slots, (uint32_t)q + 1, (uint64_t)t0, (uint64_t)n,
                                  reinterpret_cast<unsigned long long *>(dev_out),
                                  static_cast<hipStream_t>(hip_stream)));
  return POTTS_OK;
}

int potts_tune(potts_state *s, int32_t kernel, int32_t strip_rows, int32_t max_groups) {
  if (!s) return fail(POTTS_EINVAL, "state is NULL");
  if (kernel < 0 || kernel > 7) return fail(POTTS_EINVAL, "kernel must be 0 .. 7");
  if (kernel == 7 && !band_ok(s))
    return fail(POTTS_EINVAL, "band kernel needs L % 32 == 0, L <= 16384 and a band shape whose grid fits the GPU");
  if (kernel == 6 && !drawn_ok(s))
    return fail(POTTS_EINVAL, "pre-drawn resident kernel needs L % 16 == 0 and L*L <= 4096");
  if (kernel == 5 && !tiles_ok(s)) return fail(POTTS_EINVAL, "tile kernel needs L % 16 == 0 and a tile shape");
  if (kernel == 4 && !packed_ok(s))
    return fail(POTTS_EINVAL, "colour-split kernel needs L % 32 == 0 and L <= 65520");
  if (kernel == 1 && !strip_ok(s)) return fail(POTTS_EINVAL, "strip kernel needs L % 16 == 0 and L <= 65520");
  if (kernel == 3 && !resident_ok(s))
    return fail(POTTS_EINVAL, "LDS-resident kernel needs L % 16 == 0, L*L <= 65536 and LDS for q");
  if (strip_rows < 0 || strip_rows % 2 || (strip_rows && s->L % strip_rows))
    return fail(POTTS_EINVAL, "strip_rows must be 0 or an even divisor of L");
  if (max_groups < 0) return fail(POTTS_EINVAL, "max_groups must be >= 0");
  s->kernel = kernel;
  s->rows = (uint32_t)strip_rows;
  s->max_groups = (unsigned)max_groups;
  return POTTS_OK;
}

int potts_measure(potts_state *s, potts_obs *out) {
  if (!s || !out) return fail(POTTS_EINVAL, "NULL argument");
  const int rc = sync_spins(s);
  if (rc) return rc;
  const int64_t rl = s->q + 1;
  HIP_TRY(potts::launch_fill_u64(s->scratch, (uint64_t)rl, 0ull, s->stream));
  potts::MeasureParams p{};
  p.spins = s->spins;
  p.L = (uint32_t)s->L;
  p.q = (uint32_t)s->q;
  p.nchunks = n_sites(s) / 4;
  p.out = s->scratch;
  HIP_TRY(potts::launch_measure(p, s->stream));
  std::vector<int64_t> rec((size_t)rl);
  HIP_TRY(hipMemcpyAsync(rec.data(), s->scratch, (size_t)rl * 8, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  const int brc = band_check(s);
  if (brc) return brc;
  fill_obs(s, rec.data(), out);
  return POTTS_OK;
}

int potts_observables(potts_state *s, potts_obs *out) {
  if (!s || !out) return fail(POTTS_EINVAL, "NULL argument");
  if (s->t == 0 || s->rec_from >= s->t) return potts_measure(s, out);
  std::vector<int64_t> rec((size_t)(s->q + 1));
  int rc = copy_records(s, s->t - 1, 1, rec.data());
  if (rc) return rc;
  fill_obs(s, rec.data(), out);
  return POTTS_OK;
}

int potts_records(potts_state *s, int64_t t0, int64_t n, int64_t *out) {
  if (!s || (!out && n > 0)) return fail(POTTS_EINVAL, "NULL argument");
  return copy_records(s, t0, n, out);
}

int potts_stats(potts_state *s, int64_t t0, int64_t n, double beta, potts_summary *out) {
  if (!s || !out) return fail(POTTS_EINVAL, "NULL argument");
  if (n < 1 || n > (1ll << 24)) return fail(POTTS_EINVAL, "window must hold 1 .. 2^24 records");
  if (!(beta >= 0.0) || !isfinite(beta)) return fail(POTTS_EINVAL, "beta must be finite and >= 0");
  int64_t slot0 = 0;
  int rc = ring_window(s, t0, n, &slot0);
  if (rc) return rc;
  potts::StatsParams p{};
  p.ring = s->records;
  p.cap = s->rec_cap;
  p.slot0 = slot0;
  p.n = n;
  p.q = (uint32_t)s->q;
  p.N = n_sites(s);
  p.beta = beta;
  p.out = s->stats_out;
  HIP_TRY(potts::launch_stats(p, s->stream));
  double v[5];
  HIP_TRY(hipMemcpyAsync(v, s->stats_out, sizeof(v), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  rc = band_check(s);
  if (rc) return rc;
  out->n = n;
  out->e = v[0];
  out->C = v[1];
  out->V_L = v[2];
  out->m = v[3];
  out->chi = v[4];
  return POTTS_OK;
}

int potts_reweight(potts_state *s, int64_t t0, int64_t n, double beta0, const double *betas, int32_t npoints,
                   potts_summary *out) {
  if (!s || !betas || !out) return fail(POTTS_EINVAL, "NULL argument");
  if (n < 1 || n > (1ll << 24)) return fail(POTTS_EINVAL, "window must hold 1 .. 2^24 records");
  if (npoints < 1 || npoints > 65535) return fail(POTTS_EINVAL, "npoints must be 1 .. 65535");
  if (!(beta0 >= 0.0) || !isfinite(beta0)) return fail(POTTS_EINVAL, "beta0 must be finite and >= 0");
  for (int32_t i = 0; i < npoints; ++i)
    if (!(betas[i] >= 0.0) || !isfinite(betas[i])) return fail(POTTS_EINVAL, "betas must be finite and >= 0");
  int64_t slot0 = 0;
  int rc = ring_window(s, t0, n, &slot0);
  if (rc) return rc;
  double *dev = nullptr;  // npoints targets, then 5 results per target
  const size_t bytes = (size_t)npoints * 6 * sizeof(double);
  HIP_TRY(hipMalloc(&dev, bytes));
  std::vector<double> host((size_t)npoints * 5);
  potts::ReweightParams p{};
  p.ring = s->records;
  p.cap = s->rec_cap;
  p.slot0 = slot0;
  p.n = n;
  p.q = (uint32_t)s->q;
  p.N = n_sites(s);
  p.beta0 = beta0;
  p.betas = dev;
  p.out = dev + npoints;
  hipError_t e = hipMemcpyAsync(dev, betas, (size_t)npoints * sizeof(double), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = potts::launch_reweight(p, (unsigned)npoints, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(host.data(), p.out, host.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  (void)hipFree(dev);
  if (e != hipSuccess) return hip_fail(e, "potts_reweight");
  for (int32_t i = 0; i < npoints; ++i) {
    out[i].n = n;
    out[i].e = host[5 * i + 0];
    out[i].C = host[5 * i + 1];
    out[i].V_L = host[5 * i + 2];
    out[i].m = host[5 * i + 3];
    out[i].chi = host[5 * i + 4];
  }
  return POTTS_OK;
}

int potts_reserve_records(potts_state *s, int64_t capacity) {
  if (!s) return fail(POTTS_EINVAL, "state is NULL");
  if (capacity < 2 || capacity > (1ll << 40)) return fail(POTTS_EINVAL, "capacity must be in 2 .. 2^40");
  capacity = ring_slots(capacity);
  HIP_TRY(hipStreamSynchronize(s->stream));
  unsigned long long *ring = nullptr;
  const size_t bytes = (size_t)capacity * (size_t)(s->q + 1) * sizeof(unsigned long long);
  if (hipMalloc(&ring, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(POTTS_ENOMEM, "hipMalloc of the record ring failed");
  }
  HIP_TRY(hipFree(s->records));
  s->records = ring;
  s->rec_cap = capacity;
  s->rec_from = s->t;
  return POTTS_OK;
}

int potts_ramp(potts_state *s, const double *betas, int32_t npoints, int64_t t_equil, int64_t t_meas,
               potts_summary *out) {
  if (!s || !betas || !out) return fail(POTTS_EINVAL, "NULL argument");
  if (npoints < 1 || t_equil < 0 || t_meas < 1 || t_meas > (1ll << 24))
    return fail(POTTS_EINVAL, "need npoints >= 1, t_equil >= 0, 1 <= t_meas <= 2^24");
  if ((t_equil + t_meas) * (int64_t)npoints > INT64_MAX - s->t) return fail(POTTS_ERANGE, "sweep counter overflow");
  std::vector<uint32_t> tables((size_t)npoints * 4);
  for (int32_t k = 0; k < npoints; ++k) {
    int rc = build_table(betas[k], &tables[(size_t)k * 4]);
    if (rc) return rc;
  }
  if (s->rec_cap < t_meas + 1) {
    int rc = potts_reserve_records(s, t_meas + 1);
    if (rc) return rc;
  }
  double *dev_out = nullptr;
  if (hipMalloc(&dev_out, (size_t)npoints * 8 * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(POTTS_ENOMEM, "hipMalloc of the ramp results failed");
  }
  int rc = POTTS_OK;
  for (int32_t k = 0; k < npoints && rc == POTTS_OK; ++k) {
    rc = run_sweeps(s, &tables[(size_t)k * 4], t_equil + t_meas);
    if (rc) break;
    potts::StatsParams p{};
    p.ring = s->records;
    p.cap = s->rec_cap;
    p.slot0 = (s->t - t_meas) % s->rec_cap;
    p.n = t_meas;
    p.q = (uint32_t)s->q;
    p.N = n_sites(s);
    p.beta = betas[k];
    p.out = dev_out + (size_t)k * 8;
    hipError_t e = potts::launch_stats(p, s->stream);
    if (e != hipSuccess) rc = hip_fail(e, "launch_stats");
  }
  std::vector<double> host((size_t)npoints * 8);
  if (rc == POTTS_OK) {
    hipError_t e = hipMemcpyAsync(host.data(), dev_out, host.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) rc = hip_fail(e, "ramp results copy");
  } else {
    (void)hipStreamSynchronize(s->stream);
  }
  (void)hipFree(dev_out);
  if (rc) return rc;
  for (int32_t k = 0; k < npoints; ++k) {
    const double *v = &host[(size_t)k * 8];
    out[k].n = t_meas;
    out[k].e = v[0];
    out[k].C = v[1];
    out[k].V_L = v[2];
    out[k].m = v[3];
    out[k].chi = v[4];
  }
  return POTTS_OK;
}

int potts_get_spins(potts_state *s, uint8_t *host_out) {
  if (!s || !host_out) return fail(POTTS_EINVAL, "NULL argument");
  const int rc = sync_spins(s);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(host_out, s->spins, (size_t)n_sites(s), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return band_check(s);
}

int potts_set_spins(potts_state *s, const uint8_t *host_in, int64_t t) {
  if (!s || !host_in) return fail(POTTS_EINVAL, "NULL argument");
  if (t < 0) return fail(POTTS_EINVAL, "t must be >= 0");
  const uint64_t n = n_sites(s);
  for (uint64_t i = 0; i < n; ++i)
    if (host_in[i] >= s->q) return fail(POTTS_EINVAL, "spin value >= q");
  HIP_TRY(hipMemcpyAsync(s->spins, host_in, (size_t)n, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->spins_valid = true;
  s->planes_valid = false;
  s->t = t;
  s->rec_from = t;
  return POTTS_OK;
}

void *potts_device_spins(potts_state *s) {
  if (!s || sync_spins(s)) return nullptr;
  // the caller may write through the pointer: the next sweep packs again
  s->planes_valid = false;
  return (void *)s->spins;
}

int64_t potts_time(const potts_state *s) { return s ? s->t : -1; }

void *potts_stream(const potts_state *s) { return s ? (void *)s->stream : nullptr; }

int potts_save(potts_state *s, const char *path) {
  if (!s || !path) return fail(POTTS_EINVAL, "NULL argument");
  std::vector<uint8_t> host((size_t)n_sites(s));
  int rc = potts_get_spins(s, host.data());
  if (rc) return rc;
  FILE *f = fopen(path, "wb");
  if (!f) return fail(POTTS_EIO, std::string("cannot open ") + path);
  const int32_t shape[2] = {s->L, s->q};
  const int64_t tt = s->t;
  bool ok = fwrite(kMagic, sizeof(kMagic), 1, f) == 1 && fwrite(shape, sizeof(shape), 1, f) == 1 &&
            fwrite(&s->seed, sizeof(s->seed), 1, f) == 1 && fwrite(&tt, sizeof(tt), 1, f) == 1 &&
            fwrite(host.data(), 1, host.size(), f) == host.size();
  ok = (fclose(f) == 0) && ok;
  return ok ? POTTS_OK : fail(POTTS_EIO, std::string("write failed: ") + path);
}

int potts_load(const char *path, potts_state **out) {
  if (!path || !out) return fail(POTTS_EINVAL, "NULL argument");
  *out = nullptr;
  FILE *f = fopen(path, "rb");
  if (!f) return fail(POTTS_EIO, std::string("cannot open ") + path);
  uint32_t magic[2];
  int32_t shape[2];
  uint64_t seed;
  int64_t t;
  bool ok = fread(magic, sizeof(magic), 1, f) == 1 && fread(shape, sizeof(shape), 1, f) == 1 &&
            fread(&seed, sizeof(seed), 1, f) == 1 && fread(&t, sizeof(t), 1, f) == 1;
  if (!ok || magic[0] != kMagic[0] || magic[1] != kMagic[1] || !valid_shape(shape[0], shape[1]) || t < 0) {
    fclose(f);
    return fail(POTTS_EIO, std::string("not a checkpoint: ") + path);
  }
  std::vector<uint8_t> host((size_t)shape[0] * (size_t)shape[0]);
  ok = fread(host.data(), 1, host.size(), f) == host.size();
  fclose(f);
  if (!ok) return fail(POTTS_EIO, std::string("truncated checkpoint: ") + path);
  potts_state *s = nullptr;
  int rc = potts_init(shape[0], shape[1], seed, POTTS_ORDERED, &s);
  if (rc) return rc;
  rc = potts_set_spins(s, host.data(), t);
  if (rc) {
    release(s);
    return rc;
  }
  *out = s;
  return POTTS_OK;
}

void potts_free(potts_state *s) { release(s); }

const char *potts_strerror(int code) {
  switch (code) {
    case POTTS_OK: return "ok";
    case POTTS_EINVAL: return "invalid argument";
    case POTTS_ENOMEM: return "out of memory";
    case POTTS_EDEVICE: return "HIP device error";
    case POTTS_ERANGE: return "out of range";
    case POTTS_EIO: return "checkpoint I/O error";
    default: return "unknown error";
  }
}

const char *potts_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
