// kernels.hpp -- parameter blocks and launchers of the Potts sweep kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace potts {

struct Thresholds {
  uint32_t v[4];  // v[d-1] for dE = d = 1..4
};

struct SweepParams {
  uint8_t *spins;
  uint32_t L, q;
  uint64_t nchunks;               // L*L/4
  uint32_t t_lo, t_hi;            // sweep index
  uint32_t k0, k1;                // Philox key = seed
  Thresholds thr;
  unsigned long long *rec;        // record of this sweep: [0] e_sat, [1+v] N_v
  unsigned long long *rec_clear;  // record slot to zero for the next sweep, or null
  double inv_thr[4];              // heat bath: 1/thr[d] rounded (0 where thr[d] == 0), set by its launcher
};

// Main path (L % 16 == 0, L <= 65520): a work item is a 16-byte-wide strip of
// `rows` consecutive rows (rows even, nrows % rows == 0).  One StripParams per
// lattice ("job"); it does not change between sweeps, so one table serves
// every launch of a captured graph.  The updated rows are storage rows
// first_row .. first_row + nrows - 1 of `spins`: the whole lattice (0, L,
// periodic: up_row = L-1, down_row = 0), or a row slab with its two halo
// rows stored inline (1, h, up_row = 0, down_row = h+1).  Updated row 0 is
// global row y0 (even), whose first chunk has Philox word ctr0 = y0 * L/4.
struct StripParams {
  uint8_t *spins;
  uint32_t L, q;
  uint32_t ipr;         // items per row band = L/16
  uint32_t rows;        // rows per item
  uint32_t nitems;      // (nrows/rows) * (L/16)
  uint32_t nrows, first_row, up_row, down_row;
  uint32_t ctr0;
  int32_t item_shift;   // log2(ipr) when ipr is a power of two, else -1
  uint64_t item_magic;  // ceil(2^64 / ipr) otherwise
  uint32_t row_words;   // L/4: Philox counter stride between rows
  uint32_t k0, k1;      // Philox key = seed
  Thresholds thr;
  uint64_t t0;          // sweep index of launch sweep 0
  uint64_t nsweeps;     // launches with sweep >= nsweeps leave this job alone
  unsigned long long *ring;  // records of sweep t in slot t % cap
  uint64_t cap;              // a power of two
  // Optional (single lattices): instead of adding its totals to the ring slot,
  // a workgroup adds them to one of nstripes partial records (stripe =
  // workgroup % nstripes, set t & 1, stripe_words() apart), which spreads the
  // atomics of many short launches over many cache lines.  The lead
  // workgroup of colour 0 of the next launched sweep folds set t & 1 into slot
  // t and clears it; launch_fold_stripes does so after a run's last sweep.
  unsigned long long *stripes;
  uint32_t nstripes;  // a power of two
};

// distance between two partial records (1+q words rounded up to 128 bytes)
__host__ __device__ inline uint32_t stripe_words(uint32_t q) { return (q + 1 + 15) & ~15u; }

// Workgroup -> (job, item range) for launches that sweep many lattices.
struct StripTile {
  uint32_t job;
  uint32_t first;  // first item of the range
  uint32_t count;  // items in the range (at most one per lane of the workgroup)
  uint32_t lead;   // 1 for one tile per job: it clears the next record slot
};

// Launch shape of a tiled launch (batches, the serving loop): lanes, and so
// items, per workgroup tile (256 or 128), and the occupancy asked of the
// compiler (wpe 0: its own choice; 8: at least 8 waves per SIMD, at most 64
// VGPRs).  Shapes other than (256, 0) exist for q <= 16.
struct TileShape {
  uint32_t block = 256;
  uint32_t wpe = 0;
};

inline bool shape_ok(const TileShape &s, uint32_t max_q) {
  if (s.block == 256 && s.wpe == 0) return true;
  return max_q <= 16 && (s.block == 128 || s.block == 256) && (s.wpe == 0 || s.wpe == 8);
}

struct StripLaunch {
  const StripParams *jobs;  // null: run `single` over a grid-stride loop
  const StripTile *tiles;
  StripParams single;
  uint32_t sweep;           // this launch updates sweep t = t0 + sweep of every job
};

// Heat-bath draw table of the colour-split kernel, per pattern of equal
// neighbours (64 patterns of the six flags ab, ac, ad, bc, bd, cd "differ",
// a..d = up, down, left, right; pattern bit 5 = ab .. bit 0 = cd), built on
// the host from the thresholds and q: the cuts on the site's word that pick
// the ranked neighbour values, Z and S of the draw, w0 and its reciprocal.
struct HbTable {
  static constexpr uint32_t kCut = 0;       // 64 x 4 uint32: ceil(c_i 2^32 / Z) - 1 (all thresholds >= 1)
  static constexpr uint32_t kZs = 1024;     // 64 x {Z lo, Z hi, S lo, S hi}
  static constexpr uint32_t kWi = 2048;     // 64 x {w0, (1 + 2^-19)/w0 as FP32 bits, 0, 0}
  static constexpr uint32_t kCut64 = 3072;  // 64 x 4 uint64: ceil(c_i 2^32 / Z) (some threshold 0)
  static constexpr uint32_t kBytes = 5120;
  uint8_t bytes[kBytes];
};

struct HbLaunch {
  StripParams p;         // the colour-split copy, as for the Metropolis kernel
  const HbTable *table;  // device
  uint32_t sweep;        // sweep t = p.t0 + sweep
};

// fills the table for thresholds thr and q; returns true when some threshold
// is 0 (the wide form is then the one to use)
bool build_heatbath_table(const uint32_t thr[4], uint32_t q, HbTable *t);
hipError_t launch_heatbath_packed(const HbLaunch &l, int colour, unsigned grid, bool wide, hipStream_t stream);

// populations are counted in lane-private LDS columns up to this many states
constexpr uint32_t kPrivateHistMaxQ = 64;

// Several sweeps per launch on LDS tiles with recomputed halos (tiles.hip):
// one workgroup per tile of ty rows x tx bytes of a row-major L x L lattice,
// read from src with halo rows above and below and 16 bytes left and right,
// swept nsweeps <= halo / 2 times in LDS, interior written to dst (another
// buffer).  The record of sweep t0 + s is added into partial-record set s
// (nstripes stripes of stripe_words(q) words, set s at stripes + s x nstripes
// x stripe_words(q)), which launch_fold_sets sums into ring slot t0 + s.
constexpr uint32_t kTileMaxSweeps = 8;
constexpr uint32_t kTileMaxHalo = 16;          // = the 16-byte column halo: 2 x 8 sweeps
constexpr size_t kTileMaxLds = 44u * 1024u;    // dynamic LDS of one tile (static LDS up to 19 KB)

struct TileParams {
  const uint8_t *src;
  uint8_t *dst;
  uint32_t L, q;
  uint32_t k0, k1;      // Philox key = seed
  Thresholds thr;
  uint64_t t0;          // sweep index of the launch's first sweep
  uint32_t nsweeps;     // sweeps of this launch
  uint32_t tx, ty;      // tile interior: tx bytes (multiple of 16) x ty rows (even)
  uint32_t halo;        // rows above and below (even, >= 2 nsweeps)
  uint32_t tiles_x;     // L / tx
  unsigned long long *stripes;
  uint32_t nstripes;    // a power of two
};

size_t tile_lds_bytes(uint32_t tx, uint32_t ty, uint32_t halo);
bool tile_shape_ok(uint32_t L, uint32_t tx, uint32_t ty, uint32_t halo);
hipError_t launch_tiles(const TileParams &p, hipStream_t stream);
hipError_t launch_fold_sets(const TileParams &p, unsigned long long *ring, uint64_t cap, hipStream_t stream);

// One lattice run entirely in LDS by one workgroup (resident.hip).
struct ResidentJob {
  uint8_t *spins;                 // L*L bytes, updated in place
  uint32_t L, q;
  uint32_t k0, k1;                // Philox key = seed
  uint64_t t0;                    // sweep index of the first sweep
  uint32_t nsweeps;
  Thresholds thr;
  unsigned long long *ring;       // records of sweep t go to slot t % cap
  uint64_t cap;                   // a power of two
};

// A launch: jobs[blockIdx.x] from device memory, or `single` when jobs is null.
struct ResidentLaunch {
  const ResidentJob *jobs;
  ResidentJob single;
};

struct InitParams {
  uint8_t *spins;
  uint32_t L, q;
  uint64_t nchunks;
  uint32_t k0, k1;
  int random;
};

struct MeasureParams {
  const uint8_t *spins;
  uint32_t L, q;
  uint64_t nchunks;
  unsigned long long *out;  // [0] e_sat, [1+v] N_v; must start zeroed
};

// Temperature reweighting of a record window sampled at beta0 to betas[b],
// one workgroup per target (stats.hip).
struct ReweightParams {
  const unsigned long long *ring;
  int64_t cap, slot0, n;           // window as in StatsParams
  uint32_t q;
  uint64_t N;
  double beta0;
  const double *betas;             // device, one per workgroup
  double *out;                     // device, 5 per workgroup: e, C, V_L, m, chi
};

struct StatsParams {
  const unsigned long long *ring;  // record ring, cap slots of (1+q) int64
  int64_t cap, slot0, n;           // window: n records from slot0 (wrapping; cap a power of two)
  uint32_t q;
  uint64_t N;
  double beta;
  double *out;                     // e, C, V_L, m, chi
};

void fill_strip_params(StripParams &p, uint8_t *spins, uint32_t L, uint32_t q, uint64_t seed,
                       const uint32_t thr[4], uint32_t rows);
// items of `rows` rows, ipr per row band, over nrows rows
void set_items(StripParams &p, uint32_t ipr, uint32_t nrows, uint32_t rows);
// the same for a slab of h rows (global rows y0 ..) stored between its halos
void fill_slab_params(StripParams &p, uint8_t *slab, uint32_t L, uint32_t h, uint32_t y0, uint32_t q,
                      uint64_t seed, const uint32_t thr[4], uint32_t rows);
// rows per item for `nrows` rows of width L: the largest even divisor of
// nrows up to 32 that still gives at least `want` items
uint32_t auto_strip_rows(uint32_t L, uint32_t nrows, uint64_t want);

hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long value,
                           hipStream_t stream);
hipError_t launch_init(const InitParams &p, hipStream_t stream);
hipError_t launch_half_sweep(const SweepParams &p, int colour, hipStream_t stream);
// heat-bath half sweep (kernels.hip), same parameters and records
hipError_t launch_heatbath(const SweepParams &p, int colour, hipStream_t stream);
// grid: number of workgroups (tiles when l.jobs is set); max_q/wide: the
// comparison mode and table form covering every job of the launch
hipError_t launch_strip(const StripLaunch &l, int colour, unsigned grid, uint32_t max_q, bool wide,
                        hipStream_t stream);
// colour-split single-lattice kernel (packed.hip): l.single describes the
// split copy (spins = its two planes, ipr = L/32); pack/unpack convert
// qmax: the largest q of the launch's jobs (selects the comparison mode and
// histogram form); l.tiles set: batched jobs through the tile table
hipError_t launch_packed(const StripLaunch &l, int colour, unsigned grid, uint32_t qmax, bool wide,
                         hipStream_t stream);
hipError_t launch_pack(const uint8_t *row_major, uint8_t *packed, uint32_t L, hipStream_t stream);
// graph replay of a single lattice: write the device descriptor *d = p; fold
// the stripes of sweep d->t0 + sweeps - 1 and advance d->t0 by sweeps
hipError_t launch_set_desc(StripParams *d, const StripParams &p, hipStream_t stream);
hipError_t launch_fold_advance(StripParams *d, uint32_t sweeps, hipStream_t stream);
// a single lattice's colour-split launch (grid-stride) asking for at least
// wpe waves per SIMD (0: the compiler's choice; 8 exists for q <= 16)
hipError_t launch_packed_single(const StripLaunch &l, int colour, unsigned grid, uint32_t qmax, bool wide,
                                uint32_t wpe, hipStream_t stream);
// tiled launches (l.tiles set, tiles of shape.block items) in a tuner shape;
// hipErrorInvalidValue for a shape that does not exist for max_q
hipError_t launch_strip_tiled(const StripLaunch &l, int colour, unsigned ntiles, const TileShape &shape,
                              uint32_t max_q, bool wide, hipStream_t stream);
hipError_t launch_packed_tiled(const StripLaunch &l, int colour, unsigned ntiles, const TileShape &shape,
                               uint32_t max_q, bool wide, hipStream_t stream);
hipError_t launch_unpack(const uint8_t *packed, uint8_t *row_major, uint32_t L, hipStream_t stream);
// folds stripe set t & 1 of p into ring slot t and clears it
hipError_t launch_fold_stripes(const StripParams &p, uint64_t t, hipStream_t stream);
size_t resident_lds_bytes(uint32_t L, uint32_t q);
bool resident_fits(uint32_t L, uint32_t q);
// n jobs (n workgroups); LDS sized for the largest L and q among them
hipError_t launch_resident(const ResidentLaunch &p, unsigned njobs, uint32_t max_L, uint32_t max_q,
                           bool wide, hipStream_t stream);
hipError_t launch_measure(const MeasureParams &p, hipStream_t stream);
hipError_t launch_stats(const StatsParams &p, hipStream_t stream);
hipError_t launch_reweight(const ReweightParams &p, unsigned npoints, hipStream_t stream);
// out[r][w] = sum over g < nslabs of slot (t0 + r) % slots, word w, of ring g
// (rings stored one after another, slots x width words each), r < n
hipError_t launch_slab_fold(const unsigned long long *rings, uint32_t nslabs, uint64_t slots, uint32_t width,
                            uint64_t t0, uint64_t n, unsigned long long *out, hipStream_t stream);
// one workgroup per window, params in device memory
hipError_t launch_stats_many(const StatsParams *dev_params, unsigned n, hipStream_t stream);

}  // namespace potts
