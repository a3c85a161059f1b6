// batch.hip -- many independent lattices (replicas, temperatures, sizes) run
// together: the C ABI potts_batch_* of include/potts.h.
//
// Jobs with L <= 256 run in the LDS-resident kernel, one workgroup each, all
// their sweeps in one launch.  Larger jobs run through a tile table
// (workgroup -> job, item range), so one launch per colour advances every one
// of them by one sweep: jobs with L % 32 == 0 in the colour-split kernel on a
// copy of their lattice split into its two colour planes (packed before a run,
// unpacked after it), the others in the row-major strip kernel.  Because the
// random numbers are keyed by (seed, site, sweep), every job gives exactly the
// bits it gives alone.
//
// Launch shape: an in-run autotuner times, on the first sweeps of the run
// (real sweeps: the shape does not change the results), first the strip
// heights of each lattice size, then the workgroup shape of each kernel group
// (lanes per workgroup, and the occupancy asked of the compiler), and keeps
// the fastest; the choices persist in a JSON cache keyed by the kernels'
// source digest, so later runs of the same sizes skip the timing.  The remaining
// sweeps are captured once into a hipGraph: the resident launches and the
// strip chain as two branches that the GPU overlaps, then replayed.  No
// memset is recorded in the graph; record slots are cleared by the kernels.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/potts.h"
#include "kernels.hpp"
#include "tune_cache.hpp"

namespace potts {
int record_error(int code, const std::string &msg);  // capi.hip
int build_threshold_table(double beta, uint32_t thr[4]);
}  // namespace potts

namespace {

using potts::record_error;

constexpr int64_t kResidentChunk = 4096;  // sweeps per resident launch

int hip_err(hipError_t e, const char *what) {
  return record_error(POTTS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                                          \
  do {                                                         \
    hipError_t hip_err_ = (call);                              \
    if (hip_err_ != hipSuccess) return hip_err(hip_err_, #call); \
  } while (0)

int64_t pow2_at_least(int64_t n) {
  int64_t p = 2;
  while (p < n) p <<= 1;
  return p;
}

// comparison-mode class of the kernels (q <= 16, <= 64, <= 128, <= 256)
int q_class(uint32_t q) { return q <= 16 ? 0 : q <= potts::kPrivateHistMaxQ ? 1 : q <= 128 ? 2 : 3; }
uint32_t class_max_q(int c) { return c == 0 ? 16 : c == 1 ? potts::kPrivateHistMaxQ : c == 2 ? 128 : 256; }

struct StripGroup {  // strip or colour-split jobs sharing a kernel instantiation
  int qc = 0;
  bool wide = false;
  bool packed = false;    // colour-split kernel on the jobs' colour planes
  std::vector<int> jobs;  // job indices
};

struct ResidentGroup {
  int qc = 0;
  bool wide = false;
  std::vector<int> jobs;
  uint32_t max_L = 0, max_q = 0;
};

}  // namespace

struct potts_batch {
  std::vector<potts_job> jobs;
  potts_batch_opts opts{};
  hipStream_t stream = nullptr, side = nullptr;
  bool owns_stream = false;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
  uint8_t *arena = nullptr;                 // all lattices (row-major)
  uint8_t *planes = nullptr;                // colour-split copies of the colour-split jobs
  unsigned long long *rec_arena = nullptr;  // all record rings
  std::vector<size_t> lat_off, rec_off;     // per job offsets
  std::vector<size_t> plane_off;            // per colour-split job (others unused)
  std::vector<char> packed;                 // per job: runs in the colour-split kernel
  std::vector<int64_t> ring;                // slots per job (power of two)
  std::vector<int64_t> done;                // sweeps done per job
  std::vector<int64_t> target;              // sweeps each job has when the current run ends
  std::vector<uint32_t> thr;                // 4 per job
  std::vector<uint32_t> rows;               // strip rows per job (0: resident)
  std::vector<StripGroup> strip_groups;
  std::vector<potts::TileShape> shape;      // per strip group
  std::vector<ResidentGroup> res_groups;
  potts::TuneCache cache;
  // device tables
  potts::StripParams *d_strip = nullptr;    // per strip group: jobs' descriptors, contiguous
  potts::StripTile *d_tiles = nullptr;      // colour-0 tables, then (at tiles_cap) the colour-1 ones
  size_t tiles_cap = 0;
  std::vector<size_t> strip_desc_off, tile_off, tile_count;  // per strip group
  potts::ResidentJob *d_res = nullptr;      // per resident group and chunk
  std::vector<size_t> res_off;              // per (group, chunk)
  potts::StatsParams *d_stats = nullptr;
  double *d_stats_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  float last_ms = 0.0f;
  int64_t run_sweeps = 0;                   // sweeps per job of one run (max over jobs)
  std::string tuned;                        // chosen shapes, for the record
};

namespace {

void release(potts_batch *b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (void *p : {(void *)b->arena, (void *)b->planes, (void *)b->rec_arena, (void *)b->d_strip, (void *)b->d_tiles,
                  (void *)b->d_res, (void *)b->d_stats, (void *)b->d_stats_out})
    if (p) (void)hipFree(p);
  for (hipEvent_t e : {b->ev_fork, b->ev_join, b->ev_t0, b->ev_t1})
    if (e) (void)hipEventDestroy(e);
  if (b->side) (void)hipStreamDestroy(b->side);
  if (b->owns_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

bool resident_job(const potts_job &j) { return potts::resident_fits((uint32_t)j.L, (uint32_t)j.q); }

bool packed_job(const potts_job &j) { return !resident_job(j) && j.L % 32 == 0; }

// Candidate strip heights for an L (even divisors up to 32).
std::vector<uint32_t> row_candidates(uint32_t L) {
  std::vector<uint32_t> c;
  for (uint32_t r = 2; r <= 32; r *= 2)
    if (L % r == 0) c.push_back(r);
  return c;
}

// Descriptors and tiles of one strip group for the jobs' current rows; the
// sweep index of launch s is done[j] + s for every job (t0 = done[j]).
void build_strip_tables(const potts_batch *b, const StripGroup &g, const potts::TileShape &shape,
                        std::vector<potts::StripParams> &desc, std::vector<potts::StripTile> &tiles,
                        const std::vector<int> *only = nullptr) {
  desc.clear();
  tiles.clear();
  for (size_t k = 0; k < g.jobs.size(); ++k) {
    const int j = g.jobs[k];
    const potts_job &job = b->jobs[j];
    potts::StripParams p{};
    if (g.packed) {
      potts::fill_strip_params(p, b->planes + b->plane_off[j], (uint32_t)job.L, (uint32_t)job.q, job.seed,
                               &b->thr[(size_t)j * 4], b->rows[j]);
      potts::set_items(p, (uint32_t)job.L / 32, (uint32_t)job.L, b->rows[j]);
    } else {
      potts::fill_strip_params(p, b->arena + b->lat_off[j], (uint32_t)job.L, (uint32_t)job.q, job.seed,
                               &b->thr[(size_t)j * 4], b->rows[j]);
    }
    p.t0 = (uint64_t)b->done[j];
    p.nsweeps = (uint64_t)(b->target[j] - b->done[j] > 0 ? b->target[j] - b->done[j] : 0);
    p.ring = b->rec_arena + b->rec_off[j];
    p.cap = (uint64_t)b->ring[j];
    desc.push_back(p);
    if (only && std::find(only->begin(), only->end(), j) == only->end()) continue;
    for (uint32_t first = 0; first < p.nitems; first += shape.block) {
      potts::StripTile t{(uint32_t)k, first, std::min<uint32_t>(shape.block, p.nitems - first), first == 0 ? 1u : 0u};
      tiles.push_back(t);
    }
  }
  // Longest tiles first (a tile's work is its items times their rows): the
  // last workgroups of a launch, which leave CUs idle while they finish, are
  // then short ones.  Jobs of one batch differ up to 8x in rows per item.
  std::stable_sort(tiles.begin(), tiles.end(), [&desc](const potts::StripTile &x, const potts::StripTile &y) {
    return (uint64_t)desc[x.job].rows * x.count > (uint64_t)desc[y.job].rows * y.count;
  });
}

// The colour-1 launch takes its workgroups' tiles from the end of the table
// (it walks the lattice bottom-up), so it gets the table reversed: both
// launches then dispatch the longest tiles first.
std::vector<potts::StripTile> reversed(const std::vector<potts::StripTile> &t) {
  return std::vector<potts::StripTile>(t.rbegin(), t.rend());
}

int upload(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (!bytes) return POTTS_OK;
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));  // the host vectors may go away next
  return POTTS_OK;
}

// One launch pair (colour 0, colour 1) of a strip group for sweep s; tiles0
// and tiles1: the group's table and its reverse.
int launch_strip_sweep(const StripGroup &g, const potts::TileShape &shape, const potts::StripParams *d_desc,
                       const potts::StripTile *tiles0, const potts::StripTile *tiles1, size_t ntiles, uint32_t s,
                       hipStream_t st) {
  potts::StripLaunch l0{}, l1{};
  l0.jobs = l1.jobs = d_desc;
  l0.tiles = tiles0;
  l1.tiles = tiles1;
  l0.sweep = l1.sweep = s;
  const uint32_t mq = class_max_q(g.qc);
  if (g.packed) {
    HIP_TRY(potts::launch_packed_tiled(l0, 0, (unsigned)ntiles, shape, mq, g.wide, st));
    HIP_TRY(potts::launch_packed_tiled(l1, 1, (unsigned)ntiles, shape, mq, g.wide, st));
  } else {
    HIP_TRY(potts::launch_strip_tiled(l0, 0, (unsigned)ntiles, shape, mq, g.wide, st));
    HIP_TRY(potts::launch_strip_tiled(l1, 1, (unsigned)ntiles, shape, mq, g.wide, st));
  }
  return POTTS_OK;
}

// Times `reps` sweeps of the given jobs of a strip group with their current
// rows and the given shape (real sweeps), advancing done[] for them.
int timed_strip_sweeps(potts_batch *b, const StripGroup &g, const potts::TileShape &shape,
                       const std::vector<int> &jobs, int reps, float *ms) {
  std::vector<potts::StripParams> desc;
  std::vector<potts::StripTile> tiles;
  build_strip_tables(b, g, shape, desc, tiles, &jobs);
  int rc = upload(b->d_strip, desc.data(), desc.size() * sizeof(desc[0]), b->stream);
  if (rc) return rc;
  rc = upload(b->d_tiles, tiles.data(), tiles.size() * sizeof(tiles[0]), b->stream);
  if (rc) return rc;
  const std::vector<potts::StripTile> rev = reversed(tiles);
  rc = upload(b->d_tiles + b->tiles_cap, rev.data(), rev.size() * sizeof(rev[0]), b->stream);
  if (rc) return rc;
  HIP_TRY(hipEventRecord(b->ev_t0, b->stream));
  for (int s = 0; s < reps; ++s) {
    rc = launch_strip_sweep(g, shape, b->d_strip, b->d_tiles, b->d_tiles + b->tiles_cap, tiles.size(), (uint32_t)s,
                            b->stream);
    if (rc) return rc;
  }
  HIP_TRY(hipEventRecord(b->ev_t1, b->stream));
  HIP_TRY(hipEventSynchronize(b->ev_t1));
  HIP_TRY(hipEventElapsedTime(ms, b->ev_t0, b->ev_t1));
  for (int j : jobs) b->done[j] += std::min<int64_t>(reps, std::max<int64_t>(0, b->target[j] - b->done[j]));
  return POTTS_OK;
}

int64_t sweeps_left(const potts_batch *b, const std::vector<int> &jobs) {
  int64_t left = INT64_MAX;
  for (int j : jobs) left = std::min<int64_t>(left, b->target[j] - b->done[j]);
  return left;
}

std::string shape_text(const potts::TileShape &t) {
  return "block=" + std::to_string(t.block) + ",waves/SIMD=" + (t.wpe ? std::to_string(t.wpe) : std::string("auto"));
}

// In-run tuning, on real sweeps of the run (kReps timed sweeps per candidate,
// after one untimed warm-up sweep of each lattice size):
//   1. per (group, L): the strip height, with the default shape;
//   2. per group of q <= 16: the workgroup shape (lanes 256 or 128; the
//      compiler's occupancy or at least 8 waves per SIMD) at the chosen heights.
// Choices found in the cache are taken without timing; new ones are added.
constexpr int kReps = 2;

int autotune(potts_batch *b, bool time_new) {
  for (size_t gi = 0; gi < b->strip_groups.size(); ++gi) {
    StripGroup &g = b->strip_groups[gi];
    std::map<int, std::vector<int>> by_L;
    for (int j : g.jobs) by_L[b->jobs[j].L].push_back(j);
    const potts::TileShape base;
    for (auto &kv : by_L) {
      const uint32_t L = (uint32_t)kv.first;
      std::vector<int> &js = kv.second;
      const std::string key = potts::TuneCache::rows_key(g.packed, g.qc, L);
      auto hit = b->cache.rows.find(key);
      if (hit != b->cache.rows.end() && L % hit->second == 0) {
        for (int j : js) b->rows[j] = hit->second;
        b->tuned += "L=" + std::to_string(L) + ":rows=" + std::to_string(hit->second) + "(cached) ";
        continue;
      }
      const std::vector<uint32_t> cands = row_candidates(L);
      if (!time_new || sweeps_left(b, js) < 1 + kReps * (int64_t)cands.size() + 1) continue;  // too short
      float ms = 0.0f, best_ms = 0.0f;
      uint32_t best = cands[0];
      for (int j : js) b->rows[j] = best;
      int rc = timed_strip_sweeps(b, g, base, js, 1, &ms);  // warm-up
      if (rc) return rc;
      for (uint32_t r : cands) {
        for (int j : js) b->rows[j] = r;
        rc = timed_strip_sweeps(b, g, base, js, kReps, &ms);
        if (rc) return rc;
        if (r == cands[0] || ms < best_ms) {
          best_ms = ms;
          best = r;
        }
      }
      for (int j : js) b->rows[j] = best;
      b->cache.rows[key] = best;
      b->cache.dirty = true;
      b->tuned += "L=" + std::to_string(L) + ":rows=" + std::to_string(best) + " ";
    }
    // the workgroup shape of the whole group
    const std::string skey = potts::TuneCache::shape_key(g.packed, g.qc);
    auto hit = b->cache.shapes.find(skey);
    if (hit != b->cache.shapes.end() && potts::shape_ok(hit->second, class_max_q(g.qc))) {
      b->shape[gi] = hit->second;
      b->tuned += std::string(g.packed ? "packed" : "strip") + "/q" + std::to_string(class_max_q(g.qc)) + ":" +
                  shape_text(hit->second) + "(cached) ";
      continue;
    }
    if (!time_new || g.qc != 0) continue;  // one shape for q > 16
    const potts::TileShape cands[4] = {{256, 0}, {128, 0}, {256, 8}, {128, 8}};
    if (sweeps_left(b, g.jobs) < kReps * 4 + 1) continue;
    float best_ms = 0.0f;
    potts::TileShape best = cands[0];
    for (int c = 0; c < 4; ++c) {
      float ms = 0.0f;
      int rc = timed_strip_sweeps(b, g, cands[c], g.jobs, kReps, &ms);
      if (rc) return rc;
      if (c == 0 || ms < best_ms) {
        best_ms = ms;
        best = cands[c];
      }
    }
    b->shape[gi] = best;
    b->cache.shapes[skey] = best;
    b->cache.dirty = true;
    b->tuned += std::string(g.packed ? "packed" : "strip") + "/q16:" + shape_text(best) + " ";
  }
  if (!b->cache.save()) return record_error(POTTS_EIO, "cannot write the tuning cache " + b->cache.path);
  return POTTS_OK;
}

// Queues the rest of the run (every job to its nsweeps) on the stream, as a
// graph when asked.
int queue_rest(potts_batch *b) {
  // strip tables for the remaining sweeps
  std::vector<potts::StripParams> all_desc;
  std::vector<potts::StripTile> all_tiles, all_rev;
  b->strip_desc_off.clear();
  b->tile_off.clear();
  b->tile_count.clear();
  int64_t strip_sweeps = 0;
  for (const StripGroup &g : b->strip_groups) {
    std::vector<potts::StripParams> desc;
    std::vector<potts::StripTile> tiles;
    build_strip_tables(b, g, b->shape[b->strip_desc_off.size()], desc, tiles);
    b->strip_desc_off.push_back(all_desc.size());
    b->tile_off.push_back(all_tiles.size());
    b->tile_count.push_back(tiles.size());
    for (const auto &d : desc) strip_sweeps = std::max<int64_t>(strip_sweeps, (int64_t)d.nsweeps);
    all_desc.insert(all_desc.end(), desc.begin(), desc.end());
    all_tiles.insert(all_tiles.end(), tiles.begin(), tiles.end());
    all_rev.insert(all_rev.end(), tiles.rbegin(), tiles.rend());
  }
  int rc = upload(b->d_strip, all_desc.data(), all_desc.size() * sizeof(all_desc[0]), b->stream);
  if (rc) return rc;
  rc = upload(b->d_tiles, all_tiles.data(), all_tiles.size() * sizeof(all_tiles[0]), b->stream);
  if (rc) return rc;
  rc = upload(b->d_tiles + b->tiles_cap, all_rev.data(), all_rev.size() * sizeof(all_rev[0]), b->stream);
  if (rc) return rc;

  // resident descriptors, one array per (group, chunk)
  std::vector<potts::ResidentJob> all_res;
  b->res_off.clear();
  std::vector<std::pair<size_t, size_t>> res_launch;  // (group, offset) per launch
  for (size_t gi = 0; gi < b->res_groups.size(); ++gi) {
    const ResidentGroup &g = b->res_groups[gi];
    int64_t most = 0;
    for (int j : g.jobs) most = std::max<int64_t>(most, b->target[j] - b->done[j]);
    for (int64_t c0 = 0; c0 < most; c0 += kResidentChunk) {
      res_launch.push_back({gi, all_res.size()});
      for (int j : g.jobs) {
        const potts_job &job = b->jobs[j];
        potts::ResidentJob r{};
        r.spins = b->arena + b->lat_off[j];
        r.L = (uint32_t)job.L;
        r.q = (uint32_t)job.q;
        r.k0 = (uint32_t)job.seed;
        r.k1 = (uint32_t)(job.seed >> 32);
        r.t0 = (uint64_t)(b->done[j] + c0);
        const int64_t left = b->target[j] - b->done[j] - c0;
        r.nsweeps = (uint32_t)std::max<int64_t>(0, std::min<int64_t>(kResidentChunk, left));
        memcpy(r.thr.v, &b->thr[(size_t)j * 4], sizeof(r.thr.v));
        r.ring = b->rec_arena + b->rec_off[j];
        r.cap = (uint64_t)b->ring[j];
        all_res.push_back(r);
      }
    }
  }
  rc = upload(b->d_res, all_res.data(), all_res.size() * sizeof(all_res[0]), b->stream);
  if (rc) return rc;

  const bool use_graph = b->opts.graph != 0;
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  hipStream_t st = b->stream;
  if (use_graph) HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  int err = POTTS_OK;
  // branch 1: resident launches on the side stream
  if (hipEventRecord(b->ev_fork, st) != hipSuccess || hipStreamWaitEvent(b->side, b->ev_fork, 0) != hipSuccess)
    err = record_error(POTTS_EDEVICE, "fork of the batch streams failed");
  for (size_t k = 0; k < res_launch.size() && !err; ++k) {
    const ResidentGroup &g = b->res_groups[res_launch[k].first];
    potts::ResidentLaunch p{};
    p.jobs = b->d_res + res_launch[k].second;
    hipError_t e = potts::launch_resident(p, (unsigned)g.jobs.size(), g.max_L, g.max_q, g.wide, b->side);
    if (e != hipSuccess) err = hip_err(e, "launch_resident");
  }
  // branch 2: the strip chain on the main stream
  for (int64_t s = 0; s < strip_sweeps && !err; ++s) {
    for (size_t gi = 0; gi < b->strip_groups.size() && !err; ++gi) {
      if (!b->tile_count[gi]) continue;
      err = launch_strip_sweep(b->strip_groups[gi], b->shape[gi], b->d_strip + b->strip_desc_off[gi],
                               b->d_tiles + b->tile_off[gi], b->d_tiles + b->tiles_cap + b->tile_off[gi],
                               b->tile_count[gi], (uint32_t)s, st);
    }
  }
  if (!err && (hipEventRecord(b->ev_join, b->side) != hipSuccess || hipStreamWaitEvent(st, b->ev_join, 0) != hipSuccess))
    err = record_error(POTTS_EDEVICE, "join of the batch streams failed");
  if (use_graph) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (!err && e != hipSuccess) err = hip_err(e, "hipStreamEndCapture");
    if (err) {
      if (g) (void)hipGraphDestroy(g);
      return err;
    }
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    HIP_TRY(hipGraphLaunch(b->exec, st));
  }
  if (err) return err;
  b->done = b->target;
  return POTTS_OK;
}

// The colour-split jobs' lattices into their colour planes (before a run's
// sweeps) or back (after them), on the batch stream.
int convert_packed(potts_batch *b, bool to_planes) {
  for (size_t j = 0; j < b->jobs.size(); ++j) {
    if (!b->packed[j]) continue;
    const uint32_t L = (uint32_t)b->jobs[j].L;
    if (to_planes)
      HIP_TRY(potts::launch_pack(b->arena + b->lat_off[j], b->planes + b->plane_off[j], L, b->stream));
    else
      HIP_TRY(potts::launch_unpack(b->planes + b->plane_off[j], b->arena + b->lat_off[j], L, b->stream));
  }
  return POTTS_OK;
}

}  // namespace

extern "C" {

int potts_batch_create(const potts_job *jobs, int32_t n, const potts_batch_opts *opts, potts_batch **out) {
  if (!out) return record_error(POTTS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!jobs || n < 1) return record_error(POTTS_EINVAL, "need at least one job");
  for (int32_t i = 0; i < n; ++i) {
    const potts_job &j = jobs[i];
    if (j.L < 16 || j.L % 16 || j.L > 65520 || j.q < 2 || j.q > POTTS_QMAX)
      return record_error(POTTS_EINVAL, "job " + std::to_string(i) + ": need L % 16 == 0, 16 <= L <= 65520, 2 <= q <= 256");
    if (j.start != POTTS_ORDERED && j.start != POTTS_RANDOM)
      return record_error(POTTS_EINVAL, "job " + std::to_string(i) + ": bad start");
    if (j.nsweeps < 0 || j.nsweeps > (1ll << 31))
      return record_error(POTTS_EINVAL, "job " + std::to_string(i) + ": nsweeps must be in 0 .. 2^31");
  }
  if (opts && (opts->window < 0 || opts->strip_rows < 0))
    return record_error(POTTS_EINVAL, "window and strip_rows must be >= 0");
  potts_batch *b = new (std::nothrow) potts_batch();
  if (!b) return record_error(POTTS_ENOMEM, "host allocation failed");
  b->jobs.assign(jobs, jobs + n);
  if (opts) b->opts = *opts;
  b->done.assign(n, 0);
  b->target.assign(n, 0);
  b->thr.assign((size_t)n * 4, 0);
  b->rows.assign(n, 0);
  b->ring.assign(n, 0);
  int rc = POTTS_OK;
  for (int32_t i = 0; i < n && !rc; ++i) rc = potts::build_threshold_table(jobs[i].beta, &b->thr[(size_t)i * 4]);
  if (rc) {
    release(b);
    return rc;
  }
#define B_TRY(call)                           \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) {                   \
      int r_ = hip_err(e_, #call);            \
      release(b);                             \
      return r_;                              \
    }                                         \
  } while (0)
  if (b->opts.hip_stream) {
    b->stream = (hipStream_t)b->opts.hip_stream;
  } else {
    B_TRY(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    b->owns_stream = true;
  }
  B_TRY(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
  for (hipEvent_t *e : {&b->ev_fork, &b->ev_join}) B_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
  B_TRY(hipEventCreate(&b->ev_t0));
  B_TRY(hipEventCreate(&b->ev_t1));

  // memory: lattices and record rings (every sweep of a run kept)
  size_t lat_bytes = 0, rec_words = 0, plane_bytes = 0;
  b->lat_off.resize(n);
  b->rec_off.resize(n);
  b->plane_off.assign(n, 0);
  b->packed.assign(n, 0);
  for (int32_t i = 0; i < n; ++i) {
    const potts_job &j = jobs[i];
    b->lat_off[i] = lat_bytes;
    lat_bytes += ((size_t)j.L * j.L + 255) / 256 * 256;
    if (packed_job(j)) {
      b->packed[i] = 1;
      b->plane_off[i] = plane_bytes;
      plane_bytes += ((size_t)j.L * j.L + 255) / 256 * 256;
    }
    b->ring[i] = pow2_at_least(std::max<int64_t>(j.nsweeps + 1, b->opts.window + 1));
    b->rec_off[i] = rec_words;
    rec_words += (size_t)b->ring[i] * (size_t)(j.q + 1);
  }
  if (hipMalloc(&b->arena, lat_bytes) != hipSuccess || hipMalloc(&b->rec_arena, rec_words * 8) != hipSuccess ||
      (plane_bytes && hipMalloc(&b->planes, plane_bytes) != hipSuccess)) {
    (void)hipGetLastError();
    release(b);
    return record_error(POTTS_ENOMEM, "batch arena allocation failed (" +
                                          std::to_string(lat_bytes + plane_bytes + rec_words * 8) + " bytes)");
  }
  B_TRY(potts::launch_fill_u64(b->rec_arena, rec_words, 0ull, b->stream));

  // partition and groups
  std::map<std::pair<int, bool>, size_t> sg, rg;
  size_t nstrip_desc = 0, ntiles_max = 0;
  for (int32_t i = 0; i < n; ++i) {
    const potts_job &j = jobs[i];
    const bool wide = !b->thr[i * 4] || !b->thr[i * 4 + 1] || !b->thr[i * 4 + 2] || !b->thr[i * 4 + 3];
    const int qc = q_class((uint32_t)j.q);
    if (resident_job(j)) {
      auto key = std::make_pair(qc, wide);
      if (!rg.count(key)) {
        rg[key] = b->res_groups.size();
        b->res_groups.push_back(ResidentGroup{qc, wide, {}, 0, 0});
      }
      ResidentGroup &g = b->res_groups[rg[key]];
      g.jobs.push_back(i);
      g.max_L = std::max<uint32_t>(g.max_L, (uint32_t)j.L);
      g.max_q = std::max<uint32_t>(g.max_q, (uint32_t)j.q);
    } else {
      const bool pk = b->packed[i] != 0;
      auto key = std::make_pair(qc * 2 + (pk ? 1 : 0), wide);
      if (!sg.count(key)) {
        sg[key] = b->strip_groups.size();
        b->strip_groups.push_back(StripGroup{qc, wide, pk, {}});
      }
      b->strip_groups[sg[key]].jobs.push_back(i);
      b->rows[i] = b->opts.strip_rows && j.L % b->opts.strip_rows == 0 && b->opts.strip_rows % 2 == 0
                       ? (uint32_t)b->opts.strip_rows
                       : potts::auto_strip_rows((uint32_t)j.L, (uint32_t)j.L, 64 * 256);
      ++nstrip_desc;
      ntiles_max += ((size_t)j.L / 2) * ((size_t)j.L / 16) / 128 + 1;  // rows = 2, 128 lanes: the most tiles
    }
  }
  b->shape.assign(b->strip_groups.size(), potts::TileShape{});
  b->cache.load(b->opts.tune_cache);
  // resident descriptors: one per job per chunk of the longest run
  size_t nres = 0;
  for (const ResidentGroup &g : b->res_groups) {
    int64_t most = 0;
    for (int j : g.jobs) most = std::max<int64_t>(most, jobs[j].nsweeps);
    nres += g.jobs.size() * (size_t)std::max<int64_t>(1, (most + kResidentChunk - 1) / kResidentChunk);
  }
  if ((nstrip_desc && (hipMalloc(&b->d_strip, nstrip_desc * sizeof(potts::StripParams)) != hipSuccess ||
                       hipMalloc(&b->d_tiles, 2 * ntiles_max * sizeof(potts::StripTile)) != hipSuccess)) ||
      (nres && hipMalloc(&b->d_res, nres * sizeof(potts::ResidentJob)) != hipSuccess) ||
      hipMalloc(&b->d_stats, (size_t)n * sizeof(potts::StatsParams)) != hipSuccess ||
      hipMalloc(&b->d_stats_out, (size_t)n * 8 * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    release(b);
    return record_error(POTTS_ENOMEM, "batch table allocation failed");
  }
  b->tiles_cap = ntiles_max;
  // initial conditions
  for (int32_t i = 0; i < n; ++i) {
    potts::InitParams p{};
    p.spins = b->arena + b->lat_off[i];
    p.L = (uint32_t)jobs[i].L;
    p.q = (uint32_t)jobs[i].q;
    p.nchunks = (uint64_t)jobs[i].L * jobs[i].L / 4;
    p.k0 = (uint32_t)jobs[i].seed;
    p.k1 = (uint32_t)(jobs[i].seed >> 32);
    p.random = jobs[i].start == POTTS_RANDOM;
    B_TRY(potts::launch_init(p, b->stream));
  }
  B_TRY(hipStreamSynchronize(b->stream));
#undef B_TRY
  *out = b;
  return POTTS_OK;
}

int potts_batch_run(potts_batch *b) {
  if (!b) return record_error(POTTS_EINVAL, "batch is NULL");
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (size_t j = 0; j < b->jobs.size(); ++j) {
    if (b->done[j] > INT64_MAX - b->jobs[j].nsweeps) return record_error(POTTS_ERANGE, "sweep counter overflow");
    b->target[j] = b->done[j] + b->jobs[j].nsweeps;
  }
  hipEvent_t mark = nullptr;
  HIP_TRY(hipEventCreate(&mark));
  HIP_TRY(hipEventRecord(mark, b->stream));
  int rc = convert_packed(b, true);
  if (!rc) rc = autotune(b, b->opts.tune != 0);
  if (!rc) rc = queue_rest(b);
  if (!rc) rc = convert_packed(b, false);
  if (!rc) {
    hipError_t e = hipEventRecord(b->ev_t1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b->ev_t1);
    if (e == hipSuccess) e = hipEventElapsedTime(&b->last_ms, mark, b->ev_t1);
    if (e != hipSuccess) rc = hip_err(e, "batch timing");
  }
  (void)hipEventDestroy(mark);
  return rc;
}

int potts_batch_results(potts_batch *b, potts_job_result *out) {
  if (!b || !out) return record_error(POTTS_EINVAL, "NULL argument");
  const size_t n = b->jobs.size();
  std::vector<potts::StatsParams> sp(n);
  std::vector<int64_t> last(n * (POTTS_QMAX + 1));
  for (size_t j = 0; j < n; ++j) {
    const potts_job &job = b->jobs[j];
    const int64_t t = b->done[j];
    int64_t w = b->opts.window > 0 ? std::min<int64_t>(b->opts.window, t) : t;
    potts::StatsParams &p = sp[j];
    p.ring = b->rec_arena + b->rec_off[j];
    p.cap = b->ring[j];
    p.n = w > 0 ? w : 1;
    p.slot0 = ((t - p.n) & (b->ring[j] - 1));
    p.q = (uint32_t)job.q;
    p.N = (uint64_t)job.L * job.L;
    p.beta = job.beta;
    p.out = b->d_stats_out + j * 8;
  }
  int rc = upload(b->d_stats, sp.data(), n * sizeof(sp[0]), b->stream);
  if (rc) return rc;
  HIP_TRY(potts::launch_stats_many(b->d_stats, (unsigned)n, b->stream));
  std::vector<double> host(n * 8);
  HIP_TRY(hipMemcpyAsync(host.data(), b->d_stats_out, host.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  for (size_t j = 0; j < n; ++j) {
    const int64_t t = b->done[j];
    const int64_t slot = t > 0 ? ((t - 1) & (b->ring[j] - 1)) : 0;
    HIP_TRY(hipMemcpyAsync(&last[j * (POTTS_QMAX + 1)], b->rec_arena + b->rec_off[j] + slot * (b->jobs[j].q + 1),
                           (size_t)(b->jobs[j].q + 1) * 8, hipMemcpyDeviceToHost, b->stream));
  }
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (size_t j = 0; j < n; ++j) {
    potts_job_result &r = out[j];
    memset(&r, 0, sizeof(r));
    r.t = b->done[j];
    const int64_t *rec = &last[j * (POTTS_QMAX + 1)];
    if (r.t > 0) {
      r.e_sat = rec[0];
      for (int v = 0; v < b->jobs[j].q; ++v) r.nmax = std::max<int64_t>(r.nmax, rec[1 + v]);
      const double *v = &host[j * 8];
      r.stats.n = b->opts.window > 0 ? std::min<int64_t>(b->opts.window, r.t) : r.t;
      r.stats.e = v[0];
      r.stats.C = v[1];
      r.stats.V_L = v[2];
      r.stats.m = v[3];
      r.stats.chi = v[4];
    }
  }
  return POTTS_OK;
}

int potts_batch_records(potts_batch *b, int32_t job, int64_t t0, int64_t n, int64_t *out) {
  if (!b || (!out && n > 0) || job < 0 || job >= (int32_t)b->jobs.size())
    return record_error(POTTS_EINVAL, "bad batch, job index or output");
  const int64_t t = b->done[job], cap = b->ring[job];
  if (t0 < 0 || n < 0 || t0 < t - cap + 1 || t0 + n > t)
    return record_error(POTTS_ERANGE, "requested records are not kept");
  const int64_t rl = b->jobs[job].q + 1;
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (int64_t i = 0; i < n; ++i) {
    const int64_t slot = (t0 + i) & (cap - 1);
    HIP_TRY(hipMemcpy(out + i * rl, b->rec_arena + b->rec_off[job] + slot * rl, (size_t)rl * 8, hipMemcpyDeviceToHost));
  }
  return POTTS_OK;
}

int potts_batch_spins(potts_batch *b, int32_t job, uint8_t *host_out) {
  if (!b || !host_out || job < 0 || job >= (int32_t)b->jobs.size())
    return record_error(POTTS_EINVAL, "bad batch, job index or output");
  HIP_TRY(hipStreamSynchronize(b->stream));
  HIP_TRY(hipMemcpy(host_out, b->arena + b->lat_off[job], (size_t)b->jobs[job].L * b->jobs[job].L,
                    hipMemcpyDeviceToHost));
  return POTTS_OK;
}

double potts_batch_elapsed_ms(const potts_batch *b) { return b ? (double)b->last_ms : -1.0; }

const char *potts_batch_tuning(const potts_batch *b) { return b ? b->tuned.c_str() : ""; }

void potts_batch_free(potts_batch *b) { release(b); }

}  // extern "C"
