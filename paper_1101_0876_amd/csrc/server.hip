// server.hip -- serving loop with continuous batching: the C ABI
// potts_server_* of include/potts.h.
//
// A request is a simulation job: L, q, seed, start and a beta schedule (a
// ramp of points, each with its number of sweeps; the protocol of Sec. 3).
// A server thread admits queued requests in arrival order while a slot is
// free and the job's lattice and record ring fit in the HBM budget, keeps
// every admitted lattice and its sweep counter resident on the device, and
// runs iterations: each iteration advances every active job by up to
// `quantum` sweeps of its current point in shared launches (LDS-resident
// launches for L <= 256, one tiled strip launch per colour and sweep for the
// rest), so requests that arrive while others run join the next iteration.
// When a point's sweeps are done its summary (derived statistics over the last
// half of the point's sweeps) is computed on the device; when the last point
// is done the job's memory is released and its completion time recorded.
//
// Results are bit-identical to the same job run alone: random numbers are
// keyed by (seed, site, sweep), and each job's sweep counter is its own.
//
// Recovery: a job may name a checkpoint file, rewritten after each completed
// point; a later request may resume from it and ends with the bits of an
// uninterrupted run.  A failure of one job (an injected one, for tests, is
// raised on the host before the iteration that would run the chosen sweep)
// ends that job alone.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
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
using Clock = std::chrono::steady_clock;

int q_class(uint32_t q) { return q <= 16 ? 0 : q <= potts::kPrivateHistMaxQ ? 1 : q <= 128 ? 2 : 3; }
uint32_t class_max_q(int c) { return c == 0 ? 16 : c == 1 ? potts::kPrivateHistMaxQ : c == 2 ? 128 : 256; }

int64_t pow2_at_least(int64_t n) {
  int64_t p = 2;
  while (p < n) p <<= 1;
  return p;
}

struct Job {
  int64_t ticket = 0;
  potts_request req{};
  std::vector<double> betas;
  std::vector<int64_t> sweeps;
  std::vector<uint32_t> thr;  // 4 per point
  bool keep_spins = false;
  std::string ckpt_path;           // checkpoint file after each completed point ("" = none)
  int64_t fault_at = -1;           // injected failure before sweep fault_at runs (-1 = none)
  // resumed jobs: the state read from the checkpoint at submit
  bool resume = false;
  std::vector<uint8_t> resume_spins;
  int64_t resume_t = 0;
  int resume_point = 0;
  bool ckpt_due = false;           // a point completed in the last iteration
  // device state
  uint8_t *lat = nullptr;
  unsigned long long *ring = nullptr;
  int64_t cap = 0;
  size_t bytes = 0;
  int64_t t = 0;        // sweeps done
  int point = 0;        // current point
  int64_t left = 0;     // sweeps left in the current point
  uint32_t rows = 0;    // strip height (0: resident)
  bool resident = false;
  // results
  std::vector<potts_summary> points;
  std::vector<uint8_t> spins;
  potts_served info{};
};

struct Pending {  // a point summary being computed this iteration
  Job *job;
  int point;
  int64_t window;
};

}  // namespace

struct potts_server {
  potts_server_cfg cfg{};
  hipStream_t stream = nullptr;
  bool owns_stream = false;
  Clock::time_point t0;
  int device = 0;
  std::thread thread;
  std::mutex mu;  // guards queue, done, stop, failed, next_ticket, submitted, finished
  std::condition_variable cv_work, cv_done;
  std::deque<std::unique_ptr<Job>> queue;
  std::map<int64_t, std::unique_ptr<Job>> done;
  std::vector<int64_t> done_order;  // finished, not yet reported by potts_server_wait
  bool stop = false;
  int failed = 0;
  std::string fail_msg;
  int64_t next_ticket = 1;
  int64_t submitted = 0, finished = 0;
  std::map<int64_t, int64_t> faults;  // ticket -> sweep, for injected failures
  int64_t fault_next = -1;            // injected failure of the next accepted job (-1 = none)
  std::set<int64_t> running;          // tickets of admitted, unfinished jobs
  // owned by the server thread
  std::vector<std::unique_ptr<Job>> active;
  size_t used_bytes = 0;
  potts::StripParams *d_strip = nullptr;
  potts::StripTile *d_tiles = nullptr;
  potts::ResidentJob *d_res = nullptr;
  potts::StatsParams *d_stats = nullptr;
  size_t cap_strip = 0, cap_tiles = 0, cap_res = 0, cap_stats = 0;
  void *h_stage = nullptr;  // pinned staging for descriptor uploads
  size_t cap_stage = 0;
  int64_t iterations = 0;
  potts::TuneCache cache;   // launch shapes: strip heights per (q class, L), shape per q class
  std::string tuned;        // what the tuner chose, for the record (guarded by mu)
};

namespace {

double seconds_since(const potts_server *s) {
  return std::chrono::duration<double>(Clock::now() - s->t0).count();
}

const char *herr(hipError_t e) { return hipGetErrorString(e); }

// grows a device table to at least n entries of `size` bytes
bool reserve_dev(void **p, size_t *cap, size_t n, size_t size) {
  if (n <= *cap) return true;
  size_t want = std::max<size_t>(n, *cap * 2);
  void *q = nullptr;
  if (hipMalloc(&q, want * size) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (*p) (void)hipFree(*p);
  *p = q;
  *cap = want;
  return true;
}

bool reserve_stage(potts_server *s, size_t bytes) {
  if (bytes <= s->cap_stage) return true;
  size_t want = std::max<size_t>(bytes, s->cap_stage * 2);
  void *q = nullptr;
  if (hipHostMalloc(&q, want, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (s->h_stage) (void)hipHostFree(s->h_stage);
  s->h_stage = q;
  s->cap_stage = want;
  return true;
}

size_t job_bytes(const Job &j) {
  return ((size_t)j.req.L * j.req.L + 255) / 256 * 256 + (size_t)j.cap * (size_t)(j.req.q + 1) * 8;
}

// Frees a job's device memory (failure paths; synchronous).
void release_job_memory(Job &j) {
  for (void *p : {(void *)j.lat, (void *)j.ring})
    if (p) (void)hipFree(p);
  j.lat = nullptr;
  j.ring = nullptr;
}

// Job checkpoint: magic, (L, q, npoints, point, start, pad) int32, seed u64,
// t int64, `point` summaries, then the L*L lattice.
const uint32_t kJobMagic[2] = {0x54544f50u, 0x31424a53u};  // "POTTSJB1"

bool write_job_checkpoint(const Job &j, const std::vector<uint8_t> &lat, std::string &err) {
  const std::string tmp = j.ckpt_path + ".tmp";
  FILE *f = fopen(tmp.c_str(), "wb");
  if (!f) {
    err = "cannot open " + tmp;
    return false;
  }
  const int32_t hdr[6] = {j.req.L, j.req.q, j.req.npoints, j.point, j.req.start, 0};
  const uint64_t seed = j.req.seed;
  const int64_t t = j.t;
  bool ok = fwrite(kJobMagic, sizeof(kJobMagic), 1, f) == 1 && fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
            fwrite(&seed, sizeof(seed), 1, f) == 1 && fwrite(&t, sizeof(t), 1, f) == 1 &&
            (j.point == 0 || fwrite(j.points.data(), sizeof(potts_summary), (size_t)j.point, f) == (size_t)j.point) &&
            fwrite(lat.data(), 1, lat.size(), f) == lat.size();
  ok = fclose(f) == 0 && ok;
  if (!ok || rename(tmp.c_str(), j.ckpt_path.c_str()) != 0) {
    err = "cannot write checkpoint " + j.ckpt_path;
    return false;
  }
  return true;
}

// Reads a checkpoint into j's resume fields; 0 or a negative code.
int read_job_checkpoint(Job &j, const char *path) {
  FILE *f = fopen(path, "rb");
  if (!f) return record_error(POTTS_EIO, std::string("cannot open ") + path);
  uint32_t magic[2];
  int32_t hdr[6];
  uint64_t seed;
  int64_t t;
  bool ok = fread(magic, sizeof(magic), 1, f) == 1 && fread(hdr, sizeof(hdr), 1, f) == 1 &&
            fread(&seed, sizeof(seed), 1, f) == 1 && fread(&t, sizeof(t), 1, f) == 1;
  if (!ok || magic[0] != kJobMagic[0] || magic[1] != kJobMagic[1]) {
    fclose(f);
    return record_error(POTTS_EIO, std::string("not a job checkpoint: ") + path);
  }
  if (hdr[0] != j.req.L || hdr[1] != j.req.q || hdr[2] != j.req.npoints || hdr[4] != j.req.start ||
      seed != j.req.seed || hdr[3] < 1 || hdr[3] >= j.req.npoints || t < 0) {
    fclose(f);
    return record_error(POTTS_EINVAL, std::string("the checkpoint belongs to another job: ") + path);
  }
  int64_t expect = 0;  // the sweeps of the points before the resume point
  for (int k = 0; k < hdr[3]; ++k) expect += j.sweeps[(size_t)k];
  if (t != expect) {
    fclose(f);
    return record_error(POTTS_EINVAL, std::string("the checkpoint's sweep count does not fit the schedule: ") + path);
  }
  j.points.assign((size_t)j.req.npoints, potts_summary{});
  j.resume_spins.resize((size_t)j.req.L * j.req.L);
  ok = fread(j.points.data(), sizeof(potts_summary), (size_t)hdr[3], f) == (size_t)hdr[3] &&
       fread(j.resume_spins.data(), 1, j.resume_spins.size(), f) == j.resume_spins.size();
  fclose(f);
  if (!ok) return record_error(POTTS_EIO, std::string("truncated job checkpoint: ") + path);
  for (uint8_t v : j.resume_spins)
    if (v >= j.req.q) return record_error(POTTS_EIO, std::string("spin value >= q in ") + path);
  j.resume = true;
  j.resume_t = t;
  j.resume_point = hdr[3];
  return POTTS_OK;
}

std::string shape_text(const potts::TileShape &t) {
  return "block=" + std::to_string(t.block) + ",waves/SIMD=" + (t.wpe ? std::to_string(t.wpe) : std::string("auto"));
}

// Times `reps` sweeps of one throwaway lattice in the strip kernel with the
// given height and shape; ms is the device time.
bool time_shape(potts_server *s, potts::StripParams p, uint32_t rows, const potts::TileShape &shape, int reps,
                uint64_t *t, float *ms, hipEvent_t e0, hipEvent_t e1, std::string &err) {
  p.rows = rows;
  potts::set_items(p, p.L / 16, p.L, rows);
  p.t0 = *t;
  p.nsweeps = (uint64_t)reps;
  std::vector<potts::StripTile> tiles;
  for (uint32_t first = 0; first < p.nitems; first += shape.block)
    tiles.push_back(potts::StripTile{0, first, std::min<uint32_t>(shape.block, p.nitems - first), first == 0 ? 1u : 0u});
  if (!reserve_dev((void **)&s->d_strip, &s->cap_strip, 1, sizeof(potts::StripParams)) ||
      !reserve_dev((void **)&s->d_tiles, &s->cap_tiles, tiles.size(), sizeof(potts::StripTile))) {
    err = "descriptor table allocation failed";
    return false;
  }
  hipError_t e = hipMemcpyAsync(s->d_strip, &p, sizeof(p), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_tiles, tiles.data(), tiles.size() * sizeof(tiles[0]), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);  // the host tables go away next
  if (e == hipSuccess) e = hipEventRecord(e0, s->stream);
  potts::StripLaunch l{};
  l.jobs = s->d_strip;
  l.tiles = s->d_tiles;
  const uint32_t mq = (p.q <= 16) ? 16 : p.q <= potts::kPrivateHistMaxQ ? potts::kPrivateHistMaxQ : p.q <= 128 ? 128 : 256;
  const bool wide = !p.thr.v[0] || !p.thr.v[1] || !p.thr.v[2] || !p.thr.v[3];
  for (int k = 0; k < reps && e == hipSuccess; ++k) {
    l.sweep = (uint32_t)k;
    e = potts::launch_strip_tiled(l, 0, (unsigned)tiles.size(), shape, mq, wide, s->stream);
    if (e == hipSuccess) e = potts::launch_strip_tiled(l, 1, (unsigned)tiles.size(), shape, mq, wide, s->stream);
  }
  if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  if (e != hipSuccess) {
    err = std::string("tuning failed: ") + herr(e);
    return false;
  }
  *t += (uint64_t)reps;
  return true;
}

// The strip height of lattice size L in q class qc (and, on first sight of
// the class, the workgroup shape), timed on a throwaway random lattice at
// beta_c(q) unless the cache knows them; the cache is updated.
bool tune_size(potts_server *s, uint32_t L, uint32_t q, int qc, std::string &err) {
  const std::string rkey = potts::TuneCache::rows_key(false, qc, L);
  const std::string skey = potts::TuneCache::shape_key(false, qc);
  const bool need_rows = !s->cache.rows.count(rkey);
  const bool need_shape = qc == 0 && !s->cache.shapes.count(skey);
  if (!need_rows && !need_shape) return true;
  uint8_t *lat = nullptr;
  unsigned long long *ring = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const uint64_t cap = 2;
  hipError_t e = hipMallocAsync((void **)&lat, (size_t)L * L, s->stream);
  if (e == hipSuccess) e = hipMallocAsync((void **)&ring, cap * (q + 1) * 8, s->stream);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  potts::InitParams ip{};
  ip.spins = lat;
  ip.L = L;
  ip.q = q;
  ip.nchunks = (uint64_t)L * L / 4;
  ip.k0 = 1;
  ip.random = 1;
  if (e == hipSuccess) e = potts::launch_init(ip, s->stream);
  if (e == hipSuccess) e = potts::launch_fill_u64(ring, cap * (q + 1), 0ull, s->stream);
  bool ok = e == hipSuccess;
  if (!ok) err = std::string("tuning setup failed: ") + herr(e);
  uint32_t thr[4] = {0, 0, 0, 0};
  if (ok) ok = potts::build_threshold_table(log1p(sqrt((double)q)), thr) == POTTS_OK;
  potts::StripParams p{};
  if (ok) {
    potts::fill_strip_params(p, lat, L, q, 1, thr, 2);
    p.ring = ring;
    p.cap = cap;
  }
  uint64_t t = 0;
  const potts::TileShape base;
  uint32_t rows = need_rows ? 0 : s->cache.rows[rkey];
  float ms = 0.0f;
  if (ok && need_rows) {
    ok = time_shape(s, p, 2, base, 1, &t, &ms, e0, e1, err);  // warm-up
    float best_ms = 0.0f;
    for (uint32_t r = 2; r <= 32 && ok; r *= 2) {
      if (L % r) continue;
      ok = time_shape(s, p, r, base, 2, &t, &ms, e0, e1, err);
      if (ok && (rows == 0 || ms < best_ms)) {
        best_ms = ms;
        rows = r;
      }
    }
    if (ok) {
      s->cache.rows[rkey] = rows;
      s->cache.dirty = true;
      std::lock_guard<std::mutex> lk(s->mu);
      s->tuned += rkey + ":rows=" + std::to_string(rows) + " ";
    }
  }
  if (ok && need_shape) {
    const potts::TileShape cands[4] = {{256, 0}, {128, 0}, {256, 8}, {128, 8}};
    float best_ms = 0.0f;
    potts::TileShape best = cands[0];
    for (int c = 0; c < 4 && ok; ++c) {
      ok = time_shape(s, p, rows, cands[c], 2, &t, &ms, e0, e1, err);
      if (ok && (c == 0 || ms < best_ms)) {
        best_ms = ms;
        best = cands[c];
      }
    }
    if (ok) {
      s->cache.shapes[skey] = best;
      s->cache.dirty = true;
      std::lock_guard<std::mutex> lk(s->mu);
      s->tuned += skey + ":" + shape_text(best) + " ";
    }
  }
  (void)hipStreamSynchronize(s->stream);
  if (lat) (void)hipFreeAsync(lat, s->stream);
  if (ring) (void)hipFreeAsync(ring, s->stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (ok && !s->cache.save()) {
    err = "cannot write the tuning cache " + s->cache.path;
    ok = false;
  }
  return ok;
}

// Allocates and initializes an admitted job on the server stream.
bool admit(potts_server *s, Job &j, std::string &err) {
  hipError_t e = hipMallocAsync((void **)&j.lat, ((size_t)j.req.L * j.req.L + 255) / 256 * 256, s->stream);
  if (e == hipSuccess) e = hipMallocAsync((void **)&j.ring, (size_t)j.cap * (j.req.q + 1) * 8, s->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s->stream);
    release_job_memory(j);
    err = std::string("allocation failed: ") + herr(e);
    return false;
  }
  potts::InitParams p{};
  p.spins = j.lat;
  p.L = (uint32_t)j.req.L;
  p.q = (uint32_t)j.req.q;
  p.nchunks = (uint64_t)j.req.L * j.req.L / 4;
  p.k0 = (uint32_t)j.req.seed;
  p.k1 = (uint32_t)(j.req.seed >> 32);
  p.random = j.req.start == POTTS_RANDOM;
  if (j.resume) {
    e = hipMemcpyAsync(j.lat, j.resume_spins.data(), j.resume_spins.size(), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);  // the host copy goes away next
  } else {
    e = potts::launch_init(p, s->stream);
  }
  if (e == hipSuccess) e = potts::launch_fill_u64(j.ring, (uint64_t)j.cap * (j.req.q + 1), 0ull, s->stream);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(s->stream);
    release_job_memory(j);
    err = std::string("initialization failed: ") + herr(e);
    return false;
  }
  j.resident = potts::resident_fits((uint32_t)j.req.L, (uint32_t)j.req.q);
  j.rows = 0;
  if (!j.resident) {
    const int qc = q_class((uint32_t)j.req.q);
    if (s->cfg.tune && !tune_size(s, (uint32_t)j.req.L, (uint32_t)j.req.q, qc, err)) {
      (void)hipStreamSynchronize(s->stream);
      release_job_memory(j);
      return false;
    }
    auto hit = s->cache.rows.find(potts::TuneCache::rows_key(false, qc, (uint32_t)j.req.L));
    j.rows = hit != s->cache.rows.end() && j.req.L % hit->second == 0
                 ? hit->second
                 : potts::auto_strip_rows((uint32_t)j.req.L, (uint32_t)j.req.L, 64 * 256);
  }
  j.point = j.resume ? j.resume_point : 0;
  j.left = j.sweeps[(size_t)j.point];
  j.t = j.resume ? j.resume_t : 0;
  j.resume_spins.clear();
  j.resume_spins.shrink_to_fit();
  j.info.t_admit = seconds_since(s);
  return true;
}

// One iteration over the active jobs: returns 0 or a negative code (message in err).
int iterate(potts_server *s, std::string &err) {
  const int64_t quantum = s->cfg.quantum;
  struct SG {
    int qc;
    bool wide;
    std::vector<Job *> jobs;
    potts::TileShape shape;
  };
  std::vector<SG> strip_groups, res_groups;
  auto group_of = [s](std::vector<SG> &gs, int qc, bool wide) -> SG & {
    for (SG &g : gs)
      if (g.qc == qc && g.wide == wide) return g;
    potts::TileShape shape;
    auto hit = s->cache.shapes.find(potts::TuneCache::shape_key(false, qc));
    if (hit != s->cache.shapes.end() && potts::shape_ok(hit->second, class_max_q(qc))) shape = hit->second;
    gs.push_back(SG{qc, wide, {}, shape});
    return gs.back();
  };
  std::vector<int64_t> step(s->active.size());
  for (size_t k = 0; k < s->active.size(); ++k) {
    Job &j = *s->active[k];
    step[k] = std::min<int64_t>(quantum, j.left);
    const uint32_t *thr = &j.thr[(size_t)j.point * 4];
    const bool wide = !thr[0] || !thr[1] || !thr[2] || !thr[3];
    group_of(j.resident ? res_groups : strip_groups, q_class((uint32_t)j.req.q), wide).jobs.push_back(&j);
  }
  std::map<Job *, int64_t> nstep;
  for (size_t k = 0; k < s->active.size(); ++k) nstep[s->active[k].get()] = step[k];

  // descriptors
  std::vector<potts::StripParams> desc;
  std::vector<potts::StripTile> tiles;
  std::vector<size_t> desc_off, tile_off, tile_cnt;
  int64_t strip_sweeps = 0;
  for (SG &g : strip_groups) {
    desc_off.push_back(desc.size());
    tile_off.push_back(tiles.size());
    for (size_t k = 0; k < g.jobs.size(); ++k) {
      Job &j = *g.jobs[k];
      potts::StripParams p{};
      potts::fill_strip_params(p, j.lat, (uint32_t)j.req.L, (uint32_t)j.req.q, j.req.seed,
                               &j.thr[(size_t)j.point * 4], j.rows);
      p.t0 = (uint64_t)j.t;
      p.nsweeps = (uint64_t)nstep[&j];
      p.ring = j.ring;
      p.cap = (uint64_t)j.cap;
      strip_sweeps = std::max<int64_t>(strip_sweeps, nstep[&j]);
      for (uint32_t first = 0; first < p.nitems; first += g.shape.block)
        tiles.push_back(potts::StripTile{(uint32_t)k, first, std::min<uint32_t>(g.shape.block, p.nitems - first),
                                         first == 0 ? 1u : 0u});
      desc.push_back(p);
    }
    tile_cnt.push_back(tiles.size() - tile_off.back());
  }
  std::vector<potts::ResidentJob> res;
  std::vector<size_t> res_off;
  for (SG &g : res_groups) {
    res_off.push_back(res.size());
    for (Job *jp : g.jobs) {
      Job &j = *jp;
      potts::ResidentJob r{};
      r.spins = j.lat;
      r.L = (uint32_t)j.req.L;
      r.q = (uint32_t)j.req.q;
      r.k0 = (uint32_t)j.req.seed;
      r.k1 = (uint32_t)(j.req.seed >> 32);
      r.t0 = (uint64_t)j.t;
      r.nsweeps = (uint32_t)nstep[&j];
      memcpy(r.thr.v, &j.thr[(size_t)j.point * 4], sizeof(r.thr.v));
      r.ring = j.ring;
      r.cap = (uint64_t)j.cap;
      res.push_back(r);
    }
  }
  // point summaries that complete in this iteration
  std::vector<Pending> pend;
  std::vector<potts::StatsParams> stats;
  for (auto &jp : s->active) {
    Job &j = *jp;
    if (nstep[&j] == j.left) {
      const int64_t w = std::max<int64_t>(1, (j.sweeps[j.point] + 1) / 2);
      const int64_t t_end = j.t + nstep[&j];
      potts::StatsParams p{};
      p.ring = j.ring;
      p.cap = j.cap;
      p.n = w;
      p.slot0 = (t_end - w) & (j.cap - 1);
      p.q = (uint32_t)j.req.q;
      p.N = (uint64_t)j.req.L * j.req.L;
      p.beta = j.betas[j.point];
      stats.push_back(p);
      pend.push_back(Pending{&j, j.point, w});
    }
  }
  if (!reserve_dev((void **)&s->d_strip, &s->cap_strip, desc.size(), sizeof(potts::StripParams)) ||
      !reserve_dev((void **)&s->d_tiles, &s->cap_tiles, tiles.size(), sizeof(potts::StripTile)) ||
      !reserve_dev((void **)&s->d_res, &s->cap_res, res.size(), sizeof(potts::ResidentJob)) ||
      !reserve_dev((void **)&s->d_stats, &s->cap_stats, stats.size(), sizeof(potts::StatsParams))) {
    err = "descriptor table allocation failed";
    return POTTS_ENOMEM;
  }
  double *d_out = nullptr;
  if (stats.size()) {
    if (hipMallocAsync((void **)&d_out, stats.size() * 8 * sizeof(double), s->stream) != hipSuccess) {
      err = "stats buffer allocation failed";
      return POTTS_ENOMEM;
    }
    for (size_t i = 0; i < stats.size(); ++i) stats[i].out = d_out + i * 8;
  }
  const size_t b1 = desc.size() * sizeof(desc[0]), b2 = tiles.size() * sizeof(tiles[0]),
               b3 = res.size() * sizeof(res[0]), b4 = stats.size() * sizeof(stats[0]);
  if (!reserve_stage(s, b1 + b2 + b3 + b4)) {
    err = "pinned staging allocation failed";
    return POTTS_ENOMEM;
  }
  uint8_t *h = (uint8_t *)s->h_stage;
  memcpy(h, desc.data(), b1);
  memcpy(h + b1, tiles.data(), b2);
  memcpy(h + b1 + b2, res.data(), b3);
  memcpy(h + b1 + b2 + b3, stats.data(), b4);
  hipError_t e = hipSuccess;
  if (b1) e = hipMemcpyAsync(s->d_strip, h, b1, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess && b2) e = hipMemcpyAsync(s->d_tiles, h + b1, b2, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess && b3) e = hipMemcpyAsync(s->d_res, h + b1 + b2, b3, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess && b4) e = hipMemcpyAsync(s->d_stats, h + b1 + b2 + b3, b4, hipMemcpyHostToDevice, s->stream);
  // resident groups: all of this iteration's sweeps in one launch each
  for (size_t gi = 0; gi < res_groups.size() && e == hipSuccess; ++gi) {
    uint32_t max_L = 0, max_q = 0;
    for (Job *jp : res_groups[gi].jobs) {
      max_L = std::max<uint32_t>(max_L, (uint32_t)jp->req.L);
      max_q = std::max<uint32_t>(max_q, (uint32_t)jp->req.q);
    }
    potts::ResidentLaunch p{};
    p.jobs = s->d_res + res_off[gi];
    e = potts::launch_resident(p, (unsigned)res_groups[gi].jobs.size(), max_L, max_q, res_groups[gi].wide, s->stream);
  }
  // strip groups: one launch per colour and sweep covering every job
  for (int64_t sw = 0; sw < strip_sweeps && e == hipSuccess; ++sw) {
    for (size_t gi = 0; gi < strip_groups.size() && e == hipSuccess; ++gi) {
      potts::StripLaunch l{};
      l.jobs = s->d_strip + desc_off[gi];
      l.tiles = s->d_tiles + tile_off[gi];
      l.sweep = (uint32_t)sw;
      const uint32_t mq = class_max_q(strip_groups[gi].qc);
      const potts::TileShape &shape = strip_groups[gi].shape;
      e = potts::launch_strip_tiled(l, 0, (unsigned)tile_cnt[gi], shape, mq, strip_groups[gi].wide, s->stream);
      if (e == hipSuccess)
        e = potts::launch_strip_tiled(l, 1, (unsigned)tile_cnt[gi], shape, mq, strip_groups[gi].wide, s->stream);
    }
  }
  std::vector<double> out(stats.size() * 8);
  if (e == hipSuccess && stats.size()) e = potts::launch_stats_many(s->d_stats, (unsigned)stats.size(), s->stream);
  if (e == hipSuccess && stats.size())
    e = hipMemcpyAsync(out.data(), d_out, out.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream);
  if (d_out && e == hipSuccess) e = hipFreeAsync(d_out, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    err = std::string("iteration failed: ") + herr(e);
    return POTTS_EDEVICE;
  }
  ++s->iterations;
  for (size_t i = 0; i < pend.size(); ++i) {
    potts_summary &r = pend[i].job->points[(size_t)pend[i].point];
    const double *v = &out[i * 8];
    r.n = pend[i].window;
    r.e = v[0];
    r.C = v[1];
    r.V_L = v[2];
    r.m = v[3];
    r.chi = v[4];
  }
  for (auto &jp : s->active) {
    Job &j = *jp;
    const int64_t n = nstep[&j];
    j.t += n;
    j.left -= n;
    while (j.left == 0 && j.point + 1 < j.req.npoints) {
      ++j.point;
      j.left = j.sweeps[(size_t)j.point];
      j.ckpt_due = true;
    }
  }
  return POTTS_OK;
}

// Ends one active job with an error code: its memory is released and it is
// reported finished; the server and the other jobs go on.
void fail_job(potts_server *s, std::unique_ptr<Job> jp, int code) {
  Job &j = *jp;
  (void)hipStreamSynchronize(s->stream);
  release_job_memory(j);
  s->used_bytes -= j.bytes;
  j.info.status = code;
  j.info.sweeps = j.t;
  j.info.t_done = seconds_since(s);
  std::lock_guard<std::mutex> lk(s->mu);
  s->running.erase(j.ticket);
  s->done_order.push_back(j.ticket);
  s->done[j.ticket] = std::move(jp);
  ++s->finished;
  s->cv_done.notify_all();
}

// Injected failures: a job whose next iteration would run its marked sweep
// fails now, before any of that iteration's work is queued.
void apply_faults(potts_server *s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto &jp : s->active) {
      auto it = s->faults.find(jp->ticket);
      if (it != s->faults.end()) {
        jp->fault_at = it->second;
        s->faults.erase(it);
      }
    }
  }
  std::vector<std::unique_ptr<Job>> keep;
  for (auto &jp : s->active) {
    Job &j = *jp;
    const int64_t step = std::min<int64_t>(s->cfg.quantum, j.left);
    if (j.fault_at >= 0 && j.fault_at < j.t + step)
      fail_job(s, std::move(jp), POTTS_EDEVICE);
    else
      keep.push_back(std::move(jp));
  }
  s->active.swap(keep);
}

// Writes the checkpoints of jobs that completed a point (not their last) in
// the last iteration.
int write_checkpoints(potts_server *s, std::string &err) {
  for (auto &jp : s->active) {
    Job &j = *jp;
    if (!j.ckpt_due) continue;
    j.ckpt_due = false;
    if (j.ckpt_path.empty() || j.left == 0) continue;
    std::vector<uint8_t> lat((size_t)j.req.L * j.req.L);
    hipError_t e = hipMemcpyAsync(lat.data(), j.lat, lat.size(), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
      err = std::string("checkpoint copy failed: ") + herr(e);
      return POTTS_EDEVICE;
    }
    if (!write_job_checkpoint(j, lat, err)) return POTTS_EIO;
  }
  return POTTS_OK;
}

// Finishes the jobs whose last point is done: final observables, optional
// spins, memory released.
int retire(potts_server *s, std::string &err) {
  std::vector<std::unique_ptr<Job>> keep;
  for (auto &jp : s->active) {
    Job &j = *jp;
    if (j.left > 0) {
      keep.push_back(std::move(jp));
      continue;
    }
    std::vector<int64_t> rec((size_t)j.req.q + 1, 0);
    hipError_t e = hipSuccess;
    if (j.t > 0)
      e = hipMemcpyAsync(rec.data(), j.ring + ((j.t - 1) & (j.cap - 1)) * (j.req.q + 1), rec.size() * 8,
                         hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && j.keep_spins) {
      j.spins.resize((size_t)j.req.L * j.req.L);
      e = hipMemcpyAsync(j.spins.data(), j.lat, j.spins.size(), hipMemcpyDeviceToHost, s->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) e = hipFreeAsync(j.lat, s->stream);
    if (e == hipSuccess) e = hipFreeAsync(j.ring, s->stream);
    if (e != hipSuccess) {
      err = std::string("retire failed: ") + herr(e);
      return POTTS_EDEVICE;
    }
    j.lat = nullptr;
    j.ring = nullptr;
    s->used_bytes -= j.bytes;
    j.info.e_sat = j.t > 0 ? rec[0] : 0;
    int64_t nmax = 0;
    for (int v = 0; v < j.req.q; ++v) nmax = std::max<int64_t>(nmax, rec[1 + v]);
    j.info.nmax = j.t > 0 ? nmax : 0;
    j.info.sweeps = j.t;
    j.info.t_done = seconds_since(s);
    j.info.status = POTTS_OK;
    std::lock_guard<std::mutex> lk(s->mu);
    s->running.erase(j.ticket);
    s->done_order.push_back(j.ticket);
    s->done[j.ticket] = std::move(jp);
    ++s->finished;
  }
  s->active.swap(keep);
  s->cv_done.notify_all();
  return POTTS_OK;
}

void fail_all(potts_server *s, int code, const std::string &msg) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->failed = code;
  s->fail_msg = msg;
  auto finish = [&](std::unique_ptr<Job> jp) {
    release_job_memory(*jp);
    jp->info.status = code;
    jp->info.t_done = seconds_since(s);
    s->done_order.push_back(jp->ticket);
    const int64_t t = jp->ticket;
    s->done[t] = std::move(jp);
    ++s->finished;
  };
  for (auto &jp : s->active) finish(std::move(jp));
  s->active.clear();
  s->running.clear();
  while (!s->queue.empty()) {
    finish(std::move(s->queue.front()));
    s->queue.pop_front();
  }
  s->cv_done.notify_all();
}

void server_loop(potts_server *s) {
  if (hipSetDevice(s->device) != hipSuccess) {
    fail_all(s, POTTS_EDEVICE, "hipSetDevice failed in the server thread");
    return;
  }
  for (;;) {
    // admission, in arrival order, by slots and HBM budget
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->active.empty())
        s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
      if (s->stop && s->queue.empty() && s->active.empty()) return;
      while (!s->queue.empty() && (int32_t)s->active.size() < s->cfg.max_slots) {
        Job &j = *s->queue.front();
        if (s->used_bytes + j.bytes > (size_t)s->cfg.hbm_budget && !s->active.empty()) break;
        std::unique_ptr<Job> jp = std::move(s->queue.front());
        s->queue.pop_front();
        lk.unlock();
        std::string err;
        if (!admit(s, *jp, err)) {
          fail_all(s, POTTS_ENOMEM, err);
          return;
        }
        s->used_bytes += jp->bytes;
        const int64_t ticket = jp->ticket;
        s->active.push_back(std::move(jp));
        lk.lock();
        s->running.insert(ticket);
      }
    }
    apply_faults(s);
    if (s->active.empty()) continue;
    std::string err;
    int rc = iterate(s, err);
    if (rc == POTTS_OK) rc = write_checkpoints(s, err);
    if (rc == POTTS_OK) rc = retire(s, err);
    if (rc != POTTS_OK) {
      fail_all(s, rc, err);
      return;
    }
  }
}

}  // namespace

extern "C" {

int potts_server_start(const potts_server_cfg *cfg, potts_server **out) {
  if (!out) return record_error(POTTS_EINVAL, "out is NULL");
  *out = nullptr;
  potts_server *s = new (std::nothrow) potts_server();
  if (!s) return record_error(POTTS_ENOMEM, "host allocation failed");
  if (cfg) s->cfg = *cfg;
  if (s->cfg.hbm_budget <= 0) s->cfg.hbm_budget = 200ll << 30;
  if (s->cfg.max_slots <= 0) s->cfg.max_slots = 256;
  if (s->cfg.quantum <= 0) s->cfg.quantum = 32;
  s->cache.load(s->cfg.tune_cache);
  s->cfg.tune_cache = nullptr;  // the path lives on in the cache
  if (s->cfg.hip_stream) {
    s->stream = (hipStream_t)s->cfg.hip_stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete s;
      return record_error(POTTS_EDEVICE, std::string("hipStreamCreateWithFlags: ") + herr(e));
    }
    s->owns_stream = true;
  }
  s->t0 = Clock::now();
  (void)hipGetDevice(&s->device);
  try {
    s->thread = std::thread(server_loop, s);
  } catch (...) {
    if (s->owns_stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return record_error(POTTS_ENOMEM, "cannot start the server thread");
  }
  *out = s;
  return POTTS_OK;
}

int potts_server_submit(potts_server *s, const potts_request *req, int64_t *ticket) {
  if (!s || !req || !ticket) return record_error(POTTS_EINVAL, "NULL argument");
  if (req->L < 16 || req->L % 16 || req->L > 65520 || req->q < 2 || req->q > POTTS_QMAX)
    return record_error(POTTS_EINVAL, "need L % 16 == 0, 16 <= L <= 65520, 2 <= q <= 256");
  if (req->start != POTTS_ORDERED && req->start != POTTS_RANDOM) return record_error(POTTS_EINVAL, "bad start");
  if (req->npoints < 1 || req->npoints > 4096 || !req->betas || !req->sweeps)
    return record_error(POTTS_EINVAL, "need 1 .. 4096 beta points with sweeps");
  std::unique_ptr<Job> j(new (std::nothrow) Job());
  if (!j) return record_error(POTTS_ENOMEM, "host allocation failed");
  j->req = *req;
  j->betas.assign(req->betas, req->betas + req->npoints);
  j->sweeps.assign(req->sweeps, req->sweeps + req->npoints);
  j->req.betas = nullptr;
  j->req.sweeps = nullptr;
  j->keep_spins = req->keep_spins != 0;
  j->thr.resize((size_t)req->npoints * 4);
  int64_t most = 1;
  for (int32_t k = 0; k < req->npoints; ++k) {
    if (j->sweeps[k] < 1 || j->sweeps[k] > (1ll << 30))
      return record_error(POTTS_EINVAL, "every point needs 1 .. 2^30 sweeps");
    int rc = potts::build_threshold_table(j->betas[k], &j->thr[(size_t)k * 4]);
    if (rc) return rc;
    most = std::max<int64_t>(most, j->sweeps[k]);
  }
  j->points.assign(req->npoints, potts_summary{});
  if (req->checkpoint) j->ckpt_path = req->checkpoint;
  j->req.checkpoint = nullptr;
  j->req.resume_from = nullptr;
  if (req->resume_from) {
    int rc = read_job_checkpoint(*j, req->resume_from);
    if (rc) return rc;
  }
  j->cap = pow2_at_least(most + 1);
  j->bytes = job_bytes(*j);
  j->info.L = req->L;
  j->info.q = req->q;
  j->info.npoints = req->npoints;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->failed) return record_error(s->failed, "server failed: " + s->fail_msg);
  if (s->stop) return record_error(POTTS_EINVAL, "server is stopping");
  if (j->bytes > (size_t)s->cfg.hbm_budget) return record_error(POTTS_ENOMEM, "job exceeds the HBM budget");
  j->ticket = s->next_ticket++;
  j->info.ticket = j->ticket;
  if (s->fault_next >= 0) {
    j->fault_at = s->fault_next;  // attached before the server thread can see the job
    s->fault_next = -1;
  }
  j->info.t_submit = seconds_since(s);
  *ticket = j->ticket;
  s->queue.push_back(std::move(j));
  ++s->submitted;
  s->cv_work.notify_one();
  return POTTS_OK;
}

int potts_server_wait(potts_server *s, int64_t *tickets, int32_t max, int32_t timeout_ms, int32_t *n) {
  if (!s || !n || (max > 0 && !tickets)) return record_error(POTTS_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done_order.empty() && timeout_ms != 0) {
    auto pred = [&] { return !s->done_order.empty() || s->finished == s->submitted; };
    if (timeout_ms < 0)
      s->cv_done.wait(lk, pred);
    else
      s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred);
  }
  int32_t k = 0;
  while (k < max && !s->done_order.empty()) {
    tickets[k++] = s->done_order.front();
    s->done_order.erase(s->done_order.begin());
  }
  *n = k;
  return POTTS_OK;
}

int potts_server_collect(potts_server *s, int64_t ticket, potts_served *info, potts_summary *points,
                         uint8_t *spins) {
  if (!s || !info) return record_error(POTTS_EINVAL, "NULL argument");
  std::unique_ptr<Job> j;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->done.find(ticket);
    if (it == s->done.end()) return record_error(POTTS_ERANGE, "ticket not finished or already collected");
    j = std::move(it->second);
    s->done.erase(it);
  }
  *info = j->info;
  if (points) memcpy(points, j->points.data(), j->points.size() * sizeof(potts_summary));
  if (spins && !j->spins.empty()) memcpy(spins, j->spins.data(), j->spins.size());
  return j->info.status;
}

int potts_server_inject_fault(potts_server *s, int64_t ticket, int64_t at_sweep) {
  if (!s || at_sweep < 0) return record_error(POTTS_EINVAL, "need a server and at_sweep >= 0");
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticket == 0) {
    s->fault_next = at_sweep;
    return POTTS_OK;
  }
  for (auto &jp : s->queue)
    if (jp->ticket == ticket) {
      jp->fault_at = at_sweep;
      return POTTS_OK;
    }
  if (!s->running.count(ticket)) return record_error(POTTS_ERANGE, "no unfinished job with this ticket");
  s->faults[ticket] = at_sweep;  // an active job: picked up by the server thread
  return POTTS_OK;
}

int potts_server_drain(potts_server *s, int32_t timeout_ms) {
  if (!s) return record_error(POTTS_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto pred = [&] { return s->finished == s->submitted; };
  if (timeout_ms < 0)
    s->cv_done.wait(lk, pred);
  else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred))
    return record_error(POTTS_ERANGE, "drain timed out");
  return s->failed ? record_error(s->failed, "server failed: " + s->fail_msg) : POTTS_OK;
}

double potts_server_now(const potts_server *s) { return s ? seconds_since(s) : -1.0; }

int64_t potts_server_iterations(const potts_server *s) { return s ? s->iterations : -1; }

int potts_server_tuning(potts_server *s, char *out, int32_t cap) {
  if (!s || !out || cap < 1) return record_error(POTTS_EINVAL, "NULL argument or cap < 1");
  std::lock_guard<std::mutex> lk(s->mu);
  // entries are "<cache key>:<choice>"; those this server did not time
  // itself come from its cache file
  std::string text = s->tuned;
  const auto timed_here = [&](const std::string &key) {
    return (" " + s->tuned).find(" " + key + ":") != std::string::npos;
  };
  for (const auto &kv : s->cache.rows)
    if (!timed_here(kv.first)) text += kv.first + ":rows=" + std::to_string(kv.second) + "(cached) ";
  for (const auto &kv : s->cache.shapes)
    if (!timed_here(kv.first)) text += kv.first + ":" + shape_text(kv.second) + "(cached) ";
  const size_t n = std::min<size_t>(text.size(), (size_t)cap - 1);
  memcpy(out, text.data(), n);
  out[n] = 0;
  return POTTS_OK;
}

int potts_server_stop(potts_server *s) {
  if (!s) return POTTS_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->thread.joinable()) s->thread.join();
  const int rc = s->failed;
  (void)hipStreamSynchronize(s->stream);
  for (void *p : {(void *)s->d_strip, (void *)s->d_tiles, (void *)s->d_res, (void *)s->d_stats})
    if (p) (void)hipFree(p);
  if (s->h_stage) (void)hipHostFree(s->h_stage);
  if (s->owns_stream) (void)hipStreamDestroy(s->stream);
  delete s;
  return rc;
}

}  // extern "C"
