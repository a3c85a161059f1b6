// noalloc.hip -- potts_sweep_static: Metropolis sweeps of a caller-owned
// row-major lattice that allocate no device memory.
//
// The sweeps are those of potts_sweep_thr on the row-major strip kernel
// (strip.hip): same launches, same records.  The only device memory beyond
// the caller's lattice and record buffer is the strip kernel's striped
// partial records, which live in a file-scope device array (`scratch`), one
// copy per GPU for the life of the process.  Its device address is looked up
// once per device (hipGetSymbolAddress with that device current) and only
// that address is handed to kernels and fills: in host code the array's name
// is not a device pointer.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <mutex>
#include <string>

#include "../../include/potts.h"
#include "kernels.hpp"

namespace potts {
int record_error(int code, const std::string &msg);  // capi.hip
}  // namespace potts

namespace {

// two stripe sets (by sweep parity) of kStripes partial records of
// stripe_words(q) words each; stripe_words(256) = 272
constexpr uint32_t kStripes = 32;
constexpr uint64_t kScratchWords = 2ull * kStripes * 272ull;
static_assert(((POTTS_QMAX + 1 + 15) & ~15) == 272, "scratch sized for q <= 256");

static __device__ __align__(256) unsigned long long scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long *g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

int fail(int code, const std::string &msg) { return potts::record_error(code, msg); }

int hip_fail(hipError_t e, const char *what) {
  return fail(POTTS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// The device address of this GPU's copy of `scratch` (dev must be current).
int scratch_address(int dev, unsigned long long **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(POTTS_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(POTTS_EDEVICE, "hipGetSymbolAddress(scratch) gave a null address");
    g_scratch_ptr[dev] = static_cast<unsigned long long *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return POTTS_OK;
}

// rows per strip item, as the single-lattice strip path picks them: 32 when
// that still gives 2048 x 256 items, else 16
uint32_t strip_rows(uint32_t L) {
  return L % 32 == 0 && (uint64_t)(L / 32) * (L / 16) >= 2048ull * 256ull ? 32u : 16u;
}

}  // namespace

extern "C" int potts_sweep_static(uint8_t *dev_spins, int32_t L, int32_t q, uint64_t seed, int64_t t0,
                                  const uint32_t thr[4], int64_t nsweeps, int64_t *dev_records,
                                  void *hip_stream) {
  if (!dev_spins || !thr) return fail(POTTS_EINVAL, "dev_spins or thr is NULL");
  if (L < 16 || L % 16 || L > 65520 || q < 2 || q > POTTS_QMAX)
    return fail(POTTS_EINVAL, "need L % 16 == 0, 16 <= L <= 65520, 2 <= q <= 256");
  if (nsweeps < 0 || t0 < 0) return fail(POTTS_EINVAL, "nsweeps and t0 must be >= 0");
  if (nsweeps > 0 && !dev_records) return fail(POTTS_EINVAL, "dev_records is NULL");
  if (nsweeps > INT64_MAX - t0) return fail(POTTS_ERANGE, "sweep counter overflow");
  const uint64_t words = 2ull * kStripes * potts::stripe_words((uint32_t)q);
  if (words > kScratchWords)
    return fail(POTTS_ERANGE, "the partial records need more than the static scratch holds");
  if (nsweeps == 0) return POTTS_OK;

  const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (stream) {
    int sdev = 0;
    e = hipStreamGetDevice(stream, &sdev);
    if (e != hipSuccess) return hip_fail(e, "hipStreamGetDevice");
    if (sdev != dev) return fail(POTTS_EINVAL, "hip_stream belongs to another device than the current one");
  }
  unsigned long long *stripes = nullptr;
  const int rc = scratch_address(dev, &stripes);
  if (rc) return rc;

  potts::StripLaunch l{};
  potts::StripParams &p = l.single;
  potts::fill_strip_params(p, dev_spins, (uint32_t)L, (uint32_t)q, seed, thr, strip_rows((uint32_t)L));
  p.nsweeps = (uint64_t)nsweeps;
  // the record of sweep t is written to ring + (t mod cap) (1+q) words; with
  // cap = 2^63 > t and the ring placed t0 records before dev_records (modular
  // address arithmetic), record t lands at dev_records + (t - t0)(1+q)
  p.cap = 1ull << 63;
  p.ring = reinterpret_cast<unsigned long long *>(reinterpret_cast<uintptr_t>(dev_records) -
                                                  (uintptr_t)t0 * (uintptr_t)(q + 1) * sizeof(int64_t));
  p.stripes = stripes;
  p.nstripes = kStripes;
  // a previous call may have stopped between a sweep and its fold: the
  // partial records start from zero (a fill kernel, no memset node)
  e = potts::launch_fill_u64(stripes, words, 0ull, stream);
  if (e != hipSuccess) return hip_fail(e, "launch_fill_u64");
  const uint64_t need = ((uint64_t)p.nitems + 255) / 256;
  const unsigned grid = (unsigned)(need < 8192 ? need : 8192);
  const bool wide = !thr[0] || !thr[1] || !thr[2] || !thr[3];
  // segments of at most 2^30 sweeps keep the launch's sweep index in 32 bits
  const int64_t seg = 1ll << 30;
  for (int64_t base = 0; base < nsweeps; base += seg) {
    const int64_t count = nsweeps - base < seg ? nsweeps - base : seg;
    p.t0 = (uint64_t)(t0 + base);
    for (int64_t j = 0; j < count; ++j) {
      l.sweep = (uint32_t)j;
      e = potts::launch_strip(l, 0, grid, p.q, wide, stream);
      if (e == hipSuccess) e = potts::launch_strip(l, 1, grid, p.q, wide, stream);
      if (e != hipSuccess) return hip_fail(e, "launch_strip");
    }
    // the segment's last sweep: no later colour-0 launch folds its records
    e = potts::launch_fold_stripes(p, p.t0 + (uint64_t)count - 1, stream);
    if (e != hipSuccess) return hip_fail(e, "launch_fold_stripes");
  }
  return POTTS_OK;
}
