// stats.hip -- derived observables of a window of per-sweep records, computed
// on the device with exact integer moments and one FP64 evaluation at the end.
//
// For records {e_sat_t, hist_t} of n sweeps on N sites with q states:
//   S1 = sum e,  S2 = sum e^2,  S4 = sum e^4          (H = -e, Eq. 1)
//   M1 = sum (q nmax - N),  M2 = sum (q nmax - N)^2   (m = (q nmax/N - 1)/(q-1), Eq. 7)
// With e <= 2N <= 2^33 and windows of at most 2^24 records, S1 and M1 fit in
// int64, S2 and M2 in 128 bits and S4 in 256 bits.  The moments are exact, so the
// large cancellations in <H^2> - <H>^2 cost nothing.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace potts {
namespace {

typedef unsigned __int128 u128;

struct U256 {
  u128 lo, hi;
};

__device__ __forceinline__ void add256(U256 &a, const U256 &b) {
  const u128 lo = a.lo + b.lo;
  a.hi += b.hi + (lo < a.lo ? 1 : 0);
  a.lo = lo;
}

// Full 128 x 128 -> 256-bit product (schoolbook on 64-bit limbs).
__device__ __forceinline__ U256 mul256(u128 a, u128 b) {
  const uint64_t a0 = (uint64_t)a, a1 = (uint64_t)(a >> 64);
  const uint64_t b0 = (uint64_t)b, b1 = (uint64_t)(b >> 64);
  const u128 p00 = (u128)a0 * b0, p01 = (u128)a0 * b1, p10 = (u128)a1 * b0, p11 = (u128)a1 * b1;
  const u128 mid = p01 + p10;
  const u128 mid_carry = mid < p01 ? 1 : 0;  // worth 2^192
  U256 r;
  r.lo = p00 + (mid << 64);
  const u128 lo_carry = r.lo < p00 ? 1 : 0;
  r.hi = p11 + (mid >> 64) + lo_carry + (mid_carry << 64);
  return r;
}

struct Partial {
  int64_t s1;
  u128 s2;
  U256 s4;
  u128 m1;
  u128 m2;
};

__device__ __forceinline__ void add_partial(Partial &a, const Partial &b) {
  a.s1 += b.s1;
  a.s2 += b.s2;
  add256(a.s4, b.s4);
  a.m1 += b.m1;
  a.m2 += b.m2;
}

__device__ double u128_to_double(u128 v) {
  return (double)(uint64_t)(v >> 64) * 18446744073709551616.0 + (double)(uint64_t)v;
}

__device__ double u256_to_double(const U256 &v) {
  return u128_to_double(v.hi) * 340282366920938463463374607431768211456.0 + u128_to_double(v.lo);
}

// a - b for a >= b
__device__ __forceinline__ U256 sub256(const U256 &a, const U256 &b) {
  U256 r;
  r.lo = a.lo - b.lo;
  r.hi = a.hi - b.hi - (a.lo < b.lo ? 1 : 0);
  return r;
}

constexpr int kStatsBlock = 256;

__global__ __launch_bounds__(kStatsBlock) void stats_kernel(StatsParams single, const StatsParams *many) {
  const StatsParams p = many ? many[blockIdx.x] : single;
  __shared__ Partial part[kStatsBlock];
  Partial acc = {};
  for (int64_t i = threadIdx.x; i < p.n; i += kStatsBlock) {
    const int64_t slot = (p.slot0 + i) & (p.cap - 1);
    const unsigned long long *rec = p.ring + slot * (int64_t)(p.q + 1);
    const uint64_t e = rec[0];
    uint64_t nmax = 0;
    for (uint32_t v = 0; v < p.q; ++v) nmax = rec[1 + v] > nmax ? rec[1 + v] : nmax;
    // e <= 2N <= 2^33: e^2 needs 67 bits and e^4 up to 133
    const u128 e2 = (u128)e * e;
    acc.s1 += (int64_t)e;
    acc.s2 += e2;
    add256(acc.s4, mul256(e2, e2));
    const uint64_t dm = (uint64_t)p.q * nmax - p.N;  // >= 0, below 2^40
    acc.m1 += dm;
    acc.m2 += (u128)dm * dm;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kStatsBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) add_partial(part[threadIdx.x], part[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const Partial s = part[0];
  const double n = (double)p.n, N = (double)p.N, q1 = (double)(p.q - 1);
  // e = <H>/N = -S1/(n N)
  const double e = -(double)s.s1 / (n * N);
  // C = beta^2 (n S2 - S1^2) / (n^2 N): exact integer numerator (>= 0, below 2^116)
  const u128 varnum = (u128)p.n * s.s2 - (u128)s.s1 * (u128)s.s1;
  const double heat = p.beta * p.beta * (u128_to_double(varnum) / (n * n * N));
  // V_L = 1 - n S4 / (3 S2^2)
  const double s2d = u128_to_double(s.s2);
  const double vl = s.s2 == 0 ? 0.0 : 1.0 - n * u256_to_double(s.s4) / (3.0 * s2d * s2d);
  // <m> = M1 / (n N (q-1)); chi = N beta (<m^2> - <m>^2) = beta (n M2 - M1^2) / (n^2 N (q-1)^2)
  // (M1 can reach 2^64 and n M2 2^128, so this numerator is taken in 256 bits)
  const double m = u128_to_double(s.m1) / (n * N * q1);
  const U256 mvar = sub256(mul256((u128)p.n, s.m2), mul256(s.m1, s.m1));
  const double chi = p.beta * (u256_to_double(mvar) / (n * n * N * q1 * q1));
  p.out[0] = e;
  p.out[1] = heat;
  p.out[2] = vl;
  p.out[3] = m;
  p.out[4] = chi;
}

// Reweighting (Sec. 7 names the method: Ferrenberg-Swendsen single-histogram
// reweighting).  Record t of the window gets the weight
// w_t = exp((beta - beta0) (e_t - e_ref)), with e_ref the extreme of the
// window that makes every exponent <= 0 (a common factor, so the averages do
// not change and nothing overflows).  Moments are taken of the shifted
// integers d = e - e_ref and u = M - M_min (M = q nmax - N), so the variances
// lose no digits to cancellation; <E^2> and <E^4> are rebuilt from them.
__global__ __launch_bounds__(kStatsBlock) void reweight_kernel(ReweightParams p) {
  __shared__ int64_t ext[3][kStatsBlock];
  __shared__ double sums[7][kStatsBlock];
  const double beta = p.betas[blockIdx.x];
  const double db = beta - p.beta0;
  const uint32_t tid = threadIdx.x;
  int64_t emin = INT64_MAX, emax = INT64_MIN, mmin = INT64_MAX;
  for (int64_t i = tid; i < p.n; i += kStatsBlock) {
    const unsigned long long *rec = p.ring + ((p.slot0 + i) & (p.cap - 1)) * (int64_t)(p.q + 1);
    uint64_t nmax = 0;
    for (uint32_t v = 0; v < p.q; ++v) nmax = rec[1 + v] > nmax ? rec[1 + v] : nmax;
    const int64_t e = (int64_t)rec[0];
    const int64_t m = (int64_t)p.q * (int64_t)nmax - (int64_t)p.N;
    emin = e < emin ? e : emin;
    emax = e > emax ? e : emax;
    mmin = m < mmin ? m : mmin;
  }
  ext[0][tid] = emin;
  ext[1][tid] = emax;
  ext[2][tid] = mmin;
  __syncthreads();
  for (uint32_t off = kStatsBlock / 2; off > 0; off >>= 1) {
    if (tid < off) {
      ext[0][tid] = ext[0][tid + off] < ext[0][tid] ? ext[0][tid + off] : ext[0][tid];
      ext[1][tid] = ext[1][tid + off] > ext[1][tid] ? ext[1][tid + off] : ext[1][tid];
      ext[2][tid] = ext[2][tid + off] < ext[2][tid] ? ext[2][tid + off] : ext[2][tid];
    }
    __syncthreads();
  }
  const int64_t eref = db > 0.0 ? ext[1][0] : ext[0][0];
  const int64_t mref = ext[2][0];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};  // W, d, d^2, d^3, d^4, u, u^2 (weighted)
  for (int64_t i = tid; i < p.n; i += kStatsBlock) {
    const unsigned long long *rec = p.ring + ((p.slot0 + i) & (p.cap - 1)) * (int64_t)(p.q + 1);
    uint64_t nmax = 0;
    for (uint32_t v = 0; v < p.q; ++v) nmax = rec[1 + v] > nmax ? rec[1 + v] : nmax;
    const double d = (double)((int64_t)rec[0] - eref);
    const double u = (double)((int64_t)p.q * (int64_t)nmax - (int64_t)p.N - mref);
    const double w = exp(db * d);
    const double wd = w * d, wd2 = wd * d;
    acc[0] += w;
    acc[1] += wd;
    acc[2] += wd2;
    acc[3] += wd2 * d;
    acc[4] += wd2 * d * d;
    acc[5] += w * u;
    acc[6] += w * u * u;
  }
  for (int k = 0; k < 7; ++k) sums[k][tid] = acc[k];
  __syncthreads();
  for (uint32_t off = kStatsBlock / 2; off > 0; off >>= 1) {
    if (tid < off)
      for (int k = 0; k < 7; ++k) sums[k][tid] += sums[k][tid + off];
    __syncthreads();
  }
  if (tid != 0) return;
  const double W = sums[0][0];
  const double D1 = sums[1][0] / W, D2 = sums[2][0] / W, D3 = sums[3][0] / W, D4 = sums[4][0] / W;
  const double U1 = sums[5][0] / W, U2 = sums[6][0] / W;
  const double N = (double)p.N, q1 = (double)(p.q - 1), r = (double)eref;
  const double e1 = r + D1;
  const double e2 = r * r + 2.0 * r * D1 + D2;
  const double e4 = r * r * r * r + 4.0 * r * r * r * D1 + 6.0 * r * r * D2 + 4.0 * r * D3 + D4;
  double *out = p.out + 5 * blockIdx.x;
  out[0] = -e1 / N;
  out[1] = beta * beta * (D2 - D1 * D1) / N;
  out[2] = e2 == 0.0 ? 0.0 : 1.0 - e4 / (3.0 * e2 * e2);
  out[3] = ((double)mref + U1) / (N * q1);
  out[4] = beta * (U2 - U1 * U1) / (N * q1 * q1);
}

// Sum of the records of n sweeps over G slab rings stored one after another
// (ring g at rings + g * slots * width): one thread per output word.
__global__ __launch_bounds__(256) void slab_fold_kernel(const unsigned long long *rings, uint32_t nslabs,
                                                        uint64_t slots, uint32_t width, uint64_t t0, uint64_t n,
                                                        unsigned long long *out) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n * width) return;
  const uint64_t r = i / width, w = i - r * width;
  const uint64_t at = ((t0 + r) & (slots - 1)) * width + w;
  unsigned long long sum = 0;
  for (uint32_t g = 0; g < nslabs; ++g) sum += rings[g * slots * width + at];
  out[i] = sum;
}

}  // namespace

hipError_t launch_slab_fold(const unsigned long long *rings, uint32_t nslabs, uint64_t slots, uint32_t width,
                            uint64_t t0, uint64_t n, unsigned long long *out, hipStream_t stream) {
  const uint64_t total = n * width;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(slab_fold_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, rings, nslabs,
                     slots, width, t0, n, out);
  return hipGetLastError();
}

hipError_t launch_reweight(const ReweightParams &p, unsigned npoints, hipStream_t stream) {
  if (npoints == 0) return hipSuccess;
  hipLaunchKernelGGL(reweight_kernel, dim3(npoints), dim3(kStatsBlock), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_stats(const StatsParams &p, hipStream_t stream) {
  hipLaunchKernelGGL(stats_kernel, dim3(1), dim3(kStatsBlock), 0, stream, p, (const StatsParams *)nullptr);
  return hipGetLastError();
}

hipError_t launch_stats_many(const StatsParams *dev_params, unsigned n, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(stats_kernel, dim3(n), dim3(kStatsBlock), 0, stream, StatsParams{}, dev_params);
  return hipGetLastError();
}

}  // namespace potts
