// Independent Philox4x32-10 reference for the oracle's pin: PyTorch's header-only
// engine (ATen/core/PhiloxRNGEngine.h), called, not copied.  Reads lines
// "c0 c1 c2 c3 k0 k1" (decimal) from stdin, prints the four output words.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cinttypes>
#include <cstdio>

int main() {
  unsigned long long c[4], k[2];
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
    const uint64_t seed = (uint64_t)k[0] | ((uint64_t)k[1] << 32);
    const uint64_t subsequence = (uint64_t)c[2] | ((uint64_t)c[3] << 32);
    const uint64_t offset = (uint64_t)c[0] | ((uint64_t)c[1] << 32);
    // the engine keeps the counter as (offset_lo, offset_hi, subseq_lo, subseq_hi)
    at::Philox4_32 engine(seed, subsequence, offset);
    uint32_t w[4];
    for (int i = 0; i < 4; ++i) w[i] = engine();
    std::printf("%" PRIu32 " %" PRIu32 " %" PRIu32 " %" PRIu32 "\n", w[0], w[1], w[2], w[3]);
  }
  return 0;
}
