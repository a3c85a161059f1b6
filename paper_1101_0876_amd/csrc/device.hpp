// device.hpp -- gfx950 device helpers for the Potts sweep kernels.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) written for CDNA4: the
// 32x32->64 products issue as v_mad_u64_u32 at full rate, and the two
// three-input XORs of each round use gfx950's v_bitop3_b32 (truth table 0x96),
// which halves the XOR count the compiler would otherwise emit.  The key is
// wave-uniform, so its Weyl increments stay on the scalar unit.
//
// SWAR byte helpers treat a dword as four uint8 spins.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace potts {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kWeyl0 = 0x9E3779B9u;
constexpr uint32_t kWeyl1 = 0xBB67AE85u;

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

struct Words {
  uint32_t w0, w1, w2, w3;
};

// Ten rounds; round r uses key (k0 + r*W0, k1 + r*W1).  The first round is
// split off: PhiloxHead holds its outputs for counter words 0, 2, 3 and key
// (k0, k1), with output word 0 still missing the XOR of counter word 1.  The
// sweep kernels put the per-lane chunk index in word 1 and the sweep and
// colour in words 0, 2, 3, so the head is wave-uniform (scalar unit) and each
// block costs one XOR plus nine rounds of vector work.
struct PhiloxHead {
  uint32_t a0, x1, x2, x3;  // round-1 outputs (a0 before ^ counter word 1)
  uint32_t k0, k1;          // key of round 2
};

__device__ __forceinline__ PhiloxHead philox_head(uint32_t c0, uint32_t c2, uint32_t c3, uint32_t k0,
                                                  uint32_t k1) {
  const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
  const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
  return PhiloxHead{(uint32_t)(p1 >> 32) ^ k0, (uint32_t)p1, xor3((uint32_t)(p0 >> 32), c3, k1),
                    (uint32_t)p0, k0 + kWeyl0, k1 + kWeyl1};
}

// Rounds 2..10 from the head and x0 = h.a0 ^ counter word 1.
__device__ __forceinline__ Words philox_tail(uint32_t x0, const PhiloxHead &h) {
  uint32_t c0 = x0, c1 = h.x1, c2 = h.x2, c3 = h.x3, k0 = h.k0, k1 = h.k1;
#pragma unroll
  for (int r = 1; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
  return Words{c0, c1, c2, c3};
}

__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
  const PhiloxHead h = philox_head(c0, c2, c3, k0, k1);
  return philox_tail(h.a0 ^ c1, h);
}

// floor(w * q / 2^32): a 32-bit word onto 0..q-1.
__device__ __forceinline__ uint32_t scale_to_q(uint32_t w, uint32_t q) { return __umulhi(w, q); }

// 0x80 in every byte of x that is zero, 0 elsewhere (exact, no carries across bytes).
__device__ __forceinline__ uint32_t zero_bytes(uint32_t x) {
  const uint32_t t = (x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
  return ~(t | x) & 0x80808080u;
}

// Per-byte count (0..4) of the four neighbour dwords equal to v, bytewise.
__device__ __forceinline__ uint32_t count_equal(uint32_t v, uint32_t a, uint32_t b, uint32_t c,
                                                uint32_t d) {
  return (zero_bytes(v ^ a) >> 7) + (zero_bytes(v ^ b) >> 7) + (zero_bytes(v ^ c) >> 7) +
         (zero_bytes(v ^ d) >> 7);
}

__device__ __forceinline__ uint32_t byte_of(uint32_t x, uint32_t i) { return (x >> (8u * i)) & 0xFFu; }

// Wave64 sum, the same total in every lane: adds within each row of 16 lanes
// by DPP (two quad permutations, then the half-row and row mirrors) and reads
// the four row sums out, instead of six shuffles with an LDS round trip each
// (they sat on the critical path of the kernels that reduce a record every
// sweep).  Needs the whole wave active: every caller reduces after its work
// loop, outside any lane-dependent branch.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);  // row_mirror
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) + (uint32_t)__builtin_amdgcn_readlane((int)v, 16) +
         (uint32_t)__builtin_amdgcn_readlane((int)v, 32) + (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

}  // namespace potts
