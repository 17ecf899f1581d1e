// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) and the Box-Muller
// transform on the device: the counter-based words behind the residual noise
// of Alg. 2 and the inputs drawn from a seed.  Key = (seed mod 2^32,
// seed >> 32); ten rounds, each multiplying counter words 0 and 2 by
// 0xD2511F53 and 0xCD9E8D57 and mixing the product halves with the other
// words and the round key, the key bumped by the Weyl constants between
// rounds.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace rpt {
namespace {

// a ^ b ^ k in one instruction: gfx950's three-input bitwise op with the XOR
// truth table (0x96); the compiler emits two v_xor_b32 for it.  The round key
// k is uniform and goes in as the one scalar operand.
__device__ __forceinline__ unsigned xor3(unsigned a, unsigned b, unsigned k) {
  unsigned r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}

// NC independent counters advanced round by round together, so that the
// dependent product -> xor chain of one call overlaps the others'
template <int NC>
__device__ __forceinline__ void philox4x32_10_n(unsigned (&c)[NC][4], unsigned k0, unsigned k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c[q][0];
      const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c[q][2];
      const unsigned lo0 = static_cast<unsigned>(p0), hi0 = static_cast<unsigned>(p0 >> 32);
      const unsigned lo1 = static_cast<unsigned>(p1), hi1 = static_cast<unsigned>(p1 >> 32);
      const unsigned n0 = xor3(hi1, c[q][1], k0), n2 = xor3(hi0, c[q][3], k1);
      c[q][0] = n0;
      c[q][1] = lo1;
      c[q][2] = n2;
      c[q][3] = lo0;
    }
  }
}

__device__ __forceinline__ void philox4x32_10(unsigned c[4], unsigned k0, unsigned k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c[0];
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c[2];
    const unsigned lo0 = static_cast<unsigned>(p0), hi0 = static_cast<unsigned>(p0 >> 32);
    const unsigned lo1 = static_cast<unsigned>(p1), hi1 = static_cast<unsigned>(p1 >> 32);
    const unsigned n0 = xor3(hi1, c[1], k0), n2 = xor3(hi0, c[3], k1);
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Box-Muller on the hardware transcendental units: v_log_f32 is log2,
// v_sin_f32 / v_cos_f32 take their argument in revolutions (sin(2 pi x)), the
// exact form the transform needs; u lies in (0, 1).
// u = ((x >> 8) + 1/2) 2^-24 as one FMA: scaling by 2^-24 commutes with the
// single rounding, so this equals rounding the sum and then scaling
__device__ __forceinline__ float unif24(unsigned x) {
  return fmaf(static_cast<float>(x >> 8), 5.9604644775390625e-08f, 2.98023223876953125e-08f);  // 2^-24, 2^-25
}
__device__ __forceinline__ float bm_radius(unsigned x) {
  return __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(unif24(x)));  // -2 ln 2 log2(u)
}
__device__ __forceinline__ float bm_turns(unsigned x) { return unif24(x); }

// z(seed, stream, col, vox): counter (vox, col >> 2, stream, study); column
// col & 3 selects the word pair (0,1) or (2,3) and cos or sin.
__device__ __forceinline__ float noise_z(uint64_t seed, unsigned stream, unsigned col, int64_t vox, unsigned study) {
  unsigned c[4] = {static_cast<unsigned>(vox), col >> 2, stream, study};
  philox4x32_10(c, static_cast<unsigned>(seed), static_cast<unsigned>(seed >> 32));
  const int lane4 = static_cast<int>(col & 3);
  const unsigned xa = lane4 < 2 ? c[0] : c[2];
  const unsigned xb = lane4 < 2 ? c[1] : c[3];
  const float t = bm_turns(xb);
  return bm_radius(xa) * ((lane4 & 1) ? __builtin_amdgcn_sinf(t) : __builtin_amdgcn_cosf(t));
}

}  // namespace
}  // namespace rpt
