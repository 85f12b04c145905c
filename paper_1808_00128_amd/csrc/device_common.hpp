// Device helpers: wave-level GF(2) primitives and the counter-based generator.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace chsim {

__device__ __forceinline__ uint32_t par64(uint64_t x) { return (uint32_t)__popcll(x) & 1u; }

// Broadcast lane `src` (wave-uniform) of a 64-bit per-lane value.
__device__ __forceinline__ uint64_t rl64(uint64_t x, uint32_t src) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, (int)src);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), (int)src);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t rl32(uint32_t x, uint32_t src) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, (int)src);
}
__device__ __forceinline__ uint32_t uniform32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}
// Mask of lanes where pred holds (64-bit wave).
__device__ __forceinline__ uint64_t ballot64(bool pred) { return (uint64_t)__ballot(pred); }

// All-ones if bit i of x is set, else 0.
__device__ __forceinline__ uint64_t bitmask64(uint64_t x, uint32_t i) {
  return (uint64_t)0 - ((x >> i) & 1ull);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of
// (hi(M0 c0) ^ c1 ^ k0, lo(M1 c2), hi(M1 c2) ^ c3 ^ k1, lo(M0 c0)) with the
// key advanced by the Weyl increments between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint32_t lo0 = 0xD2511F53u * c0;
    uint32_t hi0 = __umulhi(0xD2511F53u, c0);
    uint32_t lo1 = 0xCD9E8D57u * c2;
    uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// 53-bit uniform in [0, 1) from the first two words: (w0 << 21) | (w1 >> 11).
__device__ __forceinline__ double philox_uniform53(uint64_t seed, uint64_t index, uint32_t sub,
                                                   uint32_t stream) {
  uint32_t w[4];
  philox4x32_10((uint32_t)index, (uint32_t)(index >> 32), sub, stream, (uint32_t)seed,
                (uint32_t)(seed >> 32), w);
  uint64_t bits = ((uint64_t)w[0] << 21) | (uint64_t)(w[1] >> 11);
  return (double)bits * (1.0 / 9007199254740992.0);
}

constexpr uint32_t kStreamSparsify = 0x53504152u;

}  // namespace chsim
