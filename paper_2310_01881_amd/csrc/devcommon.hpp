// devcommon.hpp -- small device helpers shared by the library's kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace amn {

// splitmix64 (Steele, Lea and Flood, OOPSLA 2014), used as a counter-based generator for
// the per-interval stratum offsets.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Offset u in [0,1) of the samples of interval k of ray `ray` (global ray index):
// 1/2 for centred strata, else the top 24 bits of the hash scaled by 2^-24 (exact).
__device__ __forceinline__ float stratum_u(int jitter, uint64_t seed, uint64_t ray, uint32_t k) {
  if (!jitter) return 0.5f;
  uint64_t h = splitmix64(seed ^ (ray * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)k * 0xD1B54A32D192ED03ull));
  return (float)(uint32_t)(h >> 40) * (1.0f / 16777216.0f);
}

// Position of sample j of an interval starting at t0 with segment length delta.
__device__ __forceinline__ float sample_t(float t0, float delta, uint32_t j, float u) {
  return fmaf((float)j + u, delta, t0);
}

// Interval key: leaf slot in the low 16 bits, samples per interval in the high 16 bits.
__device__ __forceinline__ uint32_t key_slot(uint32_t key) { return key & 0xFFFFu; }
__device__ __forceinline__ uint32_t key_n(uint32_t key) { return key >> 16; }

}  // namespace amn
