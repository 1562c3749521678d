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

// Lane shift within the wave's data-parallel-primitive network: lanes whose source is
// outside the selected rows (or whose row is masked off) read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_or_zero(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

// Inclusive prefix sum over the 64 lanes of a wave: shifts by 1, 2, 4, 8 within rows of
// 16 lanes, then the last lane of row 0 (2) is added to row 1 (3) and the last lane of
// row 1 to rows 2 and 3.  The association order is fixed, so results are reproducible.
__device__ __forceinline__ float wave_scan_incl(float v) {
  v += dpp_or_zero<0x111, 0xF>(v);   // row_shr:1
  v += dpp_or_zero<0x112, 0xF>(v);   // row_shr:2
  v += dpp_or_zero<0x114, 0xF>(v);   // row_shr:4
  v += dpp_or_zero<0x118, 0xF>(v);   // row_shr:8
  v += dpp_or_zero<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_or_zero<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

// Prefix maximum over the 64 lanes of a wave (signed), on the same lane-shift pattern as
// wave_scan_incl; lanes outside the pattern contribute INT32_MIN.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_or_min(int v) {
  return __builtin_amdgcn_update_dpp((int)0x80000000, v, CTRL, ROW_MASK, 0xF, false);
}
__device__ __forceinline__ int wave_max_incl(int v) {
  v = max(v, dpp_or_min<0x111, 0xF>(v));
  v = max(v, dpp_or_min<0x112, 0xF>(v));
  v = max(v, dpp_or_min<0x114, 0xF>(v));
  v = max(v, dpp_or_min<0x118, 0xF>(v));
  v = max(v, dpp_or_min<0x142, 0xA>(v));
  v = max(v, dpp_or_min<0x143, 0xC>(v));
  return v;
}

__device__ __forceinline__ float lane_value(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

}  // namespace amn
