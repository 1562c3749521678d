// mlp_layout.hpp -- kernel-ready layout of the per-leaf MLP parameters, shared by the
// forward (mlp.hip) and backward (mlp_bwd.hip) kernels and the packer.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/amnerf.h"

namespace amn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));

constexpr int kUnitBytes = 1024;   // one A fragment set: 64 lanes x 16 bytes
constexpr int kUnit8Bytes = 512;   // the same fragments as float8: 64 lanes x 8 bytes
constexpr int kFp8ScaleBytes = 64; // one float32 scale per layer (at most 9 layers), padded

// Per leaf: float32 biases (n_hidden * H + 16, padded to 16 bytes), then 1 KiB units of
// A fragments.  Forward units: layer 0 (RB x KU0), hidden layers (RB x KUh each), output
// (KUh).  bfloat16 blocks also carry, after all leaves' forward blocks, one backward block
// per leaf with the transposed weights of layers 1..n_hidden (RB x KUh each, the output
// layer RB x 1).
struct Layout {
  int H, nh, dtype, RB, KU0, KUh;
  int bias_floats, bias_bytes, units, bwd_units;
  uint32_t bytes, bwd_bytes;
  uint32_t bytes8;   // float8 blocks in memory: biases, kFp8ScaleBytes of scales, 512-byte units
  // layer of forward unit u
  __host__ __device__ int layer_of_unit(int u) const {
    const int n0 = RB * KU0;
    if (u < n0) return 0;
    if (u < n0 + (nh - 1) * RB * KUh) return 1 + (u - n0) / (RB * KUh);
    return nh;
  }
  __host__ __device__ int unit_index(int layer, int rb, int ku) const {
    if (layer == 0) return rb * KU0 + ku;
    int base = RB * KU0;
    if (layer < nh) return base + (layer - 1) * RB * KUh + rb * KUh + ku;
    return base + (nh - 1) * RB * KUh + ku;
  }
  // transposed weights of layer l (1..nh): row block rb of its inputs, K unit ku of its outputs
  __host__ __device__ int bwd_unit_index(int layer, int rb, int ku) const {
    int base = (layer - 1) * RB * KUh;
    return layer < nh ? base + rb * KUh + ku : base + rb;
  }
};

// float8 weights are staged on chip as bfloat16, so the bfloat16 layout applies on chip;
// `bytes8` is the float8 block in memory.
inline Layout make_layout(int nh, int H, int dtype) {
  Layout L;
  const bool b16 = dtype == AMNERF_BF16 || dtype == AMNERF_FP8;
  L.H = H; L.nh = nh; L.dtype = dtype; L.RB = H / 16;
  L.KU0 = b16 ? 1 : 2;
  L.KUh = b16 ? H / 32 : H / 16;
  L.bias_floats = nh * H + 16;
  L.bias_bytes = (L.bias_floats * 4 + 15) / 16 * 16;
  L.units = L.RB * L.KU0 + (nh - 1) * L.RB * L.KUh + L.KUh;
  L.bytes = (uint32_t)(L.bias_bytes + L.units * kUnitBytes);
  L.bwd_units = dtype == AMNERF_BF16 ? (nh - 1) * L.RB * L.KUh + L.RB : 0;
  L.bwd_bytes = (uint32_t)(L.bwd_units * kUnitBytes);
  L.bytes8 = dtype == AMNERF_FP8 ? (uint32_t)(L.bias_bytes + kFp8ScaleBytes + L.units * kUnit8Bytes) : 0u;
  return L;
}

// Input feature held by lane group g in slot i (0..7) of the first layer's B operand, as a
// column of the master W0[out][30] (-1 = zero feature).
// float32: group g holds frequency 2^g: sin(2^g pi p) xyz, cos(2^g pi p) xyz, then two of
//          (p_x, p_y, p_z, d_x, d_y, d_z, -, -).
// bfloat16: group g < 3 holds coordinate g at all four frequencies (sin, cos for k = 0..3),
//          obtained from k = 0 by double-angle steps; group 3 holds p and d.
__host__ __device__ __forceinline__ int first_layer_col(int g, int i) {
  if (i < 3) return 3 + 6 * g + i;
  if (i < 6) return 3 + 6 * g + 3 + (i - 3);
  int e = 2 * g + (i - 6);
  return e < 3 ? e : (e < 6 ? 27 + (e - 3) : -1);
}
__host__ __device__ __forceinline__ int first_layer_col_bf16(int g, int i) {
  if (g < 3) return 3 + 6 * (i / 2) + 3 * (i % 2) + g;
  return i < 3 ? i : (i < 6 ? 27 + (i - 3) : -1);
}

// Hidden-width input feature held in slot e (0..7) of K unit ku by lane group g (bfloat16):
// the accumulator values of row blocks 2ku and 2ku+1 of the previous layer.
__host__ __device__ __forceinline__ int hidden_col_bf16(int ku, int g, int e) {
  return 16 * (2 * ku + e / 4) + 4 * g + (e % 4);
}

// Master offsets of layer l (din x dout weights then dout biases).
__host__ __device__ __forceinline__ void master_offsets(int nh, int H, int l, int& din, int& dout,
                                                        int& off_w, int& off_b) {
  int off = 0;
  for (int k = 0; k < l; ++k) {
    int di = k == 0 ? 30 : H, dn = k == nh ? 4 : H;
    off += di * dn + dn;
  }
  din = l == 0 ? 30 : H;
  dout = l == nh ? 4 : H;
  off_w = off;
  off_b = off + din * dout;
}

__host__ __device__ __forceinline__ int master_param_count(int nh, int H) {
  int din, dout, off_w, off_b;
  master_offsets(nh, H, nh, din, dout, off_w, off_b);
  return off_b + dout;
}

// ReLU of eight values rounded to bfloat16: after the conversion the sign is the top bit,
// so a packed signed 16-bit max with 0 clears every negative value (and -0).
// Pairs are converted with one packed conversion each.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}

__device__ __forceinline__ bf16x8 cvt_bf16x8(const float v[8]) {
  uint32_t w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = bf16_pair(v[2 * i], v[2 * i + 1]);
  return __builtin_bit_cast(bf16x8, w);
}

// ReLU of a pair rounded to bfloat16, packed low (a) and high (b).
__device__ __forceinline__ uint32_t relu_bf16_pair(float a, float b) {
  s16x2 s = __builtin_bit_cast(s16x2, bf16_pair(a, b));
  s = __builtin_elementwise_max(s, (s16x2)0);
  return __builtin_bit_cast(uint32_t, s);
}

__device__ __forceinline__ bf16x8 relu_bf16x8(const float v[8]) {
  uint32_t w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    s16x2 s = __builtin_bit_cast(s16x2, bf16_pair(v[2 * i], v[2 * i + 1]));
    s = __builtin_elementwise_max(s, (s16x2)0);
    w[i] = __builtin_bit_cast(uint32_t, s);
  }
  return __builtin_bit_cast(bf16x8, w);
}

}  // namespace amn
