// prop.hip -- the learned proposal: a 43 -> 64 -> 64 -> 32 MLP evaluated per (ray, leaf
// interval) that predicts the optical thickness of 32 equal bins of the interval.
// Compositing the bins along the ray gives the ray's predicted weight histogram over its
// leaf intervals; the plain sampler's slots are ranked by the predicted weight they cover,
// the fewest slots holding mass_thresh of the predicted mass are kept (at most cap), and the
// ray falls back to every plain slot when the predicted mass is below mass_thresh or the cap
// is exceeded.  The kept slots become new intervals (runs of consecutive slots), so the
// rest of the path (sort by leaf, grouped MLP, compositing) runs unchanged on fewer samples.
//
// Training targets come from the plain render: bin opacity 1 - exp(-sum_j sigma_j |slot_j n
// bin|).  Training runs in float32 on the matrix cores (forward, backward chain and dW with
// K = items staged through LDS), with per-block partial gradients reduced in a fixed order.
#include "internal.hpp"
#include "devcommon.hpp"
#include "mlp_layout.hpp"

#include <algorithm>
#include <atomic>

namespace amn {
namespace {

constexpr int kThreads = 256;
constexpr int kIn = 43, kH = 64, kBins = 32;
constexpr int kP = kH * kIn + kH + kH * kH + kH + kBins * kH + kBins;   // 9056
// master offsets
constexpr int kW0 = 0, kB0 = kW0 + kH * kIn, kW1 = kB0 + kH, kB1 = kW1 + kH * kH, kW2 = kB1 + kH,
              kB2 = kW2 + kBins * kH;
// packed: biases (160 floats) then 1 KiB units.
// f32 forward units: layer 0: rb 0..3 x ku 0..2 (12 k-blocks of 4 inputs); layer 1: 4 x 4;
//   layer 2: rb 0..1 x 4.  Backward (transposed) units: layer 1: rb_in 0..3 x ku 0..3;
//   layer 2: rb_in 0..3 x ku 0..1.
// bf16 forward units: layer 0: rb 0..3 x ku 0..1 (K = 64 padded from 43); layer 1: 4 x 2;
//   layer 2: 2 x 2.
constexpr int kBiasBytes = (kH + kH + kBins) * 4;
constexpr int kF32Units = 12 + 16 + 8, kF32BwdUnits = 16 + 8, kBf16Units = 8 + 8 + 4;
constexpr uint32_t kF32Bytes = kBiasBytes + (kF32Units + kF32BwdUnits) * kUnitBytes;
constexpr uint32_t kBf16Bytes = kBiasBytes + kBf16Units * kUnitBytes;

__host__ __device__ __forceinline__ int f32_unit(int layer, int rb, int ku) {
  return layer == 0 ? rb * 3 + ku : (layer == 1 ? 12 + rb * 4 + ku : 28 + rb * 4 + ku);
}
__host__ __device__ __forceinline__ int f32_bwd_unit(int layer, int rb, int ku) {
  return kF32Units + (layer == 1 ? rb * 4 + ku : 16 + rb * 2 + ku);
}
__host__ __device__ __forceinline__ int bf16_unit(int layer, int rb, int ku) {
  return layer == 0 ? rb * 2 + ku : (layer == 1 ? 8 + rb * 2 + ku : 16 + rb * 2 + ku);
}

__device__ __forceinline__ float softplusf(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }
// exp(-x) with the hardware base-2 exponential
__device__ __forceinline__ float exp_neg(float x) { return __builtin_amdgcn_exp2f(-1.44269504f * x); }
// 1 - exp(-d) for d >= 0 given e = exp(-d): a quartic Taylor polynomial below 1/16
// (relative error under 2^-23 there), else 1 - e
__device__ __forceinline__ float one_minus_exp_neg(float d, float e) {
  return d < 0.0625f ? d * fmaf(d, fmaf(d, fmaf(d, -1.f / 24.f, 1.f / 6.f), -0.5f), 1.f) : 1.f - e;
}
// softplus with the hardware base-2 exponential and logarithm: log1p(e) is taken as
// e (1 - e/2) below e = 2^-12, where that is exact to float rounding.
__device__ __forceinline__ float softplus_fast(float z) {
  const float e = __builtin_amdgcn_exp2f(-fabsf(z) * 1.44269504f);
  const float l = e < 2.44140625e-4f ? e * fmaf(-0.5f, e, 1.f) : __builtin_amdgcn_logf(1.f + e) * 0.693147181f;
  return fmaxf(z, 0.f) + l;
}

// Feature (index into the 43 of an interval) held by element e of lane group g in K step
// ku of the BF16 first layer, or -1 for a zero column.  The order lets every lane compute
// only its own 16 inputs with the same operations in all four lane groups: in step 0,
// group g holds sin and cos of pi f v with v = position (g < 2) or direction (g >= 2) and
// f = 1 (g even) or 2 (g odd), plus k / S_max in group 0; in step 1, group g holds the
// position, the direction, the entry point or the exit point (g = 0..3), and the leaf
// box's lower (g = 0) or upper (g = 1) corner.
__host__ __device__ __forceinline__ int bf16_in_feature(int ku, int g, int e) {
  if (ku == 0) {
    if (e < 6) return 6 + 12 * (g >> 1) + 6 * (g & 1) + e;
    return (e == 6 && g == 0) ? 30 : -1;
  }
  if (e < 3) return g == 0 ? e : (g == 1 ? 3 + e : (g == 2 ? 37 + e : 40 + e));
  if (e < 6 && g < 2) return 31 + 3 * g + (e - 3);
  return -1;
}
__device__ __forceinline__ float logisticf(float z) { return 1.f / (1.f + expf(-z)); }

__global__ void k_prop_pack(int dtype, const float* __restrict__ master, uint8_t* __restrict__ packed) {
  const int n_units = dtype == AMNERF_BF16 ? kBf16Units : kF32Units + kF32BwdUnits;
  for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < n_units * 64 + kBiasBytes / 4;
       id += gridDim.x * blockDim.x) {
    if (id >= n_units * 64) {
      const int j = id - n_units * 64;
      const float v = j < kH ? master[kB0 + j] : (j < 2 * kH ? master[kB1 + j - kH] : master[kB2 + j - 2 * kH]);
      reinterpret_cast<float*>(packed)[j] = v;
      continue;
    }
    const int unit = id / 64, lane = id % 64, g = lane / 16, m = lane % 16;
    uint8_t* dst = packed + kBiasBytes + unit * kUnitBytes + lane * 16;
    if (dtype == AMNERF_BF16) {
      int layer, rb, ku;
      if (unit < 8) { layer = 0; rb = unit / 2; ku = unit % 2; }
      else if (unit < 16) { layer = 1; rb = (unit - 8) / 2; ku = unit % 2; }
      else { layer = 2; rb = (unit - 16) / 2; ku = unit % 2; }
      const int row = 16 * rb + m;
      bf16x8 h;
      for (int e = 0; e < 8; ++e) {
        float v;
        if (layer == 0) { const int f = bf16_in_feature(ku, g, e); v = f >= 0 ? master[kW0 + row * kIn + f] : 0.f; }
        else if (layer == 1) v = master[kW1 + row * kH + hidden_col_bf16(ku, g, e)];
        else v = master[kW2 + row * kH + hidden_col_bf16(ku, g, e)];
        h[e] = (__bf16)v;
      }
      *reinterpret_cast<bf16x8*>(dst) = h;
    } else if (unit < kF32Units) {
      int layer, rb, ku;
      if (unit < 12) { layer = 0; rb = unit / 3; ku = unit % 3; }
      else if (unit < 28) { layer = 1; rb = (unit - 12) / 4; ku = (unit - 12) % 4; }
      else { layer = 2; rb = (unit - 28) / 4; ku = (unit - 28) % 4; }
      const int row = 16 * rb + m;
      f32x4 v;
      for (int e = 0; e < 4; ++e) {
        const int kb = 4 * ku + e;
        if (layer == 0) { const int f = 4 * kb + g; v[e] = f < kIn ? master[kW0 + row * kIn + f] : 0.f; }
        else if (layer == 1) v[e] = master[kW1 + row * kH + 16 * ku + 4 * g + e];
        else v[e] = master[kW2 + row * kH + 16 * ku + 4 * g + e];
      }
      *reinterpret_cast<f32x4*>(dst) = v;
    } else {
      // transposed: lane (g, m) of unit (rb_in, ku) holds W^T[in = 16 rb_in + m][out], out =
      // 16 ku + 4 g + e (the accumulator rows of the gradient's row block ku)
      const int u = unit - kF32Units;
      const int layer = u < 16 ? 1 : 2;
      const int rb = layer == 1 ? u / 4 : (u - 16) / 2, ku = layer == 1 ? u % 4 : (u - 16) % 2;
      const int in = 16 * rb + m;
      f32x4 v;
      for (int e = 0; e < 4; ++e) {
        const int out = 16 * ku + 4 * g + e;
        v[e] = layer == 1 ? master[kW1 + out * kH + in] : master[kW2 + out * kH + in];
      }
      *reinterpret_cast<f32x4*>(dst) = v;
    }
  }
}

// The 43 features of an interval (the oracle's order).
__device__ __forceinline__ void prop_features(const float o[3], const float d[3], float t0, float t1, uint32_t k,
                                              int s_max, const float* box, float F[kIn]) {
  float q[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) q[a] = (o[a] - 0.5f) * 0.5f;
  int c = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) F[c++] = q[a];
#pragma unroll
  for (int a = 0; a < 3; ++a) F[c++] = d[a];
#pragma unroll
  for (int src = 0; src < 2; ++src) {
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const float fr = (float)(1 << kk);
#pragma unroll
      for (int a = 0; a < 3; ++a) F[c++] = sinpif(fr * (src == 0 ? q[a] : d[a]));
#pragma unroll
      for (int a = 0; a < 3; ++a) F[c++] = cospif(fr * (src == 0 ? q[a] : d[a]));
    }
  }
  F[c++] = (float)k / (float)s_max;
#pragma unroll
  for (int a = 0; a < 6; ++a) F[c++] = box[a];
#pragma unroll
  for (int a = 0; a < 3; ++a) F[c++] = 2.f * fmaf(t0, d[a], o[a]) - 1.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) F[c++] = 2.f * fmaf(t1, d[a], o[a]) - 1.f;
}

__device__ __forceinline__ float pick4(const float* F, int base, int g, int limit) {
  const float v0 = base < limit ? F[base < limit ? base : 0] : 0.f;
  const float v1 = base + 1 < limit ? F[base + 1 < limit ? base + 1 : 0] : 0.f;
  const float v2 = base + 2 < limit ? F[base + 2 < limit ? base + 2 : 0] : 0.f;
  const float v3 = base + 3 < limit ? F[base + 3 < limit ? base + 3 : 0] : 0.f;
  return g == 0 ? v0 : (g == 1 ? v1 : (g == 2 ? v2 : v3));
}

// Inputs of one item (interval i of the chunk).
__device__ __forceinline__ void item_features(const IvSet& iv, uint32_t i, const float* __restrict__ o,
                                              const float* __restrict__ d, int64_t stride, int64_t r0,
                                              const float* __restrict__ leafbox, int s_max, float F[kIn]) {
  const uint32_t ray = iv.ray[i];
  const uint32_t k = i - iv.iv_off[ray];
  const int64_t ri = r0 + ray;
  const float oo[3] = {o[ri], o[stride + ri], o[2 * stride + ri]};
  const float dd[3] = {d[ri], d[stride + ri], d[2 * stride + ri]};
  const float t0 = iv.t0[i];
  const float t1 = t0 + iv.dt[i];
  prop_features(oo, dd, t0, t1, k, s_max, leafbox + 6 * key_slot(iv.key[i]), F);
}

// ---- inference: tau^[item][32] --------------------------------------------------------
// Pieces of the bfloat16 network.
// The first layer's B operand of one column block: lane (g, m) evaluates its own 16
// inputs of item m (see bf16_in_feature).
__device__ __forceinline__ void prop_bf16_inputs(const float oo[3], const float dd[3], float t0, float t1,
                                                 const float box[3], uint32_t k, int s_max, int g, bf16x8 X[2]) {
  const float tt = g == 2 ? t0 : t1;
  const float half_f = (g & 1) ? 1.f : 0.5f;   // revolutions per unit of v
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float q = (oo[a] - 0.5f) * 0.5f;
    const float v = g < 2 ? q : dd[a];
    const float x = 2.f * fmaf(tt, dd[a], oo[a]) - 1.f;
    X[0][a] = (__bf16)__builtin_amdgcn_sinf(half_f * v);
    X[0][3 + a] = (__bf16)__builtin_amdgcn_cosf(half_f * v);
    X[1][a] = (__bf16)(g == 0 ? q : (g == 1 ? dd[a] : x));
    X[1][3 + a] = (__bf16)(g < 2 ? box[a] : 0.f);
  }
  X[0][6] = (__bf16)(g == 0 ? (float)k / (float)s_max : 0.f);
  X[0][7] = (__bf16)0.f;
  X[1][6] = (__bf16)0.f;
  X[1][7] = (__bf16)0.f;
}

// The three layers on MFMA for NCB column blocks: acc[cb][rb] holds the 32 output
// pre-activations (rb = 0, 1) of the items of column block cb.
template <int NCB>
__device__ __forceinline__ void prop_bf16_net(const uint8_t* units, const float* bias, int g, int lane,
                                              const bf16x8 X[NCB][2], f32x4 acc[NCB][4]) {
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const f32x4 bv = *reinterpret_cast<const f32x4*>(bias + 16 * rb + 4 * g);
#pragma unroll
    for (int ku = 0; ku < 2; ++ku) {
      const bf16x8 A = *reinterpret_cast<const bf16x8*>(units + bf16_unit(0, rb, ku) * kUnitBytes + lane * 16);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        acc[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, X[cb][ku], ku == 0 ? bv : acc[cb][rb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int layer = 1; layer <= 2; ++layer) {
    bf16x8 Bv[NCB][2];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int ku = 0; ku < 2; ++ku) {
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = acc[cb][2 * ku + e / 4][e % 4];
        Bv[cb][ku] = relu_bf16x8(v);
      }
    const int nrb = layer == 1 ? 4 : 2;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      if (rb >= nrb) break;
      const f32x4 bv = *reinterpret_cast<const f32x4*>(bias + layer * kH + 16 * rb + 4 * g);
#pragma unroll
      for (int ku = 0; ku < 2; ++ku) {
        const bf16x8 A = *reinterpret_cast<const bf16x8*>(units + bf16_unit(layer, rb, ku) * kUnitBytes + lane * 16);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          acc[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bv[cb][ku], ku == 0 ? bv : acc[cb][rb], 0, 0, 0);
      }
    }
  }
}

// Output of one column: v = the 32 bin thicknesses (rows 16 rb + 4 g + e), or with cum set
// the bins' local composited weights w_b = exp(-P_(b-1)) (1 - exp(-tau_b)), P_b = tau_0 +
// ... + tau_b, and the interval's total P_31 (valid in lane group 3).  Lane group g holds
// bins 4g..4g+3 and 16+4g..16+4g+3 of its column, so the offsets of its two runs are sums
// over the lower groups, gathered 16 and 32 lanes down the wave; within a run the
// transmittance steps by exp(-tau_b).
template <bool BF16>
__device__ __forceinline__ float prop_outputs(const f32x4 acc[4], int cum, int g, int m, f32x4 v[2]) {
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int e = 0; e < 4; ++e) v[rb][e] = BF16 ? softplus_fast(acc[rb][e]) : softplusf(acc[rb][e]);
  float total = 0.f;
  if (cum) {
    float run[2], off[2], last[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      float x = v[rb][0] + v[rb][1];
      x += v[rb][2];
      x += v[rb][3];
      last[rb] = x;                      // this lane's run total
      float y = __shfl_up(x, 16, 64);
      x += g >= 1 ? y : 0.f;
      y = __shfl_up(x, 32, 64);
      x += g >= 2 ? y : 0.f;
      run[rb] = x;                       // inclusive over groups 0..g
      off[rb] = x - last[rb];
    }
    const float tot0 = __shfl(run[0], 48 + m, 64);
    const float start[2] = {off[0], tot0 + off[1]};
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      float T = exp_neg(start[rb]);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float tb = v[rb][e];
        const float eb = exp_neg(tb);
        v[rb][e] = T * one_minus_exp_neg(tb, eb);
        T *= eb;
      }
    }
    total = last[1] + (tot0 + off[1]);   // P_31 in lane group 3
  }
  return total;
}

template <bool BF16>
__global__ __launch_bounds__(kThreads) void k_prop_fwd(const uint8_t* __restrict__ packed, IvSet iv,
                                                       const float* __restrict__ o, const float* __restrict__ d,
                                                       int64_t stride, int64_t r0,
                                                       const float* __restrict__ leafbox, int s_max,
                                                       int cum, float* __restrict__ tau, float* __restrict__ tot) {
  extern __shared__ __align__(16) uint8_t lds[];
  const uint32_t bytes = BF16 ? kBf16Bytes : kBiasBytes + kF32Units * kUnitBytes;
  for (uint32_t i = threadIdx.x; i < bytes / 16; i += kThreads)
    reinterpret_cast<f32x4*>(lds)[i] = reinterpret_cast<const f32x4*>(packed)[i];
  __syncthreads();
  const float* bias = reinterpret_cast<const float*>(lds);
  const uint8_t* units = lds + kBiasBytes;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, m = lane & 15;
  // items per wave and pass: 16 NCB (BF16 keeps fewer accumulators live for occupancy)
  constexpr int NCB = BF16 ? 2 : 4;
  constexpr uint32_t kTile = 4u * 16u * NCB;
  const uint32_t n_items = *iv.n_iv_dev;
  // The interval records (ray, t0, dt, key) of a wave's next tile are loaded one tile ahead;
  // the loads that depend on them (the ray's origin, direction and first interval, the leaf
  // box) are issued at the start of the tile, before that prefetch, so waiting for them
  // never waits for it.
  uint32_t p_ray[NCB], p_key[NCB];
  float p_t0[NCB], p_dt[NCB];
  auto load_records = [&](uint32_t tl) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      uint32_t it = tl * kTile + wave * 16u * NCB + cb * 16 + m;
      it = it < n_items ? it : n_items - 1;
      p_ray[cb] = iv.ray[it];
      p_t0[cb] = iv.t0[it];
      p_dt[cb] = iv.dt[it];
      p_key[cb] = iv.key[it];
    }
  };
  if (BF16 && blockIdx.x * kTile < n_items) load_records(blockIdx.x);
  for (uint32_t tile = blockIdx.x; tile * kTile < n_items; tile += gridDim.x) {
    const uint32_t base = tile * kTile + wave * 16u * NCB;
    if (base >= n_items) continue;   // so are this wave's later tiles
    f32x4 acc[NCB][4];
    if (BF16) {
      bf16x8 X[NCB][2];
      uint32_t c_ray[NCB], c_k[NCB];
      float c_t0[NCB], c_t1[NCB], c_o[NCB][3], c_d[NCB][3], c_box[NCB][3];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        uint32_t it = base + cb * 16 + m;
        it = it < n_items ? it : n_items - 1;
        c_ray[cb] = p_ray[cb];
        c_k[cb] = it - iv.iv_off[c_ray[cb]];
        const int64_t ri = r0 + c_ray[cb];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          c_o[cb][a] = o[a * stride + ri];
          c_d[cb][a] = d[a * stride + ri];
          c_box[cb][a] = leafbox[6 * key_slot(p_key[cb]) + 3 * (g & 1) + a];
        }
        c_t0[cb] = p_t0[cb];
        c_t1[cb] = p_t0[cb] + p_dt[cb];
      }
      if ((tile + gridDim.x) * kTile < n_items) load_records(tile + gridDim.x);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) prop_bf16_inputs(c_o[cb], c_d[cb], c_t0[cb], c_t1[cb], c_box[cb], c_k[cb], s_max, g, X[cb]);
      prop_bf16_net<NCB>(units, bias, g, lane, X, acc);
    } else {
      float X[NCB][12];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const uint32_t it = base + cb * 16 + m;
        float F[kIn];
        item_features(iv, it < n_items ? it : n_items - 1, o, d, stride, r0, leafbox, s_max, F);
#pragma unroll
        for (int kb = 0; kb < 12; ++kb) X[cb][kb] = pick4(F, 4 * kb, g, kIn);
      }
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const f32x4 bv = *reinterpret_cast<const f32x4*>(bias + 16 * rb + 4 * g);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[cb][rb] = bv;
#pragma unroll
        for (int ku = 0; ku < 3; ++ku) {
          const f32x4 A = *reinterpret_cast<const f32x4*>(units + f32_unit(0, rb, ku) * kUnitBytes + lane * 16);
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
              acc[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[e], X[cb][4 * ku + e], acc[cb][rb], 0, 0, 0);
        }
      }
#pragma unroll
      for (int layer = 1; layer <= 2; ++layer) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[cb][rb][e] = fmaxf(acc[cb][rb][e], 0.f);
        const int nrb = layer == 1 ? 4 : 2;
        f32x4 nacc[NCB][4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          if (rb >= nrb) break;
          const f32x4 bv = *reinterpret_cast<const f32x4*>(bias + layer * kH + 16 * rb + 4 * g);
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) nacc[cb][rb] = bv;
#pragma unroll
          for (int ku = 0; ku < 4; ++ku) {
            const f32x4 A = *reinterpret_cast<const f32x4*>(units + f32_unit(layer, rb, ku) * kUnitBytes + lane * 16);
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
              for (int cb = 0; cb < NCB; ++cb)
                nacc[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[e], acc[cb][ku][e], nacc[cb][rb], 0, 0, 0);
          }
        }
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
            if (rb < nrb) acc[cb][rb] = nacc[cb][rb];
      }
    }
    // outputs: rows 16 rb + 4 g + e of the 32 bins (with cum set, for rendering: the bins'
    // local composited weights, and the interval's total to tot)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const uint32_t it = base + cb * 16 + m;
      f32x4 v[2];
      const float total = prop_outputs<BF16>(acc[cb], cum, g, m, v);
      if (it >= n_items) continue;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
        *reinterpret_cast<f32x4*>(tau + (uint64_t)it * kBins + 16 * rb + 4 * g) = v[rb];
      if (cum && g == 3) tot[it] = total;
    }
  }
}

// ---- selection: one wave per ray ----------------------------------------------------
// Input: per interval, its total optical thickness P_31 and the local composited weights
// w_b of its 32 bins (the weights the bins would have if the ray entered the interval
// unattenuated).  The ray's optical depth before interval k, S_k, is a wave scan of the
// totals; the predicted mass is 1 - exp(-S_total), and rays below mass_thresh fall back.
// Slot j of an interval with n slots covers bins [32 j / n, 32 (j+1) / n); its weight is
// exp(-S_k) times the covered fraction of each bin's weight: c_lo w_lo + w_(lo+1) + ... +
// w_(hi-1) + c_hi w_hi, or (32 / n) w_lo when the slot lies inside one bin.
// The weights are then sorted (descending) across the wave, a prefix sum over them gives
// the number c of slots needed to reach mass_thresh * M^, and the slots kept are those with
// weight above the c-th largest value w* plus, among those equal to w*, the lowest-indexed
// ones (so ties go to the earlier slot).
constexpr int kMaxSlots = 256;   // >= AMNERF_MAX_SAMPLES + 1

// Value of lane (lane ^ J): lane permutations within rows (J <= 8, two steps for 4 and
// 8: a mirror of 8 or 16 lanes followed by a mirror of 4 or 8), a swizzle within 32 lanes
// (J = 16), or a general permute (J = 32).
template <int J>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
  const int x = (int)v;
  int r;
  if constexpr (J == 1) r = __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);        // quad_perm 1,0,3,2
  else if constexpr (J == 2) r = __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
  else if constexpr (J == 4)                                                           // i^7 then i^3
    r = __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, false), 0x1B, 0xF, 0xF, false);
  else if constexpr (J == 8)                                                           // i^15 then i^7
    r = __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, false), 0x141, 0xF, 0xF, false);
  else if constexpr (J == 16) r = __builtin_amdgcn_ds_swizzle(x, 0x401F);             // xor 16 within 32
  else r = __shfl_xor(x, J, 64);
  return (uint32_t)r;
}

// Bitonic sort, descending, of 64*E keys (element e = q*64 + lane held in key[q]).  The
// keys are the bit patterns of non-negative floats, whose unsigned order is their value
// order.  A compare-exchange at lane distance J keeps the maximum in the lower element of
// a descending block; with dir = all ones (keep maximum) or 0 (keep minimum) per lane,
// median3(key, other, dir) is that result in one instruction.  bit[j] holds all ones in
// lanes whose bit j is clear.
template <int J>
__device__ __forceinline__ uint32_t bitonic_lane_step(uint32_t key, uint32_t dir) {
  const uint32_t other = xor_lane<J>(key);
  return max(min(key, other), min(max(key, other), dir));   // median of (key, other, dir)
}

template <int E>
__device__ __forceinline__ void bitonic_desc(uint32_t key[E], int lane) {
  uint32_t bit[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) bit[j] = ((lane >> j) & 1) ? 0u : 0xFFFFFFFFu;
#pragma unroll
  for (int lk = 1; (1 << lk) <= 64 * E; ++lk) {
    const int k = 1 << lk;
#pragma unroll
    for (int lj = lk - 1; lj >= 0; --lj) {
      const int j = 1 << lj;
      if (j >= 64) {
#pragma unroll
        for (int q = 0; q < E; ++q) {
          if (((q * 64) & j) != 0) continue;
          const int q2 = q + j / 64;
          const bool desc_block = ((q * 64) & k) == 0;
          const uint32_t a = key[q], b = key[q2];
          key[q] = desc_block ? max(a, b) : min(a, b);
          key[q2] = desc_block ? min(a, b) : max(a, b);
        }
        continue;
      }
#pragma unroll
      for (int q = 0; q < E; ++q) {
        // keep the maximum where (e & j) == 0 equals (e & k) == 0, e = q * 64 + lane
        uint32_t dir;
        if (k >= 64) dir = (((q * 64) & k) == 0) ? bit[lj] : ~bit[lj];
        else dir = ~(bit[lj] ^ bit[lk]);
        switch (j) {
          case 32: key[q] = bitonic_lane_step<32>(key[q], dir); break;
          case 16: key[q] = bitonic_lane_step<16>(key[q], dir); break;
          case 8: key[q] = bitonic_lane_step<8>(key[q], dir); break;
          case 4: key[q] = bitonic_lane_step<4>(key[q], dir); break;
          case 2: key[q] = bitonic_lane_step<2>(key[q], dir); break;
          default: key[q] = bitonic_lane_step<1>(key[q], dir); break;
        }
      }
    }
  }
}

// Number of slots kept: the shortest prefix of the descending weights whose sum reaches
// target.  *reached is false when all ns slots together stay below it.  *wcut = weight of
// the last kept slot.
template <int E>
__device__ __forceinline__ uint32_t count_sorted(const float p[4], uint32_t ns, float target, int lane, bool* reached,
                                                 float* wcut) {
  // slots past ns sort last as +0 (a valid zero weight never decides the cut: adding it
  // cannot reach a positive target)
  uint32_t key[E];
#pragma unroll
  for (int q = 0; q < E; ++q) key[q] = (uint32_t)lane + 64u * q < ns ? __float_as_uint(p[q]) : 0u;
  bitonic_desc<E>(key, lane);
  float carry = 0.f, cut = 0.f;
  uint32_t count = 0;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const float v = __uint_as_float(key[q]);
    const float inc = wave_scan_incl(v);
    const uint32_t pos = (uint32_t)q * 64u + (uint32_t)lane;
    const bool take = pos < ns && carry + (inc - v) < target;
    const uint64_t b = __ballot(take);
    if (b) cut = lane_value(v, 63 - __builtin_clzll(b));
    count += (uint32_t)__popcll(b);
    carry += lane_value(inc, 63);
  }
  *reached = count < ns || carry >= target;
  *wcut = cut;
  return count;
}

// Selection of one ray (one wave): bins of interval i0 + k at wts[(i0 + k) * 32 ..], its
// total at tot[i0 + k] (global memory, or the fused kernel's LDS copy); sb: the wave's
// kMaxSlots floats of LDS.  Writes runs[r], nsel[r], mask[4 r ..] (and mass_out[r]);
// returns true when the ray falls back.  prefetch() is called once every load of the ray
// has been issued.
template <int QM, class Prefetch>
__device__ __forceinline__ bool select_ray(uint32_t r, uint32_t i0, uint32_t meff, uint32_t ns,
                                           const float* __restrict__ wts, const float* __restrict__ tot,
                                           float* __restrict__ sb, float mass_thresh, int cap, int lane,
                                           uint32_t* __restrict__ runs, uint32_t* __restrict__ nsel,
                                           uint64_t* __restrict__ mask, float* __restrict__ mass_out,
                                           Prefetch&& prefetch) {
  if (meff == 0) {
    if (lane == 0) { runs[r] = 0; nsel[r] = 0; if (mass_out) mass_out[r] = 0.f; }
    if (lane < 4) mask[4 * (uint64_t)r + lane] = 0ull;
    prefetch();
    return false;
  }
  const uint32_t n = ns / meff;
  // floor(x / n) = umulhi(x, m) with m = ceil(2^32 / n) for x < 2^16 and n >= 2 (the
  // error x (m - 2^32/n) / 2^32 stays below 1/n, so it never carries into the integer part)
  const uint32_t m32 = n > 1u ? 0xFFFFFFFFu / n + 1u : 0u;
  auto div_n = [&](uint32_t x) { return n > 1u ? __umulhi(x, m32) : x; };
  const uint32_t nq = (ns + 63u) / 64u;
  // Every load of the ray is issued before the first wait: the bin weights each slot
  // covers (its first and last bin and up to kMid whole bins between them), then the
  // interval totals, then (prefetch) the next ray's offsets.
  // The slot geometry is kept packed: interval k (8 bits), slot j in it (8 bits), first and
  // last bin (5 bits each).
  constexpr int kMid = QM == 2 ? 3 : 4;
  float wlo[QM], whi[QM], wmid[QM][kMid];
  uint32_t geo[QM];
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    wlo[q] = 0.f; whi[q] = 0.f; geo[q] = 0u;
#pragma unroll
    for (int t = 0; t < kMid; ++t) wmid[q][t] = 0.f;
    if ((uint32_t)q >= nq) continue;
    const uint32_t s = (uint32_t)lane + 64u * q;
    const uint32_t sk = div_n(s);
    const uint32_t j = s - sk * n;
    const uint32_t blo = div_n(32u * j);
    const uint32_t bhi = div_n(32u * (j + 1) + n - 1) - 1u;
    geo[q] = (sk & 255u) | ((j & 255u) << 8) | (blo << 16) | ((bhi & 31u) << 24);
    if (s >= ns) continue;
    const float* row = wts + (uint64_t)(i0 + sk) * kBins;
    wlo[q] = row[blo];
    whi[q] = row[bhi];
#pragma unroll
    for (int t = 0; t < kMid; ++t)
      if (blo + 1u + (uint32_t)t < bhi) wmid[q][t] = row[blo + 1u + t];
  }
  float tk0 = (uint32_t)lane < meff ? tot[i0 + lane] : 0.f;
  prefetch();
  // transmittance at the entry of each interval, exp(-S_k)
  float carry = 0.f;
  for (uint32_t k0 = 0; k0 < meff; k0 += 64) {
    const uint32_t k = k0 + (uint32_t)lane;
    const float tk = k0 == 0 ? tk0 : (k < meff ? tot[i0 + k] : 0.f);
    const float inc = wave_scan_incl(tk);
    if (k < meff) sb[k] = exp_neg(carry + (inc - tk));
    carry += lane_value(inc, 63);
  }
  const float M = -expm1f(-carry);
  if (mass_out && lane == 0) mass_out[r] = M;
  bool fallback = !(M >= mass_thresh);
  uint32_t count = 0;
  uint64_t sel[4] = {0ull, 0ull, 0ull, 0ull};
  uint64_t first[4] = {0ull, 0ull, 0ull, 0ull};   // slots that start an interval
  if (!fallback) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const float inv_n = 1.f / (float)n;
    float p[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < QM; ++q) {
      if ((uint32_t)q >= nq) break;
      const uint32_t s = (uint32_t)lane + 64u * q;
      const uint32_t sk = geo[q] & 255u, j = (geo[q] >> 8) & 255u;
      first[q] = __ballot(j == 0u);
      if (s >= ns) continue;
      const uint32_t blo = (geo[q] >> 16) & 31u, bhi = geo[q] >> 24;
      const float u0 = (float)(32u * j) * inv_n, u1 = (float)(32u * (j + 1)) * inv_n;
      float v;
      if (bhi == blo) {
        v = 32.f * inv_n * wlo[q];
      } else {
        v = ((float)(blo + 1) - u0) * wlo[q];
#pragma unroll
        for (int t = 0; t < kMid; ++t) v += wmid[q][t];
        const float* row = wts + (uint64_t)(i0 + sk) * kBins;
        for (uint32_t b = blo + 1u + kMid; b < bhi; ++b) v += row[b];   // slots wider than kMid + 1 bins
        v += (u1 - (float)bhi) * whi[q];
      }
      p[q] = sb[sk] * v;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const float target = mass_thresh * M;
    bool reached = true;
    float wcut = 0.f;
    if constexpr (QM == 2) count = count_sorted<2>(p, ns, target, lane, &reached, &wcut);
    else if constexpr (QM == 3) count = nq <= 2 ? count_sorted<2>(p, ns, target, lane, &reached, &wcut)
                                                : count_sorted<4>(p, ns, target, lane, &reached, &wcut);
    else count = nq <= 2 ? count_sorted<2>(p, ns, target, lane, &reached, &wcut)
                         : count_sorted<4>(p, ns, target, lane, &reached, &wcut);
    if (count > (uint32_t)cap || count == 0 || !reached) {
      fallback = true;
    } else {
      // above the cut, then the earliest slots equal to it
      uint32_t n_gt = 0;
      uint64_t eqm[4];
#pragma unroll
      for (int q = 0; q < QM; ++q) {
        const bool valid = (uint32_t)lane + 64u * q < ns;
        sel[q] = __ballot(valid && p[q] > wcut);
        eqm[q] = __ballot(valid && p[q] == wcut);
        n_gt += (uint32_t)__popcll(sel[q]);
      }
      uint32_t need = count - n_gt;
#pragma unroll
      for (int q = 0; q < QM; ++q) {
        uint64_t e = eqm[q];
        while (need && e) {
          const uint64_t low = e & (~e + 1ull);
          sel[q] |= low;
          e ^= low;
          --need;
        }
      }
    }
  }
  if (fallback) {
    if (lane == 0) { runs[r] = meff; nsel[r] = ns; }
    if (lane < 4) mask[4 * (uint64_t)r + lane] = ~0ull;
    return true;
  }
  // runs: a kept slot starts a run unless the previous slot is kept in the same interval
  uint32_t nruns = 0;
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    const uint64_t prev_kept = (sel[q] << 1) | (q > 0 ? sel[q - 1] >> 63 : 0ull);
    nruns += (uint32_t)__popcll(sel[q] & ~(prev_kept & ~first[q]));
  }
  if (lane == 0) { runs[r] = nruns; nsel[r] = count; }
  if (lane < 4) mask[4 * (uint64_t)r + lane] = sel[lane];
  return false;
}

// QM: registers of 64 slots a ray may need (2 when S_max <= 128, 3 up to 192, else 4);
// fewer live registers keep more waves resident.
template <int QM>
__global__ __launch_bounds__(kThreads, QM == 2 ? 8 : (QM == 3 ? 7 : 1)) void k_prop_select(uint32_t nr, IvSet iv, const float* __restrict__ wts,
                                                          const float* __restrict__ tot,
                                                          float mass_thresh, int cap, uint32_t* __restrict__ runs,
                                                          uint32_t* __restrict__ nsel, uint64_t* __restrict__ mask,
                                                          float* __restrict__ mass_out,
                                                          ChunkCounts* __restrict__ counts) {
  __shared__ float sbuf[kThreads / 64][kMaxSlots];
  __shared__ uint32_t fb_lds[kThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // fallback rays are counted per wave and added once per block: one global atomic per
  // fallback ray serialises on the counter's cache line
  uint32_t n_fb = 0;
  const uint32_t step = gridDim.x * (kThreads / 64);
  uint32_t r = blockIdx.x * (kThreads / 64) + (uint32_t)__builtin_amdgcn_readfirstlane(wave);
  // the ray's interval and sample offsets are loaded one ray ahead
  uint32_t nx_i0 = 0, nx_i1 = 0, nx_s0 = 0, nx_s1 = 0;
  if (r < nr) { nx_i0 = iv.iv_off[r]; nx_i1 = iv.iv_off[r + 1]; nx_s0 = iv.smp_off[r]; nx_s1 = iv.smp_off[r + 1]; }
  for (; r < nr; r += step) {
    const uint32_t i0 = nx_i0, meff = nx_i1 - nx_i0;
    const uint32_t ns = nx_s1 - nx_s0;
    const uint32_t rn = r + step;
    auto prefetch = [&]() {
      if (rn < nr) { nx_i0 = iv.iv_off[rn]; nx_i1 = iv.iv_off[rn + 1]; nx_s0 = iv.smp_off[rn]; nx_s1 = iv.smp_off[rn + 1]; }
    };
    n_fb += select_ray<QM>(r, i0, meff, ns, wts, tot, sbuf[wave], mass_thresh, cap, lane, runs, nsel, mask, mass_out,
                           prefetch) ? 1u : 0u;
  }
  if (lane == 0) fb_lds[wave] = n_fb;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kThreads / 64; ++w) t += fb_lds[w];
    if (t) atomicAdd(reinterpret_cast<unsigned long long*>(&counts->fallback), (unsigned long long)t);
  }
}

// ---- emission of the planned intervals: one lane per ray -------------------------------
// The lane walks its ray's slot mask run by run: trailing zeros skip slots that are not
// kept, trailing ones give the run's length, cut at the interval's end.  A run that is a
// whole interval keeps its endpoints exactly.  The block's rays are consecutive, so their
// planned intervals fill one contiguous output range: the first `stage_n` entries of it are
// put in LDS and written out by consecutive threads (whole cache lines), the rest go
// straight to memory.
constexpr uint32_t kEmitStage = 3072;   // 20 B each: 60 KiB of LDS

__global__ __launch_bounds__(kThreads) void k_prop_emit(uint32_t nr, IvSet iv, const uint64_t* __restrict__ mask,
                                                        const uint32_t* __restrict__ pv_off,
                                                        const uint32_t* __restrict__ ps_off,
                                                        float* __restrict__ pt0, float* __restrict__ pdt,
                                                        uint32_t* __restrict__ pkey, uint32_t* __restrict__ pray,
                                                        uint32_t* __restrict__ pbase) {
  extern __shared__ __align__(16) uint8_t dyn[];
  float* s_t0 = reinterpret_cast<float*>(dyn);
  float* s_dt = s_t0 + kEmitStage;
  uint32_t* s_key = reinterpret_cast<uint32_t*>(s_dt + kEmitStage);
  uint32_t* s_ray = s_key + kEmitStage;
  uint32_t* s_base = s_ray + kEmitStage;
  const uint32_t rb = blockIdx.x * kThreads;                     // first ray of the block
  const uint32_t re = rb + kThreads < nr ? rb + kThreads : nr;   // one past its last ray
  const uint32_t b0 = pv_off[rb], b1 = pv_off[re];               // the block's output range
  const uint32_t r = rb + threadIdx.x;
  const uint32_t i0 = r < nr ? iv.iv_off[r] : 0u, meff = r < nr ? iv.iv_off[r + 1] - i0 : 0u;
  if (meff != 0) {
    const uint32_t ns = iv.smp_off[r + 1] - iv.smp_off[r];
    const uint32_t n = ns / meff;
    const uint32_t m32 = n > 1u ? 0xFFFFFFFFu / n + 1u : 0u;   // floor(x / n) = umulhi(x, m32), x < 2^16
    uint32_t out = pv_off[r], smp = ps_off[r];
    const uint64_t w[4] = {mask[4 * (uint64_t)r], mask[4 * (uint64_t)r + 1], mask[4 * (uint64_t)r + 2],
                           mask[4 * (uint64_t)r + 3]};
    auto word = [&](uint32_t q) { return q == 0 ? w[0] : (q == 1 ? w[1] : (q == 2 ? w[2] : w[3])); };
    uint32_t s = 0;
    while (s < ns) {
      // next kept slot at or after s
      const uint64_t x = word(s >> 6) >> (s & 63u);
      if (x == 0ull) {
        s = (s | 63u) + 1u;
        continue;
      }
      s += (uint32_t)__builtin_ctzll(x);
      if (s >= ns) break;
      const uint32_t k = n > 1u ? __umulhi(s, m32) : s;
      const uint32_t j0 = s - k * n;
      // consecutive kept slots from s, word by word, cut at the interval's end
      uint32_t len = 0, pos = s;
      while (pos < ns) {
        const uint32_t b = pos & 63u;
        const uint64_t y = ~(word(pos >> 6) >> b);
        const uint32_t c = y ? (uint32_t)__builtin_ctzll(y) : 64u - b;
        len += c;
        pos += c;
        if (c < 64u - b) break;
      }
      len = min(len, min(n - j0, ns - s));
      const uint32_t i = i0 + k;
      const float delta = iv.dt[i] / (float)n;
      float t0o, dto;
      if (j0 == 0 && len == n) {          // the whole interval: keep it exactly
        t0o = iv.t0[i];
        dto = iv.dt[i];
      } else {
        t0o = fmaf((float)j0, delta, iv.t0[i]);
        dto = (float)len * delta;
      }
      const uint32_t key = key_slot(iv.key[i]) | (len << 16);
      const uint32_t q = out - b0;
      if (q < kEmitStage) {
        s_t0[q] = t0o; s_dt[q] = dto; s_key[q] = key; s_ray[q] = r; s_base[q] = smp;
      } else {
        pt0[out] = t0o; pdt[out] = dto; pkey[out] = key; pray[out] = r; pbase[out] = smp;
      }
      ++out;
      smp += len;
      s += len;
    }
  }
  __syncthreads();
  const uint32_t n_st = b1 - b0 < kEmitStage ? b1 - b0 : kEmitStage;
  for (uint32_t q = threadIdx.x; q < n_st; q += kThreads) {
    pt0[b0 + q] = s_t0[q];
    pdt[b0 + q] = s_dt[q];
    pkey[b0 + q] = s_key[q];
    pray[b0 + q] = s_ray[q];
    pbase[b0 + q] = s_base[q];
  }
}

// ---- training --------------------------------------------------------------------------
// Targets: per interval, bin opacity 1 - exp(-tau_b), tau_b = sum_j sigma_j len |slot_j n bin_b|.
__global__ __launch_bounds__(kThreads) void k_prop_targets(IvSet iv, const float* __restrict__ smp_out,
                                                           float* __restrict__ alpha) {
  const uint32_t n_iv = *iv.n_iv_dev;
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < n_iv; i += gridDim.x * kThreads) {
    const uint32_t n = key_n(iv.key[i]);
    const uint32_t base = iv.base[i];
    const float len = iv.dt[i];
    float tb[kBins];
#pragma unroll
    for (int b = 0; b < kBins; ++b) tb[b] = 0.f;
    for (uint32_t j = 0; j < n; ++j) {
      const float sig = softplusf(smp_out[4 * (uint64_t)(base + j)]);
      const float a0 = (float)j / (float)n, a1 = (float)(j + 1) / (float)n;
#pragma unroll
      for (int b = 0; b < kBins; ++b) {
        const float ov = fminf(a1, (float)(b + 1) * (1.f / 32.f)) - fmaxf(a0, (float)b * (1.f / 32.f));
        if (ov > 0.f) tb[b] = fmaf(sig * len, ov, tb[b]);
      }
    }
#pragma unroll
    for (int b = 0; b < kBins; b += 4)
      *reinterpret_cast<f32x4*>(alpha + (uint64_t)i * kBins + b) =
          f32x4{-expm1f(-tb[b]), -expm1f(-tb[b + 1]), -expm1f(-tb[b + 2]), -expm1f(-tb[b + 3])};
  }
}

constexpr int kTrNCB = 2;                       // 32 items per wave
constexpr int kTrItems = 4 * 16 * kTrNCB;       // 128 items per block step
constexpr int kTrRow = kTrItems * 4 + 16;       // staged float row + padding

__device__ __forceinline__ void stf(uint8_t* base, int row, int col, float v) {
  *reinterpret_cast<float*>(base + row * kTrRow + col * 4) = v;
}
__device__ __forceinline__ float ldf(const uint8_t* base, int row, int col) {
  return *reinterpret_cast<const float*>(base + row * kTrRow + col * 4);
}

// Forward + backward of the proposal over a contiguous range of 128-item steps per block:
// loss partial and dW/db partial per block (master layout).
__global__ __launch_bounds__(kThreads) void k_prop_train(const uint8_t* __restrict__ packed, IvSet iv,
                                                         const float* __restrict__ o, const float* __restrict__ d,
                                                         int64_t stride, int64_t r0,
                                                         const float* __restrict__ leafbox, int s_max,
                                                         const float* __restrict__ alpha, float* __restrict__ part,
                                                         float* __restrict__ loss_part) {
  extern __shared__ __align__(16) uint8_t lds[];
  const uint32_t wbytes = kF32Bytes;
  uint8_t* s_dz = lds + wbytes;
  uint8_t* s_h = s_dz + kH * kTrRow;
  for (uint32_t i = threadIdx.x; i < wbytes / 16; i += kThreads)
    reinterpret_cast<f32x4*>(lds)[i] = reinterpret_cast<const f32x4*>(packed)[i];
  __syncthreads();
  const float* bias = reinterpret_cast<const float*>(lds);
  const uint8_t* units = lds + kBiasBytes;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, m = lane & 15;
  const uint32_t n_items = *iv.n_iv_dev;
  const uint32_t steps = (n_items + kTrItems - 1) / kTrItems;
  const uint32_t sb = (uint32_t)(((uint64_t)blockIdx.x * steps) / gridDim.x);
  const uint32_t se = (uint32_t)(((uint64_t)(blockIdx.x + 1) * steps) / gridDim.x);
  const float scale = 1.f / ((float)n_items * (float)kBins);
  // dW items: layer 0: rb 0..3 x ci 0..2 (48 input slots) -> 3 per wave; layer 1: 4 x 4 -> 4;
  // layer 2: 2 x 4 -> 2.  Wave w owns rows of one output row block for each layer.
  f32x4 aW0[3], aW1[4], aW2[2], aB0, aB1, aB2;
#pragma unroll
  for (int q = 0; q < 4; ++q) { if (q < 3) aW0[q] = f32x4{0, 0, 0, 0}; aW1[q] = f32x4{0, 0, 0, 0}; if (q < 2) aW2[q] = f32x4{0, 0, 0, 0}; }
  aB0 = aB1 = aB2 = f32x4{0, 0, 0, 0};
  float lsum = 0.f;
  for (uint32_t st = sb; st < se; ++st) {
    const uint32_t base = st * kTrItems + wave * 16 * kTrNCB;
    float X[kTrNCB][12];
    bool valid[kTrNCB];
#pragma unroll
    for (int cb = 0; cb < kTrNCB; ++cb) {
      const uint32_t it = base + cb * 16 + m;
      valid[cb] = it < n_items;
      float F[kIn];
      item_features(iv, valid[cb] ? it : 0u, o, d, stride, r0, leafbox, s_max, F);
#pragma unroll
      for (int kb = 0; kb < 12; ++kb) X[cb][kb] = pick4(F, 4 * kb, g, kIn);
    }
    // forward
    f32x4 H1[kTrNCB][4], H2[kTrNCB][4], Z3[kTrNCB][2];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const f32x4 bv = *reinterpret_cast<const f32x4*>(bias + 16 * rb + 4 * g);
#pragma unroll
      for (int cb = 0; cb < kTrNCB; ++cb) H1[cb][rb] = bv;
#pragma unroll
      for (int ku = 0; ku < 3; ++ku) {
        const f32x4 A = *reinterpret_cast<const f32x4*>(units + f32_unit(0, rb, ku) * kUnitBytes + lane * 16);
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int cb = 0; cb < kTrNCB; ++cb)
            H1[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[e], X[cb][4 * ku + e], H1[cb][rb], 0, 0, 0);
      }
    }
#pragma unroll
    for (int cb = 0; cb < kTrNCB; ++cb)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) H1[cb][rb][e] = fmaxf(H1[cb][rb][e], 0.f);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const f32x4 bv = *reinterpret_cast<const f32x4*>(bias + kH + 16 * rb + 4 * g);
#pragma unroll
      for (int cb = 0; cb < kTrNCB; ++cb) H2[cb][rb] = bv;
#pragma unroll
      for (int ku = 0; ku < 4; ++ku) {
        const f32x4 A = *reinterpret_cast<const f32x4*>(units + f32_unit(1, rb, ku) * kUnitBytes + lane * 16);
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int cb = 0; cb < kTrNCB; ++cb)
            H2[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[e], H1[cb][ku][e], H2[cb][rb], 0, 0, 0);
      }
    }
#pragma unroll
    for (int cb = 0; cb < kTrNCB; ++cb)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) H2[cb][rb][e] = fmaxf(H2[cb][rb][e], 0.f);
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const f32x4 bv = *reinterpret_cast<const f32x4*>(bias + 2 * kH + 16 * rb + 4 * g);
#pragma unroll
      for (int cb = 0; cb < kTrNCB; ++cb) Z3[cb][rb] = bv;
#pragma unroll
      for (int ku = 0; ku < 4; ++ku) {
        const f32x4 A = *reinterpret_cast<const f32x4*>(units + f32_unit(2, rb, ku) * kUnitBytes + lane * 16);
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int cb = 0; cb < kTrNCB; ++cb)
            Z3[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[e], H2[cb][ku][e], Z3[cb][rb], 0, 0, 0);
      }
    }
    // loss and output gradient: alpha^ = 1 - exp(-softplus(z))
    f32x4 dZ3[kTrNCB][2];
#pragma unroll
    for (int cb = 0; cb < kTrNCB; ++cb) {
      const uint32_t it = base + cb * 16 + m;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        f32x4 tg = {0.f, 0.f, 0.f, 0.f};
        if (valid[cb]) tg = *reinterpret_cast<const f32x4*>(alpha + (uint64_t)it * kBins + 16 * rb + 4 * g);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float z = Z3[cb][rb][e];
          const float tau = softplusf(z);
          const float et = expf(-tau);
          const float err = (1.f - et) - tg[e];
          lsum += valid[cb] ? err * err : 0.f;
          dZ3[cb][rb][e] = valid[cb] ? 2.f * err * scale * et * logisticf(z) : 0.f;
        }
      }
    }
    // backward, layer 2 -> 0; stage dZ and inputs feature-major, then dW on MFMA (K = items)
#pragma unroll
    for (int layer = 2; layer >= 0; --layer) {
      const int rbo = layer == 2 ? 2 : 4;
      const int cbi = layer == 0 ? 3 : 4;
      __syncthreads();
#pragma unroll
      for (int cb = 0; cb < kTrNCB; ++cb) {
        const int col = wave * 16 * kTrNCB + cb * 16 + m;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          if (rb >= rbo) break;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float v = layer == 2 ? dZ3[cb][rb < 2 ? rb : 0][e] : (layer == 1 ? H2[cb][rb][e] : H1[cb][rb][e]);
            stf(s_dz, 16 * rb + 4 * g + e, col, v);
          }
        }
        if (layer == 0) {
#pragma unroll
          for (int kb = 0; kb < 12; ++kb) stf(s_h, 4 * kb + g, col, X[cb][kb]);
        } else {
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int e = 0; e < 4; ++e) stf(s_h, 16 * rb + 4 * g + e, col, layer == 2 ? H2[cb][rb][e] : H1[cb][rb][e]);
        }
      }
      __syncthreads();
      // H2/H1 staged into s_dz above hold dZ for layers 1 and 0 (see the chain below)
      const int n_items_l = rbo * cbi;
      const int per = (n_items_l + 3) / 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int item = wave * per + q;
        if (q >= per || item >= n_items_l) break;
        const int rb = item / cbi, ci = item % cbi;
        f32x4 acc = layer == 2 ? aW2[q < 2 ? q : 0] : (layer == 1 ? aW1[q] : aW0[q < 3 ? q : 0]);
        f32x4 accb = layer == 2 ? aB2 : (layer == 1 ? aB1 : aB0);
        for (int kb = 0; kb < kTrItems / 4; ++kb) {
          const float a = ldf(s_dz, 16 * rb + m, 4 * kb + g);
          const float bm = ldf(s_h, 16 * ci + m, 4 * kb + g);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bm, acc, 0, 0, 0);
          if (ci == 0) accb = __builtin_amdgcn_mfma_f32_16x16x4f32(a, 1.f, accb, 0, 0, 0);
        }
        if (layer == 2) { aW2[q < 2 ? q : 0] = acc; if (ci == 0) aB2 = accb; }
        else if (layer == 1) { aW1[q] = acc; if (ci == 0) aB1 = accb; }
        else { aW0[q < 3 ? q : 0] = acc; if (ci == 0) aB0 = accb; }
      }
      if (layer == 0) break;
      // chain: dH = W^T dZ, masked by the forward activation, becomes dZ of the layer below
      if (layer == 2) {
#pragma unroll
        for (int cb = 0; cb < kTrNCB; ++cb)
#pragma unroll
          for (int rb = 0; rb < 4; ++rb) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ku = 0; ku < 2; ++ku) {
              const f32x4 A = *reinterpret_cast<const f32x4*>(units + (f32_bwd_unit(2, rb, ku) - kF32Units + kF32Units) * kUnitBytes + lane * 16);
#pragma unroll
              for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[e], dZ3[cb][ku][e], acc, 0, 0, 0);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) H2[cb][rb][e] = H2[cb][rb][e] > 0.f ? acc[e] : 0.f;
          }
      } else {
#pragma unroll
        for (int cb = 0; cb < kTrNCB; ++cb) {
          f32x4 nd[4];
#pragma unroll
          for (int rb = 0; rb < 4; ++rb) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ku = 0; ku < 4; ++ku) {
              const f32x4 A = *reinterpret_cast<const f32x4*>(units + f32_bwd_unit(1, rb, ku) * kUnitBytes + lane * 16);
#pragma unroll
              for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[e], H2[cb][ku][e], acc, 0, 0, 0);
            }
            nd[rb] = acc;
          }
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int e = 0; e < 4; ++e) H1[cb][rb][e] = H1[cb][rb][e] > 0.f ? nd[rb][e] : 0.f;
        }
      }
    }
  }
  // partial gradient of this block, master layout
  float* dst = part + (uint64_t)blockIdx.x * kP;
#pragma unroll
  for (int layer = 0; layer <= 2; ++layer) {
    const int rbo = layer == 2 ? 2 : 4;
    const int cbi = layer == 0 ? 3 : 4;
    const int n_items_l = rbo * cbi;
    const int per = (n_items_l + 3) / 4;
    const int din = layer == 0 ? kIn : kH;
    const int offw = layer == 0 ? kW0 : (layer == 1 ? kW1 : kW2);
    const int offb = layer == 0 ? kB0 : (layer == 1 ? kB1 : kB2);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int item = wave * per + q;
      if (q >= per || item >= n_items_l) break;
      const int rb = item / cbi, ci = item % cbi;
      const f32x4 acc = layer == 2 ? aW2[q < 2 ? q : 0] : (layer == 1 ? aW1[q] : aW0[q < 3 ? q : 0]);
      const f32x4 accb = layer == 2 ? aB2 : (layer == 1 ? aB1 : aB0);
      const int col = 16 * ci + m;   // staged input row: feature index (layer 0: slot 4 kb + g == feature)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int out = 16 * rb + 4 * g + e;
        if (col < din) dst[offw + out * din + col] = acc[e];
        if (ci == 0 && m == 0) dst[offb + out] = accb[e];
      }
    }
  }
  // loss partial
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
  __shared__ float lsh[4];
  if (lane == 0) lsh[wave] = lsum;
  __syncthreads();
  if (threadIdx.x == 0) loss_part[blockIdx.x] = (lsh[0] + lsh[1]) + (lsh[2] + lsh[3]);
}

__global__ __launch_bounds__(kThreads) void k_prop_reduce(const float* __restrict__ part, uint32_t nb,
                                                          const float* __restrict__ loss_part,
                                                          float* __restrict__ grad,
                                                          float* __restrict__ loss, const uint32_t* __restrict__ n_iv) {
  for (uint32_t p = blockIdx.x * kThreads + threadIdx.x; p < (uint32_t)kP; p += gridDim.x * kThreads) {
    float s = 0.f;
    for (uint32_t b = 0; b < nb; ++b) s += part[(uint64_t)b * kP + p];
    grad[p] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float s = 0.f;
    for (uint32_t b = 0; b < nb; ++b) s += loss_part[b];
    loss[0] = s / ((float)(*n_iv) * (float)kBins);
  }
}

std::atomic<int> g_ncu{0};   // compute units of the device (queried once; host threads may race to it)
hipError_t ncu(int* out) {
  int n = g_ncu.load();
  if (n == 0) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    g_ncu.store(n);
  }
  *out = n;
  return hipSuccess;
}

}  // namespace

int prop_param_count() { return kP; }
size_t prop_packed_bytes(int dtype) { return dtype == AMNERF_BF16 ? kBf16Bytes : kF32Bytes; }
uint32_t prop_train_blocks() {
  int n = 0;
  if (ncu(&n) != hipSuccess || n <= 0) return 256u;   // the device's compute units, else a fixed count
  return (uint32_t)n;
}

hipError_t launch_prop_pack(int dtype, const float* master, void* packed, hipStream_t st) {
  hipLaunchKernelGGL(k_prop_pack, dim3(64), dim3(256), 0, st, dtype, master, (uint8_t*)packed);
  return hipGetLastError();
}

hipError_t launch_prop_fwd(int dtype, const void* packed, const IvSet& iv, const float* o, const float* d,
                           int64_t stride, int64_t r0, const float* leafbox, int s_max, uint32_t n_iv_max,
                           bool cum, float* tau, float* tot, hipStream_t st) {
  int n = 0;
  hipError_t e = ncu(&n);
  if (e != hipSuccess) return e;
  const uint32_t tile = dtype == AMNERF_BF16 ? 128u : 256u;
  uint32_t tiles = (n_iv_max + tile - 1) / tile;
  uint32_t grid = std::min<uint32_t>(tiles > 0 ? tiles : 1, (uint32_t)n * 8);
  if (dtype == AMNERF_BF16)
    hipLaunchKernelGGL(k_prop_fwd<true>, dim3(grid), dim3(kThreads), kBf16Bytes, st, (const uint8_t*)packed, iv, o,
                       d, stride, r0, leafbox, s_max, cum ? 1 : 0, tau, tot);
  else
    hipLaunchKernelGGL(k_prop_fwd<false>, dim3(grid), dim3(kThreads), kBiasBytes + kF32Units * kUnitBytes, st,
                       (const uint8_t*)packed, iv, o, d, stride, r0, leafbox, s_max, cum ? 1 : 0, tau, tot);
  return hipGetLastError();
}

hipError_t launch_prop_select(uint32_t nr, const IvSet& iv, const float* wts, const float* tot, float mass_thresh,
                              int cap, int s_max,
                              uint32_t* runs, uint32_t* nsel, uint64_t* mask, float* mass, ChunkCounts* counts,
                              hipStream_t st) {
  if (nr == 0) return hipSuccess;
  int n = 0;
  hipError_t e = ncu(&n);
  if (e != hipSuccess) return e;
  const uint32_t grid = std::min<uint32_t>((nr + 3) / 4, (uint32_t)n * 16);
  hipLaunchKernelGGL(s_max <= 128 ? k_prop_select<2> : (s_max <= 192 ? k_prop_select<3> : k_prop_select<4>), dim3(grid),
                     dim3(kThreads), 0, st, nr, iv, wts,
                     tot, mass_thresh, cap, runs, nsel,
                     mask, mass, counts);
  return hipGetLastError();
}

hipError_t launch_prop_emit(uint32_t nr, const IvSet& iv, const uint64_t* mask, const uint32_t* pv_off,
                            const uint32_t* ps_off, float* pt0, float* pdt, uint32_t* pkey, uint32_t* pray,
                            uint32_t* pbase, hipStream_t st) {
  if (nr == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prop_emit, dim3((nr + kThreads - 1) / kThreads), dim3(kThreads), 20u * kEmitStage, st, nr, iv,
                     mask, pv_off, ps_off, pt0, pdt, pkey, pray, pbase);
  return hipGetLastError();
}

hipError_t launch_prop_targets(const IvSet& iv, const float* smp_out, float* alpha, hipStream_t st) {
  hipLaunchKernelGGL(k_prop_targets, dim3(2048), dim3(kThreads), 0, st, iv, smp_out, alpha);
  return hipGetLastError();
}

hipError_t launch_prop_train(const void* packed, const IvSet& iv, const float* o, const float* d, int64_t stride,
                             int64_t r0, const float* leafbox, int s_max, const float* alpha, float* part,
                             float* loss_part, float* grad, float* loss, hipStream_t st) {
  const uint32_t nb = prop_train_blocks();
  const uint32_t lds = kF32Bytes + 2u * kH * kTrRow;
  hipError_t e = hipFuncSetAttribute((const void*)k_prop_train, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_prop_train, dim3(nb), dim3(kThreads), lds, st, (const uint8_t*)packed, iv, o, d, stride, r0,
                     leafbox, s_max, alpha, part, loss_part);
  hipLaunchKernelGGL(k_prop_reduce, dim3(36), dim3(kThreads), 0, st, part, nb, loss_part, grad, loss, iv.n_iv_dev);
  return hipGetLastError();
}

}  // namespace amn
