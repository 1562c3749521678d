// mlp.hip -- grouped per-leaf MLP inference on the matrix cores (Section 3.5: after the
// sort, each node's small network runs over its bucket; Section 4.4: small MLPs are fast
// when their weights stay on chip).
//
// Work: the sorted samples of leaf b form rows [bucket_off[b], bucket_off[b+1]); they are
// cut into 256-row tiles that never straddle two leaves.  A persistent grid gives each
// block a contiguous run of tiles, so consecutive tiles mostly share one leaf and the
// leaf's packed parameters are staged into LDS only when the leaf changes.
//
// Data flow inside a wave (64 rows = 4 column blocks of 16 samples): every layer is
// computed transposed, Y^T = W X^T, with the weights as the MFMA A operand (from LDS) and
// the activations as the B operand (in registers).  An MFMA accumulator leaves lane
// (g = lane/16, n = lane%16) holding rows 4g..4g+3 of its 16-row block for sample n; the
// packer orders each layer's K index so that exactly those values are the next layer's B
// operand for that lane.  Activations therefore never leave registers between layers.
// Biases enter as the C operand of the first MFMA of each output block.
//   F32  : v_mfma_f32_16x16x4_f32  (fp32 in, fp32 accumulate)
//   BF16 : v_mfma_f32_16x16x32_bf16 (bf16 in, fp32 accumulate)
//   FP8  : the BF16 kernel; the leaf's e4m3 weights are widened to bf16 (times the layer's
//          scale) while they are staged into LDS, so the block in memory is half the size.
#include <algorithm>
#include <mutex>

#include "internal.hpp"
#include "devcommon.hpp"
#include "mlp_layout.hpp"

#include "../../include/amnerf.h"

namespace amn {

namespace {

constexpr int kThreads = 256;

// float8 e4m3 in the OCP encoding (sign, 4 exponent bits with bias 7, 3 mantissa bits; no
// infinities, 0x7F is NaN, largest finite 448): round to nearest, ties to even, saturating.
__device__ __forceinline__ uint32_t e4m3_encode(float x) {
  const uint32_t sign = x < 0.f ? 0x80u : 0u;
  const float a = fabsf(x);
  if (!(a < 464.f)) return sign | 0x7Eu;            // at or beyond the midpoint above 448
  if (a < 0.015625f) return sign | (uint32_t)rintf(a * 512.f);   // subnormals, step 2^-9 (8 = 2^-6)
  int e2;
  frexpf(a, &e2);                                    // a in [2^(e2-1), 2^e2)
  int E = e2 - 1;
  uint32_t m = (uint32_t)rintf((ldexpf(a, -E) - 1.f) * 8.f);
  if (m == 8u) { m = 0u; ++E; }
  if (E > 8 || (E == 8 && m > 6u)) return sign | 0x7Eu;
  return sign | ((uint32_t)(E + 7) << 3) | m;
}

__device__ __forceinline__ float e4m3_decode(uint32_t b) {
  const uint32_t e = (b >> 3) & 15u, m = b & 7u;
  const float v = e ? __uint_as_float(((e + 120u) << 23) | (m << 20)) : (float)m * 0.001953125f;
  return (b & 0x80u) ? -v : v;
}

// float8 scales: one block per (leaf, layer), max |W| / 448 (1 for an all-zero layer).
__global__ __launch_bounds__(kThreads) void k_fp8_scales(Layout L, int P, const float* __restrict__ master,
                                                          uint8_t* __restrict__ packed) {
  __shared__ float red[kThreads];
  const int leaf = blockIdx.x / (L.nh + 1), layer = blockIdx.x % (L.nh + 1);
  int din, dout, off_w, off_b;
  master_offsets(L.nh, L.H, layer, din, dout, off_w, off_b);
  const float* W = master + (uint64_t)leaf * P + off_w;
  float mx = 0.f;
  for (int i = threadIdx.x; i < din * dout; i += kThreads) mx = fmaxf(mx, fabsf(W[i]));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    float* sc = reinterpret_cast<float*>(packed + (uint64_t)leaf * L.bytes8 + L.bias_bytes);
    sc[layer] = red[0] > 0.f ? red[0] / 448.f : 1.f;
  }
}

// One thread per (leaf, unit, lane): 16 bytes of A fragment (8 for float8).  Plus the bias
// block.
__global__ void k_mlp_pack(Layout L, int n_leaves, int P, const float* __restrict__ master,
                           uint8_t* __restrict__ packed) {
  const uint64_t per_leaf = (uint64_t)L.units * 64;
  const uint64_t total = per_leaf * n_leaves;
  for (uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; id < total;
       id += (uint64_t)gridDim.x * blockDim.x) {
    int leaf = (int)(id / per_leaf);
    int rem = (int)(id % per_leaf);
    int unit = rem / 64, lane = rem % 64;
    int g = lane / 16, m = lane % 16;
    // which layer / rb / ku is this unit
    int layer, rb, ku;
    int n0 = L.RB * L.KU0, nhid = (L.nh - 1) * L.RB * L.KUh;
    if (unit < n0) { layer = 0; rb = unit / L.KU0; ku = unit % L.KU0; }
    else if (unit < n0 + nhid) { int u = unit - n0; layer = 1 + u / (L.RB * L.KUh); u %= L.RB * L.KUh; rb = u / L.KUh; ku = u % L.KUh; }
    else { layer = L.nh; rb = 0; ku = unit - n0 - nhid; }
    int din, dout, off_w, off_b;
    master_offsets(L.nh, L.H, layer, din, dout, off_w, off_b);
    const float* W = master + (uint64_t)leaf * P + off_w;
    int row = 16 * rb + m;
    uint8_t* dst = packed + (uint64_t)leaf * L.bytes + L.bias_bytes + (uint64_t)unit * kUnitBytes + lane * 16;
    const bool b16 = L.dtype == AMNERF_BF16 || L.dtype == AMNERF_FP8;
    int ne = b16 ? 8 : 4;
    float v[8];
    for (int e = 0; e < ne; ++e) {
      int col;
      if (b16) col = layer == 0 ? first_layer_col_bf16(g, e) : 16 * (2 * ku + e / 4) + 4 * g + (e % 4);
      else { int kb = 4 * ku + e; col = layer == 0 ? first_layer_col(g, kb) : 16 * ku + 4 * g + e; }
      v[e] = (row < dout && col >= 0) ? W[row * din + col] : 0.f;
    }
    if (L.dtype == AMNERF_FP8) {
      uint8_t* blk = packed + (uint64_t)leaf * L.bytes8;
      const float sc = reinterpret_cast<const float*>(blk + L.bias_bytes)[layer];
      uint32_t lo = 0, hi = 0;
      for (int e = 0; e < 4; ++e) lo |= e4m3_encode(v[e] / sc) << (8 * e);
      for (int e = 0; e < 4; ++e) hi |= e4m3_encode(v[4 + e] / sc) << (8 * e);
      *reinterpret_cast<uint2*>(blk + L.bias_bytes + kFp8ScaleBytes + (uint64_t)unit * kUnit8Bytes + lane * 8) =
          make_uint2(lo, hi);
    } else if (L.dtype == AMNERF_BF16) {
      bf16x8 h;
      for (int e = 0; e < 8; ++e) h[e] = (__bf16)v[e];
      *(bf16x8*)dst = h;
    } else {
      *(f32x4*)dst = f32x4{v[0], v[1], v[2], v[3]};
    }
  }
  const uint64_t btotal = (uint64_t)(L.bias_bytes / 4) * n_leaves;
  for (uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; id < btotal;
       id += (uint64_t)gridDim.x * blockDim.x) {
    int leaf = (int)(id / (L.bias_bytes / 4));
    int j = (int)(id % (L.bias_bytes / 4));
    float val = 0.f;
    if (j < L.nh * L.H) {
      int l = j / L.H, o = j % L.H, din, dout, off_w, off_b;
      master_offsets(L.nh, L.H, l, din, dout, off_w, off_b);
      val = master[(uint64_t)leaf * P + off_b + o];
    } else if (j < L.nh * L.H + 4) {
      int din, dout, off_w, off_b;
      master_offsets(L.nh, L.H, L.nh, din, dout, off_w, off_b);
      val = master[(uint64_t)leaf * P + off_b + (j - L.nh * L.H)];
    }
    ((float*)(packed + (uint64_t)leaf * (L.dtype == AMNERF_FP8 ? L.bytes8 : L.bytes)))[j] = val;
  }
  // transposed weights for the backward pass: unit (layer l >= 1, rb, ku), lane (g, m)
  // holds W_l^T[in = 16 rb + m][out = hidden_col_bf16(ku, g, e)], e = 0..7
  const uint64_t bper = (uint64_t)L.bwd_units * 64;
  const uint64_t bt = bper * n_leaves;
  uint8_t* bwd = packed + (uint64_t)n_leaves * L.bytes;
  for (uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; id < bt;
       id += (uint64_t)gridDim.x * blockDim.x) {
    int leaf = (int)(id / bper);
    int rem = (int)(id % bper);
    int unit = rem / 64, lane = rem % 64;
    int g = lane / 16, m = lane % 16;
    int per_hidden = L.RB * L.KUh;
    int layer, rb, ku;
    if (unit < (L.nh - 1) * per_hidden) { layer = 1 + unit / per_hidden; rb = (unit % per_hidden) / L.KUh; ku = unit % L.KUh; }
    else { layer = L.nh; rb = unit - (L.nh - 1) * per_hidden; ku = 0; }
    int din, dout, off_w, off_b;
    master_offsets(L.nh, L.H, layer, din, dout, off_w, off_b);
    const float* W = master + (uint64_t)leaf * P + off_w;
    int in = 16 * rb + m;
    bf16x8 h;
    for (int e = 0; e < 8; ++e) {
      int out = hidden_col_bf16(ku, g, e);
      h[e] = (__bf16)((out < dout && in < din) ? W[out * din + in] : 0.f);
    }
    *(bf16x8*)(bwd + (uint64_t)leaf * L.bwd_bytes + (uint64_t)unit * kUnitBytes + lane * 16) = h;
  }
}

// ---- BF16 layer steps.  Activations between layers are ReLU'd bf16 B operands: H[cb][ku]
// packs accumulator rows 2ku (elements 0..3) and 2ku+1 (elements 4..7) of column block
// cb, two values per register.  A layer walks its output row blocks and converts the
// previous block's results while the current block's MFMAs run, so the MFMA result
// latency is not waited for in line.
template <int H, int NCB, int KIN>
__device__ __forceinline__ void bf16_layer(const Layout& L, const uint8_t* units, const float* bias, int layer, int lane,
                                           int g, const uint32_t (&Hin)[NCB][KIN][4], uint32_t (&Hout)[NCB][H / 32][4]) {
  constexpr int RB = H / 16;
  f32x4 c[2][NCB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int cur = rb & 1, prv = cur ^ 1;
    bf16x8 A[KIN];
#pragma unroll
    for (int ku = 0; ku < KIN; ++ku)
      A[ku] = *reinterpret_cast<const bf16x8*>(units + L.unit_index(layer, rb, ku) * kUnitBytes + lane * 16);
    const f32x4 bv = *reinterpret_cast<const f32x4*>(bias + layer * H + 16 * rb + 4 * g);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) c[cur][cb] = bv;
#pragma unroll
    for (int ku = 0; ku < KIN; ++ku)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        c[cur][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ku], __builtin_bit_cast(bf16x8, Hin[cb][ku]),
                                                             c[cur][cb], 0, 0, 0);
    if (rb > 0) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        Hout[cb][(rb - 1) >> 1][2 * ((rb - 1) & 1)] = relu_bf16_pair(c[prv][cb][0], c[prv][cb][1]);
        Hout[cb][(rb - 1) >> 1][2 * ((rb - 1) & 1) + 1] = relu_bf16_pair(c[prv][cb][2], c[prv][cb][3]);
      }
    }
  }
  constexpr int last = (RB - 1) & 1;
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    Hout[cb][(RB - 1) >> 1][2 * ((RB - 1) & 1)] = relu_bf16_pair(c[last][cb][0], c[last][cb][1]);
    Hout[cb][(RB - 1) >> 1][2 * ((RB - 1) & 1) + 1] = relu_bf16_pair(c[last][cb][2], c[last][cb][3]);
  }
}

// Output layer H -> 4 (padded to 16): float pre-activations of column block cb.
template <int H, int NCB>
__device__ __forceinline__ void bf16_out(const Layout& L, const uint8_t* units, const float* bias, int lane, int g,
                                         const uint32_t (&Hin)[NCB][H / 32][4], f32x4 (&out)[NCB]) {
  constexpr int KUh = H / 32;
  bf16x8 A[KUh];
#pragma unroll
  for (int ku = 0; ku < KUh; ++ku)
    A[ku] = *reinterpret_cast<const bf16x8*>(units + L.unit_index(L.nh, 0, ku) * kUnitBytes + lane * 16);
  const f32x4 bv = *reinterpret_cast<const f32x4*>(bias + L.nh * H + 4 * g);
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) out[cb] = bv;
#pragma unroll
  for (int ku = 0; ku < KUh; ++ku)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
      out[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ku], __builtin_bit_cast(bf16x8, Hin[cb][ku]), out[cb], 0, 0, 0);
}

// Stages leaf b's parameters into LDS in the on-chip bfloat16 (or float32) layout.  A
// float8 block is expanded on the way: each 8-byte lane fragment becomes the 16-byte
// bfloat16 fragment of the same unit and lane, every weight times its layer's scale.
template <bool FP8>
__device__ __forceinline__ void stage_leaf(const Layout& L, const uint8_t* __restrict__ packed, uint32_t b,
                                           uint8_t* lds, int tid) {
  if constexpr (FP8) {
    const uint8_t* blk = packed + (uint64_t)b * L.bytes8;
    const f32x4* bsrc = reinterpret_cast<const f32x4*>(blk);
    for (int i = tid; i < L.bias_bytes / 16; i += kThreads) reinterpret_cast<f32x4*>(lds)[i] = bsrc[i];
    const float* scale = reinterpret_cast<const float*>(blk + L.bias_bytes);
    const uint2* wsrc = reinterpret_cast<const uint2*>(blk + L.bias_bytes + kFp8ScaleBytes);
    for (int i = tid; i < L.units * 64; i += kThreads) {
      const uint2 q = wsrc[i];
      const float s = scale[L.layer_of_unit(i >> 6)];
      float f[8];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        f[e] = e4m3_decode((q.x >> (8 * e)) & 255u) * s;
        f[4 + e] = e4m3_decode((q.y >> (8 * e)) & 255u) * s;
      }
      *reinterpret_cast<bf16x8*>(lds + L.bias_bytes + (uint32_t)i * 16) = cvt_bf16x8(f);
    }
  } else {
    const f32x4* src = reinterpret_cast<const f32x4*>(packed + (uint64_t)b * L.bytes);
    f32x4* dst = reinterpret_cast<f32x4*>(lds);
    for (uint32_t i = tid; i < L.bytes / 16; i += kThreads) dst[i] = src[i];
  }
}

template <int H, bool BF16, bool FP8 = false>
__global__ __launch_bounds__(kThreads, BF16 ? 4 : 2) void k_mlp(
    Layout L, const uint8_t* __restrict__ packed, uint32_t n_leaves,
    const uint32_t* __restrict__ bucket_off, const uint32_t* __restrict__ tile_off,
    const ChunkCounts* __restrict__ counts, const uint32_t* __restrict__ srec_ray,
    const float* __restrict__ srec_t, const uint32_t* __restrict__ perm,
    const float* __restrict__ o, const float* __restrict__ d, int64_t stride, int64_t r0,
    float* __restrict__ out) {
  extern __shared__ __align__(16) uint8_t lds[];
  constexpr int RB = H / 16;
  constexpr int NCB = 4;                       // column blocks per wave
  constexpr int KUh = BF16 ? H / 32 : H / 16;  // K units of a hidden-width input
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, m = lane & 15;
  const float* bias = reinterpret_cast<const float*>(lds);
  const uint8_t* units = lds + L.bias_bytes;

  const uint32_t T = counts->n_tiles;
  const uint32_t tb = (uint32_t)(((uint64_t)blockIdx.x * T) / gridDim.x);
  const uint32_t te = (uint32_t)(((uint64_t)(blockIdx.x + 1) * T) / gridDim.x);
  if (tb >= te) return;
  // leaf of the first tile: largest b with tile_off[b] <= tb
  uint32_t lo = 0, hi = n_leaves;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (tile_off[mid] <= tb) lo = mid; else hi = mid;
  }
  uint32_t b = lo;
  int cur = -1;
  // Inputs of the wave's 64 rows of the next tile, one row per lane: the sample record is
  // loaded a tile ahead and the ray's origin and direction are gathered during the current
  // tile's first layer, so neither load is waited for at the start of a tile.
  uint32_t qb = lo, q_row0 = 0, q_end = 0;
  uint32_t n_ray = 0, n_perm = 0;
  float n_t = 0.f, n_o[3] = {0.f, 0.f, 0.f}, n_d[3] = {0.f, 0.f, 0.f};
  auto next_rows = [&](uint32_t tt) {
    while (tile_off[qb + 1] <= tt) ++qb;
    q_row0 = bucket_off[qb] + (tt - tile_off[qb]) * kMlpTileRows + wave * 64;
    q_end = bucket_off[qb + 1];
    const uint32_t row = q_row0 + lane;
    n_ray = 0u; n_perm = 0u; n_t = 0.f;
    if (row < q_end) {
      n_ray = srec_ray[row];
      n_t = srec_t[row];
      n_perm = perm[row];
    }
  };
  auto gather = [&]() {
    const int64_t ri = r0 + n_ray;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      n_o[a] = o[a * stride + ri];
      n_d[a] = d[a * stride + ri];
    }
  };
  next_rows(tb);
  gather();
  for (uint32_t t = tb; t < te; ++t) {
    while (tile_off[b + 1] <= t) ++b;
    if ((int)b != cur) {
      __syncthreads();
      stage_leaf<FP8>(L, packed, b, lds, tid);
      __syncthreads();
      cur = (int)b;
    }
    const uint32_t row0 = q_row0, row_end = q_end;
    const uint32_t c_perm = n_perm;
    // this lane's row: sample position mapped to [-1, 1]^3, and the direction
    float c_p[3], c_d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c_d[a] = n_d[a];
      c_p[a] = 2.f * fmaf(n_t, n_d[a], n_o[a]) - 1.f;
    }
    const bool more = t + 1 < te;
    if (more) next_rows(t + 1);
    if (row0 >= row_end) {
      if (more) gather();
      continue;
    }

    // ---- inputs: positional encoding of this lane's 8 features for 4 samples ----
    float feat[NCB][8];   // float32 inputs (the BF16 path packs them at once into X0)
    bf16x8 X0[NCB];
    uint32_t dst_idx[NCB];
    bool valid[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int src = cb * 16 + m;   // lane holding row cb * 16 + m
      valid[cb] = row0 + (uint32_t)src < row_end;
      dst_idx[cb] = (uint32_t)__shfl((int)c_perm, src, 64);
      float px = __shfl(c_p[0], src, 64), py = __shfl(c_p[1], src, 64), pz = __shfl(c_p[2], src, 64);
      float dx = __shfl(c_d[0], src, 64), dy = __shfl(c_d[1], src, 64), dz = __shfl(c_d[2], src, 64);
      if (BF16) {
        // this lane group's coordinate at frequencies 1, 2, 4, 8 (times pi): the hardware
        // sine takes revolutions, sin(2 pi r) with r = v / 2 exactly; higher frequencies by
        // sin 2a = 2 sin a cos a, cos 2a = 1 - 2 sin^2 a
        float v = g == 1 ? py : (g == 2 ? pz : px);
        float sn = __builtin_amdgcn_sinf(0.5f * v);
        float cs = __builtin_amdgcn_cosf(0.5f * v);
        float f[8];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          f[2 * k] = sn;
          f[2 * k + 1] = cs;
          float t2 = sn + sn;
          float s2 = t2 * cs;
          cs = fmaf(-t2, sn, 1.f);
          sn = s2;
        }
        if (g == 3) {
          f[0] = px; f[1] = py; f[2] = pz;
          f[3] = dx; f[4] = dy; f[5] = dz;
          f[6] = 0.f; f[7] = 0.f;
        }
        X0[cb] = cvt_bf16x8(f);
      } else {
        float sc = (float)(1 << g);
        float s0 = sinpif(px * sc), c0 = cospif(px * sc);
        float s1 = sinpif(py * sc), c1 = cospif(py * sc);
        float s2 = sinpif(pz * sc), c2 = cospif(pz * sc);
        feat[cb][0] = s0; feat[cb][1] = s1; feat[cb][2] = s2;
        feat[cb][3] = c0; feat[cb][4] = c1; feat[cb][5] = c2;
        float e0 = g == 0 ? px : (g == 1 ? pz : (g == 2 ? dy : 0.f));
        float e1 = g == 0 ? py : (g == 1 ? dx : (g == 2 ? dz : 0.f));
        feat[cb][6] = e0;
        feat[cb][7] = e1;
      }
    }

    f32x4 acc[NCB][RB];
    if constexpr (BF16) {
      // layer 0 reads the packed inputs (one K unit), then the hidden layers alternate
      // between two activation buffers, two layers per step
      uint32_t X0u[NCB][1][4];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const uint32_t* w = reinterpret_cast<const uint32_t*>(&X0[cb]);
#pragma unroll
        for (int i = 0; i < 4; ++i) X0u[cb][0][i] = w[i];
      }
      uint32_t Ha[NCB][KUh][4], Hb[NCB][KUh][4];
      bf16_layer<H, NCB, 1>(L, units, bias, 0, lane, g, X0u, Ha);
      __builtin_amdgcn_sched_barrier(0);
      if (more) gather();
      __builtin_amdgcn_sched_barrier(0);
      int layer = 1;
      for (; layer + 1 < L.nh; layer += 2) {
        bf16_layer<H, NCB, KUh>(L, units, bias, layer, lane, g, Ha, Hb);
        bf16_layer<H, NCB, KUh>(L, units, bias, layer + 1, lane, g, Hb, Ha);
      }
      f32x4 res[NCB];
      if (layer < L.nh) {
        bf16_layer<H, NCB, KUh>(L, units, bias, layer, lane, g, Ha, Hb);
        bf16_out<H, NCB>(L, units, bias, lane, g, Hb, res);
      } else {
        bf16_out<H, NCB>(L, units, bias, lane, g, Ha, res);
      }
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[cb][0] = res[cb];
    } else {
    // ---- layer 0: 32 (padded) -> H ----
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      f32x4 bv = *reinterpret_cast<const f32x4*>(bias + 16 * rb + 4 * g);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[cb][rb] = bv;
#pragma unroll
      for (int ku = 0; ku < 2; ++ku) {
        f32x4 A = *reinterpret_cast<const f32x4*>(units + L.unit_index(0, rb, ku) * kUnitBytes + lane * 16);
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
            acc[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[e], feat[cb][4 * ku + e], acc[cb][rb], 0, 0, 0);
      }
    }

    __builtin_amdgcn_sched_barrier(0);
    if (more) gather();
    __builtin_amdgcn_sched_barrier(0);
    // ---- hidden layers H -> H, then the output layer H -> 4 (padded to 16) ----
    for (int layer = 1; layer <= L.nh; ++layer) {
      const bool last = layer == L.nh;
      const int nrb = last ? 1 : RB;
      f32x4 nacc[NCB][RB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[cb][rb][e] = fmaxf(acc[cb][rb][e], 0.f);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        if (rb >= nrb) break;
        f32x4 bv = *reinterpret_cast<const f32x4*>(bias + (layer * H) + 16 * rb + 4 * g);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) nacc[cb][rb] = bv;
#pragma unroll
        for (int ku = 0; ku < KUh; ++ku) {
          f32x4 A = *reinterpret_cast<const f32x4*>(units + L.unit_index(layer, rb, ku) * kUnitBytes + lane * 16);
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
        for (int rb = 0; rb < RB; ++rb)
          if (rb < nrb) acc[cb][rb] = nacc[cb][rb];
    }
    }

    // ---- lanes of group 0 hold the pre-activations (sigma^, r^, g^, b^) of their sample;
    //      the compositing kernel applies softplus / logistic ----
    if (g == 0) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        if (valid[cb]) *reinterpret_cast<f32x4*>(out + 4 * (uint64_t)dst_idx[cb]) = acc[cb][0];
    }
  }
}

template <int H, bool BF16, bool FP8 = false>
hipError_t launch_typed(const Layout& L, const void* packed, uint32_t n_leaves, const uint32_t* bucket_off,
                        const uint32_t* tile_off, const ChunkCounts* counts, const uint32_t* srec_ray,
                        const float* srec_t, const uint32_t* perm, const float* o, const float* d,
                        int64_t stride, int64_t r0, float* out, hipStream_t st) {
  auto kern = k_mlp<H, BF16, FP8>;
  int grid = 0;
  hipError_t e = persistent_grid((const void*)kern, kThreads, L.bytes, &grid);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), L.bytes, st, L, (const uint8_t*)packed, n_leaves,
                     bucket_off, tile_off, counts, srec_ray, srec_t, perm, o, d, stride, r0, out);
  return hipGetLastError();
}

}  // namespace

hipError_t persistent_grid(const void* kern, int threads, uint32_t lds, int* grid) {
  // a fixed table (no heap allocation on this path); when full, grids are recomputed
  struct Entry {
    const void* kern;
    int dev;
    uint32_t lds;
    int grid;
  };
  constexpr int kEntries = 128;
  static std::mutex mu;
  static Entry table[kEntries];
  static int used = 0;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (int i = 0; i < used; ++i)
      if (table[i].kern == kern && table[i].dev == dev && table[i].lds == lds) {
        *grid = table[i].grid;
        return hipSuccess;
      }
  }
  int ncu = 0, per = 0;
  e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = resident_blocks(kern, threads, lds, &per);
  if (e != hipSuccess) return e;
  *grid = ncu * per;
  std::lock_guard<std::mutex> lk(mu);
  if (used < kEntries) table[used++] = {kern, dev, lds, *grid};
  return hipSuccess;
}

hipError_t resident_blocks(const void* kern, int threads, uint32_t lds, int* per_cu) {
  int dev = 0, lds_cu = 0, per_regs = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_regs, kern, threads, 0);
  if (e != hipSuccess) return e;
  int per = per_regs;
  if (lds > 0 && lds_cu > 0) per = std::min(per, (int)((uint32_t)lds_cu / lds));
  *per_cu = per > 0 ? per : 1;
  return hipSuccess;
}

bool mlp_geom(int n_hidden, int hidden, int dtype, MlpGeom* g) {
  if (n_hidden < 1 || n_hidden > 8) return false;
  if (hidden != 32 && hidden != 64) return false;
  if (dtype == AMNERF_FP8_ACT) {
    if (hidden != 64 || n_hidden > 4) return false;
    g->n_hidden = n_hidden;
    g->hidden = hidden;
    g->dtype = dtype;
    g->node_bytes = mlp8_block_bytes(n_hidden);
    g->bwd_node_bytes = 0;
    return true;
  }
  if (dtype != AMNERF_F32 && dtype != AMNERF_BF16 && dtype != AMNERF_FP8) return false;
  Layout L = make_layout(n_hidden, hidden, dtype);
  if (L.bytes > 160 * 1024) return false;
  g->n_hidden = n_hidden;
  g->hidden = hidden;
  g->dtype = dtype;
  g->node_bytes = dtype == AMNERF_FP8 ? L.bytes8 : L.bytes;
  g->bwd_node_bytes = L.bwd_bytes;
  return true;
}

hipError_t launch_mlp_pack(const MlpGeom& g, int n_leaves, const float* master, void* packed,
                           hipStream_t st) {
  if (g.dtype == AMNERF_FP8_ACT) return launch_mlp8_pack(g.n_hidden, n_leaves, master, nullptr, packed, st);
  Layout L = make_layout(g.n_hidden, g.hidden, g.dtype);
  int P = master_param_count(g.n_hidden, g.hidden);
  if (g.dtype == AMNERF_FP8)
    hipLaunchKernelGGL(k_fp8_scales, dim3(n_leaves * (g.n_hidden + 1)), dim3(kThreads), 0, st, L, P, master,
                       (uint8_t*)packed);
  hipLaunchKernelGGL(k_mlp_pack, dim3(1024), dim3(256), 0, st, L, n_leaves, P, master, (uint8_t*)packed);
  return hipGetLastError();
}

hipError_t launch_mlp(const MlpGeom& g, const void* packed, uint32_t n_leaves, const uint32_t* bucket_off,
                      const uint32_t* tile_off, const ChunkCounts* counts, const uint32_t* srec_ray,
                      const float* srec_t, const uint32_t* perm, const float* o, const float* d,
                      int64_t ray_stride, int64_t r0, float* out, hipStream_t st) {
  if (g.dtype == AMNERF_FP8_ACT)
    return launch_mlp8(g.n_hidden, packed, n_leaves, bucket_off, tile_off, counts, srec_ray, srec_t, perm, o, d,
                       ray_stride, r0, out, st);
  Layout L = make_layout(g.n_hidden, g.hidden, g.dtype);
  if (g.dtype == AMNERF_FP8) {
    if (g.hidden == 64) return launch_typed<64, true, true>(L, packed, n_leaves, bucket_off, tile_off, counts, srec_ray, srec_t, perm, o, d, ray_stride, r0, out, st);
    return launch_typed<32, true, true>(L, packed, n_leaves, bucket_off, tile_off, counts, srec_ray, srec_t, perm, o, d, ray_stride, r0, out, st);
  }
  if (g.dtype == AMNERF_BF16) {
    if (g.hidden == 64) return launch_typed<64, true>(L, packed, n_leaves, bucket_off, tile_off, counts, srec_ray, srec_t, perm, o, d, ray_stride, r0, out, st);
    return launch_typed<32, true>(L, packed, n_leaves, bucket_off, tile_off, counts, srec_ray, srec_t, perm, o, d, ray_stride, r0, out, st);
  }
  if (g.hidden == 64) return launch_typed<64, false>(L, packed, n_leaves, bucket_off, tile_off, counts, srec_ray, srec_t, perm, o, d, ray_stride, r0, out, st);
  return launch_typed<32, false>(L, packed, n_leaves, bucket_off, tile_off, counts, srec_ray, srec_t, perm, o, d, ray_stride, r0, out, st);
}

}  // namespace amn
