// mlp8.hip -- grouped per-leaf MLP with float8 e4m3 weights and activations on the float8
// matrix cores (Section 3.5: after the sort each node's small network runs over its bucket;
// Section 4.4: small MLPs are fast when their weights stay on chip).  Hidden width 64,
// 1..4 hidden layers.  Not in the paper, which computes in full precision.
//
// Model (every scale a power of two, so every rescaling is exact):
//   * layer 0 (30 inputs -> 64): bfloat16 weights and bfloat16 positional-encoding inputs on
//     v_mfma_f32_32x32x16_bf16;
//   * layers 1..n_hidden (hidden and output): e4m3 weight codes W / 2^e (e the smallest
//     exponent with max |W| <= 448 * 2^e) times e4m3 activation codes on
//     v_mfma_scale_f32_32x32x64_f8f6f4, float32 accumulation;
//   * hidden layer j's ReLU outputs a are held as e4m3(min(a / 2^k_j, 256)), k_j from the
//     calibration maximum m of that leaf and layer (the smallest k with 1.25 m <= 256 * 2^k).
// Each hidden layer's accumulator comes out already divided by 256 * 2^k of its own
// activations: layer 0's weights are pre-scaled by 2^-(k_0 + 8), and the weight operand of
// layer l >= 1 carries the block scale 2^(e_l + k_(l-1) - k_l - 8), its bias b / 2^(k_l + 8)
// (the output layer: 2^(e_n + k_(n-1)), its bias unscaled).  Conversion to the next layer's
// operand is then one bias add per value that carries the clamp bit (ReLU and saturation
// at full rate) and one packed conversion per two values that multiplies by 2^8.
//
// Data flow inside a wave (64 rows = 2 column blocks of 32 samples): every layer is
// computed transposed, Y^T = W X^T, weights as the A operand, activations as the B operand.
// A 32x32 accumulator leaves lane (h = lane / 32, c = lane % 32) holding rows 8j + 4h + i
// (register 4j + i) of its 32-row block for sample c, so with both row blocks a lane holds
// 32 of the 64 outputs of sample c -- exactly the 32 K bytes that lane supplies to the next
// layer's B operand (byte 16 rb + 4 j + i); the packer orders every weight row's K bytes
// the same way.  Activations never leave registers.  A block stages its leaf's parameter
// block (about 20 KB for 4 hidden layers) in LDS when the leaf changes, and every wave reads
// each weight operand from there as it needs it (32 bytes per lane per 32-row block), which
// leaves registers for three waves per SIMD.  Biases of the layers whose outputs are
// activations are float32, stored per layer in accumulator order (the 16 rows of each lane
// half of each row block), read from LDS at the start of the layer and added by the
// clamping add; the output layer's is broadcast over the 32 columns by one bfloat16 MFMA
// (A = its high and low parts in two K slots, B = ones) and taken as the accumulator input.
#include <algorithm>

#include "internal.hpp"
#include "devcommon.hpp"
#include "mlp_layout.hpp"

#include "../../include/amnerf.h"

namespace amn {

namespace {

typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kThreads8 = 256;
constexpr int kHdrBytes = 64;            // int32 header: k_j [0..3], e_l [4..7], block scale [8..11]
constexpr int kFrag = 1024;              // 64 lanes x 16 bytes (bfloat16 layer 0)
constexpr int kFrag8 = 2048;             // 64 lanes x 32 bytes (a float8 weight operand)
constexpr int kBiasBlock = 256;          // one layer's activation biases: float [rb][h][16]
constexpr int kBiasWord = 256;           // the output bias broadcast operand: 64 lanes x 4 bytes

struct Layout8 {
  int nh;
  uint32_t off_l0, off_hid, off_out, off_bias, off_obias, bytes;
};

__host__ __device__ inline Layout8 make_layout8(int nh) {
  Layout8 L;
  L.nh = nh;
  L.off_l0 = kHdrBytes;
  L.off_hid = L.off_l0 + 4 * kFrag;                       // (rb, s) fragments
  L.off_out = L.off_hid + (uint32_t)(nh - 1) * 2 * kFrag8; // per layer, rb: 32 bytes per lane
  L.off_bias = L.off_out + kFrag8;                        // output: 32 bytes per lane
  L.off_obias = L.off_bias + (uint32_t)nh * kBiasBlock;   // layers 0 .. nh-1: biases in C order
  const uint32_t end = L.off_obias + kBiasWord;
  L.bytes = (end + 255u) / 256u * 256u;
  return L;
}

// Input feature in byte/element e of K step s of lane half h (layer 0, bfloat16 B operand):
// half 0 holds coordinate x at the four frequencies (step 0) and y (step 1), half 1 holds z
// (step 0) and then p, d and two zero slots (-1, step 1).  sin / cos pairs alternate.
__host__ __device__ inline int l0_feature(int s, int h, int e) {
  if (s == 1 && h == 1) return e < 3 ? e : (e < 6 ? 27 + (e - 3) : -1);
  const int coord = h == 0 ? (s == 0 ? 0 : 1) : 2;
  return 3 + 6 * (e / 2) + 3 * (e % 2) + coord;
}

// Hidden unit in K byte e (0..31) of lane half h of a 64-wide layer input: accumulator
// register 4 j + i of row block rb of the previous layer, e = 16 rb + 4 j + i.
__host__ __device__ inline int hid_unit(int h, int e) {
  return 32 * (e / 16) + 8 * ((e % 16) / 4) + 4 * h + (e % 4);
}

// Smallest integer e with m <= limit * 2^e (m > 0), 0 for m <= 0; exact in double.
__device__ inline int pow2_exponent(double m, double limit) {
  if (!(m > 0.0)) return 0;
  int e;
  frexp(m / limit, &e);
  while (m > ldexp(limit, e)) ++e;
  while (m <= ldexp(limit, e - 1)) --e;
  return e;
}

__device__ inline uint32_t bf16_bits(float x) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){x, 0.f}, bf16x2)) & 0xFFFFu;
}
__device__ inline float bf16_value(uint32_t bits) { return __uint_as_float(bits << 16); }

// Exponents of one leaf per block: k_j from the calibration maxima (0 without them), e_l
// from max |W_l|, and the E8M0 block scale of each float8 layer's weight operand.
__global__ __launch_bounds__(kThreads8) void k_mlp8_exps(int nh, int P, const float* __restrict__ master,
                                                         const float* __restrict__ act_max, uint8_t* __restrict__ packed) {
  __shared__ float red[kThreads8];
  const Layout8 L = make_layout8(nh);
  const int leaf = blockIdx.x;
  const float* Wl = master + (uint64_t)leaf * P;
  int ew[4] = {0, 0, 0, 0};
  for (int l = 1; l <= nh; ++l) {
    int din, dout, off_w, off_b;
    master_offsets(nh, 64, l, din, dout, off_w, off_b);
    float mx = 0.f;
    for (int i = threadIdx.x; i < din * dout; i += kThreads8) mx = fmaxf(mx, fabsf(Wl[off_w + i]));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = kThreads8 / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
      __syncthreads();
    }
    ew[l - 1] = pow2_exponent((double)red[0], 448.0);
    __syncthreads();
  }
  {
    uint8_t* blk = packed + (uint64_t)leaf * L.bytes;
    for (uint32_t i = L.off_obias + kBiasWord + threadIdx.x; i < L.bytes; i += kThreads8) blk[i] = 0;
  }
  if (threadIdx.x == 0) {
    int* hdr = reinterpret_cast<int*>(packed + (uint64_t)leaf * L.bytes);
    int k[4] = {0, 0, 0, 0};
    for (int j = 0; j < nh; ++j) k[j] = act_max ? pow2_exponent(1.25 * (double)act_max[(uint64_t)leaf * nh + j], 256.0) : 0;
    for (int j = 0; j < 4; ++j) {
      hdr[j] = j < nh ? k[j] : 0;
      hdr[4 + j] = j < nh ? ew[j] : 0;
      int sc = 0;
      if (j < nh) {
        const int kout = j + 1 < nh ? k[j + 1] + 8 : 0;
        sc = min(254, max(0, 127 + ew[j] + k[j] - kout));
      }
      hdr[8 + j] = sc;
    }
    for (int j = 12; j < 16; ++j) hdr[j] = 0;
  }
}

// One thread per (leaf, item): a 16-byte lane fragment of a weight layer, one bias of a
// layer whose outputs are activations, or the output layer's 4-byte bias lane word.  Reads
// the exponents k_mlp8_exps wrote.
__global__ void k_mlp8_pack(int nh, int n_leaves, int P, const float* __restrict__ master, uint8_t* __restrict__ packed) {
  const Layout8 L = make_layout8(nh);
  const int frags = 4 + (nh - 1) * 4 + 2;                 // 16-byte lane fragments per leaf
  const int per_leaf = frags * 64 + nh * 64 + 64;
  const uint64_t total = (uint64_t)per_leaf * n_leaves;
  for (uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; id < total;
       id += (uint64_t)gridDim.x * blockDim.x) {
    const int leaf = (int)(id / per_leaf);
    int rem = (int)(id % per_leaf);
    uint8_t* blk = packed + (uint64_t)leaf * L.bytes;
    const int* hdr = reinterpret_cast<const int*>(blk);
    const float* Wm = master + (uint64_t)leaf * P;
    if (rem < frags * 64) {
      const int f = rem / 64, lane = rem % 64, h = lane / 32, c = lane % 32;
      if (f < 4) {                                        // layer 0: fragment (rb, s)
        const int rb = f / 2, s = f % 2;
        int din, dout, off_w, off_b;
        master_offsets(nh, 64, 0, din, dout, off_w, off_b);
        const int row = 32 * rb + c, k0 = hdr[0] + 8;
        uint32_t w[4];
        for (int q = 0; q < 4; ++q) {
          uint32_t two = 0;
          for (int t = 0; t < 2; ++t) {
            const int col = l0_feature(s, h, 2 * q + t);
            const uint32_t bits = col >= 0 ? bf16_bits(ldexpf(Wm[off_w + row * din + col], -k0)) : 0u;
            two |= bits << (16 * t);
          }
          w[q] = two;
        }
        *reinterpret_cast<i32x4*>(blk + L.off_l0 + f * kFrag + lane * 16) =
            i32x4{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
      } else {                                            // float8 layer: 16 of the lane's 32 K bytes
        const int g = f - 4;
        const int layer = g / 4 < nh - 1 ? 1 + g / 4 : nh;
        const int part = layer < nh ? g % 4 : g - 4 * (nh - 1);   // (rb, half) or (half)
        const int rb = layer < nh ? part / 2 : 0, half = layer < nh ? part % 2 : part;
        int din, dout, off_w, off_b;
        master_offsets(nh, 64, layer, din, dout, off_w, off_b);
        const int row = 32 * rb + c, e_w = hdr[4 + layer - 1];
        uint32_t w[4];
        for (int q = 0; q < 4; ++q) {
          float v[4];
          for (int t = 0; t < 4; ++t) {
            const int unit = hid_unit(h, 16 * half + 4 * q + t);
            v[t] = row < dout ? ldexpf(Wm[off_w + row * din + unit], -e_w) : 0.f;   // |v| <= 448
          }
          int lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], 0, false);
          w[q] = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], lo, true);
        }
        const uint32_t off = layer < nh ? L.off_hid + (uint32_t)((layer - 1) * 2 + rb) * kFrag8 : L.off_out;
        *reinterpret_cast<i32x4*>(blk + off + lane * 32 + half * 16) = i32x4{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
      }
    } else if (rem < frags * 64 + nh * 64) {            // bias of layer l < nh over 2^(k_l + 8)
      rem -= frags * 64;
      const int layer = rem / 64, idx = rem % 64;
      const int rb = idx / 32, h = (idx / 16) % 2, v = idx % 16;
      int din, dout, off_w, off_b;
      master_offsets(nh, 64, layer, din, dout, off_w, off_b);
      const int row = 32 * rb + 8 * (v / 4) + 4 * h + (v % 4);   // accumulator register v of half h
      *reinterpret_cast<float*>(blk + L.off_bias + (uint32_t)layer * kBiasBlock + idx * 4) =
          ldexpf(Wm[off_b + row], -(hdr[layer] + 8));      // exact
    } else {                                              // output bias word: lanes of half 0
      const int lane = rem - frags * 64 - nh * 64, h = lane / 32, c = lane % 32;
      int din, dout, off_w, off_b;
      master_offsets(nh, 64, nh, din, dout, off_w, off_b);
      uint32_t word = 0;
      if (h == 0 && c < dout) {
        const float bs = Wm[off_b + c];
        const uint32_t bhi = bf16_bits(bs);
        word = bhi | (bf16_bits(bs - bf16_value(bhi)) << 16);
      }
      *reinterpret_cast<uint32_t*>(blk + L.off_obias + lane * 4) = word;
    }
  }
}

// ReLU, saturation and e4m3 conversion of both column blocks: the next layer's 32-byte B
// operands (byte 16 rb + 4 j + i = register 4 j + i of row block rb).  The accumulators plus
// the layer's biases (b[rb][j] = the biases of registers 4 j .. 4 j + 3 of row block rb of
// this lane half) hold activations over 256 * 2^k; they are clamped to [0, 1] -- ReLU and
// saturation in the bias add itself, which carries the clamp bit at full rate -- and the
// conversion divides by the exponent of its scale operand, 2^-8, so the codes are
// e4m3(min(a / 2^k, 256)).
__device__ __forceinline__ void to_fp8(const f32x16 (&a)[2][2], const f32x4 (&b)[2][4], i32x8 (&act)[2]) {
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    const int rb = w / 4, j = w % 4;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      float x[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) x[i] = __builtin_amdgcn_fmed3f(a[rb][cb][4 * j + i] + b[rb][j][i], 0.f, 1.f);
      // the first conversion writes the low half of a register whose high half the second
      // one overwrites, so x0's own register serves (no zeroing move)
      const s16x2 lo = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(__builtin_bit_cast(s16x2, x[0]), x[0], x[1],
                                                                0.00390625f, false);
      act[cb][w] = __builtin_bit_cast(int, __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(lo, x[2], x[3], 0.00390625f, true));
    }
  }
}

template <int NH>
__global__ __launch_bounds__(kThreads8) void k_mlp8(
    const uint8_t* __restrict__ packed, uint32_t n_leaves, const uint32_t* __restrict__ bucket_off,
    const uint32_t* __restrict__ tile_off, const ChunkCounts* __restrict__ counts,
    const uint32_t* __restrict__ srec_ray, const float* __restrict__ srec_t, const uint32_t* __restrict__ perm,
    const float* __restrict__ o, const float* __restrict__ d, int64_t stride, int64_t r0, float* __restrict__ out) {
  extern __shared__ __align__(16) uint8_t lds[];
  const Layout8 L = make_layout8(NH);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, c = lane & 31;

  const uint32_t T = counts->n_tiles;
  const uint32_t tb = (uint32_t)(((uint64_t)blockIdx.x * T) / gridDim.x);
  const uint32_t te = (uint32_t)(((uint64_t)(blockIdx.x + 1) * T) / gridDim.x);
  if (tb >= te) return;
  uint32_t lo = 0, hi = n_leaves;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (tile_off[mid] <= tb) lo = mid; else hi = mid;
  }
  uint32_t b = lo;
  int cur = -1;

  // the output layer's bias word and the block scales, in registers (the weights and the
  // other biases are read from LDS)
  uint32_t bwo = 0u;
  int sc[NH];
  // B operand of the bias broadcast: K slots 0 and 1 (lanes of half 0) are 1
  uint32_t ones_u[4] = {h == 0 ? 0x3F803F80u : 0u, 0u, 0u, 0u};
  const bf16x8 ones = __builtin_bit_cast(bf16x8, ones_u);
  const f32x16 zero16 = {};

  // the wave's 64 rows of the next tile, one row per lane (see k_mlp)
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
      const f32x4* src = reinterpret_cast<const f32x4*>(packed + (uint64_t)b * L.bytes);
      for (uint32_t i = tid; i < L.bytes / 16; i += kThreads8) reinterpret_cast<f32x4*>(lds)[i] = src[i];
      __syncthreads();
      const int* hdr = reinterpret_cast<const int*>(lds);
#pragma unroll
      for (int l = 0; l < NH; ++l) sc[l] = hdr[8 + l];
      bwo = *reinterpret_cast<const uint32_t*>(lds + L.off_obias + lane * 4);
      cur = (int)b;
    }
    const uint32_t row0 = q_row0, row_end = q_end;
    const uint32_t c_perm = n_perm;
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

    // ---- inputs: lane (h, c) encodes sample cb * 32 + c for both column blocks ----
    bf16x8 X[2][2];
    uint32_t dst[2];
    bool valid[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int src = cb * 32 + c;
      valid[cb] = row0 + (uint32_t)src < row_end;
      dst[cb] = (uint32_t)__shfl((int)c_perm, src, 64);
      const float px = __shfl(c_p[0], src, 64), py = __shfl(c_p[1], src, 64), pz = __shfl(c_p[2], src, 64);
      const float dx = __shfl(c_d[0], src, 64), dy = __shfl(c_d[1], src, 64), dz = __shfl(c_d[2], src, 64);
      // sin / cos of pi * 2^k v for k = 0..3: the hardware sine takes revolutions, sin(2 pi r)
      // with r = v / 2 exactly, then double-angle steps
      float f1[8], f2[8];
      const float v1 = h ? pz : px, v2 = py;
      float s1 = __builtin_amdgcn_sinf(0.5f * v1), k1 = __builtin_amdgcn_cosf(0.5f * v1);
      float s2 = __builtin_amdgcn_sinf(0.5f * v2), k2 = __builtin_amdgcn_cosf(0.5f * v2);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        f1[2 * k] = s1; f1[2 * k + 1] = k1;
        f2[2 * k] = s2; f2[2 * k + 1] = k2;
        const float t1 = s1 + s1, t2 = s2 + s2;
        const float n1 = t1 * k1, n2 = t2 * k2;
        k1 = fmaf(-t1, s1, 1.f); k2 = fmaf(-t2, s2, 1.f);
        s1 = n1; s2 = n2;
      }
      if (h) {
        f2[0] = px; f2[1] = py; f2[2] = pz;
        f2[3] = dx; f2[4] = dy; f2[5] = dz;
        f2[6] = 0.f; f2[7] = 0.f;
      }
      X[cb][0] = cvt_bf16x8(f1);
      X[cb][1] = cvt_bf16x8(f2);
    }

    // Two compiler liberties are taken away with empty asm statements.  The bias and weight
    // loads of a layer do not depend on its input, and would all be hoisted to the top of
    // the tile (the registers of a wave per SIMD); the statement that takes a layer's whole
    // input ties them to it.  And a value used only by the final masked store would be
    // computed under that store's lane mask, but the matrix instructions combine lanes:
    // every lane's operand must be written, so each layer's input and the output are
    // consumed unconditionally.
    uint32_t wl = lane * 32u, hb = (uint32_t)h * 64u;
    f32x4 bias[2][4];
    auto load_bias = [&](int layer) {
      const uint8_t* bl = lds + L.off_bias + (uint32_t)layer * kBiasBlock + hb;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int j = 0; j < 4; ++j) bias[rb][j] = *reinterpret_cast<const f32x4*>(bl + rb * 128 + j * 16);
    };

    // ---- layer 0 (bfloat16) ----
    asm volatile("" : "+v"(hb) : "v"(X[0][0]), "v"(X[1][0]));
    load_bias(0);
    f32x16 acc[2][2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        const bf16x8 w0 = *reinterpret_cast<const bf16x8*>(lds + L.off_l0 + (2 * rb) * kFrag + lane * 16);
        const bf16x8 w1 = *reinterpret_cast<const bf16x8*>(lds + L.off_l0 + (2 * rb + 1) * kFrag + lane * 16);
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w0, X[cb][0], zero16, 0, 0, 0);
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1, X[cb][1], acc[rb][cb], 0, 0, 0);
      }
    __builtin_amdgcn_sched_barrier(0);
    if (more) gather();
    __builtin_amdgcn_sched_barrier(0);
    i32x8 act[2];
    to_fp8(acc, bias, act);

    // ---- hidden layers (float8) ----
#pragma unroll
    for (int l = 0; l < NH - 1; ++l) {
      asm volatile("" : "+v"(hb), "+v"(wl) : "v"(act[0]), "v"(act[1]));
      load_bias(l + 1);
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const i32x8 w = *reinterpret_cast<const i32x8*>(lds + L.off_hid + (l * 2 + rb) * kFrag8 + wl);
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(w, act[cb], zero16, 0, 0, 0, sc[l], 0, 127);
      }
      to_fp8(acc, bias, act);
    }

    // ---- output layer (float8; rows 0..3 are sigma^, r^, g^, b^): the bias, broadcast over
    // the columns by one bfloat16 MFMA (A = its high and low parts in two K slots, B = ones),
    // is the accumulator input ----
    {
      uint32_t bw = bwo;
      asm volatile("" : "+v"(bw), "+v"(wl) : "v"(act[0]), "v"(act[1]));
      const uint32_t bwa[4] = {bw, 0u, 0u, 0u};
      const f32x16 bo = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, bwa), ones, zero16, 0, 0, 0);
      const i32x8 wo = *reinterpret_cast<const i32x8*>(lds + L.off_out + wl);
      f32x16 r0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(wo, act[0], bo, 0, 0, 0, sc[NH - 1], 0, 127);
      f32x16 r1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(wo, act[1], bo, 0, 0, 0, sc[NH - 1], 0, 127);
      asm volatile("" : "+v"(r0), "+v"(r1));
      if (h == 0 && valid[0]) *reinterpret_cast<f32x4*>(out + 4 * (uint64_t)dst[0]) = f32x4{r0[0], r0[1], r0[2], r0[3]};
      if (h == 0 && valid[1]) *reinterpret_cast<f32x4*>(out + 4 * (uint64_t)dst[1]) = f32x4{r1[0], r1[1], r1[2], r1[3]};
    }
  }
}

// ---- calibration: float32 forward of the master parameters over the sorted samples of a
// render; act_max[leaf][j] is raised to the largest ReLU output of hidden layer j. ----
// Blocks of 128 threads take one 256-row tile (tiles never straddle leaves) in two halves,
// one row per thread; the activations live in LDS, [unit][thread], in two buffers.
constexpr int kCalThreads = 128;

template <int NH>
__global__ __launch_bounds__(kCalThreads) void k_act_max(int P, const float* __restrict__ master, uint32_t n_leaves,
                                                         const uint32_t* __restrict__ bucket_off,
                                                         const uint32_t* __restrict__ tile_off,
                                                         const ChunkCounts* __restrict__ counts,
                                                         const uint32_t* __restrict__ srec_ray,
                                                         const float* __restrict__ srec_t,
                                                         const float* __restrict__ o, const float* __restrict__ d,
                                                         int64_t stride, int64_t r0, float* __restrict__ act_max) {
  __shared__ float buf[2][64][kCalThreads];
  const int tid = threadIdx.x, lane = tid & 63;
  const uint32_t T = counts->n_tiles;
  for (uint32_t w = blockIdx.x; w < 2 * T; w += gridDim.x) {
    const uint32_t t = w >> 1;
    uint32_t lo = 0, hi = n_leaves;
    while (hi - lo > 1) {
      uint32_t mid = (lo + hi) >> 1;
      if (tile_off[mid] <= t) lo = mid; else hi = mid;
    }
    const uint32_t leaf = lo;
    const uint32_t row = bucket_off[leaf] + (t - tile_off[leaf]) * kMlpTileRows + (w & 1) * kCalThreads + tid;
    const bool valid = row < bucket_off[leaf + 1];
    float x[3], dir[3];
    {
      const uint32_t ray = valid ? srec_ray[row] : 0u;
      const float tt = valid ? srec_t[row] : 0.f;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        dir[a] = d[a * stride + r0 + ray];
        x[a] = 2.f * fmaf(tt, dir[a], o[a * stride + r0 + ray]) - 1.f;
      }
    }
    // features in the master column order
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      buf[0][a][tid] = x[a];
      buf[0][27 + a][tid] = dir[a];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float v = x[a] * (float)(1 << k);
        buf[0][3 + 6 * k + a][tid] = sinpif(v);
        buf[0][3 + 6 * k + 3 + a][tid] = cospif(v);
      }
    }
    const float* Wm = master + (uint64_t)leaf * P;
    int cur = 0;
    for (int l = 0; l < NH; ++l) {
      int din, dout, off_w, off_b;
      master_offsets(NH, 64, l, din, dout, off_w, off_b);
      float m = 0.f;
      for (int o8 = 0; o8 < 64; o8 += 8) {
        float z[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) z[k] = Wm[off_b + o8 + k];
        for (int i = 0; i < din; ++i) {
          const float a = buf[cur][i][tid];
#pragma unroll
          for (int k = 0; k < 8; ++k) z[k] = fmaf(Wm[off_w + (o8 + k) * din + i], a, z[k]);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const float r = fmaxf(z[k], 0.f);
          buf[cur ^ 1][o8 + k][tid] = r;
          m = fmaxf(m, r);
        }
      }
      cur ^= 1;
      // largest value over the wave's valid rows (non-negative floats order as integers),
      // then one atomic per wave
      int mi = valid ? __float_as_int(m) : 0;
      mi = wave_max_incl(mi);
      if (lane == 63 && mi > 0)
        atomicMax(reinterpret_cast<unsigned int*>(act_max + (uint64_t)leaf * NH + l), (unsigned)mi);
    }
  }
}

template <int NH>
hipError_t launch8(const void* packed, uint32_t n_leaves, const uint32_t* bucket_off, const uint32_t* tile_off,
                   const ChunkCounts* counts, const uint32_t* srec_ray, const float* srec_t, const uint32_t* perm,
                   const float* o, const float* d, int64_t stride, int64_t r0, float* out, hipStream_t st) {
  auto kern = k_mlp8<NH>;
  const uint32_t lds = make_layout8(NH).bytes;
  int grid = 0;
  hipError_t e = persistent_grid((const void*)kern, kThreads8, lds, &grid);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads8), lds, st, (const uint8_t*)packed, n_leaves, bucket_off, tile_off,
                     counts, srec_ray, srec_t, perm, o, d, stride, r0, out);
  return hipGetLastError();
}

template <int NH>
hipError_t launch_cal(int P, const float* master, uint32_t n_leaves, const uint32_t* bucket_off,
                      const uint32_t* tile_off, const ChunkCounts* counts, const uint32_t* srec_ray,
                      const float* srec_t, const float* o, const float* d, int64_t stride, int64_t r0,
                      float* act_max, hipStream_t st) {
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_act_max<NH>, dim3(4 * ncu), dim3(kCalThreads), 0, st, P, master, n_leaves, bucket_off, tile_off,
                     counts, srec_ray, srec_t, o, d, stride, r0, act_max);
  return hipGetLastError();
}

}  // namespace

size_t mlp8_block_bytes(int n_hidden) { return make_layout8(n_hidden).bytes; }

hipError_t launch_mlp8_pack(int n_hidden, int n_leaves, const float* master, const float* act_max, void* packed,
                            hipStream_t st) {
  const int P = master_param_count(n_hidden, 64);
  hipLaunchKernelGGL(k_mlp8_exps, dim3(n_leaves), dim3(kThreads8), 0, st, n_hidden, P, master, act_max,
                     (uint8_t*)packed);
  hipLaunchKernelGGL(k_mlp8_pack, dim3(1024), dim3(256), 0, st, n_hidden, n_leaves, P, master, (uint8_t*)packed);
  return hipGetLastError();
}

hipError_t launch_mlp8(int n_hidden, const void* packed, uint32_t n_leaves, const uint32_t* bucket_off,
                       const uint32_t* tile_off, const ChunkCounts* counts, const uint32_t* srec_ray,
                       const float* srec_t, const uint32_t* perm, const float* o, const float* d, int64_t stride,
                       int64_t r0, float* out, hipStream_t st) {
  switch (n_hidden) {
    case 1: return launch8<1>(packed, n_leaves, bucket_off, tile_off, counts, srec_ray, srec_t, perm, o, d, stride, r0, out, st);
    case 2: return launch8<2>(packed, n_leaves, bucket_off, tile_off, counts, srec_ray, srec_t, perm, o, d, stride, r0, out, st);
    case 3: return launch8<3>(packed, n_leaves, bucket_off, tile_off, counts, srec_ray, srec_t, perm, o, d, stride, r0, out, st);
    case 4: return launch8<4>(packed, n_leaves, bucket_off, tile_off, counts, srec_ray, srec_t, perm, o, d, stride, r0, out, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_act_max(int n_hidden, const float* master, uint32_t n_leaves, const uint32_t* bucket_off,
                          const uint32_t* tile_off, const ChunkCounts* counts, const uint32_t* srec_ray,
                          const float* srec_t, const float* o, const float* d, int64_t stride, int64_t r0,
                          float* act_max, hipStream_t st) {
  const int P = master_param_count(n_hidden, 64);
  switch (n_hidden) {
    case 1: return launch_cal<1>(P, master, n_leaves, bucket_off, tile_off, counts, srec_ray, srec_t, o, d, stride, r0, act_max, st);
    case 2: return launch_cal<2>(P, master, n_leaves, bucket_off, tile_off, counts, srec_ray, srec_t, o, d, stride, r0, act_max, st);
    case 3: return launch_cal<3>(P, master, n_leaves, bucket_off, tile_off, counts, srec_ray, srec_t, o, d, stride, r0, act_max, st);
    case 4: return launch_cal<4>(P, master, n_leaves, bucket_off, tile_off, counts, srec_ray, srec_t, o, d, stride, r0, act_max, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace amn
