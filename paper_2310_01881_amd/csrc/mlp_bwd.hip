// mlp_bwd.hip -- backward pass of the grouped per-leaf MLP (bfloat16 operands, float32
// accumulation), the differentiable counterpart of the grouped forward in mlp.hip.
//
// Work item: a segment of at most kSegTiles consecutive 256-row tiles of one leaf, each
// processed by a block of 16 waves (4 per SIMD: one block fills a compute unit), 16 rows per
// wave.  Every wave recomputes its forward activations (none are stored between the forward
// and backward passes) and keeps each layer's bfloat16 input in registers in B-operand
// order.  Then, from the output layer down:
//   * dZ_l (gradient at layer l's pre-activation) and the layer's input H_{l-1} are staged
//     feature-major in LDS ([feature][256 samples], rows padded by 16 bytes), and the
//     waves accumulate dW_l = sum_samples dZ_l H_{l-1}^T on MFMA with K = samples (and
//     db_l = sum_samples dZ_l against a ones operand);
//   * dH_{l-1} = W_l^T dZ_l runs on MFMA in registers (transposed weights packed in the
//     same register-chained order as the forward), then dZ_{l-1} = dH_{l-1} where the
//     forward activation was positive.
// Each segment writes its partial dW, db (master layout) to its own slot; a separate
// kernel sums the slots of each leaf in order, so the gradient is deterministic.
#include "internal.hpp"
#include "devcommon.hpp"
#include "mlp_layout.hpp"

namespace amn {
namespace {

constexpr int kThreads = 256;                    // the float32 kernel's block
constexpr int kWavesB = 16;                      // waves of a bfloat16 block (4 per SIMD)
constexpr int kThreadsB = 64 * kWavesB;
constexpr int kNCB = 1;                          // 16-sample column blocks per wave
constexpr int kTileRows = kMlpTileRows;          // 256-row tiles of the forward pass, each
constexpr int kSubRows = kWavesB * 16 * kNCB;    // processed as one sub-tile of 16 rows per wave
constexpr int kSubPerTile = kTileRows / kSubRows;
static_assert(kTileRows % kSubRows == 0, "sub-tiles must divide a tile");
constexpr int kRowBytes = kSubRows * 2 + 16;     // staged feature row (bf16) + padding
static_assert(kWavesB == 16, "the weight-gradient ownership below assumes 16 waves");

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Weight-gradient ownership, fixed so that every sum is taken in one order.  Below the
// output layer, dW_l is cut into 32x32 blocks (rows: outputs; columns: staged inputs), one
// wave each, accumulated with 32x32x16 MFMAs over the sub-tile's samples: the layers take
// waves in the order 1, 2, .., NH - 1, 0 (slot li), (H/32)^2 waves apiece.  db_l's 16-row
// blocks go to 16x16x32 MFMAs against a ones operand on waves 8 + li H/16 + j (mod 16),
// which never hold a dW block of the same layer, and each hold one layer's.  The output
// layer (its outputs padded to 16 rows) keeps 16x16 blocks: column block ci on wave ci,
// its db on wave 0.
__device__ __forceinline__ constexpr int bwd_slot(int NH, int l) { return l >= 1 ? l - 1 : NH - 1; }

__device__ __forceinline__ void stage(uint8_t* base, int row, int col, __bf16 v) {
  *reinterpret_cast<__bf16*>(base + row * kRowBytes + col * 2) = v;
}
__device__ __forceinline__ bool pos_bf16(__bf16 v) {
  return __builtin_bit_cast(short, v) > 0;
}

template <int H, int NH>
__global__ __launch_bounds__(kThreadsB) void k_mlp_bwd(
    Layout L, const uint8_t* __restrict__ packed_fwd, const uint8_t* __restrict__ packed_bwd,
    uint32_t n_leaves, const uint32_t* __restrict__ bucket_off,
    const uint32_t* __restrict__ tile_off, const uint32_t* __restrict__ seg_off,
    const uint32_t* __restrict__ srec_ray, const float* __restrict__ srec_t,
    const uint32_t* __restrict__ perm, const float* __restrict__ o, const float* __restrict__ d,
    int64_t stride, int64_t r0, const float* __restrict__ gpre, float* __restrict__ part, int P,
    uint32_t* __restrict__ seg_queue) {
  extern __shared__ __align__(16) uint8_t lds[];
  constexpr int RB = H / 16;
  constexpr int KUh = H / 32;
  uint8_t* w_fwd = lds;
  uint8_t* w_bwd = lds + L.bytes;
  uint8_t* s_dz = w_bwd + L.bwd_bytes;
  uint8_t* s_h = s_dz + H * kRowBytes;
  uint32_t& s_seg = *reinterpret_cast<uint32_t*>(s_h + H * kRowBytes);   // the segment taken
  const float* bias = reinterpret_cast<const float*>(w_fwd);
  const uint8_t* units = w_fwd + L.bias_bytes;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, m = lane & 15;
  bf16x8 ones;
#pragma unroll
  for (int e = 0; e < 8; ++e) ones[e] = (__bf16)1.f;
  // this wave's blocks (see above) and the byte offsets of its operand fragments in the
  // staged rows, which are the same for every layer
  const int h32 = lane >> 5, c32 = lane & 31;
  int big_l = -1, big_ri = 0, big_cj = 0, bias_l = -1, bias_j = 0;
#pragma unroll
  for (int l = 0; l < NH; ++l) {
    const int li = bwd_slot(NH, l);
    const int ncol = l == 0 ? 1 : H / 32;
    const int bi = wave - li * (H / 32) * (H / 32);
    if (bi >= 0 && bi < (H / 32) * ncol) { big_l = l; big_ri = bi / ncol; big_cj = bi % ncol; }
    const int bj = (wave - 8 - li * (H / 16)) & 15;
    if (bj < H / 16) { bias_l = l; bias_j = bj; }
  }
  const uint32_t big_a = (uint32_t)(32 * big_ri + c32) * kRowBytes + 16u * h32;   // + 32 bytes per K step
  const uint32_t big_b = (uint32_t)(32 * big_cj + c32) * kRowBytes + 16u * h32;
  const uint32_t bias_a = (uint32_t)(16 * bias_j + m) * kRowBytes + 16u * g;      // + 64 bytes per K step
  const uint32_t out_b = (uint32_t)(16 * (wave & (RB - 1)) + m) * kRowBytes + 16u * g;
  const uint32_t out_a = (uint32_t)m * kRowBytes + 16u * g;

  const uint32_t n_seg = seg_off[n_leaves];
  int cur = -1;
  // segments are taken from a queue (segments differ in length, so a fixed stride over them
  // leaves blocks unevenly loaded); each writes its own partial slot, so the order is free
  if (tid == 0) s_seg = atomicAdd(seg_queue, 1u);
  __syncthreads();
  uint32_t seg = __builtin_amdgcn_readfirstlane(s_seg);
  while (seg < n_seg) {
    uint32_t lo = 0, hi = n_leaves;
    while (hi - lo > 1) {
      uint32_t mid = (lo + hi) >> 1;
      if (seg_off[mid] <= seg) lo = mid; else hi = mid;
    }
    const uint32_t b = lo;
    const uint32_t t_first = tile_off[b] + (seg - seg_off[b]) * kSegTiles;
    const uint32_t t_last = t_first + kSegTiles < tile_off[b + 1] ? t_first + kSegTiles : tile_off[b + 1];
    if ((int)b != cur) {
      __syncthreads();
      const f32x4* s1 = reinterpret_cast<const f32x4*>(packed_fwd + (uint64_t)b * L.bytes);
      for (uint32_t i = tid; i < L.bytes / 16; i += kThreadsB) reinterpret_cast<f32x4*>(w_fwd)[i] = s1[i];
      const f32x4* s2 = reinterpret_cast<const f32x4*>(packed_bwd + (uint64_t)b * L.bwd_bytes);
      for (uint32_t i = tid; i < L.bwd_bytes / 16; i += kThreadsB) reinterpret_cast<f32x4*>(w_bwd)[i] = s2[i];
      __syncthreads();
      cur = (int)b;
    }
    f32x16 accW32;             // this wave's 32x32 block of some dW_l (l < NH)
#pragma unroll
    for (int i = 0; i < 16; ++i) accW32[i] = 0.f;
    f32x4 accB16 = {0.f, 0.f, 0.f, 0.f};   // its 16-row block of some db_l (l < NH)
    f32x4 accWo = {0.f, 0.f, 0.f, 0.f};    // its 16x16 block of the output layer's dW
    f32x4 accBo = {0.f, 0.f, 0.f, 0.f};    // the output layer's db (wave 0)

    for (uint32_t sub = kSubPerTile * t_first; sub < kSubPerTile * t_last; ++sub) {
      const uint32_t row0 = bucket_off[b] + (sub - kSubPerTile * tile_off[b]) * kSubRows + wave * (16 * kNCB);
      const uint32_t row_end = bucket_off[b + 1];
      // ---- forward recompute: layer inputs in B-operand order ----
      bf16x8 X0[kNCB];
      bf16x8 Hs[NH + 1][kNCB][KUh];    // Hs[l] = input of layer l (l >= 1), after ReLU
      f32x4 dz[kNCB][RB];
#pragma unroll
      for (int cb = 0; cb < kNCB; ++cb) {
        const uint32_t row = row0 + cb * 16 + m;
        const bool valid = row < row_end;
        uint32_t ray = 0;
        float ts = 0.f;
        uint32_t dst = 0;
        if (valid) {
          ray = srec_ray[row];
          ts = srec_t[row];
          dst = perm[row];
        }
        const int64_t ri = r0 + ray;
        const float ox = o[ri], oy = o[stride + ri], oz = o[2 * stride + ri];
        const float dx = d[ri], dy = d[stride + ri], dzz = d[2 * stride + ri];
        const float px = 2.f * fmaf(ts, dx, ox) - 1.f;
        const float py = 2.f * fmaf(ts, dy, oy) - 1.f;
        const float pz = 2.f * fmaf(ts, dzz, oz) - 1.f;
        float feat[8];
        const float v = g == 1 ? py : (g == 2 ? pz : px);
        float sn = __builtin_amdgcn_sinf(0.5f * v);
        float cs = __builtin_amdgcn_cosf(0.5f * v);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          feat[2 * k] = sn;
          feat[2 * k + 1] = cs;
          const float t2 = sn + sn;
          const float s2 = t2 * cs;
          cs = fmaf(-t2, sn, 1.f);
          sn = s2;
        }
        if (g == 3) {
          feat[0] = px; feat[1] = py; feat[2] = pz;
          feat[3] = dx; feat[4] = dy; feat[5] = dzz;
          feat[6] = 0.f; feat[7] = 0.f;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) X0[cb][e] = (__bf16)feat[e];
        // output-layer gradient: lanes of group 0 hold (dsigma^, dr^, dg^, db^)
        f32x4 gz = {0.f, 0.f, 0.f, 0.f};
        if (g == 0 && valid) gz = *reinterpret_cast<const f32x4*>(gpre + 4 * (uint64_t)dst);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) dz[cb][rb] = f32x4{0.f, 0.f, 0.f, 0.f};
        dz[cb][0] = gz;
      }
#pragma unroll
      for (int l = 0; l < NH; ++l) {
        f32x4 acc[kNCB][RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const f32x4 bv = *reinterpret_cast<const f32x4*>(bias + l * H + 16 * rb + 4 * g);
          if (l == 0) {
            const bf16x8 A = *reinterpret_cast<const bf16x8*>(units + L.unit_index(0, rb, 0) * kUnitBytes + lane * 16);
#pragma unroll
            for (int cb = 0; cb < kNCB; ++cb) acc[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, X0[cb], bv, 0, 0, 0);
          } else {
#pragma unroll
            for (int ku = 0; ku < KUh; ++ku) {
              const bf16x8 A = *reinterpret_cast<const bf16x8*>(units + L.unit_index(l, rb, ku) * kUnitBytes + lane * 16);
#pragma unroll
              for (int cb = 0; cb < kNCB; ++cb)
                acc[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Hs[l][cb][ku], ku == 0 ? bv : acc[cb][rb], 0, 0, 0);
            }
          }
        }
#pragma unroll
        for (int cb = 0; cb < kNCB; ++cb)
#pragma unroll
          for (int ku = 0; ku < KUh; ++ku) {
            float vv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) vv[e] = acc[cb][2 * ku + e / 4][e % 4];
            Hs[l + 1][cb][ku] = relu_bf16x8(vv);
          }
      }

      // ---- backward, output layer first ----
#pragma unroll
      for (int l = NH; l >= 0; --l) {
        const int rbo = l == NH ? 1 : RB;          // row blocks of this layer's outputs
        // stage dZ_l and the layer input, feature-major
        __syncthreads();
#pragma unroll
        for (int cb = 0; cb < kNCB; ++cb) {
          const int col = wave * (16 * kNCB) + cb * 16 + m;
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            if (rb >= rbo) break;
#pragma unroll
            for (int i = 0; i < 4; ++i) stage(s_dz, 16 * rb + 4 * g + i, col, (__bf16)dz[cb][rb][i]);
          }
          if (l == 0) {
#pragma unroll
            for (int e = 0; e < 8; ++e) stage(s_h, 8 * g + e, col, X0[cb][e]);
          } else {
#pragma unroll
            for (int ku = 0; ku < KUh; ++ku)
#pragma unroll
              for (int e = 0; e < 8; ++e) stage(s_h, hidden_col_bf16(ku, g, e), col, Hs[l][cb][ku][e]);
          }
        }
        __syncthreads();
        // dW_l += dZ_l H^T, db_l += dZ_l 1 over the sub-tile's samples
        if (l == NH) {
          if (wave < RB) {
#pragma unroll
            for (int kb = 0; kb < kSubRows / 32; ++kb) {
              const bf16x8 A = *reinterpret_cast<const bf16x8*>(s_dz + out_a + 64 * kb);
              const bf16x8 Bm = *reinterpret_cast<const bf16x8*>(s_h + out_b + 64 * kb);
              accWo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bm, accWo, 0, 0, 0);
              if (wave == 0) accBo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, ones, accBo, 0, 0, 0);
            }
          }
        } else {
          // A: lane (h, c) holds dZ row 32 ri + c at samples 16 ks + 8 h ..; B: the input
          // feature 32 cj + c at the same samples
          if (big_l == l) {
#pragma unroll 4
            for (int ks = 0; ks < kSubRows / 16; ++ks) {
              const bf16x8 A = *reinterpret_cast<const bf16x8*>(s_dz + big_a + 32 * ks);
              const bf16x8 Bm = *reinterpret_cast<const bf16x8*>(s_h + big_b + 32 * ks);
              accW32 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, Bm, accW32, 0, 0, 0);
            }
          }
          if (bias_l == l) {
#pragma unroll
            for (int kb = 0; kb < kSubRows / 32; ++kb) {
              const bf16x8 A = *reinterpret_cast<const bf16x8*>(s_dz + bias_a + 64 * kb);
              accB16 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, ones, accB16, 0, 0, 0);
            }
          }
        }
        if (l == 0) break;
        // dH = W_l^T dZ_l, then the ReLU mask of the forward activation
        const int ku_n = l == NH ? 1 : KUh;
        bf16x8 Bz[kNCB][KUh];
#pragma unroll
        for (int cb = 0; cb < kNCB; ++cb)
#pragma unroll
          for (int ku = 0; ku < KUh; ++ku) {
            if (ku >= ku_n) break;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int rbs = 2 * ku + e / 4;
              const float v = (rbs < rbo) ? dz[cb][rbs][e % 4] : 0.f;
              Bz[cb][ku][e] = (__bf16)v;
            }
          }
        f32x4 dh[kNCB][RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
          for (int ku = 0; ku < KUh; ++ku) {
            if (ku >= ku_n) break;
            const bf16x8 A = *reinterpret_cast<const bf16x8*>(w_bwd + L.bwd_unit_index(l, rb, ku) * kUnitBytes + lane * 16);
#pragma unroll
            for (int cb = 0; cb < kNCB; ++cb)
              dh[cb][rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                  A, Bz[cb][ku], ku == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : dh[cb][rb], 0, 0, 0);
          }
        }
#pragma unroll
        for (int cb = 0; cb < kNCB; ++cb)
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i)
              dz[cb][rb][i] = pos_bf16(Hs[l][cb][rb / 2][4 * (rb % 2) + i]) ? dh[cb][rb][i] : 0.f;
      }
    }

    // ---- this segment's partial gradient, master layout ----
    // (every weight and bias of the leaf is written by exactly one wave)
    float* dst = part + (uint64_t)seg * P;
    {
      int din, dout, off_w, off_b;
      master_offsets(NH, H, NH, din, dout, off_w, off_b);
      if (wave < RB) {
        const int c = 16 * wave + m;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int out = 4 * g + i;
          if (out < dout) dst[off_w + out * din + c] = accWo[i];
          if (wave == 0 && m == 0 && out < dout) dst[off_b + out] = accBo[i];
        }
      }
    }
    if (big_l >= 0) {
      int din, dout, off_w, off_b;
      master_offsets(NH, H, big_l, din, dout, off_w, off_b);
      const int cc = 32 * big_cj + c32;
      const int col = big_l == 0 ? first_layer_col_bf16(cc / 8, cc % 8) : cc;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int out = 32 * big_ri + 8 * (r / 4) + 4 * h32 + (r % 4);   // accumulator row of register r
        if (out < dout && col >= 0) dst[off_w + out * din + col] = accW32[r];
      }
    }
    if (bias_l >= 0 && m == 0) {
      int din, dout, off_w, off_b;
      master_offsets(NH, H, bias_l, din, dout, off_w, off_b);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int out = 16 * bias_j + 4 * g + i;
        if (out < dout) dst[off_b + out] = accB16[i];
      }
    }
    __syncthreads();   // every wave has read s_seg
    if (tid == 0) s_seg = atomicAdd(seg_queue, 1u);
    __syncthreads();
    seg = __builtin_amdgcn_readfirstlane(s_seg);
  }
}

// ---- float32 operands: v_mfma_f32_16x16x4_f32.  An MFMA takes A[m][k] from lane
// (k, m) and B[k][n] from lane (k, n) (one float each) and leaves C rows 4g..4g+3 of column
// n in lane (g, n).  The same work split as the bfloat16 kernel (segments of one leaf's
// tiles, partial gradients per segment), with 64-row sub-tiles of 16 rows per wave; the
// leaf's float32 forward block (the layout k_mlp reads) is staged in LDS and serves both
// the forward recomputation and, read transposed, dH = W^T dZ.
constexpr int kSub32 = 64;                 // rows of a float32 sub-tile (4 waves x 16)
constexpr int kRowF = kSub32 + 4;          // staged feature row (floats) + padding

// W_l[row][col] of a hidden or output layer inside the float32 forward block: unit
// (l, row / 16, col / 16), lane ((col % 16) / 4) * 16 + row % 16, element col % 4.
__device__ __forceinline__ float w_at(const Layout& L, const uint8_t* units, int l, int row, int col) {
  const int u = L.unit_index(l, row >> 4, col >> 4);
  return *reinterpret_cast<const float*>(units + u * kUnitBytes + ((((col & 15) >> 2) << 4) + (row & 15)) * 16 +
                                         (col & 3) * 4);
}

template <int H, int NH>
__global__ __launch_bounds__(kThreads) void k_mlp_bwd_f32(
    Layout L, const uint8_t* __restrict__ packed, uint32_t n_leaves, const uint32_t* __restrict__ bucket_off,
    const uint32_t* __restrict__ tile_off, const uint32_t* __restrict__ seg_off,
    const uint32_t* __restrict__ srec_ray, const float* __restrict__ srec_t, const uint32_t* __restrict__ perm,
    const float* __restrict__ o, const float* __restrict__ d, int64_t stride, int64_t r0,
    const float* __restrict__ gpre, float* __restrict__ part, int P) {
  extern __shared__ __align__(16) uint8_t lds[];
  constexpr int RB = H / 16;
  const float* bias = reinterpret_cast<const float*>(lds);
  const uint8_t* units = lds + L.bias_bytes;
  float* sZ = reinterpret_cast<float*>(lds + L.bytes);   // [H][kRowF]: dZ_l, feature-major
  float* sH = sZ + H * kRowF;                            // [H][kRowF]: layer input, feature-major
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, m = lane & 15;
  const uint32_t n_seg = seg_off[n_leaves];
  int cur = -1;
  for (uint32_t seg = blockIdx.x; seg < n_seg; seg += gridDim.x) {
    uint32_t lo = 0, hi = n_leaves;
    while (hi - lo > 1) {
      uint32_t mid = (lo + hi) >> 1;
      if (seg_off[mid] <= seg) lo = mid; else hi = mid;
    }
    const uint32_t b = lo;
    const uint32_t t_first = tile_off[b] + (seg - seg_off[b]) * kSegTiles;
    const uint32_t t_last = t_first + kSegTiles < tile_off[b + 1] ? t_first + kSegTiles : tile_off[b + 1];
    if ((int)b != cur) {
      __syncthreads();
      const f32x4* src = reinterpret_cast<const f32x4*>(packed + (uint64_t)b * L.bytes);
      for (uint32_t i = tid; i < L.bytes / 16; i += kThreads) reinterpret_cast<f32x4*>(lds)[i] = src[i];
      __syncthreads();
      cur = (int)b;
    }
    f32x4 accW[NH + 1][4];
    f32x4 accB[NH + 1];
#pragma unroll
    for (int l = 0; l <= NH; ++l) {
      accB[l] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) accW[l][q] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    constexpr int kSubPerTile = kMlpTileRows / kSub32;
    for (uint32_t sub = kSubPerTile * t_first; sub < kSubPerTile * t_last; ++sub) {
      const uint32_t row_end = bucket_off[b + 1];
      const uint32_t row = bucket_off[b] + (sub - kSubPerTile * tile_off[b]) * kSub32 + wave * 16 + m;
      const bool valid = row < row_end;
      // ---- this lane's sample (column m of the wave's block): inputs as in the forward ----
      uint32_t ray = 0, dst = 0;
      float ts = 0.f;
      if (valid) {
        ray = srec_ray[row];
        ts = srec_t[row];
        dst = perm[row];
      }
      const int64_t ri = r0 + ray;
      const float ox = o[ri], oy = o[stride + ri], oz = o[2 * stride + ri];
      const float dx = d[ri], dy = d[stride + ri], dz_ = d[2 * stride + ri];
      const float px = 2.f * fmaf(ts, dx, ox) - 1.f;
      const float py = 2.f * fmaf(ts, dy, oy) - 1.f;
      const float pz = 2.f * fmaf(ts, dz_, oz) - 1.f;
      float feat[8];
      {
        const float sc = (float)(1 << g);
        feat[0] = sinpif(px * sc); feat[1] = sinpif(py * sc); feat[2] = sinpif(pz * sc);
        feat[3] = cospif(px * sc); feat[4] = cospif(py * sc); feat[5] = cospif(pz * sc);
        feat[6] = g == 0 ? px : (g == 1 ? pz : (g == 2 ? dy : 0.f));
        feat[7] = g == 0 ? py : (g == 1 ? dx : (g == 2 ? dz_ : 0.f));
      }
      // ---- forward recompute: Hs[l] = ReLU output of layer l (accumulator layout) ----
      f32x4 Hs[NH][RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        f32x4 z = *reinterpret_cast<const f32x4*>(bias + 16 * rb + 4 * g);
#pragma unroll
        for (int ku = 0; ku < 2; ++ku) {
          const f32x4 A = *reinterpret_cast<const f32x4*>(units + L.unit_index(0, rb, ku) * kUnitBytes + lane * 16);
#pragma unroll
          for (int e = 0; e < 4; ++e) z = __builtin_amdgcn_mfma_f32_16x16x4f32(A[e], feat[4 * ku + e], z, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) Hs[0][rb][i] = fmaxf(z[i], 0.f);
      }
#pragma unroll
      for (int l = 1; l < NH; ++l) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          f32x4 z = *reinterpret_cast<const f32x4*>(bias + l * H + 16 * rb + 4 * g);
#pragma unroll
          for (int ku = 0; ku < RB; ++ku) {
            const f32x4 A = *reinterpret_cast<const f32x4*>(units + L.unit_index(l, rb, ku) * kUnitBytes + lane * 16);
#pragma unroll
            for (int e = 0; e < 4; ++e) z = __builtin_amdgcn_mfma_f32_16x16x4f32(A[e], Hs[l - 1][ku][e], z, 0, 0, 0);
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) Hs[l][rb][i] = fmaxf(z[i], 0.f);
        }
      }
      // ---- backward from the output layer: lanes of group 0 hold dL/d(sigma^, r^, g^, b^) ----
      f32x4 dz[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) dz[rb] = f32x4{0.f, 0.f, 0.f, 0.f};
      if (g == 0 && valid) dz[0] = *reinterpret_cast<const f32x4*>(gpre + 4 * (uint64_t)dst);
#pragma unroll
      for (int l = NH; l >= 0; --l) {
        const int rbo = l == NH ? 1 : RB;          // row blocks of this layer's outputs
        const int cbi = l == 0 ? 2 : RB;           // 16-column blocks of its inputs
        const int n_items = rbo * cbi;
        const int per = (n_items + 3) / 4;
        __syncthreads();
        const int col = wave * 16 + m;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          if (rb >= rbo) break;
#pragma unroll
          for (int i = 0; i < 4; ++i) sZ[(16 * rb + 4 * g + i) * kRowF + col] = dz[rb][i];
        }
        if (l == 0) {
#pragma unroll
          for (int i = 0; i < 8; ++i) sH[(8 * g + i) * kRowF + col] = feat[i];
        } else {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) sH[(16 * rb + 4 * g + i) * kRowF + col] = Hs[l - 1][rb][i];
        }
        __syncthreads();
        // dW_l += dZ_l X_l^T and db_l += dZ_l 1 over the sub-tile's 64 samples (K = samples)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int item = wave * per + q;
          if (q >= per || item >= n_items) break;
          const int rb = item / cbi, ci = item % cbi;
#pragma unroll 4
          for (int kk = 0; kk < kSub32 / 4; ++kk) {
            const float a = sZ[(16 * rb + m) * kRowF + 4 * kk + g];
            const float bb = sH[(16 * ci + m) * kRowF + 4 * kk + g];
            accW[l][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bb, accW[l][q], 0, 0, 0);
            if (ci == 0) accB[l] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, 1.f, accB[l], 0, 0, 0);
          }
        }
        if (l == 0) break;
        // dH = W_l^T dZ_l (rows: the layer's inputs; K: its outputs), then the ReLU mask
        f32x4 dh[RB];
#pragma unroll
        for (int rbi = 0; rbi < RB; ++rbi) {
          dh[rbi] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int ku = 0; ku < RB; ++ku) {
            if (ku >= rbo) break;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const float a = w_at(L, units, l, 16 * ku + 4 * g + e, 16 * rbi + m);
              dh[rbi] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, dz[ku][e], dh[rbi], 0, 0, 0);
            }
          }
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int i = 0; i < 4; ++i) dz[rb][i] = Hs[l - 1][rb][i] > 0.f ? dh[rb][i] : 0.f;
      }
    }

    // ---- this segment's partial gradient, master layout ----
    float* dstp = part + (uint64_t)seg * P;
#pragma unroll
    for (int l = 0; l <= NH; ++l) {
      const int rbo = l == NH ? 1 : RB;
      const int cbi = l == 0 ? 2 : RB;
      const int n_items = rbo * cbi;
      const int per = (n_items + 3) / 4;
      int din, dout, off_w, off_b;
      master_offsets(NH, H, l, din, dout, off_w, off_b);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int item = wave * per + q;
        if (q >= per || item >= n_items) break;
        const int rb = item / cbi, ci = item % cbi;
        const int c = 16 * ci + m;
        const int colm = l == 0 ? first_layer_col(c >> 3, c & 7) : c;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int out = 16 * rb + 4 * g + i;
          if (out < dout && colm >= 0) dstp[off_w + out * din + colm] = accW[l][q][i];
          if (ci == 0 && m == 0 && out < dout) dstp[off_b + out] = accB[l][i];
        }
      }
    }
  }
}

template <int H, int NH>
hipError_t launch_bwd_f32_typed(const Layout& L, const void* packed, uint32_t n_leaves,
                                const uint32_t* bucket_off, const uint32_t* tile_off,
                                const uint32_t* seg_off, const uint32_t* srec_ray, const float* srec_t,
                                const uint32_t* perm, const float* o, const float* d, int64_t stride,
                                int64_t r0, const float* gpre, float* part, hipStream_t st) {
  auto kern = k_mlp_bwd_f32<H, NH>;
  const uint32_t lds = L.bytes + 2u * H * kRowF * 4u;
  int grid = 0;
  hipError_t e = persistent_grid((const void*)kern, kThreads, lds, &grid);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, st, L, (const uint8_t*)packed, n_leaves,
                     bucket_off, tile_off, seg_off, srec_ray, srec_t, perm, o, d, stride, r0, gpre, part,
                     master_param_count(NH, H));
  return hipGetLastError();
}

template <int H, int NH>
hipError_t launch_bwd_typed(const Layout& L, const void* packed, uint32_t n_leaves,
                            const uint32_t* bucket_off, const uint32_t* tile_off,
                            uint32_t* seg_off, const uint32_t* srec_ray, const float* srec_t,
                            const uint32_t* perm, const float* o, const float* d, int64_t stride,
                            int64_t r0, const float* gpre, float* part, hipStream_t st) {
  auto kern = k_mlp_bwd<H, NH>;
  const uint32_t lds = L.bytes + L.bwd_bytes + 2u * H * kRowBytes + 16u;   // + the queue word
  int grid = 0;
  hipError_t e = persistent_grid((const void*)kern, kThreadsB, lds, &grid);
  if (e != hipSuccess) return e;
  const uint8_t* pf = (const uint8_t*)packed;
  const uint8_t* pb = pf + (uint64_t)n_leaves * L.bytes;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreadsB), lds, st, L, pf, pb, n_leaves, bucket_off, tile_off,
                     seg_off, srec_ray, srec_t, perm, o, d, stride, r0, gpre, part,
                     master_param_count(NH, H), seg_off + n_leaves + 1);
  return hipGetLastError();
}

}  // namespace

bool mlp_bwd_supported(int n_hidden, int hidden) {
  return n_hidden >= 1 && n_hidden <= 4 && (hidden == 32 || hidden == 64);
}

hipError_t launch_mlp_bwd(const MlpGeom& g, const void* packed, uint32_t n_leaves,
                          const uint32_t* bucket_off, const uint32_t* tile_off, uint32_t* seg_off,
                          const uint32_t* srec_ray, const float* srec_t, const uint32_t* perm,
                          const float* o, const float* d, int64_t ray_stride, int64_t r0,
                          const float* gpre, float* part, hipStream_t st) {
  Layout L = make_layout(g.n_hidden, g.hidden, g.dtype);
#define AMN_BWD(HH, NN)                                                                                \
  if (g.hidden == HH && g.n_hidden == NN) {                                                            \
    if (g.dtype == AMNERF_F32)                                                                         \
      return launch_bwd_f32_typed<HH, NN>(L, packed, n_leaves, bucket_off, tile_off, seg_off, srec_ray, \
                                          srec_t, perm, o, d, ray_stride, r0, gpre, part, st);        \
    return launch_bwd_typed<HH, NN>(L, packed, n_leaves, bucket_off, tile_off, seg_off, srec_ray,       \
                                    srec_t, perm, o, d, ray_stride, r0, gpre, part, st);              \
  }
  AMN_BWD(64, 4)
  AMN_BWD(64, 3)
  AMN_BWD(64, 2)
  AMN_BWD(64, 1)
  AMN_BWD(32, 4)
  AMN_BWD(32, 3)
  AMN_BWD(32, 2)
  AMN_BWD(32, 1)
#undef AMN_BWD
  return hipErrorInvalidValue;
}

}  // namespace amn
