// trav.hip -- ray / KD-tree traversal producing front-to-back leaf intervals
// (Section 3.5, Algorithm 1: Traverse), one lane per ray.
//
// Interval endpoints are carried as unevaluated float pairs (hi + lo): the plane
// crossing t = (s - o) / d is formed with an exact TwoSum of the numerator and an
// FMA-exact remainder of the division, so endpoints agree with a float64 evaluation to
// about 2^-46 relative.  Descent decisions therefore match a float64 traversal except on
// rays that graze a split edge, and interval lengths (which weight densities in the
// quadrature) keep float32 relative accuracy even far along the ray.
#include <algorithm>

#include "internal.hpp"
#include "devcommon.hpp"

namespace amn {
namespace {

struct DF {
  float hi, lo;
};

__device__ __forceinline__ DF two_sum(float a, float b) {
  float s = a + b;
  float bb = s - a;
  float e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

// (s - o) / d as a normalised pair; d != 0.
__device__ __forceinline__ DF plane_t(float s, float o, float d) {
  DF num = two_sum(s, -o);
  float q0 = num.hi / d;
  float r = fmaf(-q0, d, num.hi);   // exact remainder of the float division
  r += num.lo;
  float q1 = r / d;
  float h = q0 + q1;
  float l = q1 - (h - q0);
  return {h, l};
}

__device__ __forceinline__ bool df_lt(DF a, DF b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }

constexpr int kBlock = 256;
// LDS per block: the node table (when staged), then the traversal stack of `stack_n` =
// tree depth + 1 entries per thread as two arrays strided by kBlock (so that a wave's
// accesses fall in distinct banks): the exit parameter's high part, and the node index
// (16 bits) packed with the exit parameter's low part rounded to bfloat16 (the pair then
// still carries about 2^-32 relative precision, far below the 1e-6 perturbation under which
// node ids are compared).
constexpr int kLdsNodes = 2048;  // node tables up to this size are staged in LDS per block

__device__ __forceinline__ float axis_val(const float v[3], int a) { return a == 0 ? v[0] : (a == 1 ? v[1] : v[2]); }

// Traverses one ray.  EMIT = false: returns the interval count, stopping once it exceeds
// cap.  EMIT = true: writes the first `cap` intervals through the output pointers.
__device__ __forceinline__ uint32_t push_word(int node, float lo) {
  return (uint32_t)node | ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)lo) << 16);
}
__device__ __forceinline__ float word_lo(uint32_t w) { return (float)__builtin_bit_cast(__bf16, (uint16_t)(w >> 16)); }

template <bool EMIT, typename NodePtr, typename Put>
__device__ int traverse(NodePtr nodes, const float o[3], const float dir[3], int cap, uint32_t n_per,
                        uint32_t* st_word, float* st_hi, Put put) {
  // root box [0,1]^3
  DF tin = {0.f, 0.f}, tout = {__builtin_inff(), 0.f};
  bool hit = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (dir[a] == 0.f) {
      if (o[a] < 0.f || o[a] > 1.f) hit = false;
      continue;
    }
    DF ta = plane_t(0.f, o[a], dir[a]);
    DF tb = plane_t(1.f, o[a], dir[a]);
    if (df_lt(tb, ta)) { DF t = ta; ta = tb; tb = t; }
    if (df_lt(tin, ta)) tin = ta;
    if (df_lt(tb, tout)) tout = tb;
  }
  hit = hit && df_lt(tin, tout);
  if (!hit) return 0;
  int m = 0, sp = 0, node = 0;
  DF t0 = tin, t1 = tout;
  while (true) {
    int info = nodes[node].info;
    while (info >= 0) {
      int a = info & 3;
      int left = info >> 2;
      float s = nodes[node].plane;
      float oa = axis_val(o, a), da = axis_val(dir, a);
      if (da == 0.f) {
        node = oa >= s ? left + 1 : left;
      } else {
        DF ts = plane_t(s, oa, da);
        int before = da > 0.f ? left : left + 1;
        int after = da > 0.f ? left + 1 : left;
        if (!df_lt(ts, t1)) {
          node = before;
        } else if (!df_lt(t0, ts)) {
          node = after;
        } else {
          st_word[sp * kBlock] = push_word(after, t1.lo);
          st_hi[sp * kBlock] = t1.hi;
          ++sp;
          node = before;
          t1 = ts;
        }
      }
      info = nodes[node].info;
    }
    // leaf interval [t0, t1], t1 > t0 by construction
    if (EMIT) {
      if (m < cap) {
        float dh = t1.hi - t0.hi;
        float dt = dh + (t1.lo - t0.lo);
        put(m, t0.hi, dt, (uint32_t)(-(info + 1)) | (n_per << 16));
      }
    }
    ++m;
    if (m >= cap + (EMIT ? 0 : 1) || sp == 0) break;
    --sp;
    const uint32_t w = st_word[sp * kBlock];
    node = (int)(w & 0xFFFFu);
    t0 = t1;
    t1 = {st_hi[sp * kBlock], word_lo(w)};
  }
  return m;
}

// The block's copy of the node table (LDS = true) or the table in memory, and the stack.
struct TravLds {
  const DevNode* nodes;
  uint32_t* st_word;
  float* st_hi;
};

template <bool LDS>
__device__ __forceinline__ TravLds stage(const DevNode* __restrict__ nodes, uint32_t n_nodes, int stack_n,
                                         uint8_t* dyn) {
  TravLds t;
  uint8_t* p = dyn;
  if (LDS) {
    DevNode* s = reinterpret_cast<DevNode*>(p);
    for (uint32_t i = threadIdx.x; i < n_nodes; i += kBlock) s[i] = nodes[i];
    p += sizeof(DevNode) * n_nodes;
    t.nodes = s;
  } else {
    t.nodes = nodes;
  }
  t.st_word = reinterpret_cast<uint32_t*>(p) + threadIdx.x;
  t.st_hi = reinterpret_cast<float*>(p + 4u * stack_n * kBlock) + threadIdx.x;
  if (LDS) __syncthreads();
  return t;
}

__host__ __device__ constexpr uint32_t trav_lds_bytes(bool lds, uint32_t n_nodes, int stack_n) {
  return (lds ? (uint32_t)sizeof(DevNode) * n_nodes : 0u) + 8u * (uint32_t)stack_n * kBlock;
}

template <bool LDS>
__global__ __launch_bounds__(kBlock) void k_trav_count(const DevNode* __restrict__ nodes, uint32_t n_nodes,
                                                       int stack_n, const float* __restrict__ o,
                                                       const float* __restrict__ d,
                                                       int64_t stride, int64_t r0, uint32_t nr,
                                                       int s_max, uint32_t* __restrict__ cnt_iv,
                                                       uint32_t* __restrict__ cnt_smp) {
  extern __shared__ __align__(16) uint8_t dyn[];
  const TravLds tl = stage<LDS>(nodes, n_nodes, stack_n, dyn);
  uint32_t r = blockIdx.x * kBlock + threadIdx.x;
  bool live = r < nr;
  float oo[3] = {0.f, 0.f, 0.f}, dd[3] = {0.f, 0.f, 1.f};
  if (live) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      oo[a] = o[a * stride + r0 + r];
      dd[a] = d[a * stride + r0 + r];
    }
  }
  int m = 0;
  // skip the descent for a wave whose rays are all out of range
  if (__ballot(live) != 0 && live)
    m = traverse<false>(tl.nodes, oo, dd, s_max, 0, tl.st_word, tl.st_hi, [](int, float, float, uint32_t) {});
  if (live) {
    uint32_t meff = m <= s_max ? (uint32_t)m : (uint32_t)s_max;
    uint32_t nper = m == 0 ? 0u : (m <= s_max ? (uint32_t)(s_max / m) : 1u);
    cnt_iv[r] = meff;
    cnt_smp[r] = meff * nper;
  }
}

// Emission: the block's rays are consecutive, so its intervals fill one contiguous range of
// the output.  Each lane puts its intervals into an LDS copy of the first `stage_n` entries
// of that range (entries past it go straight to memory), and the block then writes the
// staged entries out with consecutive threads on consecutive entries, so every cache line
// is written whole at once instead of piecewise by lanes that finish at different times.
template <bool LDS>
__global__ __launch_bounds__(kBlock) void k_trav_emit(const DevNode* __restrict__ nodes, uint32_t n_nodes,
                                                      int stack_n, uint32_t stage_n, const float* __restrict__ o,
                                                      const float* __restrict__ d, int64_t stride,
                                                      int64_t r0, uint32_t nr,
                                                      const uint32_t* __restrict__ cnt_iv,
                                                      const uint32_t* __restrict__ cnt_smp,
                                                      const uint32_t* __restrict__ iv_off,
                                                      const uint32_t* __restrict__ smp_off,
                                                      float* __restrict__ iv_t0,
                                                      float* __restrict__ iv_dt,
                                                      uint32_t* __restrict__ iv_key,
                                                      uint32_t* __restrict__ iv_ray,
                                                      uint32_t* __restrict__ iv_base) {
  extern __shared__ __align__(16) uint8_t dyn[];
  const TravLds tl = stage<LDS>(nodes, n_nodes, stack_n, dyn);
  uint8_t* sp = dyn + trav_lds_bytes(LDS, n_nodes, stack_n);
  float* s_t0 = reinterpret_cast<float*>(sp);
  float* s_dt = s_t0 + stage_n;
  uint32_t* s_key = reinterpret_cast<uint32_t*>(s_dt + stage_n);
  uint32_t* s_ray = s_key + stage_n;
  uint32_t* s_base = s_ray + stage_n;
  const uint32_t rb = blockIdx.x * kBlock;                      // first ray of the block
  const uint32_t re = rb + kBlock < nr ? rb + kBlock : nr;      // one past its last ray
  const uint32_t b0 = iv_off[rb], b1 = iv_off[re];              // the block's output range
  const uint32_t r = rb + threadIdx.x;
  const uint32_t meff = r < nr ? cnt_iv[r] : 0u;
  if (__ballot(meff != 0) != 0 && meff != 0) {
    float oo[3], dd[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      oo[a] = o[a * stride + r0 + r];
      dd[a] = d[a * stride + r0 + r];
    }
    const uint32_t nper = cnt_smp[r] / meff;
    const uint32_t pos0 = iv_off[r] - b0;
    const uint32_t base = smp_off[r];
    traverse<true>(tl.nodes, oo, dd, (int)meff, nper, tl.st_word, tl.st_hi,
                   [&](int m, float t0, float dt, uint32_t key) {
                     const uint32_t q = pos0 + (uint32_t)m;
                     const uint32_t smp = base + (uint32_t)m * nper;
                     if (q < stage_n) {
                       s_t0[q] = t0; s_dt[q] = dt; s_key[q] = key; s_ray[q] = r; s_base[q] = smp;
                     } else {
                       iv_t0[b0 + q] = t0; iv_dt[b0 + q] = dt; iv_key[b0 + q] = key; iv_ray[b0 + q] = r;
                       iv_base[b0 + q] = smp;
                     }
                   });
  }
  __syncthreads();
  const uint32_t n = b1 - b0 < stage_n ? b1 - b0 : stage_n;
  for (uint32_t q = threadIdx.x; q < n; q += kBlock) {
    iv_t0[b0 + q] = s_t0[q];
    iv_dt[b0 + q] = s_dt[q];
    iv_key[b0 + q] = s_key[q];
    iv_ray[b0 + q] = s_ray[q];
    iv_base[b0 + q] = s_base[q];
  }
}

}  // namespace

static hipError_t allow_lds(const void* kern) {
  return hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
}

static hipError_t trav_setup() {
  static bool done = false;
  if (done) return hipSuccess;
  hipError_t e = allow_lds((const void*)k_trav_count<true>);
  if (e == hipSuccess) e = allow_lds((const void*)k_trav_count<false>);
  if (e == hipSuccess) e = allow_lds((const void*)k_trav_emit<true>);
  if (e == hipSuccess) e = allow_lds((const void*)k_trav_emit<false>);
  if (e == hipSuccess) done = true;
  return e;
}

hipError_t launch_trav_count(const DevNode* nodes, uint32_t n_nodes, int depth, const float* o, const float* d,
                             int64_t ray_stride, int64_t r0, uint32_t nr, int s_max,
                             uint32_t* cnt_iv, uint32_t* cnt_smp, hipStream_t st) {
  if (nr == 0) return hipSuccess;
  hipError_t e = trav_setup();
  if (e != hipSuccess) return e;
  const int stack_n = depth + 1;
  const uint32_t grid = (nr + kBlock - 1) / kBlock;
  if (n_nodes <= (uint32_t)kLdsNodes)
    hipLaunchKernelGGL(k_trav_count<true>, dim3(grid), dim3(kBlock), trav_lds_bytes(true, n_nodes, stack_n), st, nodes,
                       n_nodes, stack_n, o, d, ray_stride, r0, nr, s_max, cnt_iv, cnt_smp);
  else
    hipLaunchKernelGGL(k_trav_count<false>, dim3(grid), dim3(kBlock), trav_lds_bytes(false, n_nodes, stack_n), st,
                       nodes, n_nodes, stack_n, o, d, ray_stride, r0, nr, s_max, cnt_iv, cnt_smp);
  return hipGetLastError();
}

hipError_t launch_trav_emit(const DevNode* nodes, uint32_t n_nodes, int depth, const float* o, const float* d,
                            int64_t ray_stride, int64_t r0, uint32_t nr, const uint32_t* cnt_iv,
                            const uint32_t* cnt_smp, const uint32_t* iv_off, const uint32_t* smp_off,
                            float* iv_t0, float* iv_dt, uint32_t* iv_key, uint32_t* iv_ray,
                            uint32_t* iv_base, hipStream_t st) {
  if (nr == 0) return hipSuccess;
  hipError_t e = trav_setup();
  if (e != hipSuccess) return e;
  const int stack_n = depth + 1;
  const uint32_t grid = (nr + kBlock - 1) / kBlock;
  const bool lds = n_nodes <= (uint32_t)kLdsNodes;
  // staging sized so that two blocks still fit in a CU's 160 KiB of LDS (the traversal
  // needs the occupancy), at most 2048 entries of 20 bytes
  const uint32_t fixed = trav_lds_bytes(lds, n_nodes, stack_n);
  const uint32_t budget = 80u * 1024u;
  uint32_t stage_n = fixed + 20u * 256u <= budget ? (budget - fixed) / 20u : 256u;
  stage_n = std::min<uint32_t>(stage_n, 2048u) & ~63u;
  const uint32_t bytes = fixed + 20u * stage_n;
  if (lds)
    hipLaunchKernelGGL(k_trav_emit<true>, dim3(grid), dim3(kBlock), bytes, st, nodes, n_nodes, stack_n, stage_n, o, d,
                       ray_stride, r0, nr, cnt_iv, cnt_smp, iv_off, smp_off, iv_t0, iv_dt, iv_key, iv_ray, iv_base);
  else
    hipLaunchKernelGGL(k_trav_emit<false>, dim3(grid), dim3(kBlock), bytes, st, nodes, n_nodes, stack_n, stage_n, o,
                       d, ray_stride, r0, nr, cnt_iv, cnt_smp, iv_off, smp_off, iv_t0, iv_dt, iv_key, iv_ray, iv_base);
  return hipGetLastError();
}

}  // namespace amn
