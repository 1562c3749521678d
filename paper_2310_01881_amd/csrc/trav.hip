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

#include <atomic>

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

// Hierarchical sampling (HCheck): the descent stops at an inner node when the ray enters
// it farther than the node's stopping distance t_stop = size / footprint (size: the node's
// longest side; footprint: the caller's sample footprint per unit distance), and the node's
// own MLP then takes the ray's whole segment in it.  Both the decision (float32 entry
// parameter against float32 t_stop) and t_stop (one correctly rounded float32 division)
// are fixed to the bit.  Two views of the per-node data: staged in LDS as (t_stop, slot)
// pairs, or read from memory with t_stop formed on the fly.
struct AhsNone {
  __device__ float tstop(int) const { return __builtin_inff(); }
  __device__ uint32_t slot(int) const { return 0u; }
};
struct AhsLds {
  const float2* p;
  __device__ float tstop(int i) const { return p[i].x; }
  __device__ uint32_t slot(int i) const { return __builtin_bit_cast(uint32_t, p[i].y); }
};
struct AhsMem {
  const DevNodeAhs* p;
  float footprint;
  __device__ float tstop(int i) const { return __fdiv_rn(p[i].size, footprint); }
  __device__ uint32_t slot(int i) const { return p[i].slot; }
};

// Traverses one ray.  EMIT = false: returns the interval count, stopping once it exceeds
// cap.  EMIT = true: writes the first `cap` intervals through the output pointers.  AHS:
// stop the descent by HCheck, and key intervals by the node's preorder slot.
__device__ __forceinline__ uint32_t push_word(int node, float lo) {
  return (uint32_t)node | ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)lo) << 16);
}
__device__ __forceinline__ float word_lo(uint32_t w) { return (float)__builtin_bit_cast(__bf16, (uint16_t)(w >> 16)); }

template <bool EMIT, bool AHS, typename NodePtr, typename Ahs, typename Put>
__device__ int traverse(NodePtr nodes, const Ahs ahs, const float o[3], const float dir[3], int cap, uint32_t n_per,
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
      if (AHS && t0.hi > ahs.tstop(node)) break;
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
    // interval [t0, t1] of a leaf (or, with AHS, of a node HCheck stopped at), t1 > t0 by
    // construction
    if (EMIT) {
      if (m < cap) {
        float dh = t1.hi - t0.hi;
        float dt = dh + (t1.lo - t0.lo);
        const uint32_t slot = AHS ? ahs.slot(node) : (uint32_t)(-(info + 1));
        put(m, t0.hi, dt, slot | (n_per << 16));
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

// The block's copy of the node table (LDS = true) or the table in memory, the per-node
// hierarchical-sampling data (staged with the table when AHS), and the stack.
struct TravLds {
  const DevNode* nodes;
  const float2* ahs;
  uint32_t* st_word;
  float* st_hi;
};

template <bool LDS, bool AHS>
__device__ __forceinline__ TravLds stage(const DevNode* __restrict__ nodes, const DevNodeAhs* __restrict__ ahs,
                                         float footprint, uint32_t n_nodes, int stack_n, uint8_t* dyn) {
  TravLds t;
  uint8_t* p = dyn;
  t.ahs = nullptr;
  if (LDS) {
    DevNode* s = reinterpret_cast<DevNode*>(p);
    for (uint32_t i = threadIdx.x; i < n_nodes; i += kBlock) s[i] = nodes[i];
    p += sizeof(DevNode) * n_nodes;
    t.nodes = s;
    if (AHS) {
      float2* a = reinterpret_cast<float2*>(p);
      for (uint32_t i = threadIdx.x; i < n_nodes; i += kBlock) {
        const DevNodeAhs v = ahs[i];
        a[i] = make_float2(__fdiv_rn(v.size, footprint), __builtin_bit_cast(float, v.slot));
      }
      p += sizeof(float2) * n_nodes;
      t.ahs = a;
    }
  } else {
    t.nodes = nodes;
  }
  t.st_word = reinterpret_cast<uint32_t*>(p) + threadIdx.x;
  t.st_hi = reinterpret_cast<float*>(p + 4u * stack_n * kBlock) + threadIdx.x;
  if (LDS) __syncthreads();
  return t;
}

__host__ __device__ constexpr uint32_t trav_lds_bytes(bool lds, bool ahs, uint32_t n_nodes, int stack_n) {
  return (lds ? (uint32_t)(sizeof(DevNode) + (ahs ? sizeof(float2) : 0u)) * n_nodes : 0u) +
         8u * (uint32_t)stack_n * kBlock;
}

// Runs `f` with the hierarchical-sampling view that matches the staging.
template <bool LDS, bool AHS, typename F>
__device__ __forceinline__ int with_ahs(const TravLds& tl, const DevNodeAhs* ahs, float footprint, F f) {
  if constexpr (!AHS) return f(AhsNone{});
  else if constexpr (LDS) return f(AhsLds{tl.ahs});
  else return f(AhsMem{ahs, footprint});
}

// Counts.  Samples per interval follow the ray's leaf-interval count m (s_max / m, or 1
// when m > s_max); with AHS the intervals are those of the HCheck traversal, so a node that
// stops the descent gets one interval's share however many leaves it covers.
template <bool LDS, bool AHS>
__global__ __launch_bounds__(kBlock) void k_trav_count(const DevNode* __restrict__ nodes,
                                                       const DevNodeAhs* __restrict__ ahs, float footprint,
                                                       uint32_t n_nodes,
                                                       int stack_n, const float* __restrict__ o,
                                                       const float* __restrict__ d,
                                                       int64_t stride, int64_t r0, uint32_t nr,
                                                       int s_max, uint32_t* __restrict__ cnt_iv,
                                                       uint32_t* __restrict__ cnt_smp) {
  extern __shared__ __align__(16) uint8_t dyn[];
  const TravLds tl = stage<LDS, AHS>(nodes, ahs, footprint, n_nodes, stack_n, dyn);
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
  int m = 0, mi = 0;
  // skip the descent for a wave whose rays are all out of range
  if (__ballot(live) != 0 && live) {
    auto none = [](int, float, float, uint32_t) {};
    m = traverse<false, false>(tl.nodes, AhsNone{}, oo, dd, s_max, 0, tl.st_word, tl.st_hi, none);
    mi = m;
    if (AHS && m > 0)
      mi = with_ahs<LDS, AHS>(tl, ahs, footprint, [&](auto av) {
        return traverse<false, AHS>(tl.nodes, av, oo, dd, s_max, 0, tl.st_word, tl.st_hi, none);
      });
  }
  if (live) {
    uint32_t meff = mi <= s_max ? (uint32_t)mi : (uint32_t)s_max;
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
template <bool LDS, bool AHS>
__global__ __launch_bounds__(kBlock) void k_trav_emit(const DevNode* __restrict__ nodes,
                                                      const DevNodeAhs* __restrict__ ahs, float footprint,
                                                      uint32_t n_nodes,
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
                                                      uint32_t* __restrict__ iv_base,
                                                      ChunkCounts* __restrict__ counts) {
  extern __shared__ __align__(16) uint8_t dyn[];
  const TravLds tl = stage<LDS, AHS>(nodes, ahs, footprint, n_nodes, stack_n, dyn);
  uint8_t* sp = dyn + trav_lds_bytes(LDS, AHS, n_nodes, stack_n);
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
    auto put = [&](int m, float t0, float dt, uint32_t key) {
      const uint32_t q = pos0 + (uint32_t)m;
      const uint32_t smp = base + (uint32_t)m * nper;
      if (q < stage_n) {
        s_t0[q] = t0; s_dt[q] = dt; s_key[q] = key; s_ray[q] = r; s_base[q] = smp;
      } else {
        iv_t0[b0 + q] = t0; iv_dt[b0 + q] = dt; iv_key[b0 + q] = key; iv_ray[b0 + q] = r;
        iv_base[b0 + q] = smp;
      }
    };
    const int got = with_ahs<LDS, AHS>(tl, ahs, footprint, [&](auto av) {
      return traverse<true, AHS>(tl.nodes, av, oo, dd, (int)meff, nper, tl.st_word, tl.st_hi, put);
    });
    // The count pass walks the same way, so `got` equals meff.  Should a walk ever end
    // early, the rest of the ray's range still gets well-formed entries (zero length,
    // slot 0), so later stages never read an unwritten key, and the filled entries are
    // counted (reported by the render statistics; every test requires 0).
    if ((uint32_t)got < meff) {
      for (uint32_t q = (uint32_t)got; q < meff; ++q) put((int)q, 0.f, 0.f, nper << 16);
      atomicAdd(reinterpret_cast<unsigned long long*>(&counts->unreached), (unsigned long long)(meff - (uint32_t)got));
    }
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

template <bool AHS>
static hipError_t trav_setup_one() {
  hipError_t e = allow_lds((const void*)k_trav_count<true, AHS>);
  if (e == hipSuccess) e = allow_lds((const void*)k_trav_count<false, AHS>);
  if (e == hipSuccess) e = allow_lds((const void*)k_trav_emit<true, AHS>);
  if (e == hipSuccess) e = allow_lds((const void*)k_trav_emit<false, AHS>);
  return e;
}

// Once per device (the attribute is set on the current device).
static hipError_t trav_setup() {
  static std::atomic<uint64_t> done{0};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const uint64_t bit = dev < 64 ? 1ull << dev : 0ull;
  if (bit && (done.load() & bit)) return hipSuccess;
  e = trav_setup_one<false>();
  if (e == hipSuccess) e = trav_setup_one<true>();
  if (e == hipSuccess) done.fetch_or(bit);
  return e;
}

template <bool LDS, bool AHS>
static void count_launch(uint32_t grid, uint32_t bytes, hipStream_t st, const DevNode* nodes, const DevNodeAhs* ahs,
                         float footprint, uint32_t n_nodes, int stack_n, const float* o, const float* d,
                         int64_t ray_stride, int64_t r0, uint32_t nr, int s_max, uint32_t* cnt_iv, uint32_t* cnt_smp) {
  hipLaunchKernelGGL((k_trav_count<LDS, AHS>), dim3(grid), dim3(kBlock), bytes, st, nodes, ahs, footprint, n_nodes,
                     stack_n, o, d, ray_stride, r0, nr, s_max, cnt_iv, cnt_smp);
}

hipError_t launch_trav_count(const DevNode* nodes, const DevNodeAhs* ahs, float footprint, uint32_t n_nodes, int depth,
                             const float* o, const float* d, int64_t ray_stride, int64_t r0, uint32_t nr, int s_max,
                             uint32_t* cnt_iv, uint32_t* cnt_smp, hipStream_t st) {
  if (nr == 0) return hipSuccess;
  hipError_t e = trav_setup();
  if (e != hipSuccess) return e;
  const int stack_n = depth + 1;
  const uint32_t grid = (nr + kBlock - 1) / kBlock;
  const bool lds = n_nodes <= (uint32_t)kLdsNodes, hs = ahs != nullptr;
  const uint32_t bytes = trav_lds_bytes(lds, hs, n_nodes, stack_n);
  auto go = [&](auto fn) { fn(grid, bytes, st, nodes, ahs, footprint, n_nodes, stack_n, o, d, ray_stride, r0, nr, s_max,
                              cnt_iv, cnt_smp); };
  if (lds && hs) go(count_launch<true, true>);
  else if (lds) go(count_launch<true, false>);
  else if (hs) go(count_launch<false, true>);
  else go(count_launch<false, false>);
  return hipGetLastError();
}

template <bool LDS, bool AHS>
static void emit_launch(uint32_t grid, uint32_t bytes, hipStream_t st, const DevNode* nodes, const DevNodeAhs* ahs,
                        float footprint, uint32_t n_nodes, int stack_n, uint32_t stage_n, const float* o,
                        const float* d, int64_t ray_stride, int64_t r0, uint32_t nr, const uint32_t* cnt_iv,
                        const uint32_t* cnt_smp, const uint32_t* iv_off, const uint32_t* smp_off, float* iv_t0,
                        float* iv_dt, uint32_t* iv_key, uint32_t* iv_ray, uint32_t* iv_base, ChunkCounts* counts) {
  hipLaunchKernelGGL((k_trav_emit<LDS, AHS>), dim3(grid), dim3(kBlock), bytes, st, nodes, ahs, footprint, n_nodes,
                     stack_n, stage_n, o, d, ray_stride, r0, nr, cnt_iv, cnt_smp, iv_off, smp_off, iv_t0, iv_dt,
                     iv_key, iv_ray, iv_base, counts);
}

hipError_t launch_trav_emit(const DevNode* nodes, const DevNodeAhs* ahs, float footprint, uint32_t n_nodes, int depth,
                            const float* o, const float* d, int64_t ray_stride, int64_t r0, uint32_t nr,
                            const uint32_t* cnt_iv, const uint32_t* cnt_smp, const uint32_t* iv_off,
                            const uint32_t* smp_off, float* iv_t0, float* iv_dt, uint32_t* iv_key, uint32_t* iv_ray,
                            uint32_t* iv_base, ChunkCounts* counts, hipStream_t st) {
  if (nr == 0) return hipSuccess;
  hipError_t e = trav_setup();
  if (e != hipSuccess) return e;
  const int stack_n = depth + 1;
  const uint32_t grid = (nr + kBlock - 1) / kBlock;
  const bool lds = n_nodes <= (uint32_t)kLdsNodes, hs = ahs != nullptr;
  // staging sized so that two blocks still fit in a CU's 160 KiB of LDS (the traversal
  // needs the occupancy), at most 2048 entries of 20 bytes
  const uint32_t fixed = trav_lds_bytes(lds, hs, n_nodes, stack_n);
  const uint32_t budget = 80u * 1024u;
  uint32_t stage_n = fixed + 20u * 256u <= budget ? (budget - fixed) / 20u : 256u;
  stage_n = std::min<uint32_t>(stage_n, 2048u) & ~63u;
  const uint32_t bytes = fixed + 20u * stage_n;
  auto go = [&](auto fn) { fn(grid, bytes, st, nodes, ahs, footprint, n_nodes, stack_n, stage_n, o, d, ray_stride, r0,
                              nr, cnt_iv, cnt_smp, iv_off, smp_off, iv_t0, iv_dt, iv_key, iv_ray, iv_base, counts); };
  if (lds && hs) go(emit_launch<true, true>);
  else if (lds) go(emit_launch<true, false>);
  else if (hs) go(emit_launch<false, true>);
  else go(emit_launch<false, false>);
  return hipGetLastError();
}

}  // namespace amn
