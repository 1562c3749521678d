// comp.hip -- front-to-back volume rendering of each ray's samples with early ray
// termination (Section 3.1 defers the accumulation to the NeRF quadrature; Section 4.1
// uses early termination).
//
// Per ray: tau_j = sigma_j delta_j, S_j = sum_{i<j} tau_i accumulated in float32 with
// compensation (log-space transmittance), T_j = exp(-S_j), w_j = T_j * (1 - exp(-tau_j))
// via expm1, stop after the first j with T_{j+1} < eps.
#include <algorithm>

#include "internal.hpp"
#include "devcommon.hpp"

namespace amn {
namespace {

constexpr int kThreads = 256;

// Output heads and exponentials from the hardware base-2 exponential, logarithm and
// reciprocal (about 1 ulp each; the float32 result stays far inside the 1e-5 parity
// tolerance).
constexpr float kLog2e = 1.44269504f, kLn2 = 0.693147181f;
__device__ __forceinline__ float exp_neg(float x) { return __builtin_amdgcn_exp2f(-kLog2e * x); }
// softplus z = max(z, 0) + log(1 + e^-|z|), with log1p(e) = e (1 - e/2) below 2^-12
__device__ __forceinline__ float softplusf(float z) {
  const float e = exp_neg(fabsf(z));
  const float l = e < 2.44140625e-4f ? e * fmaf(-0.5f, e, 1.f) : __builtin_amdgcn_logf(1.f + e) * kLn2;
  return fmaxf(z, 0.f) + l;
}
__device__ __forceinline__ float logisticf(float z) { return __builtin_amdgcn_rcpf(1.f + exp_neg(z)); }
// 1 - e^-t for t >= 0: a quartic Taylor polynomial below 1/16, else from the exponential
__device__ __forceinline__ float one_minus_exp_neg(float t) {
  if (t < 0.0625f) return t * fmaf(t, fmaf(t, fmaf(t, -1.f / 24.f, 1.f / 6.f), -0.5f), 1.f);
  return 1.f - exp_neg(t);
}

// Unevaluated float pair hi + lo (compensated sums).
struct DF {
  float hi, lo;
};

__device__ __forceinline__ DF df_add(DF a, DF b) {
  float s = a.hi + b.hi;
  float bb = s - a.hi;
  float e = (a.hi - (s - bb)) + (b.hi - bb);   // TwoSum error of the high parts
  e += a.lo + b.lo;
  float h = s + e;
  return {h, e - (h - s)};
}

// exp(-(hi + lo)) for |lo| << 1: exp(-hi) * (1 - lo).
__device__ __forceinline__ float df_exp_neg(DF a) { return exp_neg(a.hi) * (1.f - a.lo); }

// Inclusive compensated prefix sum over the wave on wave_scan_incl's shift pattern (within
// rows of 16 by 1, 2, 4, 8, then the last lane of row 0 (2) into row 1 (3) and the last
// lane of row 1 into rows 2 and 3; lanes whose source is outside the pattern add 0).  The
// high parts are added with an exact TwoSum; the low parts, and each TwoSum's rounding
// error, go into a plain running sum of low parts, normalised once at the end.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void df_scan_step(float& hi, float& lo) {
  const float b = dpp_or_zero<CTRL, ROW_MASK>(hi);
  const float s = hi + b;
  const float bb = s - hi;
  const float e = (hi - (s - bb)) + (b - bb);
  lo = lo + dpp_or_zero<CTRL, ROW_MASK>(lo) + e;
  hi = s;
}

__device__ __forceinline__ DF df_scan_incl(DF v) {
  float hi = v.hi, lo = v.lo;
  df_scan_step<0x111, 0xF>(hi, lo);
  df_scan_step<0x112, 0xF>(hi, lo);
  df_scan_step<0x114, 0xF>(hi, lo);
  df_scan_step<0x118, 0xF>(hi, lo);
  df_scan_step<0x142, 0xA>(hi, lo);
  df_scan_step<0x143, 0xC>(hi, lo);
  const float h = hi + lo;
  return {h, lo - (h - hi)};
}

__device__ __forceinline__ float wave_sum(float v) { return lane_value(wave_scan_incl(v), 63); }

// One wave per ray, 64 samples per step.  Lane j of a step handles sample base + j:
// tau_j, then S_j = sum_{i<j} tau_i by a compensated (float pair) prefix scan across the
// wave plus the running total of earlier steps; T_j = exp(-S_j), w_j = T_j (1 - e^-tau_j).
// Early termination: the first lane whose T_{j+1} < eps keeps its sample and later lanes
// (and steps) contribute nothing.  T_j is the neighbouring lane's T_{j+1} (the exclusive
// sum of lane j is the inclusive sum of lane j - 1), so one exponential per sample serves
// both.  Each step's weighted sums are reduced across the wave and added to the ray's
// running totals, so the state carried from one step to the next is a handful of scalars.
// Lane j finds its interval by binary search over the intervals' first-sample indices.
//
// ROUND: one 64-sample window (step `round`) of every ray that is still marching, the state
// of the earlier windows read from and written back to `carry`; a ray's outputs are written
// when it terminates or its last window is done.  The arithmetic of each step is the same
// as in the single pass, so a render in rounds is bit-identical to one in a single pass.
constexpr uint32_t kStage = 256;   // intervals of a ray searched in LDS (more: in memory)
constexpr uint32_t kDone = 0x80000000u;

template <bool ROUND>
__global__ __launch_bounds__(kThreads) void k_composite(
    uint32_t nr, IvSet iv, const float* __restrict__ smp_out, int64_t r0, int jitter,
    uint64_t seed, float eps, float* __restrict__ rgb, float* __restrict__ depth,
    float* __restrict__ opac, float* __restrict__ weights, uint32_t* __restrict__ ray_used,
    ChunkCounts* __restrict__ counts, CompCarry* __restrict__ carry_st, uint32_t round) {
  __shared__ uint32_t sbase[kThreads / 64][kStage];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t r = blockIdx.x * (kThreads / 64) + wave;
  if (r >= nr) return;
  const uint32_t i0 = iv.iv_off[r], i1 = iv.iv_off[r + 1];
  const uint32_t s0 = iv.smp_off[r], ns = iv.smp_off[r + 1] - s0;
  uint32_t sb = 0, se = ns;                    // this launch's samples of the ray
  DF S = {0.f, 0.f};                           // sum of tau before sample sb
  float tot[5] = {0.f, 0.f, 0.f, 0.f, 0.f};    // rgb, depth, opacity so far
  if (ROUND) {
    sb = 64u * round;
    if (sb >= ns && !(ns == 0 && round == 0)) return;   // finished in an earlier window
    if (round > 0) {
      const CompCarry c = carry_st[r];
      if (c.state & kDone) return;
      S = {c.s_hi, c.s_lo};
      tot[0] = c.cr; tot[1] = c.cg; tot[2] = c.cb; tot[3] = c.dep; tot[4] = c.acc;
    }
    se = sb + 64u < ns ? sb + 64u : ns;
  }
  // the ray's interval start samples (relative to s0), searched in LDS
  const uint32_t m = i1 - i0;
  const bool staged = m <= kStage;
  if (staged) {
    for (uint32_t k = lane; k < m; k += 64) sbase[wave][k] = iv.base[i0 + k] - s0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  const uint64_t wbase = counts->smp_global + s0;
  uint32_t used = ns;   // samples composited: up to and including the stop sample
  bool done = false;
  uint32_t next = sb;   // first sample after the last step processed
  for (uint32_t base = sb; base < se; base += 64) {
    next = base + 64u;
    const uint32_t j = base + lane;
    const bool valid = !done && j < ns;
    float tau = 0.f, sig_c[3] = {0.f, 0.f, 0.f}, t = 0.f;
    if (valid) {
      uint32_t i;
      if (staged) {
        uint32_t lo = 0, hi = m;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (sbase[wave][mid] <= j) lo = mid; else hi = mid;
        }
        i = i0 + lo;
      } else {
        i = find_interval(iv.base, i0, i1, s0 + j);
      }
      const uint32_t jj = s0 + j - iv.base[i];
      const float4 z = *reinterpret_cast<const float4*>(smp_out + 4 * (uint64_t)(s0 + j));
      const float delta = iv.dt[i] / (float)key_n(iv.key[i]);
      const float u = stratum_u(jitter, seed, (uint64_t)(r0 + r), i - i0);
      t = sample_t(iv.t0[i], delta, jj, u);
      tau = softplusf(z.x) * delta;       // sigma = softplus, rgb = logistic
      sig_c[0] = logisticf(z.y);
      sig_c[1] = logisticf(z.z);
      sig_c[2] = logisticf(z.w);
    }
    // inclusive compensated scan of tau across the wave; exclusive = shifted by one lane
    const DF inc = df_scan_incl({tau, 0.f});
    const DF Sn = df_add(S, inc);
    const float Tn = df_exp_neg(Sn);                        // T_{j+1}
    const float Tsh = dpp_or_zero<0x138, 0xF>(Tn);          // wave_shr:1: lane j - 1's T_j
    const float T = lane == 0 ? df_exp_neg(S) : Tsh;
    float w = valid ? T * one_minus_exp_neg(tau) : 0.f;
    const bool stop = valid && eps > 0.f && Tn < eps;
    const uint64_t stops = __ballot(stop);
    if (stops) {
      const int first = __ffsll((unsigned long long)stops) - 1;
      if (lane > first) w = 0.f;
      done = true;
      used = base + (uint32_t)first + 1u;
    }
    tot[0] += wave_sum(w * sig_c[0]);
    tot[1] += wave_sum(w * sig_c[1]);
    tot[2] += wave_sum(w * sig_c[2]);
    tot[3] += wave_sum(w * t);
    tot[4] += wave_sum(w);
    if (weights && j < ns) weights[wbase + j] = w;
    S = {lane_value(Sn.hi, 63), lane_value(Sn.lo, 63)};
    if (done) break;
  }
  // a ray that stopped has weight 0 on every later sample
  if (weights && done)
    for (uint32_t j = next + lane; j < ns; j += 64) weights[wbase + j] = 0.f;
  if (ROUND && !done && se < ns) {
    if (lane == 0) carry_st[r] = {S.hi, S.lo, tot[0], tot[1], tot[2], tot[3], tot[4], 0u};
    return;
  }
  if (lane == 0) {
    if (ROUND) carry_st[r].state = kDone;
    ray_used[r] = used;
    rgb[3 * (uint64_t)(r0 + r) + 0] = tot[0];
    rgb[3 * (uint64_t)(r0 + r) + 1] = tot[1];
    rgb[3 * (uint64_t)(r0 + r) + 2] = tot[2];
    if (depth) depth[r0 + r] = tot[3];
    if (opac) opac[r0 + r] = tot[4];
    if (!isfinite(tot[0]) || !isfinite(tot[1]) || !isfinite(tot[2]) || !isfinite(tot[3]) || !isfinite(tot[4]))
      atomicAdd(reinterpret_cast<unsigned long long*>(&counts->nonfinite), 1ull);
  }
}

// counts->composited += sum of ray_used[0, nr): block sums in a fixed order, one integer
// atomic per block.
__global__ __launch_bounds__(kThreads) void k_sum_used(uint32_t nr, const uint32_t* __restrict__ ray_used,
                                                       ChunkCounts* __restrict__ counts) {
  __shared__ uint32_t sh[kThreads / 64];
  uint32_t s = 0;
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < nr; i += gridDim.x * kThreads) s += ray_used[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int w = 0; w < kThreads / 64; ++w) t += sh[w];
    if (t) atomicAdd(reinterpret_cast<unsigned long long*>(&counts->composited), (unsigned long long)t);
  }
}

// Records the chunk's totals for the host and advances the global sample base.
__global__ void k_chunk_finish(ChunkCounts* counts, const uint32_t* smp_total, const uint32_t* iv_total,
                               const uint32_t* plain_total, int rounds) {
  if (threadIdx.x != 0) return;
  if (!rounds) counts->evaluated += *smp_total;   // (in rounds: added by each round's selection)
  counts->smp_global += *smp_total;
  counts->iv_global += *iv_total;
  counts->plain_smp += *plain_total;
}

__global__ void k_chunk_begin(ChunkCounts* counts, const uint32_t* iv_total, uint32_t seg, uint32_t n_leaves) {
  if (threadIdx.x != 0) return;
  const uint32_t n = *iv_total;
  counts->n_iv = n;
  counts->mat_n = n_leaves * ((n + seg - 1) / seg);
}

// Adds the second lane's running totals into the first lane's counters.
__global__ void k_counts_merge(ChunkCounts* a, const ChunkCounts* b) {
  if (threadIdx.x != 0) return;
  a->smp_global += b->smp_global;
  a->iv_global += b->iv_global;
  a->nonfinite += b->nonfinite;
  a->fallback += b->fallback;
  a->plain_smp += b->plain_smp;
  a->unreached += b->unreached;
  a->composited += b->composited;
  a->evaluated += b->evaluated;
}

__global__ void k_counts_reset(ChunkCounts* counts) {
  if (threadIdx.x != 0) return;
  ChunkCounts z = {};
  *counts = z;
}

}  // namespace

hipError_t launch_composite(uint32_t nr, const IvSet& iv, const float* smp_out, int64_t r0,
                            int jitter, uint64_t seed, float ert_eps, float* rgb, float* depth,
                            float* opac, float* weights, uint32_t* ray_used, ChunkCounts* counts,
                            hipStream_t st) {
  if (nr == 0) return hipSuccess;
  const uint32_t rays_per_block = kThreads / 64;
  uint32_t grid = (nr + rays_per_block - 1) / rays_per_block;
  hipLaunchKernelGGL(k_composite<false>, dim3(grid), dim3(kThreads), 0, st, nr, iv, smp_out, r0, jitter, seed,
                     ert_eps, rgb, depth, opac, weights, ray_used, counts, nullptr, 0u);
  return launch_sum_used(nr, ray_used, counts, st);
}

hipError_t launch_composite_round(uint32_t nr, const IvSet& iv, const float* smp_out, int64_t r0, int jitter,
                                  uint64_t seed, float ert_eps, float* rgb, float* depth, float* opac,
                                  float* weights, uint32_t* ray_used, ChunkCounts* counts, CompCarry* carry,
                                  uint32_t round, hipStream_t st) {
  if (nr == 0) return hipSuccess;
  const uint32_t rays_per_block = kThreads / 64;
  uint32_t grid = (nr + rays_per_block - 1) / rays_per_block;
  hipLaunchKernelGGL(k_composite<true>, dim3(grid), dim3(kThreads), 0, st, nr, iv, smp_out, r0, jitter, seed,
                     ert_eps, rgb, depth, opac, weights, ray_used, counts, carry, round);
  return hipGetLastError();
}

hipError_t launch_sum_used(uint32_t nr, const uint32_t* ray_used, ChunkCounts* counts, hipStream_t st) {
  if (nr == 0) return hipSuccess;
  const uint32_t sgrid = std::min<uint32_t>(256u, (nr + 4 * kThreads - 1) / (4 * kThreads));
  hipLaunchKernelGGL(k_sum_used, dim3(sgrid), dim3(kThreads), 0, st, nr, ray_used, counts);
  return hipGetLastError();
}

hipError_t launch_chunk_finish(ChunkCounts* counts, const uint32_t* smp_off_total,
                               const uint32_t* iv_off_total, const uint32_t* plain_smp_total, int rounds,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_chunk_finish, dim3(1), dim3(64), 0, st, counts, smp_off_total, iv_off_total,
                     plain_smp_total, rounds);
  return hipGetLastError();
}

hipError_t launch_counts_merge(ChunkCounts* a, const ChunkCounts* b, hipStream_t st) {
  hipLaunchKernelGGL(k_counts_merge, dim3(1), dim3(64), 0, st, a, b);
  return hipGetLastError();
}

hipError_t launch_counts_reset(ChunkCounts* counts, hipStream_t st) {
  hipLaunchKernelGGL(k_counts_reset, dim3(1), dim3(64), 0, st, counts);
  return hipGetLastError();
}

hipError_t launch_chunk_begin(ChunkCounts* counts, const uint32_t* iv_total, uint32_t seg, uint32_t n_leaves,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_chunk_begin, dim3(1), dim3(64), 0, st, counts, iv_total, seg, n_leaves);
  return hipGetLastError();
}

}  // namespace amn
