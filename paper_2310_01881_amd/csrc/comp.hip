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
// both.  Lane j finds its interval by binary search over the intervals' first-sample
// indices.
constexpr uint32_t kStage = 256;   // intervals of a ray searched in LDS (more: in memory)

__global__ __launch_bounds__(kThreads) void k_composite(
    uint32_t nr, IvSet iv, const float* __restrict__ smp_out, int64_t r0, int jitter,
    uint64_t seed, float eps, float* __restrict__ rgb, float* __restrict__ depth,
    float* __restrict__ opac, float* __restrict__ weights, uint32_t* __restrict__ ray_used,
    ChunkCounts* __restrict__ counts) {
  __shared__ uint32_t sbase[kThreads / 64][kStage];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t r = blockIdx.x * (kThreads / 64) + wave;
  if (r >= nr) return;
  const uint32_t i0 = iv.iv_off[r], i1 = iv.iv_off[r + 1];
  const uint32_t s0 = iv.smp_off[r], ns = iv.smp_off[r + 1] - s0;
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
  float cr = 0.f, cg = 0.f, cb = 0.f, dep = 0.f, acc = 0.f;
  uint32_t used = ns;   // samples composited: up to and including the stop sample
  if (ns > 0) {
    DF carry = {0.f, 0.f};
    bool done = false;
    for (uint32_t base = 0; base < ns; base += 64) {
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
      const DF Sn = df_add(carry, inc);
      const float Tn = df_exp_neg(Sn);                        // T_{j+1}
      const float Tsh = dpp_or_zero<0x138, 0xF>(Tn);          // wave_shr:1: lane j - 1's T_j
      const float T = lane == 0 ? df_exp_neg(carry) : Tsh;
      float w = valid ? T * one_minus_exp_neg(tau) : 0.f;
      const bool stop = valid && eps > 0.f && Tn < eps;
      const uint64_t stops = __ballot(stop);
      if (stops) {
        const int first = __ffsll((unsigned long long)stops) - 1;
        if (lane > first) w = 0.f;
        done = true;
        used = base + (uint32_t)first + 1u;
      }
      cr = fmaf(w, sig_c[0], cr);
      cg = fmaf(w, sig_c[1], cg);
      cb = fmaf(w, sig_c[2], cb);
      dep = fmaf(w, t, dep);
      acc += w;
      if (weights && j < ns) weights[wbase + j] = w;
      carry = {lane_value(Sn.hi, 63), lane_value(Sn.lo, 63)};
      if (done && !weights) break;
    }
    cr = wave_sum(cr);
    cg = wave_sum(cg);
    cb = wave_sum(cb);
    dep = wave_sum(dep);
    acc = wave_sum(acc);
  }
  if (lane == 0) {
    ray_used[r] = used;
    rgb[3 * (uint64_t)(r0 + r) + 0] = cr;
    rgb[3 * (uint64_t)(r0 + r) + 1] = cg;
    rgb[3 * (uint64_t)(r0 + r) + 2] = cb;
    if (depth) depth[r0 + r] = dep;
    if (opac) opac[r0 + r] = acc;
    if (!isfinite(cr) || !isfinite(cg) || !isfinite(cb) || !isfinite(dep) || !isfinite(acc))
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
                               const uint32_t* plain_total) {
  if (threadIdx.x != 0) return;
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
  hipLaunchKernelGGL(k_composite, dim3(grid), dim3(kThreads), 0, st, nr, iv, smp_out, r0, jitter, seed,
                     ert_eps, rgb, depth, opac, weights, ray_used, counts);
  const uint32_t sgrid = std::min<uint32_t>(256u, (nr + 4 * kThreads - 1) / (4 * kThreads));
  hipLaunchKernelGGL(k_sum_used, dim3(sgrid), dim3(kThreads), 0, st, nr, ray_used, counts);
  return hipGetLastError();
}

hipError_t launch_chunk_finish(ChunkCounts* counts, const uint32_t* smp_off_total,
                               const uint32_t* iv_off_total, const uint32_t* plain_smp_total,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_chunk_finish, dim3(1), dim3(64), 0, st, counts, smp_off_total, iv_off_total,
                     plain_smp_total);
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
