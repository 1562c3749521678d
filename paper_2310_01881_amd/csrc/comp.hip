// comp.hip -- front-to-back volume rendering of each ray's samples with early ray
// termination (Section 3.1 defers the accumulation to the NeRF quadrature; Section 4.1
// uses early termination).
//
// Per ray: tau_j = sigma_j delta_j, S_j = sum_{i<j} tau_i accumulated in float32 with
// Kahan compensation (log-space transmittance), T_j = exp(-S_j),
// w_j = T_j * (1 - exp(-tau_j)) via expm1, stop after the first j with T_{j+1} < eps.
#include "internal.hpp"
#include "devcommon.hpp"

namespace amn {
namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_composite(
    uint32_t nr, const uint32_t* __restrict__ iv_off, const uint32_t* __restrict__ smp_off,
    const float* __restrict__ iv_t0, const float* __restrict__ iv_dt,
    const uint32_t* __restrict__ iv_key, const float* __restrict__ smp_out, int64_t r0, int jitter,
    uint64_t seed, float eps, float* __restrict__ rgb, float* __restrict__ depth,
    float* __restrict__ opac, float* __restrict__ weights, ChunkCounts* __restrict__ counts) {
  uint32_t r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= nr) return;
  const uint32_t i0 = iv_off[r], i1 = iv_off[r + 1];
  uint32_t s = smp_off[r];
  const uint64_t wbase = counts->smp_global;
  float S = 0.f, comp = 0.f;
  float cr = 0.f, cg = 0.f, cb = 0.f, dep = 0.f, acc = 0.f;
  bool done = false;
  for (uint32_t i = i0; i < i1; ++i) {
    const uint32_t n = key_n(iv_key[i]);
    const float t0 = iv_t0[i];
    const float delta = iv_dt[i] / (float)n;
    const float u = stratum_u(jitter, seed, (uint64_t)(r0 + r), i - i0);
    for (uint32_t j = 0; j < n; ++j, ++s) {
      if (done) {
        if (weights) weights[wbase + s] = 0.f;
        continue;
      }
      const float4 v = *reinterpret_cast<const float4*>(smp_out + 4 * (uint64_t)s);
      const float tau = v.x * delta;
      const float T = expf(-S);
      const float w = T * -expm1f(-tau);
      cr = fmaf(w, v.y, cr);
      cg = fmaf(w, v.z, cg);
      cb = fmaf(w, v.w, cb);
      dep = fmaf(w, sample_t(t0, delta, j, u), dep);
      acc += w;
      if (weights) weights[wbase + s] = w;
      // Kahan-compensated S += tau
      const float y = tau - comp;
      const float tsum = S + y;
      comp = (tsum - S) - y;
      S = tsum;
      if (eps > 0.f && expf(-S) < eps) done = true;
    }
  }
  rgb[3 * (uint64_t)(r0 + r) + 0] = cr;
  rgb[3 * (uint64_t)(r0 + r) + 1] = cg;
  rgb[3 * (uint64_t)(r0 + r) + 2] = cb;
  if (depth) depth[r0 + r] = dep;
  if (opac) opac[r0 + r] = acc;
  if (!isfinite(cr) || !isfinite(cg) || !isfinite(cb) || !isfinite(dep) || !isfinite(acc))
    atomicAdd(reinterpret_cast<unsigned long long*>(&counts->nonfinite), 1ull);
}

// Records the chunk's totals for the host and advances the global sample base.
__global__ void k_chunk_finish(ChunkCounts* counts, const uint32_t* smp_total, const uint32_t* iv_total) {
  if (threadIdx.x != 0) return;
  counts->smp_global += *smp_total;
  counts->iv_global += *iv_total;
}

__global__ void k_chunk_begin(ChunkCounts* counts, const uint32_t* iv_total) {
  if (threadIdx.x != 0) return;
  counts->n_iv = *iv_total;
}

__global__ void k_counts_reset(ChunkCounts* counts) {
  if (threadIdx.x != 0) return;
  ChunkCounts z = {};
  *counts = z;
}

}  // namespace

hipError_t launch_composite(uint32_t nr, const uint32_t* iv_off, const uint32_t* smp_off,
                            const float* iv_t0, const float* iv_dt, const uint32_t* iv_key,
                            const float* smp_out, int64_t r0, int jitter, uint64_t seed,
                            float ert_eps, float* rgb, float* depth, float* opac, float* weights,
                            ChunkCounts* counts, hipStream_t st) {
  if (nr == 0) return hipSuccess;
  uint32_t grid = (nr + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_composite, dim3(grid), dim3(kThreads), 0, st, nr, iv_off, smp_off, iv_t0, iv_dt,
                     iv_key, smp_out, r0, jitter, seed, ert_eps, rgb, depth, opac, weights, counts);
  return hipGetLastError();
}

hipError_t launch_chunk_finish(ChunkCounts* counts, const uint32_t* smp_off_total,
                               const uint32_t* iv_off_total, hipStream_t st) {
  hipLaunchKernelGGL(k_chunk_finish, dim3(1), dim3(64), 0, st, counts, smp_off_total, iv_off_total);
  return hipGetLastError();
}

hipError_t launch_counts_reset(ChunkCounts* counts, hipStream_t st) {
  hipLaunchKernelGGL(k_counts_reset, dim3(1), dim3(64), 0, st, counts);
  return hipGetLastError();
}

hipError_t launch_chunk_begin(ChunkCounts* counts, const uint32_t* iv_total, hipStream_t st) {
  hipLaunchKernelGGL(k_chunk_begin, dim3(1), dim3(64), 0, st, counts, iv_total);
  return hipGetLastError();
}

}  // namespace amn
