// train.hip -- kernels of the training step: backward of the compositing quadrature, the
// squared-error loss, the per-leaf gradient reduction and Adam.
#include "internal.hpp"
#include "devcommon.hpp"

#include <algorithm>

#include "../../include/amnerf.h"

namespace amn {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float softplusf(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }
__device__ __forceinline__ float logisticf(float z) { return 1.f / (1.f + expf(-z)); }

struct DF {
  float hi, lo;
};
__device__ __forceinline__ DF df_add(DF a, DF b) {
  float s = a.hi + b.hi;
  float bb = s - a.hi;
  float e = (a.hi - (s - bb)) + (b.hi - bb);
  e += a.lo + b.lo;
  float h = s + e;
  return {h, e - (h - s)};
}
__device__ __forceinline__ float df_exp_neg(DF a) { return expf(-a.hi) * (1.f - a.lo); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Exclusive prefix (S before each lane) and inclusive prefix of tau across the wave, as
// compensated pairs, offset by `carry`.
__device__ __forceinline__ void tau_scan(float tau, DF carry, int lane, DF& S, DF& Sn) {
  DF inc = {tau, 0.f};
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    DF y = {__shfl_up(inc.hi, off, 64), __shfl_up(inc.lo, off, 64)};
    if (lane >= off) inc = df_add(inc, y);
  }
  DF exc = {__shfl_up(inc.hi, 1, 64), __shfl_up(inc.lo, 1, 64)};
  if (lane == 0) exc = {0.f, 0.f};
  S = df_add(carry, exc);
  Sn = df_add(carry, inc);
}

// Sum over the lanes above this one.
__device__ __forceinline__ float suffix_excl(float v, int lane) {
  float x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    float y = __shfl_down(x, off, 64);
    if (lane + off < 64) x += y;
  }
  return x - v;
}

// Backward of the quadrature, one wave per ray.  The forward's count of composited samples
// U = ray_used[r] fixes the early-termination sample J = U - 1 (the backward never decides
// termination again, so it differentiates exactly the sum the forward computed).  Pass 1
// recomputes the transmittance carried into each 64-sample step up to J.
// Pass 2 walks the steps in reverse: with T_{j+1} = exp(-S_{j+1}) and the suffix sums
// sum_{i>j} w_i c_i (and of w_i t_i, w_i) from a reverse scan,
//   dL/dtau_j = g . (T_{j+1} c_j - sum_{i>j} w_i c_i) + g_D (T_{j+1} t_j - sum_{i>j} w_i t_i)
//             + g_A (T_{j+1} - sum_{i>j} w_i),
// dL/dsigma^_j = dL/dtau_j delta_j logistic(sigma^_j), dL/dc^_j = g w_j c_j (1 - c_j).
__global__ __launch_bounds__(kThreads) void k_comp_bwd(
    uint32_t nr, IvSet iv, const float* __restrict__ smp_out, int64_t r0, int jitter,
    uint64_t seed, const uint32_t* __restrict__ ray_used, const float* __restrict__ g_rgb,
    const float* __restrict__ g_depth, const float* __restrict__ g_opac, float* __restrict__ gpre) {
  const int lane = threadIdx.x & 63;
  const uint32_t r = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (r >= nr) return;
  const uint32_t i0 = iv.iv_off[r], i1 = iv.iv_off[r + 1];
  const uint32_t s0 = iv.smp_off[r], ns = iv.smp_off[r + 1] - s0;
  if (ns == 0) return;
  const float gr = g_rgb[3 * (uint64_t)(r0 + r)], gg = g_rgb[3 * (uint64_t)(r0 + r) + 1],
              gb = g_rgb[3 * (uint64_t)(r0 + r) + 2];
  const float gd = g_depth ? g_depth[r0 + r] : 0.f;
  const float ga = g_opac ? g_opac[r0 + r] : 0.f;
  constexpr int kMaxSteps = (AMNERF_MAX_SAMPLES + 63) / 64;
  DF carry_at[kMaxSteps];
  auto sample = [&](uint32_t j, float& tau, float& delta, float& t, float4& z) {
    const uint32_t i = find_interval(iv.base, i0, i1, s0 + j);
    const uint32_t jj = s0 + j - iv.base[i];
    z = *reinterpret_cast<const float4*>(smp_out + 4 * (uint64_t)(s0 + j));
    delta = iv.dt[i] / (float)key_n(iv.key[i]);
    const float u = stratum_u(jitter, seed, (uint64_t)(r0 + r), i - i0);
    t = sample_t(iv.t0[i], delta, jj, u);
    tau = softplusf(z.x) * delta;
  };
  // pass 1: forward scan of the steps up to the termination sample
  const uint32_t U = ray_used[r] < ns ? ray_used[r] : ns;
  const uint32_t J = U > 0 ? U - 1 : 0;
  const uint32_t steps = (U + 63) / 64;
  DF carry = {0.f, 0.f};
  for (uint32_t st = 0; st < steps; ++st) {
    carry_at[st] = carry;
    const uint32_t j = st * 64u + lane;
    float tau = 0.f, delta, t;
    float4 z;
    if (j < ns) sample(j, tau, delta, t, z);
    DF S, Sn;
    tau_scan(tau, carry, lane, S, Sn);
    carry = {__shfl(Sn.hi, 63, 64), __shfl(Sn.lo, 63, 64)};
  }
  // pass 2: reverse over steps
  float sufR = 0.f, sufG = 0.f, sufB = 0.f, sufD = 0.f, sufA = 0.f;
  for (int st = (int)steps - 1; st >= 0; --st) {
    const uint32_t base = (uint32_t)st * 64u;
    const uint32_t j = base + lane;
    const bool valid = j <= J && U > 0;
    float tau = 0.f, delta = 0.f, t = 0.f;
    float4 z = {0.f, 0.f, 0.f, 0.f};
    if (j < ns) sample(j, tau, delta, t, z);
    DF S, Sn;
    tau_scan(valid ? tau : 0.f, carry_at[st], lane, S, Sn);
    const float cr = logisticf(z.y), cg = logisticf(z.z), cbv = logisticf(z.w);
    const float w = valid ? df_exp_neg(S) * -expm1f(-tau) : 0.f;
    const float Tn = df_exp_neg(Sn);
    const float vR = w * cr, vG = w * cg, vB = w * cbv, vD = w * t;
    const float aR = suffix_excl(vR, lane) + sufR, aG = suffix_excl(vG, lane) + sufG;
    const float aB = suffix_excl(vB, lane) + sufB, aD = suffix_excl(vD, lane) + sufD;
    const float aA = suffix_excl(w, lane) + sufA;
    if (j < ns) {
      float4 out = {0.f, 0.f, 0.f, 0.f};
      if (valid) {
        const float dtau = gr * (Tn * cr - aR) + gg * (Tn * cg - aG) + gb * (Tn * cbv - aB) +
                           gd * (Tn * t - aD) + ga * (Tn - aA);
        out.x = dtau * delta * logisticf(z.x);
        out.y = gr * w * cr * (1.f - cr);
        out.z = gg * w * cg * (1.f - cg);
        out.w = gb * w * cbv * (1.f - cbv);
      }
      *reinterpret_cast<float4*>(gpre + 4 * (uint64_t)(s0 + j)) = out;
    }
    sufR += wave_sum(vR);
    sufG += wave_sum(vG);
    sufB += wave_sum(vB);
    sufD += wave_sum(vD);
    sufA += wave_sum(w);
  }
  // samples after the termination step carry no gradient
  for (uint32_t j = steps * 64u + lane; j < ns; j += 64)
    *reinterpret_cast<float4*>(gpre + 4 * (uint64_t)(s0 + j)) = float4{0.f, 0.f, 0.f, 0.f};
}

// Segments of at most kSegTiles tiles per leaf: seg_off[b] (exclusive scan) and the total.
__global__ __launch_bounds__(1024) void k_seg_offsets(const uint32_t* __restrict__ tile_off,
                                                      uint32_t n_leaves, uint32_t* __restrict__ seg_off) {
  __shared__ uint32_t sh[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t carry = 0;
  for (uint32_t c = 0; c < n_leaves; c += 1024) {
    const uint32_t b = c + threadIdx.x;
    const uint32_t nt = b < n_leaves ? tile_off[b + 1] - tile_off[b] : 0u;
    const uint32_t ns = (nt + kSegTiles - 1) / kSegTiles;
    uint32_t x = ns;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      uint32_t s = sh[w];
      if (w < wave) pre += s;
      tot += s;
    }
    if (b < n_leaves) seg_off[b] = carry + pre + x - ns;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    seg_off[n_leaves] = carry;
    seg_off[n_leaves + 1] = 0u;   // the backward's segment queue
  }
}

// grad[b][p] = sum over the segments of leaf b, in order, of part[seg][p].
__global__ __launch_bounds__(kThreads) void k_grad_reduce(const float* __restrict__ part,
                                                          const uint32_t* __restrict__ seg_off,
                                                          uint32_t n_leaves, uint32_t P,
                                                          float* __restrict__ grad) {
  const uint64_t total = (uint64_t)n_leaves * P;
  for (uint64_t id = (uint64_t)blockIdx.x * kThreads + threadIdx.x; id < total;
       id += (uint64_t)gridDim.x * kThreads) {
    const uint32_t b = (uint32_t)(id / P), p = (uint32_t)(id % P);
    const uint32_t s1 = seg_off[b + 1];
    const float* q = part + p;
    float s = 0.f;
    uint32_t seg = seg_off[b];
    // eight loads in flight, then their sum in segment order (the order of one at a time)
    for (; seg + 8 <= s1; seg += 8) {
      float v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = q[(uint64_t)(seg + k) * P];
#pragma unroll
      for (int k = 0; k < 8; ++k) s += v[k];
    }
    for (; seg < s1; ++seg) s += q[(uint64_t)seg * P];
    grad[id] = s;
  }
}

// Per ray: g = dL/drgb = 2 (rgb - target) / (3 R); block partial sums of squared errors.
__global__ __launch_bounds__(kThreads) void k_loss_grad(uint32_t R, const float* __restrict__ rgb,
                                                        const float* __restrict__ target,
                                                        float* __restrict__ g_rgb,
                                                        float* __restrict__ partial) {
  __shared__ float sh[kThreads / 64];
  const uint32_t r = blockIdx.x * kThreads + threadIdx.x;
  float s = 0.f;
  if (r < R) {
    const float scale = 2.f / (3.f * (float)R);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float e = rgb[3 * (uint64_t)r + c] - target[3 * (uint64_t)r + c];
      g_rgb[3 * (uint64_t)r + c] = scale * e;
      s = fmaf(e, e, s);
    }
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(1024) void k_loss_final(const float* __restrict__ partial, uint32_t nb,
                                                     uint32_t R, float* __restrict__ loss) {
  __shared__ float sh[1024];
  float s = 0.f;
  for (uint32_t i = threadIdx.x; i < nb; i += 1024) s += partial[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 512; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = sh[0] / (3.f * (float)R);
}

__global__ __launch_bounds__(kThreads) void k_adam(int64_t n, float* __restrict__ p, float* __restrict__ m,
                                                   float* __restrict__ v, const float* __restrict__ g,
                                                   float lr, float b1, float b2, float eps, float c1,
                                                   float c2) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

}  // namespace

hipError_t launch_comp_bwd(uint32_t nr, const IvSet& iv, const float* smp_out, int64_t r0, int jitter,
                           uint64_t seed, const uint32_t* ray_used, const float* g_rgb, const float* g_depth,
                           const float* g_opac, float* gpre, hipStream_t st) {
  if (nr == 0) return hipSuccess;
  const uint32_t rays_per_block = kThreads / 64;
  hipLaunchKernelGGL(k_comp_bwd, dim3((nr + rays_per_block - 1) / rays_per_block), dim3(kThreads), 0, st, nr,
                     iv, smp_out, r0, jitter, seed, ray_used, g_rgb, g_depth, g_opac, gpre);
  return hipGetLastError();
}

hipError_t launch_seg_offsets(const uint32_t* tile_off, uint32_t n_leaves, uint32_t* seg_off, hipStream_t st) {
  hipLaunchKernelGGL(k_seg_offsets, dim3(1), dim3(1024), 0, st, tile_off, n_leaves, seg_off);
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const float* part, const uint32_t* seg_off, uint32_t n_leaves, uint32_t P,
                              float* grad, hipStream_t st) {
  // one thread per parameter (its loads are what it waits for)
  const uint64_t total = (uint64_t)n_leaves * P;
  const uint64_t blocks = std::max<uint64_t>(1, std::min<uint64_t>((total + kThreads - 1) / kThreads, 1u << 20));
  hipLaunchKernelGGL(k_grad_reduce, dim3((uint32_t)blocks), dim3(kThreads), 0, st, part, seg_off, n_leaves, P, grad);
  return hipGetLastError();
}

hipError_t launch_loss_grad(uint32_t R, const float* rgb, const float* target, float* g_rgb, float* partial,
                            float* loss, hipStream_t st) {
  const uint32_t nb = R == 0 ? 1 : (R + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_loss_grad, dim3(nb), dim3(kThreads), 0, st, R, rgb, target, g_rgb, partial);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1024), 0, st, partial, nb, R, loss);
  return hipGetLastError();
}

size_t loss_partial_words(uint64_t R) { return R == 0 ? 1 : (R + kThreads - 1) / kThreads; }

hipError_t launch_adam(int64_t n, float* p, float* m, float* v, const float* g, float lr, float b1, float b2,
                       float eps, int step, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  int64_t blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_adam, dim3((uint32_t)blocks), dim3(kThreads), 0, st, n, p, m, v, g, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace amn
