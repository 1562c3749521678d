// scan.hip -- exclusive prefix sums of uint32 arrays whose length may live on the device
// (reduce, scan of block sums, rescan), used for ray offsets, bucket bases and tiles.
#include "internal.hpp"

namespace amn {
namespace {

constexpr int kThreads = 256;
constexpr int kPer = kScanItems / kThreads;   // 8
constexpr int kMaxGrid = 2048;

__device__ __forceinline__ uint64_t scan_n(uint64_t n_cap, const uint32_t* n_dev) {
  if (!n_dev) return n_cap;
  uint64_t n = *n_dev;
  return n < n_cap ? n : n_cap;
}

// Inclusive scan of one value per thread across a 256-thread block; returns the block total.
__device__ __forceinline__ uint32_t block_incl_scan(uint32_t v, uint32_t* sh_wave, uint32_t& incl) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(v, off, 64);
    if (lane >= off) v += y;
  }
  if (lane == 63) sh_wave[wave] = v;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    uint32_t s = sh_wave[w];
    if (w < wave) pre += s;
    tot += s;
  }
  __syncthreads();
  incl = v + pre;
  return tot;
}

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t* __restrict__ in,
                                                          uint64_t n_cap, const uint32_t* n_dev,
                                                          uint32_t* __restrict__ bsum) {
  __shared__ uint32_t sh[kThreads / 64];
  const uint64_t n = scan_n(n_cap, n_dev);
  const uint64_t nb = (n + kScanItems - 1) / kScanItems;
  for (uint64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    uint64_t base = b * kScanItems + (uint64_t)threadIdx.x * kPer;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i)
      if (base + i < n) s += in[base + i];
    uint32_t incl;
    uint32_t tot = block_incl_scan(s, sh, incl);
    if (threadIdx.x == 0) bsum[b] = tot;
  }
}

// Single block: exclusive scan of the block sums in place; writes the grand total to out[n].
__global__ __launch_bounds__(1024) void k_scan_blocks(uint32_t* __restrict__ bsum, uint64_t n_cap,
                                                      const uint32_t* n_dev,
                                                      uint32_t* __restrict__ out) {
  __shared__ uint32_t sh[1024 / 64];
  __shared__ uint32_t carry_sh;
  const uint64_t n = scan_n(n_cap, n_dev);
  const uint64_t nb = (n + kScanItems - 1) / kScanItems;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t carry = 0;
  for (uint64_t c = 0; c < nb; c += 1024) {
    uint64_t i = c + threadIdx.x;
    uint32_t v = i < nb ? bsum[i] : 0u;
    uint32_t x = v;
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
    if (i < nb) bsum[i] = carry + pre + x - v;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[n] = carry;
    carry_sh = carry;
  }
}

__global__ __launch_bounds__(kThreads) void k_scan_final(const uint32_t* __restrict__ in,
                                                         uint32_t* __restrict__ out, uint64_t n_cap,
                                                         const uint32_t* n_dev,
                                                         const uint32_t* __restrict__ bsum) {
  __shared__ uint32_t sh[kThreads / 64];
  const uint64_t n = scan_n(n_cap, n_dev);
  const uint64_t nb = (n + kScanItems - 1) / kScanItems;
  for (uint64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    uint64_t base = b * kScanItems + (uint64_t)threadIdx.x * kPer;
    uint32_t v[kPer];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      v[i] = base + i < n ? in[base + i] : 0u;
      s += v[i];
    }
    uint32_t incl;
    block_incl_scan(s, sh, incl);
    uint32_t run = bsum[b] + incl - s;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      if (base + i < n) out[base + i] = run;
      run += v[i];
    }
  }
}

}  // namespace

size_t scan_tmp_words(uint64_t n_cap) { return (n_cap + kScanItems - 1) / kScanItems + 1; }

hipError_t launch_scan_u32(const uint32_t* in, uint32_t* out, uint64_t n_cap, const uint32_t* n_dev,
                           uint32_t* tmp, hipStream_t st) {
  uint64_t nb = (n_cap + kScanItems - 1) / kScanItems;
  uint32_t grid = (uint32_t)(nb < kMaxGrid ? (nb > 0 ? nb : 1) : kMaxGrid);
  hipLaunchKernelGGL(k_scan_reduce, dim3(grid), dim3(kThreads), 0, st, in, n_cap, n_dev, tmp);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, tmp, n_cap, n_dev, out);
  hipLaunchKernelGGL(k_scan_final, dim3(grid), dim3(kThreads), 0, st, in, out, n_cap, n_dev, tmp);
  return hipGetLastError();
}

}  // namespace amn
