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

// Elements are uint32 (one array) or, for a pair of arrays scanned together, uint64 with
// the first array in the high and the second in the low half: the sums of both stay below
// 2^32 (a pass holds at most 2^28 samples), so the halves never carry into each other.
template <bool PAIR>
struct Elem {
  typedef uint32_t T;
  __device__ static T load(const uint32_t* a, const uint32_t*, uint64_t i) { return a[i]; }
  __device__ static void store(uint32_t* a, uint32_t*, uint64_t i, T v) { a[i] = v; }
};
template <>
struct Elem<true> {
  typedef uint64_t T;
  __device__ static T load(const uint32_t* a, const uint32_t* b, uint64_t i) {
    return ((uint64_t)a[i] << 32) | b[i];
  }
  __device__ static void store(uint32_t* a, uint32_t* b, uint64_t i, T v) {
    a[i] = (uint32_t)(v >> 32);
    b[i] = (uint32_t)v;
  }
};

// Inclusive scan of one value per thread across a 256-thread block; returns the block total.
template <typename T>
__device__ __forceinline__ T block_incl_scan(T v, T* sh_wave, T& incl) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T y = __shfl_up(v, off, 64);
    if (lane >= off) v += y;
  }
  if (lane == 63) sh_wave[wave] = v;
  __syncthreads();
  T pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    T s = sh_wave[w];
    if (w < wave) pre += s;
    tot += s;
  }
  __syncthreads();
  incl = v + pre;
  return tot;
}

template <bool PAIR>
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t* __restrict__ in,
                                                          const uint32_t* __restrict__ in2,
                                                          uint64_t n_cap, const uint32_t* n_dev,
                                                          typename Elem<PAIR>::T* __restrict__ bsum) {
  typedef typename Elem<PAIR>::T T;
  __shared__ T sh[kThreads / 64];
  const uint64_t n = scan_n(n_cap, n_dev);
  const uint64_t nb = (n + kScanItems - 1) / kScanItems;
  for (uint64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    uint64_t base = b * kScanItems + (uint64_t)threadIdx.x * kPer;
    T s = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i)
      if (base + i < n) s += Elem<PAIR>::load(in, in2, base + i);
    T incl;
    T tot = block_incl_scan<T>(s, sh, incl);
    if (threadIdx.x == 0) bsum[b] = tot;
  }
}

// Single block: exclusive scan of the block sums in place; writes the grand total to out[n].
template <bool PAIR>
__global__ __launch_bounds__(1024) void k_scan_blocks(typename Elem<PAIR>::T* __restrict__ bsum, uint64_t n_cap,
                                                      const uint32_t* n_dev, uint32_t* __restrict__ out,
                                                      uint32_t* __restrict__ out2) {
  typedef typename Elem<PAIR>::T T;
  __shared__ T sh[1024 / 64];
  const uint64_t n = scan_n(n_cap, n_dev);
  const uint64_t nb = (n + kScanItems - 1) / kScanItems;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T carry = 0;
  for (uint64_t c = 0; c < nb; c += 1024) {
    uint64_t i = c + threadIdx.x;
    T v = i < nb ? bsum[i] : (T)0;
    T x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      T y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    T pre = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      T s = sh[w];
      if (w < wave) pre += s;
      tot += s;
    }
    if (i < nb) bsum[i] = carry + pre + x - v;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) Elem<PAIR>::store(out, out2, n, carry);
}

template <bool PAIR>
__global__ __launch_bounds__(kThreads) void k_scan_final(const uint32_t* __restrict__ in,
                                                         const uint32_t* __restrict__ in2,
                                                         uint32_t* __restrict__ out, uint32_t* __restrict__ out2,
                                                         uint64_t n_cap, const uint32_t* n_dev,
                                                         const typename Elem<PAIR>::T* __restrict__ bsum) {
  typedef typename Elem<PAIR>::T T;
  __shared__ T sh[kThreads / 64];
  const uint64_t n = scan_n(n_cap, n_dev);
  const uint64_t nb = (n + kScanItems - 1) / kScanItems;
  for (uint64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    uint64_t base = b * kScanItems + (uint64_t)threadIdx.x * kPer;
    T v[kPer];
    T s = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      v[i] = base + i < n ? Elem<PAIR>::load(in, in2, base + i) : (T)0;
      s += v[i];
    }
    T incl;
    block_incl_scan<T>(s, sh, incl);
    T run = bsum[b] + incl - s;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      if (base + i < n) Elem<PAIR>::store(out, out2, base + i, run);
      run += v[i];
    }
  }
}

}  // namespace

// Block sums of up to 64 bits each, plus the total.
size_t scan_tmp_words(uint64_t n_cap) { return 2 * ((n_cap + kScanItems - 1) / kScanItems + 1); }

hipError_t launch_scan_u32(const uint32_t* in, uint32_t* out, uint64_t n_cap, const uint32_t* n_dev,
                           uint32_t* tmp, hipStream_t st) {
  uint64_t nb = (n_cap + kScanItems - 1) / kScanItems;
  uint32_t grid = (uint32_t)(nb < kMaxGrid ? (nb > 0 ? nb : 1) : kMaxGrid);
  hipLaunchKernelGGL(k_scan_reduce<false>, dim3(grid), dim3(kThreads), 0, st, in, nullptr, n_cap, n_dev, tmp);
  hipLaunchKernelGGL(k_scan_blocks<false>, dim3(1), dim3(1024), 0, st, tmp, n_cap, n_dev, out, nullptr);
  hipLaunchKernelGGL(k_scan_final<false>, dim3(grid), dim3(kThreads), 0, st, in, nullptr, out, nullptr, n_cap, n_dev,
                     tmp);
  return hipGetLastError();
}

hipError_t launch_scan_u32_pair(const uint32_t* in_a, uint32_t* out_a, const uint32_t* in_b, uint32_t* out_b,
                                uint64_t n_cap, uint32_t* tmp, hipStream_t st) {
  uint64_t nb = (n_cap + kScanItems - 1) / kScanItems;
  uint32_t grid = (uint32_t)(nb < kMaxGrid ? (nb > 0 ? nb : 1) : kMaxGrid);
  uint64_t* t64 = reinterpret_cast<uint64_t*>(tmp);
  hipLaunchKernelGGL(k_scan_reduce<true>, dim3(grid), dim3(kThreads), 0, st, in_a, in_b, n_cap, nullptr, t64);
  hipLaunchKernelGGL(k_scan_blocks<true>, dim3(1), dim3(1024), 0, st, t64, n_cap, nullptr, out_a, out_b);
  hipLaunchKernelGGL(k_scan_final<true>, dim3(grid), dim3(kThreads), 0, st, in_a, in_b, out_a, out_b, n_cap, nullptr,
                     t64);
  return hipGetLastError();
}

}  // namespace amn
