// ert.hip -- early ray termination in rounds (Section 4.1: the framework stops marching a
// ray once its transmittance is spent).  A render in rounds evaluates, in round k, only the
// samples of window k (sample index 64k .. 64k + 63 of their ray) of the rays that have not
// terminated yet, so the leaf MLPs never see samples that lie past a termination decided in
// an earlier window.
//
// The samples are already sorted by leaf; a round keeps that order: flags over the sorted
// positions, an exclusive scan, a compaction of the sample records, and each leaf's bucket
// and tile offsets read off the scan at the leaf's first sorted position.
#include "internal.hpp"
#include "devcommon.hpp"

namespace amn {
namespace {

constexpr int kThreads = 256;
constexpr uint32_t kDoneBit = 0x80000000u;

__global__ __launch_bounds__(kThreads) void k_round_flags(const uint32_t* __restrict__ perm,
                                                          const uint32_t* __restrict__ srec_ray,
                                                          const uint32_t* __restrict__ smp_off,
                                                          const CompCarry* __restrict__ carry,
                                                          const ChunkCounts* __restrict__ counts, uint32_t round,
                                                          uint32_t* __restrict__ flags) {
  const uint32_t n = counts->n_smp;
  for (uint32_t p = blockIdx.x * kThreads + threadIdx.x; p < n; p += gridDim.x * kThreads) {
    const uint32_t ray = srec_ray[p];
    const uint32_t j = perm[p] - smp_off[ray];   // the sample's index along its ray
    bool keep = (j >> 6) == round;
    if (keep && round > 0) keep = (carry[ray].state & kDoneBit) == 0u;
    flags[p] = keep ? 1u : 0u;
  }
}

__global__ __launch_bounds__(kThreads) void k_round_compact(const uint32_t* __restrict__ flags,
                                                            const uint32_t* __restrict__ pos,
                                                            const uint32_t* __restrict__ srec_ray,
                                                            const float* __restrict__ srec_t,
                                                            const uint32_t* __restrict__ perm,
                                                            const ChunkCounts* __restrict__ counts,
                                                            uint32_t* __restrict__ c_ray, float* __restrict__ c_t,
                                                            uint32_t* __restrict__ c_perm) {
  const uint32_t n = counts->n_smp;
  for (uint32_t p = blockIdx.x * kThreads + threadIdx.x; p < n; p += gridDim.x * kThreads) {
    if (!flags[p]) continue;
    const uint32_t q = pos[p];
    c_ray[q] = srec_ray[p];
    c_t[q] = srec_t[p];
    c_perm[q] = perm[p];
  }
}

// One block: c_bucket_off[b] = pos[bucket_off[b]], and the tiles of each compacted bucket
// (an exclusive scan of ceil(count / tile rows) over the leaves).
__global__ __launch_bounds__(1024) void k_round_tiles(const uint32_t* __restrict__ bucket_off,
                                                      const uint32_t* __restrict__ pos, uint32_t n_leaves,
                                                      uint32_t* __restrict__ c_bucket_off,
                                                      uint32_t* __restrict__ c_tile_off,
                                                      ChunkCounts* __restrict__ counts) {
  __shared__ uint32_t sh[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t carry = 0;
  for (uint32_t c = 0; c < n_leaves; c += 1024) {
    const uint32_t b = c + threadIdx.x;
    uint32_t nt = 0;
    if (b < n_leaves) {
      const uint32_t lo = pos[bucket_off[b]], hi = pos[bucket_off[b + 1]];
      c_bucket_off[b] = lo;
      nt = (hi - lo + kMlpTileRows - 1) / kMlpTileRows;
    }
    uint32_t x = nt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      const uint32_t s = sh[w];
      if (w < wave) pre += s;
      tot += s;
    }
    if (b < n_leaves) c_tile_off[b] = carry + pre + x - nt;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const uint32_t total = pos[bucket_off[n_leaves]];
    c_bucket_off[n_leaves] = total;
    c_tile_off[n_leaves] = carry;
    counts->n_tiles = carry;
    counts->evaluated += total;
  }
}

uint32_t grid_for(uint32_t ns_cap) {
  const uint32_t g = (ns_cap + kThreads * 8 - 1) / (kThreads * 8);
  return g == 0 ? 1u : (g > 8192u ? 8192u : g);
}

}  // namespace

hipError_t launch_round_flags(const uint32_t* perm, const uint32_t* srec_ray, const uint32_t* smp_off,
                              const CompCarry* carry, const ChunkCounts* counts, uint32_t round, uint32_t ns_cap,
                              uint32_t* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_round_flags, dim3(grid_for(ns_cap)), dim3(kThreads), 0, st, perm, srec_ray, smp_off, carry,
                     counts, round, flags);
  return hipGetLastError();
}

hipError_t launch_round_compact(const uint32_t* flags, const uint32_t* pos, const uint32_t* srec_ray,
                                const float* srec_t, const uint32_t* perm, const ChunkCounts* counts,
                                uint32_t ns_cap, uint32_t* c_ray, float* c_t, uint32_t* c_perm, hipStream_t st) {
  hipLaunchKernelGGL(k_round_compact, dim3(grid_for(ns_cap)), dim3(kThreads), 0, st, flags, pos, srec_ray, srec_t,
                     perm, counts, c_ray, c_t, c_perm);
  return hipGetLastError();
}

hipError_t launch_round_tiles(const uint32_t* bucket_off, const uint32_t* pos, uint32_t n_leaves,
                              uint32_t* c_bucket_off, uint32_t* c_tile_off, ChunkCounts* counts, hipStream_t st) {
  hipLaunchKernelGGL(k_round_tiles, dim3(1), dim3(1024), 0, st, bucket_off, pos, n_leaves, c_bucket_off, c_tile_off,
                     counts);
  return hipGetLastError();
}

}  // namespace amn
