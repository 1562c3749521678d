// sort.hip -- stable sort of samples by leaf slot and bucket compaction (Section 3.5:
// samples are sorted with their ray id and node id, then inferred per node).
//
// All samples of one leaf interval share its slot and are contiguous in ray-major order,
// so the stable sort of samples equals the stable sort of intervals, each expanded into
// its samples in place.  The sort therefore runs on intervals (about S_max / n fewer keys
// than samples):
//   hist    one wave per segment of `seg` consecutive intervals: LDS histogram of slots,
//           written column-wise into a [slot][segment] count matrix (row length = the
//           chunk's actual segment count, so the matrix and its scan scale with the
//           intervals present, and there is a segment per wave across the machine);
//   scan    exclusive scan of that matrix in slot-major order = the first sorted position
//           of (slot, segment);
//   scatter one wave per segment again, 64 intervals at a time: lanes holding the same
//           slot find each other with one ballot per key bit; rank = earlier lanes of the
//           same slot, base = a per-slot running counter in LDS -> stable positions;
//   expand  each sorted interval writes its samples' records at its sorted sample base.
#include "internal.hpp"
#include "devcommon.hpp"

namespace amn {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr uint32_t kMaxGrid = 4096;

__device__ __forceinline__ uint64_t lanemask_lt(int lane) { return (1ull << lane) - 1ull; }

__global__ __launch_bounds__(kThreads) void k_sort_hist(const uint32_t* __restrict__ iv_key,
                                                        const uint32_t* __restrict__ n_iv_dev,
                                                        uint32_t seg, uint32_t n_leaves,
                                                        uint32_t* __restrict__ mat) {
  extern __shared__ uint32_t sh[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t* hist = sh + wave * n_leaves;
  const uint32_t n_iv = *n_iv_dev;
  const uint32_t nseg = (n_iv + seg - 1) / seg;
  for (uint32_t s = blockIdx.x * kWaves + wave; s < nseg; s += gridDim.x * kWaves) {
    for (uint32_t b = lane; b < n_leaves; b += 64) hist[b] = 0u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint64_t begin = (uint64_t)s * seg;
    uint64_t end = begin + seg < n_iv ? begin + seg : n_iv;
    for (uint64_t i = begin + lane; i < end; i += 64) atomicAdd(&hist[key_slot(iv_key[i])], 1u);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (uint32_t b = lane; b < n_leaves; b += 64) mat[(uint64_t)b * nseg + s] = hist[b];
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ __launch_bounds__(kThreads) void k_sort_scatter(const uint32_t* __restrict__ iv_key,
                                                           const uint32_t* __restrict__ n_iv_dev,
                                                           uint32_t seg, uint32_t n_leaves,
                                                           uint32_t key_bits,
                                                           const uint32_t* __restrict__ mat_scan,
                                                           uint32_t* __restrict__ sidx,
                                                           uint32_t* __restrict__ sn) {
  extern __shared__ uint32_t sh[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t* base = sh + wave * n_leaves;
  const uint32_t n_iv = *n_iv_dev;
  const uint32_t nseg = (n_iv + seg - 1) / seg;
  for (uint32_t s = blockIdx.x * kWaves + wave; s < nseg; s += gridDim.x * kWaves) {
    for (uint32_t b = lane; b < n_leaves; b += 64) base[b] = mat_scan[(uint64_t)b * nseg + s];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint64_t begin = (uint64_t)s * seg;
    uint64_t end = begin + seg < n_iv ? begin + seg : n_iv;
    for (uint64_t c = begin; c < end; c += 64) {
      uint64_t i = c + lane;
      bool valid = i < end;
      uint32_t key = valid ? iv_key[i] : 0u;
      uint32_t slot = key_slot(key);
      // lanes with the same slot: intersect one ballot per key bit
      uint64_t peers = __ballot(valid);
      for (uint32_t bit = 0; bit < key_bits; ++bit) {
        uint64_t ones = __ballot(valid && ((slot >> bit) & 1u));
        peers &= ((slot >> bit) & 1u) ? ones : ~ones;
      }
      uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt(lane));
      uint32_t pos = 0;
      if (valid) pos = base[slot] + rank;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      // the highest lane of each group advances that slot's counter
      bool last = valid && (peers >> lane) == 1ull;
      if (last) base[slot] = pos + 1;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (valid) {
        sidx[pos] = (uint32_t)i;
        sn[pos] = key_n(key);
      }
    }
  }
}

// One block: leaf bucket offsets in sorted samples and MLP tile offsets.
__global__ __launch_bounds__(1024) void k_bucket_tiles(const uint32_t* __restrict__ mat_scan,
                                                       uint32_t seg, uint32_t n_leaves,
                                                       const uint32_t* __restrict__ ssb,
                                                       uint32_t* __restrict__ bucket_off,
                                                       uint32_t* __restrict__ tile_off,
                                                       ChunkCounts* counts) {
  __shared__ uint32_t sh[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t n_iv = counts->n_iv;
  const uint32_t nseg = (n_iv + seg - 1) / seg;
  const uint32_t n_smp = ssb[n_iv];
  uint32_t carry = 0;
  for (uint32_t c = 0; c < n_leaves; c += 1024) {
    uint32_t b = c + threadIdx.x;
    uint32_t lo = 0, hi = 0;
    if (b < n_leaves) {
      lo = ssb[mat_scan[(uint64_t)b * nseg]];
      hi = b + 1 < n_leaves ? ssb[mat_scan[(uint64_t)(b + 1) * nseg]] : n_smp;
      bucket_off[b] = lo;
    }
    uint32_t nt = (hi - lo + kMlpTileRows - 1) / kMlpTileRows;
    uint32_t x = nt;
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
    if (b < n_leaves) tile_off[b] = carry + pre + x - nt;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    bucket_off[n_leaves] = n_smp;
    tile_off[n_leaves] = carry;
    counts->n_smp = n_smp;
    counts->n_tiles = carry;
  }
}

// One block per 256 consecutive sorted intervals: their records go to LDS, then each wave
// writes windows of 64 consecutive sorted samples (coalesced).  A sample's interval is
// found without a search: the intervals starting inside the window mark their first
// lane in a per-wave LDS row, and a prefix maximum over the row (seeded with the last
// interval of the previous window) gives every lane the latest interval started at or
// before it.
__global__ __launch_bounds__(kThreads) void k_expand(
    const uint32_t* __restrict__ sidx, const uint32_t* __restrict__ ssb, IvSet iv, int64_t r0,
    int jitter, uint64_t seed, uint32_t* __restrict__ srec_ray, float* __restrict__ srec_t,
    uint32_t* __restrict__ perm) {
  __shared__ uint32_t sh_base[kThreads + 1];
  __shared__ uint32_t sh_ray[kThreads], sh_rm[kThreads];
  __shared__ float sh_t0[kThreads], sh_delta[kThreads], sh_u[kThreads];
  __shared__ int sh_mark[kWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t n_iv = *iv.n_iv_dev;
  const uint32_t n_groups = (n_iv + kThreads - 1) / kThreads;
  for (uint32_t grp = blockIdx.x; grp < n_groups; grp += gridDim.x) {
    const uint32_t p0 = grp * kThreads;
    const uint32_t cnt = n_iv - p0 < (uint32_t)kThreads ? n_iv - p0 : (uint32_t)kThreads;
    const uint32_t p = p0 + threadIdx.x;
    if (threadIdx.x < cnt) {
      uint32_t i = sidx[p];
      uint32_t ray = iv.ray[i];
      uint32_t n = key_n(iv.key[i]);
      uint32_t k = i - iv.iv_off[ray];
      sh_base[threadIdx.x] = ssb[p];
      sh_ray[threadIdx.x] = ray;
      sh_rm[threadIdx.x] = iv.base[i];   // ray-major index of the first sample
      sh_t0[threadIdx.x] = iv.t0[i];
      sh_delta[threadIdx.x] = iv.dt[i] / (float)n;
      sh_u[threadIdx.x] = stratum_u(jitter, seed, (uint64_t)(r0 + ray), k);
    }
    if (threadIdx.x == 0) sh_base[cnt] = ssb[p0 + cnt];
    __syncthreads();
    const uint32_t q0 = sh_base[0], q1 = sh_base[cnt];
    // this lane's view of the staged intervals' first samples (intervals lane + 64 c)
    uint32_t st[kWaves];
#pragma unroll
    for (int c = 0; c < kWaves; ++c) {
      const uint32_t a = (uint32_t)lane + 64u * c;
      st[c] = a < cnt ? sh_base[a] : 0xFFFFFFFFu;
    }
    // windows of 64 samples: wave w takes windows w, w + 4, ...; the interval covering a
    // window's first sample is the last one starting at or before it
    for (uint32_t qw = q0 + 64u * wave; qw < q1; qw += 64u * kWaves) {
      sh_mark[wave][lane] = -1;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      int before = 0;   // intervals starting at or before qw (at least interval 0 does)
#pragma unroll
      for (int c = 0; c < kWaves; ++c) {
        const uint32_t a = (uint32_t)lane + 64u * c;
        if (st[c] != 0xFFFFFFFFu && st[c] >= qw && st[c] < qw + 64u) sh_mark[wave][st[c] - qw] = (int)a;
        if (st[c] <= qw) before = max(before, (int)a);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const int first = wave_max_incl(before);                       // lane 63 holds the maximum
      const int seed_iv = __builtin_amdgcn_readlane(first, 63);
      const int lo = max(wave_max_incl(sh_mark[wave][lane]), seed_iv);
      const uint32_t q = qw + (uint32_t)lane;
      if (q < q1) {
        const uint32_t j = q - sh_base[lo];
        srec_ray[q] = sh_ray[lo];
        srec_t[q] = sample_t(sh_t0[lo], sh_delta[lo], j, sh_u[lo]);
        perm[q] = sh_rm[lo] + j;
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
  }
}

}  // namespace

SortPlan make_sort_plan(uint64_t n_iv_max, uint32_t n_leaves) {
  SortPlan p;
  p.n_leaves = n_leaves;
  uint32_t bits = 0;
  while ((1u << bits) < n_leaves) ++bits;
  p.key_bits = bits;
  // a segment per wave; at least as many intervals per segment as slots, so the count
  // matrix (n_leaves x segments) has no more entries than there are intervals
  uint64_t seg = ((uint64_t)n_leaves + 63) / 64 * 64;
  if (seg < 512) seg = 512;
  p.seg = (uint32_t)seg;
  p.nseg_max = (uint32_t)((n_iv_max + seg - 1) / seg);
  if (p.nseg_max == 0) p.nseg_max = 1;
  return p;
}

hipError_t launch_sort_hist(const SortPlan& p, const uint32_t* iv_key, const uint32_t* n_iv_dev,
                            uint32_t* mat, hipStream_t st) {
  uint32_t grid = (p.nseg_max + kWaves - 1) / kWaves;
  if (grid > kMaxGrid) grid = kMaxGrid;
  size_t lds = sizeof(uint32_t) * kWaves * p.n_leaves;
  hipLaunchKernelGGL(k_sort_hist, dim3(grid), dim3(kThreads), lds, st, iv_key, n_iv_dev, p.seg, p.n_leaves,
                     mat);
  return hipGetLastError();
}

hipError_t launch_sort_scatter(const SortPlan& p, const uint32_t* iv_key, const uint32_t* n_iv_dev,
                               const uint32_t* mat_scan, uint32_t* sidx, uint32_t* sn,
                               hipStream_t st) {
  uint32_t grid = (p.nseg_max + kWaves - 1) / kWaves;
  if (grid > kMaxGrid) grid = kMaxGrid;
  size_t lds = sizeof(uint32_t) * kWaves * p.n_leaves;
  hipLaunchKernelGGL(k_sort_scatter, dim3(grid), dim3(kThreads), lds, st, iv_key, n_iv_dev, p.seg, p.n_leaves,
                     p.key_bits, mat_scan, sidx, sn);
  return hipGetLastError();
}

hipError_t launch_bucket_tiles(const SortPlan& p, const uint32_t* mat_scan, const uint32_t* ssb,
                               uint32_t* bucket_off, uint32_t* tile_off, ChunkCounts* counts,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_bucket_tiles, dim3(1), dim3(1024), 0, st, mat_scan, p.seg, p.n_leaves,
                     ssb, bucket_off, tile_off, counts);
  return hipGetLastError();
}

hipError_t launch_expand(const uint32_t* sidx, const uint32_t* ssb, const IvSet& iv, int64_t r0,
                         int jitter, uint64_t seed, uint32_t* srec_ray, float* srec_t, uint32_t* perm,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_expand, dim3(4096), dim3(kThreads), 0, st, sidx, ssb, iv, r0, jitter, seed,
                     srec_ray, srec_t, perm);
  return hipGetLastError();
}

}  // namespace amn
