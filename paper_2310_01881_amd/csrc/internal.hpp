// internal.hpp -- declarations shared by the host orchestration and the HIP kernels of the
// adaptive multi-NeRF library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace amn {

// Device node table.  Children of an inner node are stored next to each other, so one
// index reaches both.  info >= 0: inner node, (left_index << 2) | split_axis;
// info < 0: leaf with slot -(info + 1).  plane is the split plane's coordinate in [0,1]
// (a multiple of 1/grid_n, exact in float32).
struct DevNode {
  float plane;
  int32_t info;
};

// Per node, for hierarchical sampling: the longest side of its box in [0,1] units and its
// rank among all nodes in left-first depth-first preorder (its MLP slot).
struct DevNodeAhs {
  float size;
  uint32_t slot;
};

// Per-chunk totals produced on the device (the host never waits for them mid-render).
struct ChunkCounts {
  uint32_t n_iv;        // intervals that carry samples (this chunk)
  uint32_t n_smp;       // samples (this chunk)
  uint32_t n_tiles;     // MLP work tiles (this chunk)
  uint32_t mat_n;       // entries of the sort's slot x segment count matrix (this chunk)
  uint64_t smp_global;  // ray-major sample index of this chunk's first sample
  uint64_t iv_global;   // intervals of the chunks before this one
  uint64_t nonfinite;   // rays with a non-finite output (accumulated over chunks)
  uint64_t fallback;    // rays that fell back to plain sampling under a proposal
  uint64_t plain_smp;   // samples of the plain sampler (before any proposal)
  uint64_t unreached;   // interval entries the emission walk did not reach (filled with
                        // zero-length slot-0 entries; 0 unless the two traversal passes disagree)
  uint64_t composited;  // samples composited before early termination (accumulated)
  uint64_t evaluated;   // samples the leaf MLPs evaluated (accumulated)
};

// State of a ray between the windows of a render in rounds: the compensated sum of tau so
// far, rgb, depth and opacity so far, and kDone once the ray's outputs are written.
struct CompCarry {
  float s_hi, s_lo, cr, cg, cb, dep, acc;
  uint32_t state;
};

constexpr int kMlpTileRows = 256;       // rows of one MLP work tile (4 waves x 64)
constexpr int kSegTiles = 16;           // tiles per backward work segment (one leaf)
constexpr int kScanItems = 2048;        // elements per scan block (256 threads x 8)

// ---- traversal (Algorithm 1: Traverse) -------------------------------------------------
// Pass 1: per ray, the number of leaf intervals that receive samples (min(m, s_max)) and
// the number of samples.  Pass 2: the intervals themselves, ray-major, at iv_off.
// `ahs` NULL: leaf intervals; else hierarchical sampling with the given footprint.
hipError_t launch_trav_count(const DevNode* nodes, const DevNodeAhs* ahs, float footprint, uint32_t n_nodes, int depth,
                             const float* o, const float* d, int64_t ray_stride, int64_t r0, uint32_t nr, int s_max,
                             uint32_t* cnt_iv, uint32_t* cnt_smp, hipStream_t st);
hipError_t launch_trav_emit(const DevNode* nodes, const DevNodeAhs* ahs, float footprint, uint32_t n_nodes, int depth,
                            const float* o, const float* d, int64_t ray_stride, int64_t r0, uint32_t nr,
                            const uint32_t* cnt_iv, const uint32_t* cnt_smp,
                            const uint32_t* iv_off, const uint32_t* smp_off, float* iv_t0,
                            float* iv_dt, uint32_t* iv_key, uint32_t* iv_ray, uint32_t* iv_base,
                            ChunkCounts* counts, hipStream_t st);

// Intervals of one chunk, ray-major: per ray the interval range [iv_off[r], iv_off[r+1]) and
// sample range [smp_off[r], smp_off[r+1]); per interval t0, length dt, key (slot | n << 16),
// chunk-local ray, and base = ray-major index of its first sample.
struct IvSet {
  const uint32_t* iv_off;
  const uint32_t* smp_off;
  const float* t0;
  const float* dt;
  const uint32_t* key;
  const uint32_t* ray;
  const uint32_t* base;
  const uint32_t* n_iv_dev;   // total intervals (device)
};

// Interval holding ray-major sample s among intervals [i0, i1) (largest i with base[i] <= s).
__device__ __forceinline__ uint32_t find_interval(const uint32_t* __restrict__ base, uint32_t i0,
                                                  uint32_t i1, uint32_t s) {
  uint32_t lo = i0, hi = i1;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (base[mid] <= s) lo = mid; else hi = mid;
  }
  return lo;
}

// ---- scans -----------------------------------------------------------------------------
// Exclusive prefix sum of n uint32 values (n given on the host, or read from n_dev when
// n_dev != nullptr, capped at n_cap); out[n] receives the total.  tmp needs
// scan_tmp_words(n_cap) words.
size_t scan_tmp_words(uint64_t n_cap);
hipError_t launch_scan_u32(const uint32_t* in, uint32_t* out, uint64_t n_cap,
                           const uint32_t* n_dev, uint32_t* tmp, hipStream_t st);
// Exclusive scans of two uint32 arrays of the same length n_cap at once (out_x[n_cap] = the
// totals), each total below 2^32; tmp as above, 8-byte aligned.
hipError_t launch_scan_u32_pair(const uint32_t* in_a, uint32_t* out_a, const uint32_t* in_b, uint32_t* out_b,
                                uint64_t n_cap, uint32_t* tmp, hipStream_t st);

// ---- sort by leaf slot (Section 3.5: sort, then infer per node) ------------------------
struct SortPlan {
  uint32_t seg;         // intervals per segment (multiple of 64)
  uint32_t nseg_max;    // segments for the worst-case interval count (the kernels use the
                        // actual count, ceil(n_iv / seg), as the matrix's row length)
  uint32_t key_bits;    // bits of the leaf slot
  uint32_t n_leaves;
};
SortPlan make_sort_plan(uint64_t n_iv_max, uint32_t n_leaves);
hipError_t launch_sort_hist(const SortPlan& p, const uint32_t* iv_key, const uint32_t* n_iv_dev,
                            uint32_t* mat, hipStream_t st);
hipError_t launch_sort_scatter(const SortPlan& p, const uint32_t* iv_key, const uint32_t* n_iv_dev,
                               const uint32_t* mat_scan, uint32_t* sidx, uint32_t* sn,
                               hipStream_t st);
// bucket_off[b] = first sorted sample of leaf b; tile_off[b] = first MLP tile of leaf b;
// also fills counts->n_smp and counts->n_tiles.
hipError_t launch_bucket_tiles(const SortPlan& p, const uint32_t* mat_scan, const uint32_t* ssb,
                               uint32_t* bucket_off, uint32_t* tile_off, ChunkCounts* counts,
                               hipStream_t st);
// One record per sorted sample: ray (chunk-local), t, ray-major sample index.
hipError_t launch_expand(const uint32_t* sidx, const uint32_t* ssb, const IvSet& iv,
                         int64_t r0, int jitter, uint64_t seed, uint32_t* srec_ray,
                         float* srec_t, uint32_t* perm, hipStream_t st);

// ---- grouped per-leaf MLP ---------------------------------------------------------------
struct MlpGeom {
  int n_hidden, hidden, dtype;
  size_t node_bytes;      // packed forward bytes of one leaf
  size_t bwd_node_bytes;  // packed backward bytes of one leaf (bfloat16 only)
};
bool mlp_geom(int n_hidden, int hidden, int dtype, MlpGeom* g);
// Error report: partial sums of kErrBlocks blocks (4 doubles each), then the totals
// {max |x - ref|, sum (x - ref)^2, count, sum |x - ref|} in out[4] (device).
constexpr int kErrBlocks = 1024;
hipError_t launch_error_stats(const float* x, const double* ref, const uint8_t* sel, int64_t n, double* part,
                              double* out, hipStream_t st);

// Blocks of `kern` (threads per block, dynamic LDS bytes) resident per compute unit on the
// current device: the register/wave limit from the runtime, the LDS limit from the
// device's LDS size per compute unit.
hipError_t resident_blocks(const void* kern, int threads, uint32_t lds, int* per_cu);
// Grid of a persistent launch of `kern` on the current device: compute units x resident
// blocks at `lds` bytes of dynamic LDS (allowing up to 160 KiB of it first).  Cached per
// (kernel, device, lds); safe to call from several host threads.
hipError_t persistent_grid(const void* kern, int threads, uint32_t lds, int* grid);

hipError_t launch_mlp_pack(const MlpGeom& g, int n_leaves, const float* master, void* packed,
                           hipStream_t st);
hipError_t launch_mlp(const MlpGeom& g, const void* packed, uint32_t n_leaves,
                      const uint32_t* bucket_off, const uint32_t* tile_off,
                      const ChunkCounts* counts, const uint32_t* srec_ray, const float* srec_t,
                      const uint32_t* perm, const float* o, const float* d, int64_t ray_stride,
                      int64_t r0, float* out, hipStream_t st);

// ---- float8 weights and activations on the float8 matrix cores (hidden width 64,
// n_hidden 1..4) ----------------------------------------------------------------------------
size_t mlp8_block_bytes(int n_hidden);
// act_max: device float32[n_leaves][n_hidden] calibration maxima, or null (every activation
// exponent 0).
hipError_t launch_mlp8_pack(int n_hidden, int n_leaves, const float* master, const float* act_max, void* packed,
                            hipStream_t st);
hipError_t launch_mlp8(int n_hidden, const void* packed, uint32_t n_leaves, const uint32_t* bucket_off,
                       const uint32_t* tile_off, const ChunkCounts* counts, const uint32_t* srec_ray,
                       const float* srec_t, const uint32_t* perm, const float* o, const float* d, int64_t stride,
                       int64_t r0, float* out, hipStream_t st);
// Raises act_max[leaf][j] to the largest ReLU output of hidden layer j over the sorted
// samples (float32 forward of the master parameters).
hipError_t launch_act_max(int n_hidden, const float* master, uint32_t n_leaves, const uint32_t* bucket_off,
                          const uint32_t* tile_off, const ChunkCounts* counts, const uint32_t* srec_ray,
                          const float* srec_t, const float* o, const float* d, int64_t stride, int64_t r0,
                          float* act_max, hipStream_t st);

// ---- compositing (Section 3.1 -> NeRF quadrature, early ray termination) ---------------
// ray_used[r] receives the number of samples of ray r that were composited (the stop
// sample included), and counts->composited their sum.
hipError_t launch_composite(uint32_t nr, const IvSet& iv, const float* smp_out, int64_t r0,
                            int jitter, uint64_t seed, float ert_eps, float* rgb, float* depth,
                            float* opac, float* weights, uint32_t* ray_used, ChunkCounts* counts,
                            hipStream_t st);
// One 64-sample window (`round`) of every ray still marching, continuing from `carry`;
// ray_used and the outputs are written as rays finish.  counts->composited is added by
// launch_sum_used once every round has run.
hipError_t launch_composite_round(uint32_t nr, const IvSet& iv, const float* smp_out, int64_t r0, int jitter,
                                  uint64_t seed, float ert_eps, float* rgb, float* depth, float* opac,
                                  float* weights, uint32_t* ray_used, ChunkCounts* counts, CompCarry* carry,
                                  uint32_t round, hipStream_t st);
hipError_t launch_sum_used(uint32_t nr, const uint32_t* ray_used, ChunkCounts* counts, hipStream_t st);

// ---- early termination in rounds (Section 4.1) -------------------------------------------
// Round k selects, in sorted order, the samples of window k (sample index 64k .. 64k + 63 of
// their ray) of the rays still marching (carry state not done; every ray in round 0):
// flags[p] = 1 for each, then (after an exclusive scan into pos) their sample records are
// compacted and each leaf's bucket and tile offsets recomputed over the compacted list
// (counts->n_tiles, counts->evaluated).
hipError_t launch_round_flags(const uint32_t* perm, const uint32_t* srec_ray, const uint32_t* smp_off,
                              const CompCarry* carry, const ChunkCounts* counts, uint32_t round, uint32_t ns_cap,
                              uint32_t* flags, hipStream_t st);
hipError_t launch_round_compact(const uint32_t* flags, const uint32_t* pos, const uint32_t* srec_ray,
                                const float* srec_t, const uint32_t* perm, const ChunkCounts* counts,
                                uint32_t ns_cap, uint32_t* c_ray, float* c_t, uint32_t* c_perm, hipStream_t st);
hipError_t launch_round_tiles(const uint32_t* bucket_off, const uint32_t* pos, uint32_t n_leaves,
                              uint32_t* c_bucket_off, uint32_t* c_tile_off, ChunkCounts* counts, hipStream_t st);

// ---- training ----------------------------------------------------------------------------
bool mlp_bwd_supported(int n_hidden, int hidden);
// Backward of the quadrature; ray_used[r] = samples of ray r the forward composited (the
// samples after them get zero gradient).
hipError_t launch_comp_bwd(uint32_t nr, const IvSet& iv, const float* smp_out, int64_t r0, int jitter,
                           uint64_t seed, const uint32_t* ray_used, const float* g_rgb, const float* g_depth,
                           const float* g_opac, float* gpre, hipStream_t st);
// seg_off: n_leaves + 2 words; the last is the bfloat16 backward's segment queue, which
// launch_seg_offsets resets to 0 and launch_mlp_bwd advances.
hipError_t launch_seg_offsets(const uint32_t* tile_off, uint32_t n_leaves, uint32_t* seg_off, hipStream_t st);
hipError_t launch_mlp_bwd(const MlpGeom& g, const void* packed, uint32_t n_leaves, const uint32_t* bucket_off,
                          const uint32_t* tile_off, uint32_t* seg_off, const uint32_t* srec_ray,
                          const float* srec_t, const uint32_t* perm, const float* o, const float* d,
                          int64_t ray_stride, int64_t r0, const float* gpre, float* part, hipStream_t st);
hipError_t launch_grad_reduce(const float* part, const uint32_t* seg_off, uint32_t n_leaves, uint32_t P,
                              float* grad, hipStream_t st);
size_t loss_partial_words(uint64_t R);
hipError_t launch_loss_grad(uint32_t R, const float* rgb, const float* target, float* g_rgb, float* partial,
                            float* loss, hipStream_t st);
hipError_t launch_adam(int64_t n, float* p, float* m, float* v, const float* g, float lr, float b1, float b2,
                       float eps, int step, hipStream_t st);

// ---- learned proposal ----------------------------------------------------------------------
int prop_param_count();
size_t prop_packed_bytes(int dtype);
uint32_t prop_train_blocks();
hipError_t launch_prop_pack(int dtype, const float* master, void* packed, hipStream_t st);
hipError_t launch_prop_fwd(int dtype, const void* packed, const IvSet& iv, const float* o, const float* d,
                           int64_t stride, int64_t r0, const float* leafbox, int s_max, uint32_t n_iv_max,
                           bool cum, float* tau, float* tot, hipStream_t st);
hipError_t launch_prop_select(uint32_t nr, const IvSet& iv, const float* wts, const float* tot, float mass_thresh,
                              int cap, int s_max,
                              uint32_t* runs, uint32_t* nsel, uint64_t* mask, float* mass, ChunkCounts* counts,
                              hipStream_t st);
// Empty-space skipping: per ray, the mask of plain slots whose centred sample lies in an
// occupied cell of the G^3 bit grid, with its run and kept-slot counts (emitted by
// launch_prop_emit).
hipError_t launch_occ_select(uint32_t nr, const IvSet& iv, const float* o, const float* d, int64_t stride, int64_t r0,
                             const uint32_t* bits, int g, uint32_t* runs, uint32_t* nsel, uint64_t* mask,
                             hipStream_t st);
hipError_t launch_prop_emit(uint32_t nr, const IvSet& iv, const uint64_t* mask, const uint32_t* pv_off,
                            const uint32_t* ps_off, float* pt0, float* pdt, uint32_t* pkey, uint32_t* pray,
                            uint32_t* pbase, hipStream_t st);
hipError_t launch_prop_targets(const IvSet& iv, const float* smp_out, float* alpha, hipStream_t st);
hipError_t launch_prop_train(const void* packed, const IvSet& iv, const float* o, const float* d, int64_t stride,
                             int64_t r0, const float* leafbox, int s_max, const float* alpha, float* part,
                             float* loss_part, float* grad, float* loss, hipStream_t st);

// ---- small helpers ----------------------------------------------------------------------
hipError_t launch_counts_merge(ChunkCounts* a, const ChunkCounts* b, hipStream_t st);
hipError_t launch_counts_reset(ChunkCounts* counts, hipStream_t st);
hipError_t launch_chunk_begin(ChunkCounts* counts, const uint32_t* iv_total, uint32_t seg, uint32_t n_leaves,
                              hipStream_t st);
hipError_t launch_chunk_finish(ChunkCounts* counts, const uint32_t* smp_off_total,
                               const uint32_t* iv_off_total, const uint32_t* plain_smp_total, int rounds,
                               hipStream_t st);

}  // namespace amn
