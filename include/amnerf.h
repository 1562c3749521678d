/*
 * amnerf.h -- C ABI of the adaptive multi-NeRF rendering library for AMD Instinct MI355X
 * (gfx950).
 *
 * The library renders a scene represented by many small same-shaped MLPs, one per leaf of
 * a KD tree of axis-aligned boxes built from a guidance density grid (Section 3.2 and 3.4
 * of the paper).  A render intersects every ray with the tree, places an equal number of
 * samples in every leaf interval the ray crosses (Section 3.5, Algorithm 1), sorts the
 * samples by leaf so that each leaf's MLP runs over one contiguous bucket (Section 3.5,
 * parallel scheduling), and composites the samples front to back with early ray
 * termination (Section 3.1, which defers to the NeRF volume-rendering quadrature, and
 * Section 4.1).
 *
 * Conventions shared by every call
 *   - Every call returns AMNERF_OK (0) or a negative status; amnerf_last_error() then gives
 *     a message (thread-local; valid until the next failing call on the same thread).
 *     No call aborts, throws or prints.
 *   - Pointers documented as "device" address memory on the context's GPU; pointers
 *     documented as "host" address CPU memory.  All such memory is owned by the caller;
 *     the library only reads or writes it during the call (for device pointers: until the
 *     work enqueued on the given stream has finished) and keeps no reference to it.
 *   - Handles (amnerf_ctx, amnerf_tree) are created and destroyed by the library.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls that take
 *     a stream only enqueue work on it and return without waiting, unless stated.
 *   - Results are deterministic: the same inputs give bit-identical outputs run to run
 *     (stable sorts, fixed-order reductions, no floating-point atomics).
 *   - The scene box is [0,1]^3.  Rays are float32 SoA: o[3][R] then d[3][R] (x row, then
 *     y, then z); d need not be exactly unit length.
 */
#ifndef AMNERF_H
#define AMNERF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------ */
#define AMNERF_OK 0
#define AMNERF_EINVAL (-1)    /* bad argument (null pointer, size or value out of range) */
#define AMNERF_ENOMEM (-2)    /* host allocation failed, or the workspace cap is too small */
#define AMNERF_EDEVICE (-3)   /* a HIP runtime call failed */
#define AMNERF_ECAPACITY (-4) /* a size exceeds a documented limit */
#define AMNERF_ESTATE (-5)    /* the call is not valid in the current state */

/* ---- arithmetic types of the per-leaf MLP -------------------------------------------- */
#define AMNERF_F32 0          /* float32 weights and activations, float32 accumulate */
#define AMNERF_BF16 1         /* bfloat16 weights and activations, float32 accumulate */
#define AMNERF_FP8 2          /* float8 e4m3 weights (OCP encoding: bias 7, 3 mantissa bits, max 448,
                                 no infinities) with a float32 scale per leaf and layer
                                 (max |W| / 448), widened to bfloat16 when a leaf's block is
                                 staged on chip; bfloat16 activations, float32 accumulate.
                                 Render only (no backward). */
#define AMNERF_FP8_ACT 3      /* float8 e4m3 weights AND activations on the float8 matrix cores
                                 (hidden 64, n_hidden 1 .. 4): the first layer in bfloat16
                                 (inputs and weights); the hidden and output layers take e4m3
                                 weight codes W / 2^e (e the smallest exponent with
                                 max |W| <= 448 * 2^e, per leaf and layer) and e4m3 activation
                                 codes a / 2^k (per leaf and hidden layer, see
                                 amnerf_mlp_pack_fp8_act; values above 256 * 2^k saturate);
                                 float32 accumulate, float32 biases (the output layer's carried
                                 as a bfloat16 high and low part, about 16 significant bits).
                                 Render only. */

/* ---- limits -------------------------------------------------------------------------- */
#define AMNERF_MAX_GRID 512   /* guidance grid side */
#define AMNERF_MAX_DEPTH 16
#define AMNERF_MAX_LEAVES 4096
#define AMNERF_MAX_SAMPLES 255 /* samples per ray (S_max) */

typedef struct amnerf_ctx amnerf_ctx;
typedef struct amnerf_tree amnerf_tree;
typedef struct amnerf_occ amnerf_occ;

/* Message of the last failing call on this thread ("" if none). */
const char* amnerf_last_error(void);

/* Library ABI version (major * 10000 + minor * 100 + patch). */
int amnerf_version(void);

/* ---- context ------------------------------------------------------------------------- */
/* Creates a context on HIP device `device`.  Device workspace is allocated lazily by the
 * calls that need it and grows on demand up to `workspace_cap` bytes (0 = no cap); a call
 * that would need more fails with AMNERF_ENOMEM and says how many bytes it needed.
 * Growing the workspace synchronises the device.  A context must not be used by two host
 * threads at once. */
int amnerf_ctx_create(int device, size_t workspace_cap, amnerf_ctx** out);

/* Synchronises the device, frees the workspace and the handle.  NULL is accepted. */
int amnerf_ctx_destroy(amnerf_ctx* ctx);

/* Render lanes of a render that runs in several chunks (see amnerf_render): the number of
 * chunks in flight at once, 1 .. AMNERF_MAX_RENDER_LANES (the default).  Each lane beyond
 * the first holds a chunk workspace of its own (about 16 GB when s_max is at most the leaf
 * count: 2^28 intervals and 2^28 samples), so fewer lanes hold less device memory; results
 * do not depend on it.
 * AMNERF_EINVAL outside the range. */
#define AMNERF_MAX_RENDER_LANES 4
int amnerf_ctx_set_render_lanes(amnerf_ctx* ctx, int n_lanes);

/* ---- tree (Section 3.4) -------------------------------------------------------------- */
#define AMNERF_SPLIT_MEDIAN 0  /* density-median subdivision (the method) */
#define AMNERF_SPLIT_MIDDLE 1  /* regular subdivision, for the ablation without it */

typedef struct {
  int32_t max_depth;   /* 0 .. AMNERF_MAX_DEPTH */
  int32_t max_leaves;  /* 1 .. AMNERF_MAX_LEAVES */
  int32_t split;       /* AMNERF_SPLIT_MEDIAN or AMNERF_SPLIT_MIDDLE */
} amnerf_tree_params;

typedef struct {
  int32_t n_nodes;     /* inner nodes + leaves = 2 * n_leaves - 1 */
  int32_t n_leaves;
  int32_t depth;       /* deepest leaf */
  int32_t grid_n;
} amnerf_tree_info;

/* Builds the density-aware KD tree from a guidance density grid (Section 3.4, BuildKDTree).
 *   grid_host: host float32[n^3], cell (i,j,k) at index i + n*(j + n*k), the density at the
 *              cell centre ((i+1/2)/n, (j+1/2)/n, (k+1/2)/n).  Negative values count as 0;
 *              NaN or infinity is AMNERF_EINVAL.  The grid is read during the call only.
 *   n:         a power of two, 1 .. AMNERF_MAX_GRID.
 * Densities are quantised to integers q = floor(g / max(g) * 2^24 + 1/2).  Starting from
 * the root box (all cells), the splittable leaf of largest integer mass (ties: smallest
 * node code) is split until there are max_leaves leaves or no leaf is splittable (a leaf
 * is splittable when its depth < max_depth and its longest side is >= 2 cells).  A split
 * cuts the longest side (ties: x, then y, then z) at the first cell plane whose lower side
 * holds at least half of the node's mass (the last plane if none; the middle plane for a
 * massless node).  Node codes are binary: root 1, children 2c (lower) and 2c+1 (upper).
 * Leaves are numbered 0..L-1 ("slots") in left-first depth-first order; a leaf's slot is
 * the node id samples are sorted by.  Runs synchronously on the host, then uploads the
 * node table to the context's device.
 * With split = AMNERF_SPLIT_MIDDLE the subdivision ignores the density (the regular-grid
 * subdivision that Section 4.2's ablation removes the adaptive split against): the
 * splittable leaf of smallest depth (ties: smallest node code) is split, at the middle
 * cell plane (lo + hi) / 2 of its longest side.  A power-of-two leaf count on a
 * power-of-two grid then gives equal boxes.  Masses are recorded as in the median mode. */
int amnerf_build_tree(amnerf_ctx* ctx, const float* grid_host, int32_t n,
                      const amnerf_tree_params* params, amnerf_tree** out);

int amnerf_tree_info_get(const amnerf_tree* tree, amnerf_tree_info* out);

/* Copies the tree into caller arrays, one row per node, sorted by node code.
 *   rows_host: host int32[n_nodes][12]: code, depth, lo[3], hi[3] (integer cell box
 *              [lo, hi)), split axis (-1 for a leaf), split plane (cell index, -1 for a
 *              leaf), leaf slot (-1 for an inner node), node slot (the node's rank among
              all nodes in left-first depth-first preorder: root 0, a node's lower child
              right after it, its upper child after the lower child's subtree).
 *   mass_host: host uint64[n_nodes] integer masses, or NULL. */
int amnerf_tree_export(const amnerf_tree* tree, int32_t* rows_host, uint64_t* mass_host);

/* The tree whose inner nodes are exactly the given node codes (binary: root 1, children 2c
 * (lower) and 2c + 1 (upper)), each split at the density median as above: the codes are
 * taken in increasing order, and each must name a leaf of the tree built so far whose
 * longest side is >= 2 cells (AMNERF_EINVAL otherwise).  The recursion of BuildKDTree
 * (Section 3.4) driven by a stopping rule made outside the library. */
int amnerf_build_tree_codes(amnerf_ctx* ctx, const float* grid_host, int32_t n, const uint32_t* codes_host,
                            int32_t n_codes, amnerf_tree** out);

/* Frees the tree (host and device copies).  NULL is accepted. */
int amnerf_tree_destroy(amnerf_tree* tree);

/* ---- occupancy grid for empty-space skipping (Section 4.1: the framework's density grid
 *      also serves empty-space detection) ---------------------------------------------- */
/* Builds a bit grid of G^3 cells, G = n / block, from the guidance grid: densities are
 * quantised as for the tree (q = floor(g / max(g) * 2^24 + 1/2)); a cell is occupied iff the
 * largest q over its block^3 guidance cells is >= floor(thresh * 2^24 + 1/2) and at least 1.
 *   grid_host: host float32[n^3] as for amnerf_build_tree (NaN/inf: AMNERF_EINVAL).
 *   n:         a power of two, 1 .. AMNERF_MAX_GRID;  block: a power of two dividing n.
 *   thresh:    in [0, 1].
 * A render given the grid drops every sample whose position falls in an empty cell
 * (cell index floor(x * G) per axis, clamped to [0, G-1]) before the sort: its density is
 * taken as 0, so the MLPs never see it.  This changes the result wherever the MLPs have
 * density in empty cells.  Synchronous on the host, then uploads the bits. */
int amnerf_build_occupancy(amnerf_ctx* ctx, const float* grid_host, int32_t n, int32_t block, float thresh,
                           amnerf_occ** out);

/* G, and the number of occupied cells. */
int amnerf_occupancy_info_get(const amnerf_occ* occ, int32_t* g_out, int64_t* n_occupied_out);

/* Copies the cells into host uint8[G^3] (0 or 1), cell (i,j,k) at i + G*(j + G*k). */
int amnerf_occupancy_export(const amnerf_occ* occ, uint8_t* cells_host);

/* Frees the grid (host and device copies).  NULL is accepted. */
int amnerf_occupancy_destroy(amnerf_occ* occ);

/* ---- per-leaf MLPs (Section 3.1, Section 3.2) ----------------------------------------- */
/* Every leaf holds the same MLP shape (the paper keeps one MLP size for all nodes):
 *   input 30 = positional encoding of p = 2x - 1 (x the sample position):
 *              [p, sin(2^k pi p), cos(2^k pi p) for k = 0..3] (27 values, each a 3-vector)
 *              followed by the ray direction d (3);
 *   n_hidden linear layers of width `hidden`, each followed by ReLU;
 *   an output linear layer of width 4: sigma = softplus(o0), rgb = logistic(o1..o3).
 * Master parameters of one leaf are float32, P floats: for each linear layer in order,
 * W[out][in] row-major then b[out].  All leaves are stored back to back: [L][P]. */
typedef struct {
  int32_t n_hidden;    /* 1 .. 8 */
  int32_t hidden;      /* 32 or 64 */
} amnerf_mlp_shape;

/* P, the float32 parameter count of one leaf, or -1 for an invalid shape. */
int64_t amnerf_mlp_param_count(const amnerf_mlp_shape* shape);

/* Bytes of the kernel-ready parameter block for `n_leaves` leaves in `dtype`. */
int amnerf_mlp_packed_bytes(const amnerf_mlp_shape* shape, int32_t dtype, int32_t n_leaves,
                            size_t* out);

/* Converts device master parameters float32[n_leaves][P] into the kernel-ready block
 * (matrix-core fragment order, weights in `dtype` rounded to nearest even, biases float32;
 * for AMNERF_BF16 it also holds the transposed weights the backward pass uses; for
 * AMNERF_FP8 each leaf and layer gets the scale max |W| / 448 (1 for an all-zero layer)
 * and the weights W / scale are rounded to the nearest e4m3 value, saturating at 448) in the
 * caller's device buffer `packed_dev` of amnerf_mlp_packed_bytes bytes.
 * An AMNERF_FP8 block is n_leaves equal leaf blocks, each: the float32 biases (the hidden
 * layers' n_hidden * hidden, then the output layer's 4, zero-padded to n_hidden * hidden + 16
 * floats and then to a multiple of 16 bytes), 16 float32 scale slots (slot l = layer l, the
 * rest unused), then the e4m3 codes of the weights, layer after layer, each layer's codes in
 * fragment order, in which every weight appears once and zero codes fill the padding (layer
 * 0's 30 inputs are padded to 32 and the output layer's 4 rows to 16, so the layers hold
 * 32 * hidden, hidden * hidden and 16 * hidden codes).  The pack launches on `stream`; errors come back as
 * AMNERF_EINVAL (bad shape, dtype, count or NULL pointer) or AMNERF_EDEVICE. */
int amnerf_mlp_pack(amnerf_ctx* ctx, const amnerf_mlp_shape* shape, int32_t dtype,
                    int32_t n_leaves, const float* master_dev, void* packed_dev, void* stream);

/* Packs device master parameters float32[n_leaves][P] as an AMNERF_FP8_ACT block (shape:
 * hidden 64, n_hidden 1 .. 4) with the activation exponents derived from calibration maxima:
 * k[leaf][j] = the smallest integer with 1.25 * act_max[leaf][j] <= 256 * 2^k (evaluated
 * exactly; 0 where the maximum is 0), so hidden layer j's ReLU outputs a are held as
 * 2^k * e4m3(min(a / 2^k, 256)) (256: the largest power of two e4m3 holds).  act_max_dev: device float32[n_leaves][n_hidden]
 * (amnerf_mlp_calibrate), or NULL for every k = 0 (what amnerf_mlp_pack does for this
 * dtype).  The block is n_leaves equal leaf blocks of amnerf_mlp_packed_bytes / n_leaves
 * bytes, each: 16 int32 (k[0..3], the weight exponents e of layers 1..4, then the E8M0 block
 * scale of each float8 layer's weight operand, 127 + e_l + k_(l-1) - k_l - 8 for a hidden
 * layer and 127 + e_n + k_(n-1) for the output layer, clamped to 0 .. 254, and 4 zeros);
 * 4096 bytes of layer 0's bfloat16 weights times 2^-(k_0 + 8) (64 rows x 32 inputs: the 30
 * features and two zero columns); 4096 bytes of e4m3 codes W / 2^e per hidden layer
 * 1 .. n_hidden - 1 and 2048 bytes for the output layer (32 rows, of which the first 4 are
 * the outputs and the rest zero), each in fragment order, in which every weight appears
 * once; n_hidden blocks of 256 bytes holding the biases of layers 0 .. n_hidden - 1 over
 * 2^(k_l + 8) as float32 (rows in accumulator order); 256 bytes holding the output layer's
 * biases as bfloat16 high and low parts (one 4-byte word per lane); zero
 * padding to a multiple of 256 bytes.  Launches on `stream`; AMNERF_EINVAL for a bad shape,
 * count or NULL pointer, AMNERF_EDEVICE. */
int amnerf_mlp_pack_fp8_act(amnerf_ctx* ctx, const amnerf_mlp_shape* shape, int32_t n_leaves,
                            const float* master_dev, const float* act_max_dev, void* packed_dev,
                            void* stream);

typedef struct {
  amnerf_mlp_shape shape;
  int32_t dtype;          /* AMNERF_F32, AMNERF_BF16, AMNERF_FP8 or AMNERF_FP8_ACT */
  int32_t n_leaves;       /* parameter sets: the tree's leaf count (its node count for a
                             render with hierarchical sampling) */
  const void* packed_dev; /* device block written by amnerf_mlp_pack with the same
                             shape, dtype and n_leaves */
} amnerf_mlp;

/* ---- rays ---------------------------------------------------------------------------- */
typedef struct {
  const float* o_dev;  /* device float32[3][n_rays] */
  const float* d_dev;  /* device float32[3][n_rays] */
  int64_t n_rays;      /* >= 0 */
} amnerf_rays;

/* ---- render (Section 3.5, Algorithm 1; Section 3.1) ----------------------------------- */
#define AMNERF_JITTER 1u        /* stratified jitter instead of interval-centred samples */
#define AMNERF_ERT_ROUNDS 2u    /* early termination in rounds (Section 4.1): the leaf MLPs
                                   evaluate each ray's samples 64 at a time, front to back,
                                   window k of every ray in round k, and a ray that terminated
                                   in an earlier window has no samples evaluated after it.  The
                                   outputs are bit-identical to a single-pass render (which
                                   evaluates every sample and composites up to the stop); only
                                   the evaluated sample count (stats n_samples) drops.  Needs
                                   about 24 more bytes of workspace per worst-case sample; with
                                   s_max <= 64 there is one window and the flag changes nothing.
                                   The stage timing then counts the rounds' selection and all
                                   but the last round's compositing as MLP time */

/* Learned proposal used by a render (see amnerf_propose below). */
typedef struct {
  int32_t dtype;          /* AMNERF_F32 or AMNERF_BF16 inference */
  const void* packed_dev; /* block written by amnerf_prop_pack with the same dtype */
  float mass_thresh;      /* keep slots holding this fraction of the predicted mass; fall
                             back to all plain slots when the predicted mass is below it */
  int32_t cap;            /* at most this many kept samples per ray, 1 .. s_max */
} amnerf_proposal;

typedef struct {
  int32_t s_max;          /* samples per ray budget, 1 .. AMNERF_MAX_SAMPLES */
  float ert_eps;          /* stop after the sample where transmittance drops below this;
                             0 disables early termination */
  uint32_t flags;         /* AMNERF_JITTER */
  uint64_t jitter_seed;   /* seed of the per-interval offsets when AMNERF_JITTER is set */
  const amnerf_proposal* proposal;  /* NULL: plain sampling; else proposal sampling (the
                             strata are then centred: AMNERF_JITTER is rejected) */
  float hcheck_footprint; /* 0: samples in leaf intervals only.  > 0: hierarchical sampling
                             (Section 3.5, HCheck): the descent stops at an inner node when
                             the ray enters it at t > size / hcheck_footprint (size = the
                             node's longest side in [0,1] units; the quotient rounded once
                             to float32, compared with the float32 entry parameter), and that
                             node's MLP takes the ray's whole segment inside it.  The MLP then
                             holds one parameter set per node, indexed by the node's preorder
                             slot (amnerf_tree_export column 11), so n_nodes <=
                             AMNERF_MAX_LEAVES (else AMNERF_ECAPACITY).  Samples per interval
                             stay those of the leaf intervals (s_max / m with m the ray's
                             leaf-interval count), so a node that stops the descent gets one
                             interval's share.  Not combined with a proposal (AMNERF_EINVAL).
                             The footprint is a sample spacing per unit distance, e.g.
                             kappa times the pixel angle */
  const amnerf_occ* occupancy; /* NULL, or empty-space skipping: samples in empty cells are
                             dropped before the sort (centred strata only: AMNERF_JITTER
                             is rejected; not combined with a proposal).  Kept samples keep
                             their positions and segment lengths, so the render is the
                             plain quadrature with the dropped samples' densities set to 0.
                             Not differentiated: amnerf_render_backward (and so
                             amnerf_train_step) after such a render returns AMNERF_ESTATE */
} amnerf_render_params;

typedef struct {
  float* rgb_dev;         /* device float32[n_rays][3] (background 0) */
  float* depth_dev;       /* device float32[n_rays]: sum of w_j t_j; may be NULL */
  float* opacity_dev;     /* device float32[n_rays]: sum of w_j; may be NULL */
  float* weights_dev;     /* device float32[n_placed_samples] per-sample weights in
                             ray-major sample order, or NULL; its size is only known after
                             the render (amnerf_render_stats_get), so a caller passes a
                             buffer of n_rays * s_max floats */
} amnerf_render_out;

/* Renders `rays`.  Per ray r: m intervals (t0_k, t1_k, leaf_k) of the leaves the ray
 * crosses inside [0,1]^3 for t >= 0, front to back; n = s_max / m samples per interval
 * (if m > s_max, one sample in each of the first s_max intervals); sample j of interval k
 * at t = t0_k + (j + u) * (t1_k - t0_k) / n with u = 1/2 (or a hash of (seed, r, k) when
 * jittered) and segment length delta = (t1_k - t0_k) / n.  Samples are then sorted by leaf
 * slot (stably, so each bucket keeps ray-major order), each leaf's MLP evaluates its
 * bucket, and per ray tau_j = sigma_j delta_j, T_j = exp(-sum_{i<j} tau_i),
 * w_j = T_j (1 - exp(-tau_j)), rgb = sum w_j c_j, depth = sum w_j t_j,
 * opacity = sum w_j, stopping after the first j with T_{j+1} < ert_eps.
 * Asynchronous on `stream`, except that with a proposal or an occupancy grid each pass
 * waits on the host for its plain interval count (to size the planned intervals).  Rays
 * are processed in chunks of at most 2^28 / s_max rays.
 * With several chunks (and weights_dev NULL), chunk k runs on lane k mod n, n the
 * context's render lanes (amnerf_ctx_set_render_lanes, 4 by default) or the chunk count if
 * smaller: lane 0 is `stream`, the others are streams owned by the context, each with a
 * chunk workspace of its own.  Those streams first wait for `stream`, and `stream` waits
 * for them before the call returns, so the call stays ordered on `stream` and its outputs
 * equal those of chunk-by-chunk calls.  With a proposal or an occupancy grid the host waits
 * for a chunk's count only after the next chunk's traversal is queued.  Calls on one
 * context must not overlap (the workspaces are reused). */
int amnerf_render(amnerf_ctx* ctx, const amnerf_tree* tree, const amnerf_mlp* mlp,
                  const amnerf_rays* rays, const amnerf_render_params* params,
                  amnerf_render_out* out, void* stream);

/* Allocation-free render, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): amnerf_render with
 * the same arguments and results (bit-identical), whose workspace is a static array of
 * amnerf_render_static_capacity() bytes (64 MiB) on each GPU, set up when the first context
 * on that GPU is created and held until the process ends; the call itself allocates nothing
 * and never waits on the host.  The whole call must fit one pass and that workspace: about
 * 20 + 40 * min(s_max, n_leaves) + 28 * s_max bytes per ray (7 500 rays at s_max 128 with
 * 512 leaves); larger calls fail with AMNERF_ECAPACITY and the bytes they need, before any
 * work is enqueued.  No proposal or occupancy grid (AMNERF_EINVAL: their buffers are sized
 * from a count measured on the host).  Every call on a GPU shares that GPU's array and
 * overwrites it, so calls that overlap on one GPU race: a caller with several streams or
 * contexts on one GPU must order them.  The render's intermediate arrays cannot be
 * inspected or differentiated afterwards (AMNERF_ESTATE); its statistics can be read. */
int amnerf_render_static(amnerf_ctx* ctx, const amnerf_tree* tree, const amnerf_mlp* mlp,
                         const amnerf_rays* rays, const amnerf_render_params* params,
                         amnerf_render_out* out, void* stream);

/* Bytes of the static workspace of amnerf_render_static on each GPU. */
size_t amnerf_render_static_capacity(void);

typedef struct {
  int64_t n_rays;
  int64_t n_intervals;    /* leaf intervals that received samples */
  int64_t n_samples;      /* samples evaluated by the MLPs (fewer than the samples placed
                             when AMNERF_ERT_ROUNDS skipped samples past termination) */
  int64_t n_tiles;        /* MLP work tiles of the last chunk */
  int64_t n_chunks;
  int64_t n_nonfinite;    /* rays whose rgb, depth or opacity is not finite */
  int64_t n_fallback;     /* rays rendered with every plain slot under a proposal */
  int64_t n_plain_samples;/* samples the plain sampler would have taken */
  int64_t n_unreached;    /* interval entries the traversal's emission pass did not reach and
                             filled with zero-length entries (0 unless its two passes disagree;
                             such entries add samples of zero weight to leaf 0's bucket) */
  int64_t n_composited;   /* samples composited before early termination (the stop sample
                             included); n_samples - n_composited were evaluated by the MLPs
                             but lie past the termination point */
  int64_t n_placed_samples; /* samples placed along the rays (the length of the per-sample
                             arrays: weights_dev, inspect's perm and sample_out); equals
                             n_samples unless AMNERF_ERT_ROUNDS skipped some */
} amnerf_render_stats;

/* Waits for the last render's stream and reports its totals. */
int amnerf_render_stats_get(amnerf_ctx* ctx, amnerf_render_stats* out);

/* Intermediate arrays of the last render (only if it ran as a single chunk), copied on
 * `stream` into caller device buffers (any pointer may be NULL to skip that array):
 *   ray_iv_off   uint32[n_rays+1]   first interval of each ray (ray-major), and the total
 *   ray_smp_off  uint32[n_rays+1]   first sample of each ray (ray-major), and the total
 *   iv_t0        float32[n_intervals]  interval start t
 *   iv_dt        float32[n_intervals]  interval length
 *   iv_slot      uint32[n_intervals]   leaf slot (the node id samples are sorted by); the
 *                                      node's preorder slot under hierarchical sampling
 *   iv_n         uint32[n_intervals]   samples in the interval
 *   bucket_off   uint32[n_sets+1]      first sorted sample of each bucket, and the total
 *                                      (n_sets = the MLP's parameter sets: leaves, or nodes
 *                                      under hierarchical sampling)
 *   perm         uint32[n_samples]     ray-major index of the sample at each sorted
 *                                      position (the stable sort of samples by slot)
 *   sample_out   float32[n_samples][4] MLP output pre-activations (sigma^, r^, g^, b^) in
 *                                      ray-major order: sigma = softplus(sigma^),
 *                                      rgb = logistic(r^, g^, b^)
 *   ray_used     uint32[n_rays]        samples of each ray composited before early
 *                                      termination (the stop sample included)
 *   slot_mask    uint64[n_rays][4]     proposal or empty-space renders only (else
 *                                      AMNERF_ESTATE): bit s % 64 of word s / 64 is set when
 *                                      plain slot s of the ray (its plain samples numbered
 *                                      front to back) is kept; all bits for a ray that fell
 *                                      back; unspecified for rays with no interval */
typedef struct {
  uint32_t* ray_iv_off;
  uint32_t* ray_smp_off;
  float* iv_t0;
  float* iv_dt;
  uint32_t* iv_slot;
  uint32_t* iv_n;
  uint32_t* bucket_off;
  uint32_t* perm;
  float* sample_out;
  uint32_t* ray_used;
  uint64_t* slot_mask;
} amnerf_inspect;

int amnerf_render_inspect(amnerf_ctx* ctx, const amnerf_inspect* out, void* stream);

/* ---- stage timing -------------------------------------------------------------------- */
#define AMNERF_STAGE_TRAVERSE 0   /* both traversal passes and the per-ray offset scans */
#define AMNERF_STAGE_PROPOSAL 1   /* proposal inference, selection and planned intervals */
#define AMNERF_STAGE_SORT 2       /* slot histogram, scans, stable scatter, bucket/tile offsets */
#define AMNERF_STAGE_EXPAND 3     /* sorted interval -> per-sample records */
#define AMNERF_STAGE_MLP 4        /* grouped per-leaf MLP */
#define AMNERF_STAGE_COMPOSITE 5  /* front-to-back compositing */
#define AMNERF_N_STAGES 6

/* Turns per-stage timing on or off.  When on, every render records HIP events between
 * its stages on the render stream (no host synchronisation). */
int amnerf_ctx_set_timing(amnerf_ctx* ctx, int enable);

/* Waits for the events recorded since the last collection and returns, per stage, the
 * summed GPU time in milliseconds (host double[AMNERF_N_STAGES]) and the number of
 * render passes (chunks) timed; then restarts the sums. */
int amnerf_timing_collect(amnerf_ctx* ctx, double* stage_ms_host, int64_t* n_passes);

/* Backward stages, timed the same way (events on the backward's stream) when timing is on. */
#define AMNERF_BWD_STAGE_COMPOSITE 0  /* loss gradient (training step) and compositing backward */
#define AMNERF_BWD_STAGE_MLP 1        /* per-leaf MLP backward: segment offsets and k_mlp_bwd */
#define AMNERF_BWD_STAGE_REDUCE 2     /* reduction of the per-segment weight gradients */
#define AMNERF_BWD_STAGE_ADAM 3       /* Adam and the repack of the bfloat16 weights (training step) */
#define AMNERF_N_BWD_STAGES 4

/* As amnerf_timing_collect, for the backward passes (amnerf_render_backward and the backward
 * of amnerf_train_step; a backward alone has no Adam stage, timed as 0): the summed GPU time
 * per backward stage (host double[AMNERF_N_BWD_STAGES]) and the number of passes timed. */
int amnerf_timing_collect_backward(amnerf_ctx* ctx, double* stage_ms_host, int64_t* n_passes);

/* ---- training (not in the paper, which distils its leaf MLPs offline: differentiable
 *      rendering so the leaf MLPs can be fitted to images) --------------------------------- */

/* Gradient of a scalar loss L with respect to every leaf parameter, given dL/d(outputs) of
 * the rays of the most recent amnerf_render on this context.  That render must have used
 * the same tree, MLP (dtype AMNERF_BF16 or AMNERF_F32), rays and params and run as a single
 * chunk (else AMNERF_ESTATE); its intermediate arrays are reused, and per-sample
 * activations are recomputed (none are kept from the forward pass).  Backward through the
 * quadrature: dL/dc_j = w_j g, dL/dtau_j = T_{j+1} c_j g - g . sum_{i>j} w_i c_i (likewise
 * for depth with t_j and for opacity with 1), zero after the early-termination sample,
 * which is the one the forward pass stopped at (recorded per ray by the render, never
 * decided again); then softplus' = logistic, logistic' = c (1 - c), and the chain rule
 * through the ReLU MLP (operands in the MLP's dtype, float32 accumulation).
 *   g_rgb_dev     device float32[n_rays][3]
 *   g_depth_dev   device float32[n_rays] or NULL (zero)
 *   g_opacity_dev device float32[n_rays] or NULL (zero)
 *   grad_dev      device float32[n_leaves][P], overwritten (master parameter layout)
 * Supported shapes: n_hidden 1 .. 4, hidden 32 or 64. */
int amnerf_render_backward(amnerf_ctx* ctx, const amnerf_tree* tree, const amnerf_mlp* mlp,
                           const amnerf_rays* rays, const float* g_rgb_dev,
                           const float* g_depth_dev, const float* g_opacity_dev,
                           float* grad_dev, void* stream);

/* Calibration for AMNERF_FP8_ACT (not in the paper): over every sample the most recent
 * amnerf_render on this context evaluated, the float32 forward of the master parameters
 * master_dev float32[n_leaves][P] (shape: hidden 64, n_hidden 1 .. 4); act_max_dev[leaf][j]
 * (device float32[n_leaves][n_hidden]) is raised to the largest ReLU output of hidden layer j
 * of that leaf.  The caller zeroes it before the first call; calls over several renders
 * accumulate.  That render must have used these rays and n_leaves parameter sets and run as
 * a single chunk, without AMNERF_ERT_ROUNDS and not in the static workspace (else
 * AMNERF_ESTATE).  Launches on `stream`. */
int amnerf_mlp_calibrate(amnerf_ctx* ctx, const amnerf_mlp_shape* shape, int32_t n_leaves,
                         const float* master_dev, const amnerf_rays* rays, float* act_max_dev,
                         void* stream);

/* Copies the per-sample gradient of the last amnerf_render_backward with respect to the
 * MLP output pre-activations, dL/d(sigma^, r^, g^, b^), into the caller's device
 * float32[n_samples][4] (ray-major sample order, as amnerf_render_inspect's sample_out), on
 * `stream`.  AMNERF_ESTATE if no backward pass of the last render is available. */
int amnerf_render_backward_inspect(amnerf_ctx* ctx, float* sample_grad_dev, void* stream);

typedef struct {
  float lr, beta1, beta2, eps;  /* Adam (Kingma & Ba) with bias correction */
  int32_t step;                 /* 1-based step number */
} amnerf_adam_params;

/* param -= lr * mhat / (sqrt(vhat) + eps) elementwise on n float32 values, updating the
 * moments m and v in place (all device arrays of n floats). */
int amnerf_adam_step(amnerf_ctx* ctx, int64_t n, float* param_dev, float* m_dev, float* v_dev,
                     const float* grad_dev, const amnerf_adam_params* p, void* stream);

typedef struct {
  amnerf_mlp_shape shape;
  int32_t n_leaves;
  float* master_dev;   /* float32[n_leaves][P] parameters, updated in place */
  float* grad_dev;     /* float32[n_leaves][P] gradient of the last step (written) */
  float* m_dev;        /* float32[n_leaves][P] Adam first moments */
  float* v_dev;        /* float32[n_leaves][P] Adam second moments */
  void* packed_dev;    /* AMNERF_BF16 packed block (amnerf_mlp_packed_bytes), re-packed */
} amnerf_mlp_train;

#define AMNERF_GRAD_ONLY 1u   /* compute loss and gradient, skip the Adam update */
#define AMNERF_TRAIN_F32 2u   /* float32 render and backward; packed_dev holds an AMNERF_F32 block */

typedef struct {
  amnerf_render_params render;
  amnerf_adam_params adam;
  uint32_t flags;           /* AMNERF_GRAD_ONLY, AMNERF_TRAIN_F32 */
} amnerf_train_params;

/* One training step on a batch of rays: bfloat16 render (float32 with AMNERF_TRAIN_F32), loss
 * L = mean over rays and channels of (rgb - target)^2, backward, Adam on the float32
 * masters, and re-packing of the bfloat16 (float32) block.  target_rgb_dev: device float32
 * [n_rays][3]; loss_dev: device float32[1] receives L. */
int amnerf_train_step(amnerf_ctx* ctx, const amnerf_tree* tree, amnerf_mlp_train* m,
                      const amnerf_rays* rays, const float* target_rgb_dev,
                      const amnerf_train_params* p, float* loss_dev, void* stream);

/* ---- distillation-driven subdivision (Section 3.4: BuildKDTree with the TestLeaf rule) ----
 * The recursion of BuildKDTree (node, then its lower subtree, then its upper subtree), each
 * split at the density median as amnerf_build_tree does, with the stopping rule of
 * Section 3.4: to test a node, the tree built so far with that node split is distilled for
 * n_max iterations (every leaf MLP starting from init_dev; step s = 1..n_max is
 * amnerf_train_step on batch (s - 1) mod n_batches with Adam step s, lr, beta1 0.9,
 * beta2 0.999, eps 1e-8, fresh moments), and its PSNR on the evaluation rays
 * (10 log10(1 / mean squared error over the colour channels) against eval_target_dev) is
 * compared with that of the tree built so far (distilled the same way).  The split is kept
 * iff PSNR_split - PSNR >= gain_thresh * PSNR (the paper's example threshold: 1 %);
 * otherwise the node is a leaf.  A node is tested only when its depth < max_depth, its
 * longest side >= 2 cells and the tree has fewer than max_leaves leaves.  Build-time only:
 * synchronous, allocates its own device buffers (4 float32 arrays of max_leaves * P, the
 * packed block, the evaluation colours) and frees them before returning. */
#define AMNERF_TESTLEAF_F32 1u   /* distil in float32 (render and backward); default bfloat16 */

typedef struct {
  amnerf_mlp_shape student;        /* node MLP shape (the paper: width 32, depth 4); its
                                      backward needs n_hidden 1 .. 4, hidden 32 or 64 */
  const float* init_dev;           /* device float32[P]: the initial parameters of every leaf */
  int32_t n_max;                   /* distillation steps per trial tree, >= 0 */
  float gain_thresh;               /* relative PSNR gain a split must reach */
  float lr;                        /* Adam step size */
  int32_t n_batches;               /* >= 1 when n_max > 0 */
  const amnerf_rays* batches;      /* host array [n_batches] of device ray sets (one pass each) */
  const float* const* targets;     /* host array [n_batches] of device float32[rays][3] colours */
  amnerf_rays eval;                /* held-out device rays, >= 1 */
  const double* eval_target_dev;   /* device float64[eval rays][3] colours */
  amnerf_render_params render;     /* s_max, ert_eps, flags; no proposal, occupancy or footprint */
  uint32_t flags;                  /* AMNERF_TESTLEAF_F32 */
} amnerf_testleaf_params;

typedef struct {
  uint32_t code;                   /* node tested */
  int32_t depth;
  int32_t leaves_of_trial;         /* leaves of the tree with the node split */
  int32_t kept;                    /* 1: split kept */
  double psnr_current;             /* PSNR of the tree built so far */
  double psnr_split;               /* PSNR of the tree with the node split */
} amnerf_testleaf_record;

/* Builds the tree; log_host[0 .. min(*n_log, log_cap)) receives one record per test, in the
 * order made (*n_log counts every test).  The tree is on ctx's device. */
int amnerf_build_tree_distilled(amnerf_ctx* ctx, const float* grid_host, int32_t n, int32_t max_depth,
                                int32_t max_leaves, const amnerf_testleaf_params* params, amnerf_tree** out,
                                amnerf_testleaf_record* log_host, int32_t log_cap, int32_t* n_log);

/* ---- learned proposal (not in the paper; it cites sample-predicting networks as prior
 *      art).  A 43 -> 64 -> 64 -> 32 ReLU MLP maps features of a (ray, leaf interval) --
 *      (o - 1/2)/2, d, sin/cos(2^k pi .) of both for k = 0, 1, k/S_max, the leaf box centre
 *      (2c - 1) and size, entry and exit points (2x - 1) -- to the optical thickness
 *      softplus(.) of 32 equal bins of the interval.  Compositing the bins front to back over
 *      the ray's intervals gives its predicted weight histogram; plain slot j of an interval
 *      with n slots receives the weight of the bins it overlaps.  A render keeps the fewest
 *      slots of largest predicted weight (ties: earlier slot) holding mass_thresh of the
 *      predicted mass M^ = 1 - T^_end, and skips the others (a subset of the plain
 *      quadrature); it falls back to every plain slot when M^ < mass_thresh or more than cap
 *      slots would be needed.  Parameters: float32, per layer W[out][in] then b[out]. ----- */
#define AMNERF_PROP_BINS 32

int64_t amnerf_prop_param_count(void);
int amnerf_prop_packed_bytes(int32_t dtype, size_t* out);
/* Converts the float32 parameters into the kernel-ready block (dtype AMNERF_F32 also holds
 * the transposed weights the training step uses). */
int amnerf_prop_pack(amnerf_ctx* ctx, int32_t dtype, const float* master_dev, void* packed_dev,
                     void* stream);

#define AMNERF_PROPOSE_INFER 0
#define AMNERF_PROPOSE_TRAIN 1

typedef struct {
  int32_t mode;             /* AMNERF_PROPOSE_INFER or AMNERF_PROPOSE_TRAIN */
  int32_t s_max;            /* plain sampling budget the proposal is used with */
  /* INFER: predicted thicknesses of every sampled interval of the rays, ray-major */
  int32_t infer_dtype;      /* AMNERF_F32 or AMNERF_BF16 */
  const void* infer_packed_dev;
  float* tau_dev;           /* device float32[tau_cap][32] */
  int64_t tau_cap;
  /* TRAIN: one Adam step on the loss mean over intervals and bins of
   * (1 - exp(-tau^_b) - alpha_b)^2, alpha_b = 1 - exp(-sum_j sigma_j |slot_j n bin_b|) from
   * a plain render of the rays with the scene's leaf MLPs (float32 forward and backward) */
  float* master_dev;        /* float32[P], updated */
  float* grad_dev;          /* float32[P], written */
  float* m_dev;             /* float32[P] Adam moments */
  float* v_dev;
  void* packed_dev;         /* AMNERF_F32 block of master_dev, re-packed after the step */
  amnerf_adam_params adam;
  float* loss_dev;          /* device float32[1] */
} amnerf_propose_params;

/* INFER or TRAIN as above.  scene_mlp renders the plain targets (TRAIN only, any dtype).
 * Asynchronous on the stream except that TRAIN and INFER wait once for the interval count. */
int amnerf_propose(amnerf_ctx* ctx, const amnerf_tree* tree, const amnerf_mlp* scene_mlp,
                   const amnerf_rays* rays, const amnerf_propose_params* p, int64_t* n_intervals,
                   void* stream);

/* ---- error report (Section 4 reports rendering quality as PSNR) ---------------------- */
/* Compares a device float32 result x_dev[n] with device float64 reference values
 * ref_dev[n] (for instance reference outputs uploaded to the device) over the elements
 * with sel_dev[i] != 0 (sel_dev may be NULL: all elements).  Writes to the host array
 * out[4]: max |x - ref| (infinite if a difference is NaN), the sum of (x - ref)^2, the
 * number of elements compared, and the sum of |x - ref|, accumulated in float64 on the
 * device in a fixed order (bit-identical from run to run).  PSNR with peak 1 is
 * 10 log10(out[2] / out[1]).  Synchronous: returns once out[] is written.  Uses 32 KiB of
 * device memory held by the context.  EINVAL for a null ctx/out or n < 0, or null arrays
 * with n > 0. */
int amnerf_error_stats(amnerf_ctx* ctx, const float* x_dev, const double* ref_dev, const uint8_t* sel_dev,
                       int64_t n, double out[4], void* stream);

#ifdef __cplusplus
}
#endif

#endif /* AMNERF_H */
