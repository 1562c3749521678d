// amnerf.cpp -- host side of the C ABI declared in include/amnerf.h: argument checks,
// the integer KD-tree builder, the device workspace and the per-chunk launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <queue>
#include <string>
#include <vector>

#include "../../include/amnerf.h"
#include "internal.hpp"

using namespace amn;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(AMNERF_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr uint64_t kChunkSamples = 1ull << 28;   // worst-case samples of one render pass
// lanes of a render that runs in several chunks: chunk k runs on lane k mod kLanes, lane 0
// being the caller's stream
constexpr int kLanes = AMNERF_MAX_RENDER_LANES;

}  // namespace

// ---------------------------------------------------------------------------------------
// static workspace of the allocation-free render (amnerf_render_static)
// ---------------------------------------------------------------------------------------
// One array per GPU the library runs on, held until the process ends.  In host code the
// array's name is only a stand-in: its device address on each device is taken once, at
// context creation with that device current, and only that address is ever used.
static constexpr size_t kStaticBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current); once per device.
int static_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return AMNERF_OK;   // static renders unavailable there
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (g_static_ptr[device]) return AMNERF_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(AMNERF_EDEVICE, "static workspace address on device %d: %s", device, hipGetErrorString(e));
  g_static_ptr[device] = ptr;
  return AMNERF_OK;
}

void* static_workspace(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_static_mu);
  return g_static_ptr[device];
}
}  // namespace

// ---------------------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------------------
namespace {
constexpr int kStages = AMNERF_N_STAGES;
constexpr int kRing = 64;
struct EvSet {
  hipEvent_t ev[kStages + 1] = {};
  bool pending = false;
};
constexpr int kBwdStages = AMNERF_N_BWD_STAGES;
struct BwdEvSet {
  hipEvent_t ev[kBwdStages + 1] = {};
  bool pending = false;
  bool no_adam = false;   // a backward pass alone: its last event ends the reduction stage
};
}  // namespace

struct amnerf_ctx {
  int device = 0;
  bool timing = false;
  std::vector<EvSet> ring;
  int ring_next = 0;
  double stage_ms[kStages] = {};
  int64_t timed_passes = 0;
  std::vector<BwdEvSet> bring;   // the same for backward passes
  int bring_next = 0;
  double bwd_ms[kBwdStages] = {};
  int64_t bwd_passes = 0;
  size_t cap = 0;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  ChunkCounts* counts = nullptr;        // device
  ChunkCounts* counts_host = nullptr;   // pinned, one per render lane (the first also for statistics)
  int render_lanes = kLanes;          // lanes a multi-chunk render spreads its chunks over
  hipStream_t last_stream = nullptr;
  bool have_render = false;
  // last render, for stats and inspection
  int64_t last_rays = 0;
  int64_t last_chunks = 0;
  uint32_t last_leaves = 0;
  bool last_ess = false;          // the last render skipped empty space
  uint64_t last_niv_max = 0, last_ns_max = 0;
  // workspace views of the last chunk: the intervals the samples came from (plain or
  // planned by the proposal) and the sorted sample arrays
  IvSet use = {};
  uint32_t *bucket_off = nullptr, *perm = nullptr, *tile_off = nullptr, *srec_ray = nullptr;
  float *smp_out = nullptr, *srec_t = nullptr;
  uint32_t* ray_used = nullptr;   // samples composited per ray (the early-termination count)
  bool last_uses_arena3 = false;  // the last render's intervals live in the third arena
  bool last_static = false;       // the last render ran in the device's static workspace
  const uint64_t* last_mask = nullptr;   // kept plain slots per ray (proposal or empty-space renders)
  // last backward: per-sample pre-activation gradients (second arena), for inspection
  bool have_backward = false;
  const float* last_gpre = nullptr;
  // third arena: proposal stage buffers, sized from the measured interval count
  void* arena3 = nullptr;
  size_t arena3_bytes = 0;
  const amnerf_tree* last_tree = nullptr;
  const void* last_packed = nullptr;
  int32_t last_dtype = -1;
  amnerf_render_params last_params = {};
  const float* last_o = nullptr;
  // second arena: backward and training buffers
  void* arena2 = nullptr;
  size_t arena2_bytes = 0;
  // error report: block partials and totals (device), totals (pinned host)
  double* err_dev = nullptr;
  double* err_host = nullptr;
  // lanes 1 .. kLanes - 1 of a render that runs in several chunks: each a stream (default
  // priority), fork and join events, and its own chunk workspace, proposal arena and counters
  struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    void* arena3 = nullptr;
    size_t arena3_bytes = 0;
    ChunkCounts* counts = nullptr;
  } lanes[kLanes - 1];
};

struct amnerf_tree {
  int device = 0;
  int grid_n = 0;
  int n_leaves = 0;
  int depth = 0;
  std::vector<int32_t> rows;     // [n][12] sorted by code
  std::vector<uint64_t> mass;
  DevNode* dev_nodes = nullptr;
  float* dev_leafbox = nullptr;   // per leaf slot: 2*centre-1 (3), size (3), in [0,1] units
  DevNodeAhs* dev_ahs = nullptr;  // per device-table node: longest side, preorder node slot
};

struct amnerf_occ {
  int device = 0;
  int g = 0;                      // cells per side
  int64_t n_occupied = 0;
  std::vector<uint8_t> cells;     // G^3, 0 or 1
  uint32_t* dev_bits = nullptr;   // G^3 bits, cell c at word c / 32, bit c % 32
};

// ---------------------------------------------------------------------------------------
// misc
// ---------------------------------------------------------------------------------------
extern "C" const char* amnerf_last_error(void) { return g_err.c_str(); }
extern "C" int amnerf_version(void) { return 201; }

extern "C" int amnerf_ctx_create(int device, size_t workspace_cap, amnerf_ctx** out) {
  if (!out) return fail(AMNERF_EINVAL, "amnerf_ctx_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(AMNERF_EINVAL, "amnerf_ctx_create: device %d of %d", device, ndev);
  HIP_TRY(hipSetDevice(device));
  amnerf_ctx* c = new (std::nothrow) amnerf_ctx();
  if (!c) return fail(AMNERF_ENOMEM, "amnerf_ctx_create: host allocation");
  c->device = device;
  c->cap = workspace_cap;
  int rc = static_setup(device);
  if (rc) {
    delete c;
    return rc;
  }
  hipError_t e = hipMalloc((void**)&c->counts, sizeof(ChunkCounts));
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->counts_host, sizeof(ChunkCounts) * kLanes, hipHostMallocDefault);
  if (e != hipSuccess) {
    if (c->counts) (void)hipFree(c->counts);
    delete c;
    return fail(AMNERF_EDEVICE, "amnerf_ctx_create: %s", hipGetErrorString(e));
  }
  *out = c;
  return AMNERF_OK;
}

extern "C" int amnerf_ctx_destroy(amnerf_ctx* ctx) {
  if (!ctx) return AMNERF_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (EvSet& s : ctx->ring)
    for (hipEvent_t e : s.ev)
      if (e) (void)hipEventDestroy(e);
  for (BwdEvSet& s : ctx->bring)
    for (hipEvent_t e : s.ev)
      if (e) (void)hipEventDestroy(e);
  if (ctx->arena) (void)hipFree(ctx->arena);
  if (ctx->arena2) (void)hipFree(ctx->arena2);
  if (ctx->arena3) (void)hipFree(ctx->arena3);
  if (ctx->counts) (void)hipFree(ctx->counts);
  if (ctx->counts_host) (void)hipHostFree(ctx->counts_host);
  if (ctx->err_dev) (void)hipFree(ctx->err_dev);
  if (ctx->err_host) (void)hipHostFree(ctx->err_host);
  for (auto& ln : ctx->lanes) {
    if (ln.arena) (void)hipFree(ln.arena);
    if (ln.arena3) (void)hipFree(ln.arena3);
    if (ln.counts) (void)hipFree(ln.counts);
    if (ln.fork) (void)hipEventDestroy(ln.fork);
    if (ln.join) (void)hipEventDestroy(ln.join);
    if (ln.stream) (void)hipStreamDestroy(ln.stream);
  }
  delete ctx;
  return AMNERF_OK;
}

// Folds a completed event set into the stage sums.
static int drain_set(amnerf_ctx* ctx, EvSet& s) {
  if (!s.pending) return AMNERF_OK;
  HIP_TRY(hipEventSynchronize(s.ev[kStages]));
  for (int k = 0; k < kStages; ++k) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, s.ev[k], s.ev[k + 1]));
    ctx->stage_ms[k] += ms;
  }
  ctx->timed_passes += 1;
  s.pending = false;
  return AMNERF_OK;
}

extern "C" int amnerf_ctx_set_render_lanes(amnerf_ctx* ctx, int n_lanes) {
  if (!ctx) return fail(AMNERF_EINVAL, "amnerf_ctx_set_render_lanes: ctx is NULL");
  if (n_lanes < 1 || n_lanes > kLanes)
    return fail(AMNERF_EINVAL, "amnerf_ctx_set_render_lanes: %d lanes, the range is 1 .. %d", n_lanes, kLanes);
  ctx->render_lanes = n_lanes;
  return AMNERF_OK;
}

extern "C" int amnerf_ctx_set_timing(amnerf_ctx* ctx, int enable) {
  if (!ctx) return fail(AMNERF_EINVAL, "amnerf_ctx_set_timing: ctx is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  if (enable && ctx->ring.empty()) {
    ctx->ring.resize(kRing);
    for (EvSet& s : ctx->ring)
      for (hipEvent_t& e : s.ev) HIP_TRY(hipEventCreate(&e));
    ctx->bring.resize(kRing);
    for (BwdEvSet& s : ctx->bring)
      for (hipEvent_t& e : s.ev) HIP_TRY(hipEventCreate(&e));
  }
  ctx->timing = enable != 0;
  return AMNERF_OK;
}

extern "C" int amnerf_timing_collect(amnerf_ctx* ctx, double* stage_ms, int64_t* n_passes) {
  if (!ctx || !stage_ms) return fail(AMNERF_EINVAL, "amnerf_timing_collect: null argument");
  HIP_TRY(hipSetDevice(ctx->device));
  for (EvSet& s : ctx->ring) {
    int rc = drain_set(ctx, s);
    if (rc) return rc;
  }
  for (int k = 0; k < kStages; ++k) {
    stage_ms[k] = ctx->stage_ms[k];
    ctx->stage_ms[k] = 0.0;
  }
  if (n_passes) *n_passes = ctx->timed_passes;
  ctx->timed_passes = 0;
  return AMNERF_OK;
}

// Event set for the next timed pass (drained first if it is still pending).
static int next_set(amnerf_ctx* ctx, EvSet** out) {
  EvSet& s = ctx->ring[ctx->ring_next];
  ctx->ring_next = (ctx->ring_next + 1) % kRing;
  int rc = drain_set(ctx, s);
  if (rc) return rc;
  *out = &s;
  return AMNERF_OK;
}

static int drain_bwd_set(amnerf_ctx* ctx, BwdEvSet& s) {
  if (!s.pending) return AMNERF_OK;
  const int last = s.no_adam ? AMNERF_BWD_STAGE_ADAM : kBwdStages;
  HIP_TRY(hipEventSynchronize(s.ev[last]));
  for (int k = 0; k < last; ++k) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, s.ev[k], s.ev[k + 1]));
    ctx->bwd_ms[k] += ms;
  }
  ctx->bwd_passes += 1;
  s.pending = false;
  return AMNERF_OK;
}

static int next_bwd_set(amnerf_ctx* ctx, BwdEvSet** out) {
  BwdEvSet& s = ctx->bring[ctx->bring_next];
  ctx->bring_next = (ctx->bring_next + 1) % kRing;
  int rc = drain_bwd_set(ctx, s);
  if (rc) return rc;
  *out = &s;
  return AMNERF_OK;
}

extern "C" int amnerf_timing_collect_backward(amnerf_ctx* ctx, double* stage_ms, int64_t* n_passes) {
  if (!ctx || !stage_ms) return fail(AMNERF_EINVAL, "amnerf_timing_collect_backward: null argument");
  HIP_TRY(hipSetDevice(ctx->device));
  for (BwdEvSet& s : ctx->bring) {
    int rc = drain_bwd_set(ctx, s);
    if (rc) return rc;
  }
  for (int k = 0; k < kBwdStages; ++k) {
    stage_ms[k] = ctx->bwd_ms[k];
    ctx->bwd_ms[k] = 0.0;
  }
  if (n_passes) *n_passes = ctx->bwd_passes;
  ctx->bwd_passes = 0;
  return AMNERF_OK;
}

static int ensure_arena2(amnerf_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->arena2_bytes) return AMNERF_OK;
  if (ctx->cap && bytes + ctx->arena_bytes > ctx->cap)
    return fail(AMNERF_ENOMEM, "workspace needs %zu more bytes, cap is %zu", bytes, ctx->cap);
  HIP_TRY(hipDeviceSynchronize());
  ctx->have_backward = false;
  if (ctx->arena2) HIP_TRY(hipFree(ctx->arena2));
  ctx->arena2 = nullptr;
  ctx->arena2_bytes = 0;
  hipError_t e = hipMalloc(&ctx->arena2, bytes);
  if (e != hipSuccess) return fail(AMNERF_ENOMEM, "workspace hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  ctx->arena2_bytes = bytes;
  return AMNERF_OK;
}

static int ensure_arena3(amnerf_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->arena3_bytes) return AMNERF_OK;
  if (ctx->cap && bytes + ctx->arena_bytes + ctx->arena2_bytes > ctx->cap)
    return fail(AMNERF_ENOMEM, "workspace needs %zu more bytes, cap is %zu", bytes, ctx->cap);
  HIP_TRY(hipDeviceSynchronize());
  if (ctx->last_uses_arena3) ctx->have_render = false;
  if (ctx->arena3) HIP_TRY(hipFree(ctx->arena3));
  ctx->arena3 = nullptr;
  ctx->arena3_bytes = 0;
  size_t grow = bytes + bytes / 4;
  hipError_t e = hipMalloc(&ctx->arena3, grow);
  if (e != hipSuccess) return fail(AMNERF_ENOMEM, "workspace hipMalloc(%zu): %s", grow, hipGetErrorString(e));
  ctx->arena3_bytes = grow;
  return AMNERF_OK;
}

// Grows a lane buffer to `bytes` (plus `extra` of slack), within the context's cap.
static int grow_lane_buffer(amnerf_ctx* ctx, void** buf, size_t* have, size_t bytes, size_t extra) {
  if (bytes <= *have) return AMNERF_OK;
  size_t others = ctx->arena_bytes + ctx->arena2_bytes + ctx->arena3_bytes - *have;
  for (const auto& ln : ctx->lanes) others += ln.arena_bytes + ln.arena3_bytes;
  if (ctx->cap && bytes + others > ctx->cap)
    return fail(AMNERF_ENOMEM, "workspace needs %zu more bytes, cap is %zu", bytes, ctx->cap);
  HIP_TRY(hipDeviceSynchronize());
  ctx->have_render = false;   // a lane buffer may hold the last render's arrays
  if (*buf) HIP_TRY(hipFree(*buf));
  *buf = nullptr;
  *have = 0;
  const size_t grow = bytes + extra;
  hipError_t e = hipMalloc(buf, grow);
  if (e != hipSuccess) return fail(AMNERF_ENOMEM, "workspace hipMalloc(%zu): %s", grow, hipGetErrorString(e));
  *have = grow;
  return AMNERF_OK;
}

// Lane i's (1 .. kLanes - 1) stream, events, counters and chunk workspace (`need` bytes).
static int lane_prepare(amnerf_ctx* ctx, int i, size_t need) {
  auto& ln = ctx->lanes[i - 1];
  if (!ln.stream) {
    // all four or none: a failure leaves the context without this lane
    hipStream_t s = nullptr;
    hipEvent_t f = nullptr, j = nullptr;
    ChunkCounts* c = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&f, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc((void**)&c, sizeof(ChunkCounts));
    if (e != hipSuccess) {
      if (c) (void)hipFree(c);
      if (j) (void)hipEventDestroy(j);
      if (f) (void)hipEventDestroy(f);
      if (s) (void)hipStreamDestroy(s);
      return fail(AMNERF_EDEVICE, "render lane %d: %s", i, hipGetErrorString(e));
    }
    ln.stream = s;
    ln.fork = f;
    ln.join = j;
    ln.counts = c;
  }
  return grow_lane_buffer(ctx, &ln.arena, &ln.arena_bytes, need, need / 8);
}

// The proposal arena of the main context (lane 0) or of lane i.
static int ensure_arena3(amnerf_ctx* ctx, size_t bytes);
static int ensure_arena3_for(amnerf_ctx* ctx, int i, size_t bytes) {
  if (i == 0) return ensure_arena3(ctx, bytes);
  return grow_lane_buffer(ctx, &ctx->lanes[i - 1].arena3, &ctx->lanes[i - 1].arena3_bytes, bytes, bytes / 4);
}

static int ensure_arena(amnerf_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->arena_bytes) return AMNERF_OK;
  if (ctx->cap && bytes + ctx->arena2_bytes > ctx->cap)
    return fail(AMNERF_ENOMEM, "workspace needs %zu bytes, cap is %zu", bytes, ctx->cap);
  HIP_TRY(hipDeviceSynchronize());
  if (ctx->arena) HIP_TRY(hipFree(ctx->arena));
  ctx->arena = nullptr;
  ctx->arena_bytes = 0;
  ctx->have_render = false;
  size_t grow = bytes + bytes / 8;
  if (ctx->cap && grow > ctx->cap) grow = ctx->cap;
  hipError_t e = hipMalloc(&ctx->arena, grow);
  if (e != hipSuccess) return fail(AMNERF_ENOMEM, "workspace hipMalloc(%zu): %s", grow, hipGetErrorString(e));
  ctx->arena_bytes = grow;
  return AMNERF_OK;
}

// ---------------------------------------------------------------------------------------
// tree (Section 3.4)
// ---------------------------------------------------------------------------------------
namespace {

struct HNode {
  int lo[3], hi[3];
  uint32_t code;
  int depth;
  int axis = -1, plane = -1;
  int left = -1;     // index of the lower child; the upper child follows it
  int slot = -1;
  int nslot = -1;    // rank among all nodes in left-first depth-first preorder
  uint64_t mass = 0;
};

// Summed-volume table of the quantised grid: V(i,j,k) = sum of q over [0,i)x[0,j)x[0,k).
struct Svt {
  int n;
  std::vector<uint64_t> v;
  uint64_t at(int i, int j, int k) const { return v[((size_t)k * (n + 1) + j) * (n + 1) + i]; }
  uint64_t box(const int lo[3], const int hi[3]) const {
    return at(hi[0], hi[1], hi[2]) - at(lo[0], hi[1], hi[2]) - at(hi[0], lo[1], hi[2]) -
           at(hi[0], hi[1], lo[2]) + at(lo[0], lo[1], hi[2]) + at(lo[0], hi[1], lo[2]) +
           at(hi[0], lo[1], lo[2]) - at(lo[0], lo[1], lo[2]);
  }
};

int longest_axis(const HNode& nd) {
  int a = 0;
  for (int x = 1; x < 3; ++x)
    if (nd.hi[x] - nd.lo[x] > nd.hi[a] - nd.lo[a]) a = x;
  return a;
}

struct Cand {
  uint64_t prio;   // the mass (median split) or 64 - depth (middle split)
  uint32_t code;
  int idx;
};
struct CandLess {
  bool operator()(const Cand& a, const Cand& b) const {
    // priority_queue pops the largest: larger priority first, then the smaller code
    if (a.prio != b.prio) return a.prio < b.prio;
    return a.code > b.code;
  }
};

}  // namespace

namespace {

// Quantised grid (summed-volume table) and the growing node list of one tree build.
struct TreeBuild {
  int n = 0;
  Svt S;
  std::vector<HNode> nodes;
  int leaves = 1;
};

int tree_build_begin(const float* grid, int32_t n, TreeBuild& B, const char* who) {
  if (n < 1 || n > 512 || (n & (n - 1)) != 0)
    return fail(AMNERF_EINVAL, "%s: grid side %d must be a power of two <= 512", who, n);
  const size_t ncell = (size_t)n * n * n;
  double gmax = 0.0;
  for (size_t i = 0; i < ncell; ++i) {
    float g = grid[i];
    if (!std::isfinite(g)) return fail(AMNERF_EINVAL, "%s: grid[%zu] is not finite", who, i);
    if ((double)g > gmax) gmax = g;
  }
  B.n = n;
  B.S.n = n;
  try {
    B.S.v.assign((size_t)(n + 1) * (n + 1) * (n + 1), 0ull);
  } catch (...) {
    return fail(AMNERF_ENOMEM, "%s: summed-volume table", who);
  }
  const size_t N1 = n + 1;
  std::vector<uint64_t>& V = B.S.v;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double g = grid[(size_t)i + (size_t)n * ((size_t)j + (size_t)n * k)];
        uint64_t q = (gmax > 0.0 && g > 0.0) ? (uint64_t)std::floor(std::ldexp(g / gmax, 24) + 0.5) : 0ull;
        size_t o = ((size_t)(k + 1) * N1 + (j + 1)) * N1 + (i + 1);
        V[o] = q + V[o - 1] + V[o - N1] + V[o - N1 * N1] - V[o - 1 - N1] - V[o - 1 - N1 * N1] -
               V[o - N1 - N1 * N1] + V[o - 1 - N1 - N1 * N1];
      }
  B.nodes.clear();
  HNode root;
  for (int a = 0; a < 3; ++a) { root.lo[a] = 0; root.hi[a] = n; }
  root.code = 1;
  root.depth = 0;
  root.mass = B.S.box(root.lo, root.hi);
  B.nodes.push_back(root);
  B.leaves = 1;
  return AMNERF_OK;
}

bool longest_side_splittable(const HNode& nd) {
  int a = longest_axis(nd);
  return nd.hi[a] - nd.lo[a] >= 2;
}

// Splits leaf idx on its longest side: at the first cell plane whose lower side holds at
// least half of the node's mass (the last plane if none; the middle plane for a massless
// node), or at the middle plane.  Returns the index of the lower child (the upper follows).
int tree_split(TreeBuild& B, int idx, bool middle) {
  HNode nd = B.nodes[idx];
  const int a = longest_axis(nd);
  const int lo = nd.lo[a], hi = nd.hi[a];
  int plane;
  auto lower_mass = [&](int pl) {
    int h2[3] = {nd.hi[0], nd.hi[1], nd.hi[2]};
    h2[a] = pl;
    return B.S.box(nd.lo, h2);
  };
  if (middle || nd.mass == 0) {
    plane = (lo + hi) / 2;
  } else {
    // smallest plane in [lo+1, hi-1] with 2 * lower mass >= node mass (binary search on
    // the monotone lower mass); the last plane when none qualifies
    int L = lo + 1, R = hi - 1, ans = hi - 1;
    while (L <= R) {
      int mid = (L + R) / 2;
      if (2 * lower_mass(mid) >= nd.mass) { ans = mid; R = mid - 1; }
      else L = mid + 1;
    }
    plane = ans;
  }
  HNode lc = nd, rc = nd;
  lc.hi[a] = plane;
  rc.lo[a] = plane;
  lc.code = 2 * nd.code;
  rc.code = 2 * nd.code + 1;
  lc.depth = rc.depth = nd.depth + 1;
  lc.axis = rc.axis = lc.plane = rc.plane = lc.left = rc.left = -1;
  lc.mass = B.S.box(lc.lo, lc.hi);
  rc.mass = nd.mass - lc.mass;
  int li = (int)B.nodes.size();
  B.nodes[idx].axis = a;
  B.nodes[idx].plane = plane;
  B.nodes[idx].left = li;
  B.nodes.push_back(lc);
  B.nodes.push_back(rc);
  ++B.leaves;
  return li;
}

// Slots, the exported rows and the device tables of the nodes built; uploads them.
int tree_build_finish(amnerf_ctx* ctx, TreeBuild& B, amnerf_tree** out, const char* who) {
  std::vector<HNode>& nodes = B.nodes;
  const int n = B.n;
  const int leaves = B.leaves;
  // slots: left-first depth-first order (leaves among leaves; every node among all nodes);
  // a node split since an earlier finish loses its leaf slot
  for (HNode& nd : nodes) nd.slot = -1;
  int next_slot = 0, next_nslot = 0, max_depth = 0;
  std::vector<int> stack = {0};
  while (!stack.empty()) {
    int i = stack.back();
    stack.pop_back();
    nodes[i].nslot = next_nslot++;
    if (nodes[i].left < 0) {
      nodes[i].slot = next_slot++;
      max_depth = std::max(max_depth, nodes[i].depth);
    } else {
      stack.push_back(nodes[i].left + 1);
      stack.push_back(nodes[i].left);
    }
  }
  amnerf_tree* t = new (std::nothrow) amnerf_tree();
  if (!t) return fail(AMNERF_ENOMEM, "%s: host allocation", who);
  t->device = ctx->device;
  t->grid_n = n;
  t->n_leaves = leaves;
  t->depth = max_depth;
  std::vector<int> order(nodes.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return nodes[x].code < nodes[y].code; });
  t->rows.resize(nodes.size() * 12);
  t->mass.resize(nodes.size());
  for (size_t k = 0; k < order.size(); ++k) {
    const HNode& nd = nodes[order[k]];
    int32_t* r = &t->rows[k * 12];
    r[0] = (int32_t)nd.code;
    r[1] = nd.depth;
    for (int a = 0; a < 3; ++a) { r[2 + a] = nd.lo[a]; r[5 + a] = nd.hi[a]; }
    r[8] = nd.left < 0 ? -1 : nd.axis;
    r[9] = nd.left < 0 ? -1 : nd.plane;
    r[10] = nd.left < 0 ? nd.slot : -1;
    r[11] = nd.nslot;
    t->mass[k] = nd.mass;
  }
  // device table: breadth-first, siblings adjacent
  std::vector<DevNode> dev(nodes.size());
  std::vector<DevNodeAhs> ahs(nodes.size());
  std::vector<int> bfs = {0};
  std::vector<int> at(nodes.size(), -1);
  at[0] = 0;
  int next = 1;
  for (size_t q = 0; q < bfs.size(); ++q) {
    int i = bfs[q];
    DevNode& dn = dev[at[i]];
    int ext = 0;
    for (int a = 0; a < 3; ++a) ext = std::max(ext, nodes[i].hi[a] - nodes[i].lo[a]);
    ahs[at[i]].size = (float)ext / (float)n;   // exact: a small integer over a power of two
    ahs[at[i]].slot = (uint32_t)nodes[i].nslot;
    if (nodes[i].left < 0) {
      dn.plane = 0.f;
      dn.info = -(nodes[i].slot + 1);
    } else {
      int l = nodes[i].left;
      at[l] = next;
      at[l + 1] = next + 1;
      dn.plane = (float)nodes[i].plane / (float)n;
      dn.info = (next << 2) | nodes[i].axis;
      next += 2;
      bfs.push_back(l);
      bfs.push_back(l + 1);
    }
  }
  std::vector<float> box(6 * (size_t)leaves);
  for (const HNode& nd : nodes) {
    if (nd.left >= 0) continue;
    for (int a = 0; a < 3; ++a) {
      box[6 * nd.slot + a] = (float)(nd.lo[a] + nd.hi[a]) / (float)n - 1.f;
      box[6 * nd.slot + 3 + a] = (float)(nd.hi[a] - nd.lo[a]) / (float)n;
    }
  }
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipMalloc((void**)&t->dev_nodes, sizeof(DevNode) * dev.size());
  if (e == hipSuccess) e = hipMemcpy(t->dev_nodes, dev.data(), sizeof(DevNode) * dev.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void**)&t->dev_leafbox, sizeof(float) * box.size());
  if (e == hipSuccess) e = hipMemcpy(t->dev_leafbox, box.data(), sizeof(float) * box.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void**)&t->dev_ahs, sizeof(DevNodeAhs) * ahs.size());
  if (e == hipSuccess) e = hipMemcpy(t->dev_ahs, ahs.data(), sizeof(DevNodeAhs) * ahs.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (t->dev_nodes) (void)hipFree(t->dev_nodes);
    if (t->dev_leafbox) (void)hipFree(t->dev_leafbox);
    if (t->dev_ahs) (void)hipFree(t->dev_ahs);
    delete t;
    return fail(AMNERF_EDEVICE, "%s: upload: %s", who, hipGetErrorString(e));
  }
  *out = t;
  return AMNERF_OK;
}

// Index of the node with the given code, or -1.
int find_code(const TreeBuild& B, uint32_t code) {
  for (size_t i = 0; i < B.nodes.size(); ++i)
    if (B.nodes[i].code == code) return (int)i;
  return -1;
}

}  // namespace

extern "C" int amnerf_build_tree(amnerf_ctx* ctx, const float* grid, int32_t n,
                                 const amnerf_tree_params* p, amnerf_tree** out) {
  if (!ctx || !grid || !p || !out) return fail(AMNERF_EINVAL, "amnerf_build_tree: null argument");
  *out = nullptr;
  if (p->max_depth < 0 || p->max_depth > AMNERF_MAX_DEPTH)
    return fail(AMNERF_EINVAL, "amnerf_build_tree: max_depth %d out of [0, %d]", p->max_depth, AMNERF_MAX_DEPTH);
  if (p->split != AMNERF_SPLIT_MEDIAN && p->split != AMNERF_SPLIT_MIDDLE)
    return fail(AMNERF_EINVAL, "amnerf_build_tree: bad split mode %d", p->split);
  if (p->max_leaves < 1 || p->max_leaves > AMNERF_MAX_LEAVES)
    return fail(AMNERF_EINVAL, "amnerf_build_tree: max_leaves %d out of [1, %d]", p->max_leaves, AMNERF_MAX_LEAVES);
  TreeBuild B;
  int rc = tree_build_begin(grid, n, B, "amnerf_build_tree");
  if (rc) return rc;
  B.nodes.reserve(2 * (size_t)p->max_leaves);
  auto splittable = [&](const HNode& nd) { return nd.depth < p->max_depth && longest_side_splittable(nd); };
  const bool middle = p->split == AMNERF_SPLIT_MIDDLE;
  auto prio = [&](const HNode& nd) { return middle ? (uint64_t)(64 - nd.depth) : nd.mass; };
  std::priority_queue<Cand, std::vector<Cand>, CandLess> pq;
  if (splittable(B.nodes[0])) pq.push({prio(B.nodes[0]), 1u, 0});
  while (B.leaves < p->max_leaves && !pq.empty()) {
    Cand c = pq.top();
    pq.pop();
    const int li = tree_split(B, c.idx, middle);
    if (splittable(B.nodes[li])) pq.push({prio(B.nodes[li]), B.nodes[li].code, li});
    if (splittable(B.nodes[li + 1])) pq.push({prio(B.nodes[li + 1]), B.nodes[li + 1].code, li + 1});
  }
  return tree_build_finish(ctx, B, out, "amnerf_build_tree");
}

extern "C" int amnerf_build_tree_codes(amnerf_ctx* ctx, const float* grid, int32_t n, const uint32_t* codes,
                                       int32_t n_codes, amnerf_tree** out) {
  if (!ctx || !grid || !out || n_codes < 0 || (n_codes > 0 && !codes))
    return fail(AMNERF_EINVAL, "amnerf_build_tree_codes: bad argument");
  *out = nullptr;
  if (n_codes + 1 > AMNERF_MAX_LEAVES)
    return fail(AMNERF_EINVAL, "amnerf_build_tree_codes: %d splits exceed %d leaves", n_codes, AMNERF_MAX_LEAVES);
  TreeBuild B;
  int rc = tree_build_begin(grid, n, B, "amnerf_build_tree_codes");
  if (rc) return rc;
  std::vector<uint32_t> sorted(codes, codes + n_codes);
  std::sort(sorted.begin(), sorted.end());
  for (uint32_t code : sorted) {
    const int at = find_code(B, code);
    if (at < 0 || B.nodes[at].left >= 0 || !longest_side_splittable(B.nodes[at]) ||
        B.nodes[at].depth >= AMNERF_MAX_DEPTH)
      return fail(AMNERF_EINVAL, "amnerf_build_tree_codes: code %u is not a splittable leaf", code);
    tree_split(B, at, false);
  }
  return tree_build_finish(ctx, B, out, "amnerf_build_tree_codes");
}

extern "C" int amnerf_tree_info_get(const amnerf_tree* t, amnerf_tree_info* out) {
  if (!t || !out) return fail(AMNERF_EINVAL, "amnerf_tree_info_get: null argument");
  out->n_nodes = (int32_t)t->mass.size();
  out->n_leaves = t->n_leaves;
  out->depth = t->depth;
  out->grid_n = t->grid_n;
  return AMNERF_OK;
}

extern "C" int amnerf_tree_export(const amnerf_tree* t, int32_t* rows, uint64_t* mass) {
  if (!t || !rows) return fail(AMNERF_EINVAL, "amnerf_tree_export: null argument");
  std::memcpy(rows, t->rows.data(), sizeof(int32_t) * t->rows.size());
  if (mass) std::memcpy(mass, t->mass.data(), sizeof(uint64_t) * t->mass.size());
  return AMNERF_OK;
}

extern "C" int amnerf_tree_destroy(amnerf_tree* t) {
  if (!t) return AMNERF_OK;
  if (t->dev_nodes) {
    (void)hipSetDevice(t->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(t->dev_nodes);
    if (t->dev_leafbox) (void)hipFree(t->dev_leafbox);
    if (t->dev_ahs) (void)hipFree(t->dev_ahs);
  }
  delete t;
  return AMNERF_OK;
}

// ---------------------------------------------------------------------------------------
// occupancy grid
// ---------------------------------------------------------------------------------------
extern "C" int amnerf_build_occupancy(amnerf_ctx* ctx, const float* grid, int32_t n, int32_t block, float thresh,
                                      amnerf_occ** out) {
  if (!ctx || !grid || !out) return fail(AMNERF_EINVAL, "amnerf_build_occupancy: null argument");
  *out = nullptr;
  if (n < 1 || n > AMNERF_MAX_GRID || (n & (n - 1)) != 0)
    return fail(AMNERF_EINVAL, "amnerf_build_occupancy: grid side %d must be a power of two <= %d", n, AMNERF_MAX_GRID);
  if (block < 1 || (block & (block - 1)) != 0 || block > n)
    return fail(AMNERF_EINVAL, "amnerf_build_occupancy: block %d must be a power of two dividing %d", block, n);
  if (!(thresh >= 0.f && thresh <= 1.f)) return fail(AMNERF_EINVAL, "amnerf_build_occupancy: thresh must be in [0, 1]");
  const size_t ncell = (size_t)n * n * n;
  double gmax = 0.0;
  for (size_t i = 0; i < ncell; ++i) {
    float g = grid[i];
    if (!std::isfinite(g)) return fail(AMNERF_EINVAL, "amnerf_build_occupancy: grid[%zu] is not finite", i);
    if ((double)g > gmax) gmax = g;
  }
  const uint64_t q_thr = std::max<uint64_t>(1ull, (uint64_t)std::floor(std::ldexp((double)thresh, 24) + 0.5));
  const int G = n / block;
  amnerf_occ* o = new (std::nothrow) amnerf_occ();
  if (!o) return fail(AMNERF_ENOMEM, "amnerf_build_occupancy: host allocation");
  o->device = ctx->device;
  o->g = G;
  std::vector<uint32_t> bits;
  try {
    o->cells.assign((size_t)G * G * G, 0);
    bits.assign(((size_t)G * G * G + 31) / 32, 0u);
  } catch (...) {
    delete o;
    return fail(AMNERF_ENOMEM, "amnerf_build_occupancy: host allocation");
  }
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const double g = grid[(size_t)i + (size_t)n * ((size_t)j + (size_t)n * k)];
        const uint64_t q = (gmax > 0.0 && g > 0.0) ? (uint64_t)std::floor(std::ldexp(g / gmax, 24) + 0.5) : 0ull;
        if (q >= q_thr) o->cells[(size_t)(i / block) + (size_t)G * ((size_t)(j / block) + (size_t)G * (k / block))] = 1;
      }
  for (size_t c = 0; c < o->cells.size(); ++c)
    if (o->cells[c]) {
      bits[c >> 5] |= 1u << (c & 31);
      ++o->n_occupied;
    }
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipMalloc((void**)&o->dev_bits, sizeof(uint32_t) * bits.size());
  if (e == hipSuccess) e = hipMemcpy(o->dev_bits, bits.data(), sizeof(uint32_t) * bits.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (o->dev_bits) (void)hipFree(o->dev_bits);
    delete o;
    return fail(AMNERF_EDEVICE, "amnerf_build_occupancy: upload: %s", hipGetErrorString(e));
  }
  *out = o;
  return AMNERF_OK;
}

extern "C" int amnerf_occupancy_info_get(const amnerf_occ* o, int32_t* g, int64_t* n_occupied) {
  if (!o) return fail(AMNERF_EINVAL, "amnerf_occupancy_info_get: null argument");
  if (g) *g = o->g;
  if (n_occupied) *n_occupied = o->n_occupied;
  return AMNERF_OK;
}

extern "C" int amnerf_occupancy_export(const amnerf_occ* o, uint8_t* cells) {
  if (!o || !cells) return fail(AMNERF_EINVAL, "amnerf_occupancy_export: null argument");
  std::memcpy(cells, o->cells.data(), o->cells.size());
  return AMNERF_OK;
}

extern "C" int amnerf_occupancy_destroy(amnerf_occ* o) {
  if (!o) return AMNERF_OK;
  if (o->dev_bits) {
    (void)hipSetDevice(o->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(o->dev_bits);
  }
  delete o;
  return AMNERF_OK;
}

// ---------------------------------------------------------------------------------------
// MLP parameters
// ---------------------------------------------------------------------------------------
extern "C" int64_t amnerf_mlp_param_count(const amnerf_mlp_shape* s) {
  if (!s || s->n_hidden < 1 || s->n_hidden > 8 || (s->hidden != 32 && s->hidden != 64)) return -1;
  int64_t P = 0;
  for (int l = 0; l <= s->n_hidden; ++l) {
    int64_t di = l == 0 ? 30 : s->hidden, dn = l == s->n_hidden ? 4 : s->hidden;
    P += di * dn + dn;
  }
  return P;
}

static int check_geom(const amnerf_mlp_shape* s, int32_t dtype, MlpGeom* g, const char* who) {
  if (!s) return fail(AMNERF_EINVAL, "%s: shape is NULL", who);
  if (!mlp_geom(s->n_hidden, s->hidden, dtype, g))
    return fail(AMNERF_EINVAL, "%s: unsupported MLP n_hidden=%d hidden=%d dtype=%d", who, s->n_hidden, s->hidden, dtype);
  return AMNERF_OK;
}

extern "C" int amnerf_mlp_packed_bytes(const amnerf_mlp_shape* s, int32_t dtype, int32_t n_leaves, size_t* out) {
  MlpGeom g;
  int rc = check_geom(s, dtype, &g, "amnerf_mlp_packed_bytes");
  if (rc) return rc;
  if (!out || n_leaves < 1 || n_leaves > AMNERF_MAX_LEAVES) return fail(AMNERF_EINVAL, "amnerf_mlp_packed_bytes: bad argument");
  *out = (g.node_bytes + g.bwd_node_bytes) * (size_t)n_leaves;
  return AMNERF_OK;
}

extern "C" int amnerf_mlp_pack(amnerf_ctx* ctx, const amnerf_mlp_shape* s, int32_t dtype, int32_t n_leaves,
                               const float* master, void* packed, void* stream) {
  MlpGeom g;
  int rc = check_geom(s, dtype, &g, "amnerf_mlp_pack");
  if (rc) return rc;
  if (!ctx || !master || !packed || n_leaves < 1 || n_leaves > AMNERF_MAX_LEAVES)
    return fail(AMNERF_EINVAL, "amnerf_mlp_pack: bad argument");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(launch_mlp_pack(g, n_leaves, master, packed, (hipStream_t)stream));
  return AMNERF_OK;
}

extern "C" int amnerf_mlp_pack_fp8_act(amnerf_ctx* ctx, const amnerf_mlp_shape* s, int32_t n_leaves,
                                       const float* master, const float* act_max, void* packed, void* stream) {
  MlpGeom g;
  int rc = check_geom(s, AMNERF_FP8_ACT, &g, "amnerf_mlp_pack_fp8_act");
  if (rc) return rc;
  if (!ctx || !master || !packed || n_leaves < 1 || n_leaves > AMNERF_MAX_LEAVES)
    return fail(AMNERF_EINVAL, "amnerf_mlp_pack_fp8_act: bad argument");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(launch_mlp8_pack(s->n_hidden, n_leaves, master, act_max, packed, (hipStream_t)stream));
  return AMNERF_OK;
}

// ---------------------------------------------------------------------------------------
// render
// ---------------------------------------------------------------------------------------
namespace {

struct Carve {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(uint64_t count) {
    off = (off + 255) / 256 * 256;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * count;
    return p;
  }
};

struct Work {
  uint32_t *cnt_iv, *cnt_smp, *iv_off, *smp_off, *scan_tmp;
  float *iv_t0, *iv_dt;
  uint32_t *iv_key, *iv_ray, *iv_base;
  uint32_t *mat, *mat_scan, *sidx, *sn, *ssb, *bucket_off, *tile_off;
  uint32_t *srec_ray, *perm;
  float *srec_t, *smp_out;
  uint32_t* ray_used;
  // early termination in rounds: selection flags and their scan, compacted sample records,
  // the compacted buckets' offsets, and each ray's state between windows
  uint32_t *r_flags, *r_pos, *r_tmp, *c_ray, *c_perm, *c_boff, *c_toff;
  float* c_t;
  CompCarry* carry;
};

size_t carve(char* base, uint64_t nr, uint64_t niv, uint64_t ns, const SortPlan& sp, Work& w, bool rounds) {
  Carve c{base};
  uint64_t scan_n = std::max<uint64_t>({nr, niv, (uint64_t)sp.n_leaves * sp.nseg_max});
  w.cnt_iv = c.take<uint32_t>(nr);
  w.cnt_smp = c.take<uint32_t>(nr);
  w.iv_off = c.take<uint32_t>(nr + 1);
  w.smp_off = c.take<uint32_t>(nr + 1);
  w.scan_tmp = c.take<uint32_t>(scan_tmp_words(scan_n));
  w.iv_t0 = c.take<float>(niv);
  w.iv_dt = c.take<float>(niv);
  w.iv_key = c.take<uint32_t>(niv);
  w.iv_ray = c.take<uint32_t>(niv);
  w.iv_base = c.take<uint32_t>(niv);
  w.mat = c.take<uint32_t>((uint64_t)sp.n_leaves * sp.nseg_max);
  w.mat_scan = c.take<uint32_t>((uint64_t)sp.n_leaves * sp.nseg_max + 1);
  w.sidx = c.take<uint32_t>(niv);
  w.sn = c.take<uint32_t>(niv);
  w.ssb = c.take<uint32_t>(niv + 1);
  w.bucket_off = c.take<uint32_t>(sp.n_leaves + 1);
  w.tile_off = c.take<uint32_t>(sp.n_leaves + 1);
  w.srec_ray = c.take<uint32_t>(ns);
  w.srec_t = c.take<float>(ns);
  w.perm = c.take<uint32_t>(ns);
  w.smp_out = c.take<float>(4 * ns);
  w.ray_used = c.take<uint32_t>(nr);
  const uint64_t nsr = rounds ? ns : 0, nrr = rounds ? nr : 0, lr = rounds ? sp.n_leaves + 1 : 0;
  w.r_flags = c.take<uint32_t>(nsr + 1);
  w.r_pos = c.take<uint32_t>(nsr + 1);
  w.r_tmp = c.take<uint32_t>(rounds ? scan_tmp_words(ns) : 0);
  w.c_ray = c.take<uint32_t>(nsr);
  w.c_t = c.take<float>(nsr);
  w.c_perm = c.take<uint32_t>(nsr);
  w.c_boff = c.take<uint32_t>(lr);
  w.c_toff = c.take<uint32_t>(lr);
  w.carry = c.take<CompCarry>(nrr);
  return c.off + 256;
}

// Proposal-stage buffers of one chunk (sized from the measured plain interval count).
struct PropWork {
  float *wts, *tot;
  uint32_t *runs, *nsel, *pv_off, *ps_off;
  uint64_t* mask;
  float *pt0, *pdt;
  uint32_t *pkey, *pray, *pbase;
  uint32_t *mat, *mat_scan, *sidx, *sn, *ssb, *scan_tmp;
};

size_t carve_prop(char* base, uint64_t nr, uint64_t niv_plain, uint64_t niv_plan, const SortPlan& sp, PropWork& w) {
  Carve c{base};
  w.wts = c.take<float>(32 * std::max<uint64_t>(niv_plain, 1));
  w.tot = c.take<float>(std::max<uint64_t>(niv_plain, 1));
  w.runs = c.take<uint32_t>(nr);
  w.nsel = c.take<uint32_t>(nr);
  w.pv_off = c.take<uint32_t>(nr + 1);
  w.ps_off = c.take<uint32_t>(nr + 1);
  w.mask = c.take<uint64_t>(4 * nr);
  w.pt0 = c.take<float>(niv_plan);
  w.pdt = c.take<float>(niv_plan);
  w.pkey = c.take<uint32_t>(niv_plan);
  w.pray = c.take<uint32_t>(niv_plan);
  w.pbase = c.take<uint32_t>(niv_plan);
  w.mat = c.take<uint32_t>((uint64_t)sp.n_leaves * sp.nseg_max);
  w.mat_scan = c.take<uint32_t>((uint64_t)sp.n_leaves * sp.nseg_max + 1);
  w.sidx = c.take<uint32_t>(niv_plan);
  w.sn = c.take<uint32_t>(niv_plan);
  w.ssb = c.take<uint32_t>(niv_plan + 1);
  w.scan_tmp = c.take<uint32_t>(scan_tmp_words(std::max<uint64_t>({nr, niv_plan, (uint64_t)sp.n_leaves * sp.nseg_max})));
  return c.off + 256;
}

}  // namespace

static int check_proposal(const amnerf_render_params* p) {
  if (!p->proposal) return AMNERF_OK;
  const amnerf_proposal* q = p->proposal;
  if (!q->packed_dev) return fail(AMNERF_EINVAL, "proposal: packed parameters are NULL");
  if (q->dtype != AMNERF_F32 && q->dtype != AMNERF_BF16) return fail(AMNERF_EINVAL, "proposal: bad dtype %d", q->dtype);
  if (!(q->mass_thresh > 0.f)) return fail(AMNERF_EINVAL, "proposal: mass_thresh must be > 0");
  if (q->cap < 1 || q->cap > p->s_max) return fail(AMNERF_EINVAL, "proposal: cap %d out of [1, s_max]", q->cap);
  if (p->flags & AMNERF_JITTER) return fail(AMNERF_EINVAL, "proposal sampling uses centred strata (no jitter)");
  return AMNERF_OK;
}

// The render pipeline.  static_ws == nullptr: the workspace is the context's arenas, grown
// on demand.  Otherwise it is the static_bytes of static_ws (the allocation-free entry
// point): the call must then fit one pass and that workspace, and runs no proposal or
// empty-space selection (their buffers are sized on the host from a measured count).
static int render_impl(amnerf_ctx* ctx, const amnerf_tree* tree, const amnerf_mlp* mlp,
                       const amnerf_rays* rays, const amnerf_render_params* p,
                       amnerf_render_out* out, void* stream, char* static_ws, size_t static_bytes) {
  if (!ctx || !tree || !mlp || !rays || !p || !out) return fail(AMNERF_EINVAL, "amnerf_render: null argument");
  MlpGeom g;
  int rc = check_geom(&mlp->shape, mlp->dtype, &g, "amnerf_render");
  if (rc) return rc;
  if (!(p->hcheck_footprint >= 0.f) || !std::isfinite(p->hcheck_footprint))
    return fail(AMNERF_EINVAL, "amnerf_render: hcheck_footprint must be finite and >= 0");
  const bool ahs = p->hcheck_footprint > 0.f;
  const int n_nodes = (int)tree->mass.size();
  // MLP parameter sets: one per leaf, or one per node under hierarchical sampling
  const int n_sets = ahs ? n_nodes : tree->n_leaves;
  if (ahs && n_sets > AMNERF_MAX_LEAVES)
    return fail(AMNERF_ECAPACITY, "amnerf_render: hierarchical sampling needs %d node MLPs (at most %d)", n_sets,
                AMNERF_MAX_LEAVES);
  if (mlp->n_leaves != n_sets)
    return fail(AMNERF_EINVAL, "amnerf_render: MLP has %d parameter sets, the render needs %d (one per %s)",
                mlp->n_leaves, n_sets, ahs ? "node" : "leaf");
  if (ahs && p->proposal)
    return fail(AMNERF_EINVAL, "amnerf_render: proposal sampling runs on leaf intervals (no hierarchical sampling)");
  const amnerf_occ* occ = p->occupancy;
  if (occ && p->proposal)
    return fail(AMNERF_EINVAL, "amnerf_render: empty-space skipping is not combined with a proposal");
  if (occ && (p->flags & AMNERF_JITTER))
    return fail(AMNERF_EINVAL, "amnerf_render: empty-space skipping uses centred strata (no jitter)");
  if (occ && occ->device != ctx->device) return fail(AMNERF_EINVAL, "amnerf_render: occupancy grid lives on another device");
  if (!mlp->packed_dev) return fail(AMNERF_EINVAL, "amnerf_render: packed parameters are NULL");
  if (rays->n_rays < 0) return fail(AMNERF_EINVAL, "amnerf_render: n_rays < 0");
  if (rays->n_rays > 0 && (!rays->o_dev || !rays->d_dev)) return fail(AMNERF_EINVAL, "amnerf_render: ray arrays are NULL");
  if (rays->n_rays > 0 && !out->rgb_dev) return fail(AMNERF_EINVAL, "amnerf_render: rgb output is NULL");
  if (p->s_max < 1 || p->s_max > AMNERF_MAX_SAMPLES)
    return fail(AMNERF_EINVAL, "amnerf_render: s_max %d out of [1, %d]", p->s_max, AMNERF_MAX_SAMPLES);
  if (!(p->ert_eps >= 0.f) || !(p->ert_eps < 1.f)) return fail(AMNERF_EINVAL, "amnerf_render: ert_eps must be in [0, 1)");
  if (tree->device != ctx->device) return fail(AMNERF_EINVAL, "amnerf_render: tree lives on another device");
  rc = check_proposal(p);
  if (rc) return rc;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int64_t R = rays->n_rays;
  const uint32_t L = (uint32_t)n_sets;
  // the workspaces are about to be overwritten: the previous render can no longer be
  // inspected or differentiated, whether or not this one completes
  ctx->have_render = false;
  ctx->have_backward = false;
  const int jitter = (p->flags & AMNERF_JITTER) ? 1 : 0;
  // a ray has at most one interval per leaf, and hierarchical sampling only merges them
  const uint64_t iv_per_ray = std::min<uint64_t>((uint64_t)p->s_max, (uint64_t)tree->n_leaves);
  const DevNodeAhs* ahs_tab = ahs ? tree->dev_ahs : nullptr;
  uint64_t chunk = std::max<uint64_t>(1, kChunkSamples / (uint64_t)p->s_max);
  if (R > 0 && (uint64_t)R < chunk) chunk = (uint64_t)R;
  const uint64_t niv_max = chunk * iv_per_ray, ns_max = chunk * (uint64_t)p->s_max;
  SortPlan sp = make_sort_plan(niv_max, L);
  Work ws[kLanes];
  Work& w0 = ws[0];
  // early termination in rounds of 64-sample windows (a single window needs no rounds)
  const bool rounds = (p->flags & AMNERF_ERT_ROUNDS) && p->s_max > 64;
  size_t need = carve(nullptr, chunk, niv_max, ns_max, sp, w0, rounds);
  if (static_ws) {
    if ((uint64_t)R > chunk)
      return fail(AMNERF_ECAPACITY, "amnerf_render_static: %lld rays exceed one pass (%llu at s_max %d)",
                  (long long)R, (unsigned long long)chunk, p->s_max);
    if (need > static_bytes)
      return fail(AMNERF_ECAPACITY, "amnerf_render_static: the call needs %zu bytes of workspace, the static "
                  "workspace holds %zu", need, static_bytes);
    carve(static_ws, chunk, niv_max, ns_max, sp, w0, rounds);
  } else {
    rc = ensure_arena(ctx, need);
    if (rc) return rc;
    carve((char*)ctx->arena, chunk, niv_max, ns_max, sp, w0, rounds);
  }
  // More than one chunk (and no per-sample weights, whose offsets need the chunks in
  // order): chunk k runs on lane k mod n_lanes -- lanes beyond the caller's stream have their
  // own stream, workspace and counters -- so one chunk's latency-bound stages overlap
  // another's matrix-core stage.  The lanes wait for the caller's stream on entry and the
  // caller's stream waits for them on exit, so the call stays asynchronous on `stream`.
  const bool pipe = (uint64_t)R > chunk && !out->weights_dev && !static_ws;
  const int n_lanes = pipe ? (int)std::min<uint64_t>((uint64_t)ctx->render_lanes, ((uint64_t)R + chunk - 1) / chunk) : 1;
  for (int i = 1; i < n_lanes; ++i) {
    rc = lane_prepare(ctx, i, need);
    if (rc) return rc;
    carve((char*)ctx->lanes[i - 1].arena, chunk, niv_max, ns_max, sp, ws[i], rounds);
  }
  HIP_TRY(launch_counts_reset(ctx->counts, st));
  for (int i = 1; i < n_lanes; ++i) {
    auto& ln = ctx->lanes[i - 1];
    HIP_TRY(launch_counts_reset(ln.counts, st));
    HIP_TRY(hipEventRecord(ln.fork, st));
    HIP_TRY(hipStreamWaitEvent(ln.stream, ln.fork, 0));
  }
  int64_t n_chunks = 0;
  IvSet use = {};
  const uint64_t* sel_mask = nullptr;   // the last chunk's kept-slot mask, if it selected slots
  Work* wl = &w0;   // the last chunk's workspace
  uint32_t *mat = w0.mat, *mat_scan = w0.mat_scan, *sidx = w0.sidx, *sn = w0.sn, *ssb = w0.ssb, *scan_tmp = w0.scan_tmp;
  // A proposal or an occupancy grid sizes its buffers from the chunk's plain interval count,
  // which the host reads back.  The chunk loop is therefore split in two phases, and with
  // more than one lane chunk k's second phase is enqueued after chunk k + 1's first (which
  // runs on another lane, in another workspace): while the host waits for chunk k's count,
  // the next chunk's traversal is already queued.
  const bool wait_count = p->proposal || occ;
  struct Pending {
    int64_t r0;
    uint32_t nr;
    int li;
    EvSet* ev;
  };
  // phase 1: traversal, and the plain interval count on its way to the host (lane li's slot)
  auto phase1 = [&](int64_t r0, uint32_t nr, int li, Pending* pd) -> int {
    const hipStream_t cs = li ? ctx->lanes[li - 1].stream : st;
    ChunkCounts* const cc = li ? ctx->lanes[li - 1].counts : ctx->counts;
    Work& w = ws[li];
    EvSet* ev = nullptr;
    if (ctx->timing) {
      int r = next_set(ctx, &ev);
      if (r) return r;
    }
    auto mark = [&](int k) -> hipError_t { return ev ? hipEventRecord(ev->ev[k], cs) : hipSuccess; };
    HIP_TRY(mark(0));
    HIP_TRY(launch_trav_count(tree->dev_nodes, ahs_tab, p->hcheck_footprint, (uint32_t)n_nodes, tree->depth, rays->o_dev, rays->d_dev, R, r0, nr, p->s_max, w.cnt_iv, w.cnt_smp, cs));
    HIP_TRY(launch_scan_u32_pair(w.cnt_iv, w.iv_off, w.cnt_smp, w.smp_off, nr, w.scan_tmp, cs));
    HIP_TRY(launch_trav_emit(tree->dev_nodes, ahs_tab, p->hcheck_footprint, (uint32_t)n_nodes, tree->depth, rays->o_dev, rays->d_dev, R, r0, nr, w.cnt_iv, w.cnt_smp, w.iv_off,
                             w.smp_off, w.iv_t0, w.iv_dt, w.iv_key, w.iv_ray, w.iv_base, cc, cs));
    HIP_TRY(mark(1));
    if (wait_count)
      HIP_TRY(hipMemcpyAsync(&ctx->counts_host[li].n_iv, w.iv_off + nr, sizeof(uint32_t), hipMemcpyDeviceToHost, cs));
    *pd = {r0, nr, li, ev};
    return AMNERF_OK;
  };
  // phase 2: proposal or occupancy selection, sort, expansion, leaf MLPs, compositing
  auto phase2 = [&](const Pending& pd) -> int {
    const int64_t r0 = pd.r0;
    const uint32_t nr = pd.nr;
    const int li = pd.li;
    EvSet* const ev = pd.ev;
    const hipStream_t cs = li ? ctx->lanes[li - 1].stream : st;
    ChunkCounts* const cc = li ? ctx->lanes[li - 1].counts : ctx->counts;
    Work& w = ws[li];
    wl = &w;
    int rc = AMNERF_OK;
    auto mark = [&](int k) -> hipError_t { return ev ? hipEventRecord(ev->ev[k], cs) : hipSuccess; };
    const IvSet plain = {w.iv_off, w.smp_off, w.iv_t0, w.iv_dt, w.iv_key, w.iv_ray, w.iv_base, w.iv_off + nr};
    use = plain;
    SortPlan spu = sp;
    mat = w.mat; mat_scan = w.mat_scan; sidx = w.sidx; sn = w.sn; ssb = w.ssb; scan_tmp = w.scan_tmp;
    uint64_t niv_use_max = niv_max;
    if (wait_count) HIP_TRY(hipStreamSynchronize(cs));   // the chunk's plain interval count has arrived
    if (p->proposal) {
      const uint32_t niv_plain = ctx->counts_host[li].n_iv;
      const amnerf_proposal* q = p->proposal;
      const uint64_t niv_plan = (uint64_t)niv_plain + (uint64_t)nr * (uint64_t)std::min(q->cap, p->s_max);
      SortPlan spp = make_sort_plan(niv_plan, L);
      PropWork pw;
      rc = ensure_arena3_for(ctx, li, carve_prop(nullptr, nr, niv_plain, niv_plan, spp, pw));
      if (rc) return rc;
      carve_prop((char*)(li ? ctx->lanes[li - 1].arena3 : ctx->arena3), nr, niv_plain, niv_plan, spp, pw);
      HIP_TRY(launch_prop_fwd(q->dtype, q->packed_dev, plain, rays->o_dev, rays->d_dev, R, r0, tree->dev_leafbox,
                              p->s_max, niv_plain, true, pw.wts, pw.tot, cs));
      HIP_TRY(launch_prop_select(nr, plain, pw.wts, pw.tot, q->mass_thresh, q->cap, p->s_max, pw.runs, pw.nsel, pw.mask, nullptr,
                                 cc, cs));
      HIP_TRY(launch_scan_u32_pair(pw.runs, pw.pv_off, pw.nsel, pw.ps_off, nr, pw.scan_tmp, cs));
      HIP_TRY(launch_prop_emit(nr, plain, pw.mask, pw.pv_off, pw.ps_off, pw.pt0, pw.pdt, pw.pkey, pw.pray, pw.pbase, cs));
      use = {pw.pv_off, pw.ps_off, pw.pt0, pw.pdt, pw.pkey, pw.pray, pw.pbase, pw.pv_off + nr};
      sel_mask = pw.mask;
      spu = spp;
      mat = pw.mat; mat_scan = pw.mat_scan; sidx = pw.sidx; sn = pw.sn; ssb = pw.ssb; scan_tmp = pw.scan_tmp;
      niv_use_max = niv_plan;
    } else if (occ) {
      // empty-space skipping: the kept samples of each ray as runs of consecutive slots
      // (within an interval of n slots at most ceil(n/2) runs, so a ray has at most
      // (s_max + m) / 2 of them); buffers sized from the plain interval count
      const uint64_t niv_plain = ctx->counts_host[li].n_iv;
      const uint64_t niv_plan = (niv_plain + (uint64_t)nr * (uint64_t)p->s_max) / 2 + nr;
      SortPlan spp = make_sort_plan(niv_plan, L);
      PropWork pw;
      rc = ensure_arena3_for(ctx, li, carve_prop(nullptr, nr, 1, niv_plan, spp, pw));
      if (rc) return rc;
      carve_prop((char*)(li ? ctx->lanes[li - 1].arena3 : ctx->arena3), nr, 1, niv_plan, spp, pw);
      HIP_TRY(launch_occ_select(nr, plain, rays->o_dev, rays->d_dev, R, r0, occ->dev_bits, occ->g, pw.runs, pw.nsel,
                                pw.mask, cs));
      HIP_TRY(launch_scan_u32_pair(pw.runs, pw.pv_off, pw.nsel, pw.ps_off, nr, pw.scan_tmp, cs));
      HIP_TRY(launch_prop_emit(nr, plain, pw.mask, pw.pv_off, pw.ps_off, pw.pt0, pw.pdt, pw.pkey, pw.pray, pw.pbase, cs));
      use = {pw.pv_off, pw.ps_off, pw.pt0, pw.pdt, pw.pkey, pw.pray, pw.pbase, pw.pv_off + nr};
      sel_mask = pw.mask;
      spu = spp;
      mat = pw.mat; mat_scan = pw.mat_scan; sidx = pw.sidx; sn = pw.sn; ssb = pw.ssb; scan_tmp = pw.scan_tmp;
      niv_use_max = niv_plan;
    }
    HIP_TRY(launch_chunk_begin(cc, use.n_iv_dev, spu.seg, L, cs));
    HIP_TRY(mark(2));
    HIP_TRY(launch_sort_hist(spu, use.key, use.n_iv_dev, mat, cs));
    HIP_TRY(launch_scan_u32(mat, mat_scan, (uint64_t)L * spu.nseg_max, &cc->mat_n, scan_tmp, cs));
    HIP_TRY(launch_sort_scatter(spu, use.key, use.n_iv_dev, mat_scan, sidx, sn, cs));
    HIP_TRY(launch_scan_u32(sn, ssb, niv_use_max, use.n_iv_dev, scan_tmp, cs));
    HIP_TRY(launch_bucket_tiles(spu, mat_scan, ssb, w.bucket_off, w.tile_off, cc, cs));
    HIP_TRY(mark(3));
    HIP_TRY(launch_expand(sidx, ssb, use, r0, jitter, p->jitter_seed, w.srec_ray, w.srec_t, w.perm, cs));
    HIP_TRY(mark(4));
    if (!rounds) {
      HIP_TRY(launch_mlp(g, mlp->packed_dev, L, w.bucket_off, w.tile_off, cc, w.srec_ray, w.srec_t, w.perm,
                         rays->o_dev, rays->d_dev, R, r0, w.smp_out, cs));
      HIP_TRY(mark(5));
      HIP_TRY(launch_composite(nr, use, w.smp_out, r0, jitter, p->jitter_seed, p->ert_eps, out->rgb_dev,
                               out->depth_dev, out->opacity_dev, out->weights_dev, w.ray_used, cc, cs));
    } else {
      // round k: the samples of window k of the rays still marching, compacted in sorted
      // order, through the leaf MLPs, then composited from the state of the earlier windows
      // (the stage timing counts every round but the last one's compositing as MLP work)
      const uint32_t n_rounds = (uint32_t)(p->s_max + 63) / 64;
      for (uint32_t k = 0; k < n_rounds; ++k) {
        HIP_TRY(launch_round_flags(w.perm, w.srec_ray, use.smp_off, w.carry, cc, k, (uint32_t)ns_max, w.r_flags, cs));
        HIP_TRY(launch_scan_u32(w.r_flags, w.r_pos, ns_max, &cc->n_smp, w.r_tmp, cs));
        HIP_TRY(launch_round_compact(w.r_flags, w.r_pos, w.srec_ray, w.srec_t, w.perm, cc, (uint32_t)ns_max, w.c_ray,
                                     w.c_t, w.c_perm, cs));
        HIP_TRY(launch_round_tiles(w.bucket_off, w.r_pos, L, w.c_boff, w.c_toff, cc, cs));
        HIP_TRY(launch_mlp(g, mlp->packed_dev, L, w.c_boff, w.c_toff, cc, w.c_ray, w.c_t, w.c_perm, rays->o_dev,
                           rays->d_dev, R, r0, w.smp_out, cs));
        if (k + 1 == n_rounds) HIP_TRY(mark(5));
        HIP_TRY(launch_composite_round(nr, use, w.smp_out, r0, jitter, p->jitter_seed, p->ert_eps, out->rgb_dev,
                                       out->depth_dev, out->opacity_dev, out->weights_dev, w.ray_used, cc, w.carry,
                                       k, cs));
      }
      HIP_TRY(launch_sum_used(nr, w.ray_used, cc, cs));
    }
    HIP_TRY(mark(6));
    if (ev) ev->pending = true;
    HIP_TRY(launch_chunk_finish(cc, use.smp_off + nr, use.n_iv_dev, w.smp_off + nr, rounds ? 1 : 0, cs));
    return rc;
  };
  Pending prev = {};
  bool have_prev = false;
  for (int64_t r0 = 0; r0 < R; r0 += (int64_t)chunk, ++n_chunks) {
    const uint32_t nr = (uint32_t)std::min<int64_t>((int64_t)chunk, R - r0);
    Pending cur;
    rc = phase1(r0, nr, (int)(n_chunks % n_lanes), &cur);
    if (rc) return rc;
    if (n_lanes == 1) {   // one workspace: the next chunk's traversal must wait for this chunk
      rc = phase2(cur);
      if (rc) return rc;
      continue;
    }
    if (have_prev) {
      rc = phase2(prev);
      if (rc) return rc;
    }
    prev = cur;
    have_prev = true;
  }
  if (have_prev) {
    rc = phase2(prev);
    if (rc) return rc;
  }
  for (int i = 1; i < n_lanes; ++i) {
    auto& ln = ctx->lanes[i - 1];
    HIP_TRY(hipEventRecord(ln.join, ln.stream));
    HIP_TRY(hipStreamWaitEvent(st, ln.join, 0));
    HIP_TRY(launch_counts_merge(ctx->counts, ln.counts, st));
  }
  ctx->last_stream = st;
  ctx->have_render = true;
  ctx->last_rays = R;
  ctx->last_chunks = n_chunks;
  ctx->last_leaves = L;
  ctx->last_niv_max = niv_max;
  ctx->last_ns_max = ns_max;
  ctx->use = use;
  ctx->bucket_off = wl->bucket_off;
  ctx->perm = wl->perm;
  ctx->smp_out = wl->smp_out;
  ctx->tile_off = wl->tile_off;
  ctx->srec_ray = wl->srec_ray;
  ctx->srec_t = wl->srec_t;
  ctx->ray_used = wl->ray_used;
  ctx->last_uses_arena3 = p->proposal != nullptr || occ != nullptr;
  ctx->last_tree = tree;
  ctx->last_packed = mlp->packed_dev;
  ctx->last_dtype = mlp->dtype;
  ctx->last_params = *p;
  ctx->last_params.proposal = nullptr;
  ctx->last_params.occupancy = nullptr;
  ctx->last_ess = occ != nullptr;
  ctx->last_o = rays->o_dev;
  ctx->last_static = static_ws != nullptr;
  ctx->last_mask = sel_mask;
  return AMNERF_OK;
}

extern "C" int amnerf_render(amnerf_ctx* ctx, const amnerf_tree* tree, const amnerf_mlp* mlp,
                             const amnerf_rays* rays, const amnerf_render_params* p,
                             amnerf_render_out* out, void* stream) {
  return render_impl(ctx, tree, mlp, rays, p, out, stream, nullptr, 0);
}

extern "C" int amnerf_render_static(amnerf_ctx* ctx, const amnerf_tree* tree, const amnerf_mlp* mlp,
                                    const amnerf_rays* rays, const amnerf_render_params* p,
                                    amnerf_render_out* out, void* stream) {
  if (!ctx || !p) return fail(AMNERF_EINVAL, "amnerf_render_static: null argument");
  if (p->proposal || p->occupancy)
    return fail(AMNERF_EINVAL, "amnerf_render_static: proposal and empty-space renders size their buffers on the host "
                "(use amnerf_render)");
  char* ws = (char*)static_workspace(ctx->device);
  if (!ws) return fail(AMNERF_ESTATE, "amnerf_render_static: no static workspace on device %d", ctx->device);
  return render_impl(ctx, tree, mlp, rays, p, out, stream, ws, kStaticBytes);
}

extern "C" size_t amnerf_render_static_capacity(void) { return kStaticBytes; }

static int read_counts(amnerf_ctx* ctx) {
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipMemcpyAsync(ctx->counts_host, ctx->counts, sizeof(ChunkCounts), hipMemcpyDeviceToHost, ctx->last_stream));
  HIP_TRY(hipStreamSynchronize(ctx->last_stream));
  return AMNERF_OK;
}

extern "C" int amnerf_render_stats_get(amnerf_ctx* ctx, amnerf_render_stats* out) {
  if (!ctx || !out) return fail(AMNERF_EINVAL, "amnerf_render_stats_get: null argument");
  if (!ctx->have_render) return fail(AMNERF_ESTATE, "amnerf_render_stats_get: no render yet");
  int rc = read_counts(ctx);
  if (rc) return rc;
  const ChunkCounts& c = *ctx->counts_host;
  out->n_rays = ctx->last_rays;
  out->n_intervals = (int64_t)c.iv_global;
  out->n_samples = (int64_t)c.evaluated;
  out->n_tiles = c.n_tiles;
  out->n_chunks = ctx->last_chunks;
  out->n_nonfinite = (int64_t)c.nonfinite;
  out->n_fallback = (int64_t)c.fallback;
  out->n_plain_samples = (int64_t)c.plain_smp;
  out->n_unreached = (int64_t)c.unreached;
  out->n_composited = (int64_t)c.composited;
  out->n_placed_samples = (int64_t)c.smp_global;
  return AMNERF_OK;
}

extern "C" int amnerf_render_inspect(amnerf_ctx* ctx, const amnerf_inspect* o, void* stream) {
  if (!ctx || !o) return fail(AMNERF_EINVAL, "amnerf_render_inspect: null argument");
  if (!ctx->have_render) return fail(AMNERF_ESTATE, "amnerf_render_inspect: no render yet");
  if (ctx->last_static)
    return fail(AMNERF_ESTATE, "amnerf_render_inspect: the last render ran in the shared static workspace");
  if (ctx->last_chunks != 1) return fail(AMNERF_ESTATE, "amnerf_render_inspect: last render ran in %lld chunks", (long long)ctx->last_chunks);
  int rc = read_counts(ctx);
  if (rc) return rc;
  const ChunkCounts& c = *ctx->counts_host;
  const uint64_t nr = (uint64_t)ctx->last_rays, niv = c.n_iv, ns = c.n_smp, L = ctx->last_leaves;
  hipStream_t st = (hipStream_t)stream;
  auto cp = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (!dst || bytes == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
  };
  const IvSet& u = ctx->use;
  HIP_TRY(cp(o->ray_iv_off, u.iv_off, 4 * (nr + 1)));
  HIP_TRY(cp(o->ray_smp_off, u.smp_off, 4 * (nr + 1)));
  HIP_TRY(cp(o->iv_t0, u.t0, 4 * niv));
  HIP_TRY(cp(o->iv_dt, u.dt, 4 * niv));
  HIP_TRY(cp(o->bucket_off, ctx->bucket_off, 4 * (L + 1)));
  HIP_TRY(cp(o->perm, ctx->perm, 4 * ns));
  HIP_TRY(cp(o->sample_out, ctx->smp_out, 16 * ns));
  HIP_TRY(cp(o->ray_used, ctx->ray_used, 4 * nr));
  if (o->slot_mask) {
    if (!ctx->last_mask)
      return fail(AMNERF_ESTATE, "amnerf_render_inspect: slot_mask needs a proposal or empty-space render");
    HIP_TRY(cp(o->slot_mask, ctx->last_mask, 32 * nr));
  }
  if (o->iv_slot || o->iv_n) {
    // split the packed keys on the host (inspection only)
    std::vector<uint32_t> keys(niv);
    if (niv) {
      HIP_TRY(hipMemcpyAsync(keys.data(), u.key, 4 * niv, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
    }
    std::vector<uint32_t> slot(niv), nn(niv);
    for (uint64_t i = 0; i < niv; ++i) { slot[i] = keys[i] & 0xFFFFu; nn[i] = keys[i] >> 16; }
    if (o->iv_slot && niv) HIP_TRY(hipMemcpy(o->iv_slot, slot.data(), 4 * niv, hipMemcpyHostToDevice));
    if (o->iv_n && niv) HIP_TRY(hipMemcpy(o->iv_n, nn.data(), 4 * niv, hipMemcpyHostToDevice));
  }
  HIP_TRY(hipStreamSynchronize(st));
  return AMNERF_OK;
}

// ---------------------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------------------
namespace {

struct BwdWork {
  float* gpre;
  uint32_t* seg_off;
  float* part;
  float* rgb;
  float* g_rgb;
  float* loss_partial;
};

size_t carve_bwd(char* base, uint64_t ns, uint64_t L, uint64_t nseg, uint64_t P, uint64_t R, BwdWork& w) {
  Carve c{base};
  w.gpre = c.take<float>(4 * ns);
  w.seg_off = c.take<uint32_t>(L + 2);   // segment offsets, total, and the backward's queue
  w.part = c.take<float>(nseg * P);
  w.rgb = c.take<float>(3 * R);
  w.g_rgb = c.take<float>(3 * R);
  w.loss_partial = c.take<float>(loss_partial_words(R));
  return c.off + 256;
}

// in_step: called by a training step, whose backward stage events (stage 0 already marked)
// are ev, null when timing is off; a backward pass alone takes an event set of its own when
// timing is on.
int backward_impl(amnerf_ctx* ctx, const amnerf_tree* tree, const amnerf_mlp* mlp, const amnerf_rays* rays,
                  const float* g_rgb, const float* g_depth, const float* g_opac, float* grad, hipStream_t st,
                  BwdWork* w_out, bool in_step, BwdEvSet* ev) {
  MlpGeom g;
  int rc = check_geom(&mlp->shape, mlp->dtype, &g, "amnerf_render_backward");
  if (rc) return rc;
  if (mlp->dtype != AMNERF_BF16 && mlp->dtype != AMNERF_F32)
    return fail(AMNERF_EINVAL, "amnerf_render_backward: the backward pass runs in bfloat16 or float32 (dtype %d)",
                mlp->dtype);
  if (!mlp_bwd_supported(mlp->shape.n_hidden, mlp->shape.hidden))
    return fail(AMNERF_EINVAL, "amnerf_render_backward: n_hidden must be 1 .. 4 (got %d)", mlp->shape.n_hidden);
  if (!ctx->have_render || ctx->last_tree != tree || ctx->last_packed != mlp->packed_dev ||
      ctx->last_dtype != mlp->dtype || ctx->last_rays != rays->n_rays || ctx->last_o != rays->o_dev)
    return fail(AMNERF_ESTATE, "amnerf_render_backward: the last render on this context used other inputs");
  if (ctx->last_chunks != 1) return fail(AMNERF_ESTATE, "amnerf_render_backward: the last render ran in %lld chunks",
                                         (long long)ctx->last_chunks);
  if (ctx->last_static)
    return fail(AMNERF_ESTATE, "amnerf_render_backward: the last render ran in the shared static workspace");
  if (!grad || (rays->n_rays > 0 && !g_rgb)) return fail(AMNERF_EINVAL, "amnerf_render_backward: null gradient pointer");
  if (ctx->last_ess)
    return fail(AMNERF_ESTATE, "amnerf_render_backward: the last render skipped empty space (not differentiated)");
  if (mlp->n_leaves != (int)ctx->last_leaves)
    return fail(AMNERF_EINVAL, "amnerf_render_backward: MLP has %d parameter sets, the last render used %u",
                mlp->n_leaves, ctx->last_leaves);
  const uint64_t L = (uint64_t)ctx->last_leaves;   // parameter sets of that render
  const uint64_t P = (uint64_t)amnerf_mlp_param_count(&mlp->shape);
  const uint64_t ns = ctx->last_ns_max, R = (uint64_t)rays->n_rays;
  const uint64_t tiles = ns / kMlpTileRows + L;
  const uint64_t nseg = tiles / kSegTiles + L;
  BwdWork w;
  size_t need = carve_bwd(nullptr, ns, L, nseg, P, R, w);
  rc = ensure_arena2(ctx, need);
  if (rc) return rc;
  carve_bwd((char*)ctx->arena2, ns, L, nseg, P, R, w);
  if (w_out) *w_out = w;
  const amnerf_render_params& p = ctx->last_params;
  const int jitter = (p.flags & AMNERF_JITTER) ? 1 : 0;
  const uint32_t nr = (uint32_t)R;
  const bool alone = !in_step;
  if (alone && ctx->timing) {
    rc = next_bwd_set(ctx, &ev);
    if (rc) return rc;
  }
  auto mark = [&](int k) -> hipError_t { return ev ? hipEventRecord(ev->ev[k], st) : hipSuccess; };
  if (alone) HIP_TRY(mark(AMNERF_BWD_STAGE_COMPOSITE));
  HIP_TRY(launch_comp_bwd(nr, ctx->use, ctx->smp_out, 0, jitter, p.jitter_seed, ctx->ray_used, g_rgb, g_depth,
                          g_opac, w.gpre, st));
  HIP_TRY(mark(AMNERF_BWD_STAGE_MLP));
  HIP_TRY(launch_seg_offsets(ctx->tile_off, (uint32_t)L, w.seg_off, st));
  HIP_TRY(launch_mlp_bwd(g, mlp->packed_dev, (uint32_t)L, ctx->bucket_off, ctx->tile_off, w.seg_off, ctx->srec_ray,
                         ctx->srec_t, ctx->perm, rays->o_dev, rays->d_dev, rays->n_rays, 0, w.gpre, w.part, st));
  HIP_TRY(mark(AMNERF_BWD_STAGE_REDUCE));
  HIP_TRY(launch_grad_reduce(w.part, w.seg_off, (uint32_t)L, (uint32_t)P, grad, st));
  HIP_TRY(mark(AMNERF_BWD_STAGE_ADAM));
  if (alone && ev) {
    ev->no_adam = true;
    ev->pending = true;
  }
  ctx->have_backward = true;
  ctx->last_gpre = w.gpre;
  return AMNERF_OK;
}

}  // namespace

extern "C" int amnerf_render_backward(amnerf_ctx* ctx, const amnerf_tree* tree, const amnerf_mlp* mlp,
                                      const amnerf_rays* rays, const float* g_rgb, const float* g_depth,
                                      const float* g_opac, float* grad, void* stream) {
  if (!ctx || !tree || !mlp || !rays) return fail(AMNERF_EINVAL, "amnerf_render_backward: null argument");
  HIP_TRY(hipSetDevice(ctx->device));
  return backward_impl(ctx, tree, mlp, rays, g_rgb, g_depth, g_opac, grad, (hipStream_t)stream, nullptr, false, nullptr);
}

extern "C" int amnerf_mlp_calibrate(amnerf_ctx* ctx, const amnerf_mlp_shape* s, int32_t n_leaves, const float* master,
                                    const amnerf_rays* rays, float* act_max, void* stream) {
  MlpGeom g;
  int rc = check_geom(s, AMNERF_FP8_ACT, &g, "amnerf_mlp_calibrate");
  if (rc) return rc;
  if (!ctx || !master || !rays || !act_max || n_leaves < 1)
    return fail(AMNERF_EINVAL, "amnerf_mlp_calibrate: bad argument");
  if (!ctx->have_render || ctx->last_rays != rays->n_rays || ctx->last_o != rays->o_dev)
    return fail(AMNERF_ESTATE, "amnerf_mlp_calibrate: the last render on this context used other rays");
  if (ctx->last_chunks != 1 || ctx->last_static || (ctx->last_params.flags & AMNERF_ERT_ROUNDS))
    return fail(AMNERF_ESTATE, "amnerf_mlp_calibrate: the last render ran in several chunks, in rounds or in the "
                "static workspace");
  if ((uint32_t)n_leaves != ctx->last_leaves)
    return fail(AMNERF_EINVAL, "amnerf_mlp_calibrate: %d parameter sets, the last render used %u", n_leaves,
                ctx->last_leaves);
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(launch_act_max(s->n_hidden, master, (uint32_t)n_leaves, ctx->bucket_off, ctx->tile_off, ctx->counts,
                         ctx->srec_ray, ctx->srec_t, rays->o_dev, rays->d_dev, rays->n_rays, 0, act_max,
                         (hipStream_t)stream));
  return AMNERF_OK;
}

extern "C" int amnerf_render_backward_inspect(amnerf_ctx* ctx, float* sample_grad_dev, void* stream) {
  if (!ctx || !sample_grad_dev) return fail(AMNERF_EINVAL, "amnerf_render_backward_inspect: null argument");
  if (!ctx->have_backward || !ctx->have_render)
    return fail(AMNERF_ESTATE, "amnerf_render_backward_inspect: no backward pass of the last render");
  int rc = read_counts(ctx);
  if (rc) return rc;
  const uint64_t ns = ctx->counts_host->n_smp;
  if (ns) HIP_TRY(hipMemcpyAsync(sample_grad_dev, ctx->last_gpre, 16 * ns, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return AMNERF_OK;
}

extern "C" int amnerf_error_stats(amnerf_ctx* ctx, const float* x, const double* ref, const uint8_t* sel, int64_t n,
                                  double out[4], void* stream) {
  if (!ctx || !out || n < 0 || (n > 0 && (!x || !ref))) return fail(AMNERF_EINVAL, "amnerf_error_stats: bad argument");
  HIP_TRY(hipSetDevice(ctx->device));
  if (!ctx->err_dev) {
    HIP_TRY(hipMalloc((void**)&ctx->err_dev, sizeof(double) * (4 * kErrBlocks + 4)));
    HIP_TRY(hipHostMalloc((void**)&ctx->err_host, sizeof(double) * 4, 0));
  }
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(launch_error_stats(x, ref, sel, n, ctx->err_dev, ctx->err_dev + 4 * kErrBlocks, st));
  HIP_TRY(hipMemcpyAsync(ctx->err_host, ctx->err_dev + 4 * kErrBlocks, sizeof(double) * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int i = 0; i < 4; ++i) out[i] = ctx->err_host[i];
  return AMNERF_OK;
}

extern "C" int amnerf_adam_step(amnerf_ctx* ctx, int64_t n, float* param, float* m, float* v, const float* grad,
                                const amnerf_adam_params* p, void* stream) {
  if (!ctx || !p || n < 0 || (n > 0 && (!param || !m || !v || !grad)))
    return fail(AMNERF_EINVAL, "amnerf_adam_step: bad argument");
  if (p->step < 1 || !(p->lr >= 0.f) || !(p->beta1 >= 0.f && p->beta1 < 1.f) || !(p->beta2 >= 0.f && p->beta2 < 1.f) ||
      !(p->eps > 0.f))
    return fail(AMNERF_EINVAL, "amnerf_adam_step: bad hyper-parameters");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(launch_adam(n, param, m, v, grad, p->lr, p->beta1, p->beta2, p->eps, p->step, (hipStream_t)stream));
  return AMNERF_OK;
}

extern "C" int amnerf_train_step(amnerf_ctx* ctx, const amnerf_tree* tree, amnerf_mlp_train* m,
                                 const amnerf_rays* rays, const float* target, const amnerf_train_params* p,
                                 float* loss, void* stream) {
  if (!ctx || !tree || !m || !rays || !p || !loss || (rays->n_rays > 0 && !target))
    return fail(AMNERF_EINVAL, "amnerf_train_step: null argument");
  if (!m->master_dev || !m->grad_dev || !m->m_dev || !m->v_dev || !m->packed_dev)
    return fail(AMNERF_EINVAL, "amnerf_train_step: null parameter buffer");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int32_t dtype = (p->flags & AMNERF_TRAIN_F32) ? AMNERF_F32 : AMNERF_BF16;
  amnerf_mlp mlp;
  mlp.shape = m->shape;
  mlp.dtype = dtype;
  mlp.n_leaves = m->n_leaves;
  mlp.packed_dev = m->packed_dev;
  const uint64_t R = (uint64_t)rays->n_rays;
  // outputs of the forward pass live in the second arena: size it before rendering
  BwdWork w;
  {
    const uint64_t L = (uint64_t)std::max(1, m->n_leaves);
    const uint64_t P = (uint64_t)amnerf_mlp_param_count(&m->shape);
    uint64_t chunk = std::max<uint64_t>(1, kChunkSamples / (uint64_t)std::max(1, p->render.s_max));
    if (R > chunk) return fail(AMNERF_ECAPACITY, "amnerf_train_step: %llu rays exceed one pass (%llu)",
                               (unsigned long long)R, (unsigned long long)chunk);
    const uint64_t ns = std::max<uint64_t>(R, 1) * (uint64_t)std::max(1, p->render.s_max);
    const uint64_t nseg = (ns / kMlpTileRows + L) / kSegTiles + L;
    int rc = ensure_arena2(ctx, carve_bwd(nullptr, ns, L, nseg, P, R, w));
    if (rc) return rc;
    carve_bwd((char*)ctx->arena2, ns, L, nseg, P, R, w);
  }
  amnerf_render_out out = {w.rgb, nullptr, nullptr, nullptr};
  int rc = amnerf_render(ctx, tree, &mlp, rays, &p->render, &out, stream);
  if (rc) return rc;
  BwdEvSet* ev = nullptr;
  if (ctx->timing) {
    rc = next_bwd_set(ctx, &ev);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(ev->ev[AMNERF_BWD_STAGE_COMPOSITE], st));
  }
  HIP_TRY(launch_loss_grad((uint32_t)R, w.rgb, target, w.g_rgb, w.loss_partial, loss, st));
  rc = backward_impl(ctx, tree, &mlp, rays, w.g_rgb, nullptr, nullptr, m->grad_dev, st, nullptr, true, ev);
  if (rc) return rc;
  if (!(p->flags & AMNERF_GRAD_ONLY)) {
    const int64_t n = (int64_t)m->n_leaves * amnerf_mlp_param_count(&m->shape);
    rc = amnerf_adam_step(ctx, n, m->master_dev, m->m_dev, m->v_dev, m->grad_dev, &p->adam, stream);
    if (rc) return rc;
    rc = amnerf_mlp_pack(ctx, &m->shape, dtype, m->n_leaves, m->master_dev, m->packed_dev, stream);
    if (rc) return rc;
  }
  if (ev) {
    HIP_TRY(hipEventRecord(ev->ev[kBwdStages], st));
    ev->no_adam = false;
    ev->pending = true;
  }
  return AMNERF_OK;
}

// ---------------------------------------------------------------------------------------
// distillation-driven subdivision (Section 3.4, TestLeaf)
// ---------------------------------------------------------------------------------------
namespace {

struct Distiller {
  amnerf_ctx* ctx = nullptr;
  const amnerf_testleaf_params* p = nullptr;
  int32_t dtype = AMNERF_BF16;
  int64_t P = 0;
  float *master = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr, *loss = nullptr, *rgb = nullptr;
  void* packed = nullptr;
  ~Distiller() {
    for (void* q : {(void*)master, (void*)grad, (void*)m, (void*)v, (void*)loss, (void*)rgb, packed})
      if (q) (void)hipFree(q);
  }
};

// PSNR of the evaluation rays after n_max distillation steps of one parameter set per leaf of
// `tree`, every set starting from the same initial parameters.
int distil_psnr(Distiller& D, const amnerf_tree* tree, double* psnr) {
  const amnerf_testleaf_params* p = D.p;
  const int32_t L = tree->n_leaves;
  const size_t bytes = (size_t)D.P * 4;
  const hipStream_t st = nullptr;
  // tile the initial set over the leaves by doubling copies
  HIP_TRY(hipMemcpyAsync(D.master, p->init_dev, bytes, hipMemcpyDeviceToDevice, st));
  for (int32_t have = 1; have < L;) {
    const int32_t k = std::min(have, L - have);
    HIP_TRY(hipMemcpyAsync(D.master + (size_t)have * D.P, D.master, bytes * k, hipMemcpyDeviceToDevice, st));
    have += k;
  }
  HIP_TRY(hipMemsetAsync(D.m, 0, bytes * L, st));
  HIP_TRY(hipMemsetAsync(D.v, 0, bytes * L, st));
  int rc = amnerf_mlp_pack(D.ctx, &p->student, D.dtype, L, D.master, D.packed, st);
  if (rc) return rc;
  amnerf_mlp_train mt;
  mt.shape = p->student;
  mt.n_leaves = L;
  mt.master_dev = D.master;
  mt.grad_dev = D.grad;
  mt.m_dev = D.m;
  mt.v_dev = D.v;
  mt.packed_dev = D.packed;
  for (int32_t s = 1; s <= p->n_max; ++s) {
    amnerf_train_params tp;
    tp.render = p->render;
    tp.adam.lr = p->lr;
    tp.adam.beta1 = 0.9f;
    tp.adam.beta2 = 0.999f;
    tp.adam.eps = 1e-8f;
    tp.adam.step = s;
    tp.flags = D.dtype == AMNERF_F32 ? AMNERF_TRAIN_F32 : 0u;
    const int32_t b = (s - 1) % p->n_batches;
    rc = amnerf_train_step(D.ctx, tree, &mt, &p->batches[b], p->targets[b], &tp, D.loss, st);
    if (rc) return rc;
  }
  amnerf_mlp mlp;
  mlp.shape = p->student;
  mlp.dtype = D.dtype;
  mlp.n_leaves = L;
  mlp.packed_dev = D.packed;
  amnerf_render_out ro = {D.rgb, nullptr, nullptr, nullptr};
  rc = amnerf_render(D.ctx, tree, &mlp, &p->eval, &p->render, &ro, st);
  if (rc) return rc;
  double e[4];
  rc = amnerf_error_stats(D.ctx, D.rgb, p->eval_target_dev, nullptr, 3 * (int64_t)p->eval.n_rays, e, st);
  if (rc) return rc;
  *psnr = e[1] > 0.0 ? 10.0 * std::log10(e[2] / e[1]) : INFINITY;
  return AMNERF_OK;
}

}  // namespace

extern "C" int amnerf_build_tree_distilled(amnerf_ctx* ctx, const float* grid, int32_t n, int32_t max_depth,
                                           int32_t max_leaves, const amnerf_testleaf_params* p, amnerf_tree** out,
                                           amnerf_testleaf_record* log, int32_t log_cap, int32_t* n_log) {
  const char* who = "amnerf_build_tree_distilled";
  if (!ctx || !grid || !p || !out || log_cap < 0 || (log_cap > 0 && !log))
    return fail(AMNERF_EINVAL, "%s: null argument", who);
  *out = nullptr;
  if (n_log) *n_log = 0;
  if (max_depth < 0 || max_depth > AMNERF_MAX_DEPTH || max_leaves < 1 || max_leaves > AMNERF_MAX_LEAVES)
    return fail(AMNERF_EINVAL, "%s: max_depth %d / max_leaves %d out of range", who, max_depth, max_leaves);
  const int64_t P = amnerf_mlp_param_count(&p->student);
  if (P <= 0) return fail(AMNERF_EINVAL, "%s: bad student shape", who);
  if (!mlp_bwd_supported(p->student.n_hidden, p->student.hidden))
    return fail(AMNERF_EINVAL, "%s: the student's backward needs n_hidden 1 .. 4 and hidden 32 or 64", who);
  if (!p->init_dev || p->n_max < 0 || (p->n_max > 0 && (p->n_batches < 1 || !p->batches || !p->targets)) ||
      !(p->lr >= 0.f) || !std::isfinite(p->gain_thresh) || p->eval.n_rays < 1 || !p->eval_target_dev)
    return fail(AMNERF_EINVAL, "%s: bad distillation parameters", who);
  if (p->render.proposal || p->render.occupancy || p->render.hcheck_footprint != 0.f)
    return fail(AMNERF_EINVAL, "%s: distillation renders take no proposal, occupancy or footprint", who);
  for (int32_t b = 0; b < (p->n_max > 0 ? p->n_batches : 0); ++b)
    if (!p->targets[b] || p->batches[b].n_rays < 1)
      return fail(AMNERF_EINVAL, "%s: batch %d is empty or has no targets", who, b);
  HIP_TRY(hipSetDevice(ctx->device));
  Distiller D;
  D.ctx = ctx;
  D.p = p;
  D.dtype = (p->flags & AMNERF_TESTLEAF_F32) ? AMNERF_F32 : AMNERF_BF16;
  D.P = P;
  size_t packed_bytes = 0;
  int rc = amnerf_mlp_packed_bytes(&p->student, D.dtype, max_leaves, &packed_bytes);
  if (rc) return rc;
  const size_t pb = (size_t)P * 4 * max_leaves;
  HIP_TRY(hipMalloc((void**)&D.master, pb));
  HIP_TRY(hipMalloc((void**)&D.grad, pb));
  HIP_TRY(hipMalloc((void**)&D.m, pb));
  HIP_TRY(hipMalloc((void**)&D.v, pb));
  HIP_TRY(hipMalloc((void**)&D.loss, 4));
  HIP_TRY(hipMalloc((void**)&D.rgb, 12 * (size_t)p->eval.n_rays));
  HIP_TRY(hipMalloc(&D.packed, packed_bytes));

  TreeBuild B;
  rc = tree_build_begin(grid, n, B, who);
  if (rc) return rc;
  amnerf_tree* current = nullptr;
  rc = tree_build_finish(ctx, B, &current, who);
  if (rc) return rc;
  double psnr_cur = 0.0;
  rc = distil_psnr(D, current, &psnr_cur);
  int32_t logged = 0;
  // BuildKDTree: the node, then its lower subtree, then its upper subtree (explicit stack)
  std::vector<uint32_t> todo = {1u};
  while (rc == AMNERF_OK && !todo.empty()) {
    const uint32_t code = todo.back();
    todo.pop_back();
    const int at = find_code(B, code);
    const HNode nd = B.nodes[at];
    if (nd.depth >= max_depth || !longest_side_splittable(nd) || B.leaves >= max_leaves) continue;
    const std::vector<HNode> saved = B.nodes;
    const int saved_leaves = B.leaves;
    tree_split(B, at, false);
    amnerf_tree* trial = nullptr;
    rc = tree_build_finish(ctx, B, &trial, who);
    if (rc) break;
    double psnr_t = 0.0;
    rc = distil_psnr(D, trial, &psnr_t);
    if (rc) {
      amnerf_tree_destroy(trial);
      break;
    }
    const bool kept = psnr_t - psnr_cur >= (double)p->gain_thresh * psnr_cur;
    if (logged < log_cap) {
      amnerf_testleaf_record& r = log[logged];
      r.code = code;
      r.depth = nd.depth;
      r.leaves_of_trial = B.leaves;
      r.kept = kept ? 1 : 0;
      r.psnr_current = psnr_cur;
      r.psnr_split = psnr_t;
    }
    ++logged;
    if (!kept) {
      amnerf_tree_destroy(trial);
      B.nodes = saved;
      B.leaves = saved_leaves;
      continue;
    }
    amnerf_tree_destroy(current);
    current = trial;
    psnr_cur = psnr_t;
    todo.push_back(2 * code + 1);
    todo.push_back(2 * code);
  }
  HIP_TRY(hipDeviceSynchronize());
  if (rc) {
    amnerf_tree_destroy(current);
    return rc;
  }
  if (n_log) *n_log = logged;
  *out = current;
  return AMNERF_OK;
}

// ---------------------------------------------------------------------------------------
// learned proposal
// ---------------------------------------------------------------------------------------
extern "C" int64_t amnerf_prop_param_count(void) { return prop_param_count(); }

extern "C" int amnerf_prop_packed_bytes(int32_t dtype, size_t* out) {
  if (!out || (dtype != AMNERF_F32 && dtype != AMNERF_BF16)) return fail(AMNERF_EINVAL, "amnerf_prop_packed_bytes: bad argument");
  *out = prop_packed_bytes(dtype);
  return AMNERF_OK;
}

extern "C" int amnerf_prop_pack(amnerf_ctx* ctx, int32_t dtype, const float* master, void* packed, void* stream) {
  if (!ctx || !master || !packed || (dtype != AMNERF_F32 && dtype != AMNERF_BF16))
    return fail(AMNERF_EINVAL, "amnerf_prop_pack: bad argument");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(launch_prop_pack(dtype, master, packed, (hipStream_t)stream));
  return AMNERF_OK;
}

namespace {
struct PropTrainWork {
  float *rgb, *tau, *alpha, *part, *loss_part;
};
size_t carve_prop_train(char* base, uint64_t R, uint64_t niv, uint64_t nb, PropTrainWork& w) {
  Carve c{base};
  w.rgb = c.take<float>(3 * std::max<uint64_t>(R, 1));
  w.tau = c.take<float>(32 * std::max<uint64_t>(niv, 1));
  w.alpha = c.take<float>(32 * std::max<uint64_t>(niv, 1));
  w.part = c.take<float>(nb * (uint64_t)prop_param_count());
  w.loss_part = c.take<float>(nb);
  return c.off + 256;
}
}  // namespace

extern "C" int amnerf_propose(amnerf_ctx* ctx, const amnerf_tree* tree, const amnerf_mlp* scene_mlp,
                              const amnerf_rays* rays, const amnerf_propose_params* p, int64_t* n_intervals,
                              void* stream) {
  if (!ctx || !tree || !scene_mlp || !rays || !p) return fail(AMNERF_EINVAL, "amnerf_propose: null argument");
  if (p->mode != AMNERF_PROPOSE_INFER && p->mode != AMNERF_PROPOSE_TRAIN)
    return fail(AMNERF_EINVAL, "amnerf_propose: bad mode %d", p->mode);
  if (p->mode == AMNERF_PROPOSE_TRAIN &&
      (!p->master_dev || !p->grad_dev || !p->m_dev || !p->v_dev || !p->packed_dev || !p->loss_dev))
    return fail(AMNERF_EINVAL, "amnerf_propose: null training buffer");
  if (p->mode == AMNERF_PROPOSE_INFER && (!p->infer_packed_dev || !p->tau_dev ||
                                          (p->infer_dtype != AMNERF_F32 && p->infer_dtype != AMNERF_BF16)))
    return fail(AMNERF_EINVAL, "amnerf_propose: bad inference arguments");
  if (p->s_max < 1 || p->s_max > AMNERF_MAX_SAMPLES)
    return fail(AMNERF_EINVAL, "amnerf_propose: s_max %d out of [1, %d]", p->s_max, AMNERF_MAX_SAMPLES);
  if (rays->n_rays < 0) return fail(AMNERF_EINVAL, "amnerf_propose: n_rays < 0");
  const uint64_t R = (uint64_t)rays->n_rays;
  if (R * (uint64_t)std::max(1, p->s_max) > kChunkSamples)
    return fail(AMNERF_ECAPACITY, "amnerf_propose: %llu rays x %d samples exceed one pass", (unsigned long long)R, p->s_max);
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  // a plain render of the rays provides the intervals (and, for training, the samples' sigma)
  uint32_t niv_guess = 0;
  {
    PropTrainWork tw;
    int rc = ensure_arena3(ctx, carve_prop_train(nullptr, R, 0, prop_train_blocks(), tw));
    if (rc) return rc;
    carve_prop_train((char*)ctx->arena3, R, 0, prop_train_blocks(), tw);
    amnerf_render_params rp = {};
    rp.s_max = p->s_max;
    rp.ert_eps = 0.f;
    amnerf_render_out out = {tw.rgb, nullptr, nullptr, nullptr};
    rc = amnerf_render(ctx, tree, scene_mlp, rays, &rp, &out, stream);
    if (rc) return rc;
    rc = read_counts(ctx);
    if (rc) return rc;
    niv_guess = ctx->counts_host->n_iv;
  }
  if (n_intervals) *n_intervals = niv_guess;
  PropTrainWork tw;
  const uint32_t nb = prop_train_blocks();
  // the render used the main arena only, so the third arena can be re-carved freely
  int rc = ensure_arena3(ctx, carve_prop_train(nullptr, R, niv_guess, nb, tw));
  if (rc) return rc;
  carve_prop_train((char*)ctx->arena3, R, niv_guess, nb, tw);
  const IvSet& iv = ctx->use;
  if (p->mode == AMNERF_PROPOSE_INFER) {
    if ((int64_t)niv_guess > p->tau_cap)
      return fail(AMNERF_ECAPACITY, "amnerf_propose: %u intervals exceed tau_cap %lld", niv_guess, (long long)p->tau_cap);
    HIP_TRY(launch_prop_fwd(p->infer_dtype, p->infer_packed_dev, iv, rays->o_dev, rays->d_dev, rays->n_rays, 0,
                            tree->dev_leafbox, p->s_max, niv_guess, false, p->tau_dev, nullptr, st));
    return AMNERF_OK;
  }
  HIP_TRY(launch_prop_targets(iv, ctx->smp_out, tw.alpha, st));
  HIP_TRY(launch_prop_train(p->packed_dev, iv, rays->o_dev, rays->d_dev, rays->n_rays, 0, tree->dev_leafbox, p->s_max,
                            tw.alpha, tw.part, tw.loss_part, p->grad_dev, p->loss_dev, st));
  rc = amnerf_adam_step(ctx, prop_param_count(), p->master_dev, p->m_dev, p->v_dev, p->grad_dev, &p->adam, stream);
  if (rc) return rc;
  HIP_TRY(launch_prop_pack(AMNERF_F32, p->master_dev, p->packed_dev, st));
  return AMNERF_OK;
}
