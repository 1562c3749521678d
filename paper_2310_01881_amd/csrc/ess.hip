// ess.hip -- empty-space skipping with an occupancy bit grid: per ray, the mask of plain
// sample slots whose centred sample lies in an occupied cell.  The kept slots are then
// emitted as runs of consecutive slots (the same planned-interval form the proposal
// produces), so only they are sorted, evaluated and composited; a dropped sample's density
// counts as 0.
#include "internal.hpp"
#include "devcommon.hpp"

namespace amn {
namespace {

constexpr int kThreads = 256;

// One lane per ray.  Slot s = k * n + j (interval k, sample j) is bit s % 64 of mask word
// s / 64; the sample sits at the interval's centred stratum position, as the expansion
// places it.
__global__ __launch_bounds__(kThreads) void k_occ_select(uint32_t nr, IvSet iv, const float* __restrict__ o,
                                                         const float* __restrict__ d, int64_t stride, int64_t r0,
                                                         const uint32_t* __restrict__ bits, int g,
                                                         uint32_t* __restrict__ runs, uint32_t* __restrict__ nsel,
                                                         uint64_t* __restrict__ mask) {
  const uint32_t r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= nr) return;
  const uint32_t i0 = iv.iv_off[r], meff = iv.iv_off[r + 1] - i0;
  uint64_t* mw = mask + 4 * (uint64_t)r;
  if (meff == 0) {
    runs[r] = 0u;
    nsel[r] = 0u;
    for (int q = 0; q < 4; ++q) mw[q] = 0ull;
    return;
  }
  const uint32_t ns = iv.smp_off[r + 1] - iv.smp_off[r];
  const uint32_t n = ns / meff;
  float oo[3], dd[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    oo[a] = o[a * stride + r0 + r];
    dd[a] = d[a * stride + r0 + r];
  }
  const float G = (float)g, gmax = (float)(g - 1);
  uint32_t kept = 0, nrun = 0, s = 0, q = 0;
  uint64_t cur = 0ull;
  bool prev = false;
  // interval by interval; inside an interval the slots go in groups of 8 whose occupancy
  // words are loaded together (slots past the interval's end re-read its last slot and
  // are masked off)
  constexpr uint32_t kGroup = 8;
  for (uint32_t k = 0; k < meff; ++k) {
    const float t0 = iv.t0[i0 + k];
    const float delta = iv.dt[i0 + k] / (float)n;
    for (uint32_t j0 = 0; j0 < n; j0 += kGroup) {
      uint32_t word[kGroup], sh[kGroup];
#pragma unroll
      for (uint32_t e = 0; e < kGroup; ++e) {
        const uint32_t j = j0 + e < n ? j0 + e : n - 1u;
        const float t = sample_t(t0, delta, j, 0.5f);
        uint32_t c[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float x = fmaf(t, dd[a], oo[a]);
          c[a] = (uint32_t)fminf(fmaxf(floorf(x * G), 0.f), gmax);   // NaN -> 0
        }
        const uint32_t idx = c[0] + (uint32_t)g * (c[1] + (uint32_t)g * c[2]);
        word[e] = bits[idx >> 5];
        sh[e] = idx & 31u;
      }
#pragma unroll
      for (uint32_t e = 0; e < kGroup; ++e) {
        if (j0 + e >= n) break;
        const bool occ = (word[e] >> sh[e]) & 1u;
        cur |= (uint64_t)occ << (s & 63u);
        kept += occ;
        // a kept slot starts a run unless its left neighbour in the same interval is kept
        nrun += occ && (j0 + e == 0u || !prev);
        prev = occ;
        ++s;
        if ((s & 63u) == 0u) {
          mw[q++] = cur;
          cur = 0ull;
        }
      }
    }
  }
  if (s & 63u) mw[q++] = cur;
  for (; q < 4; ++q) mw[q] = 0ull;
  runs[r] = nrun;
  nsel[r] = kept;
}

}  // namespace

hipError_t launch_occ_select(uint32_t nr, const IvSet& iv, const float* o, const float* d, int64_t stride, int64_t r0,
                             const uint32_t* bits, int g, uint32_t* runs, uint32_t* nsel, uint64_t* mask,
                             hipStream_t st) {
  if (nr == 0) return hipSuccess;
  hipLaunchKernelGGL(k_occ_select, dim3((nr + kThreads - 1) / kThreads), dim3(kThreads), 0, st, nr, iv, o, d, stride,
                     r0, bits, g, runs, nsel, mask);
  return hipGetLastError();
}

}  // namespace amn
