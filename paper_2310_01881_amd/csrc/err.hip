// err.hip -- float64 error report of a float32 result against float64 reference values
// (Section 4: quality is reported as PSNR against ground truth): max |x - ref|, sum of
// (x - ref)^2, count and sum |x - ref| over the selected elements.
//
// Deterministic: a fixed grid, each thread a fixed strided subset, fixed-order tree
// reductions inside a block, and the block partials reduced in block order.
#include "internal.hpp"

namespace amn {
namespace {

constexpr int kThreads = 256;
constexpr int kBlocks = kErrBlocks;

struct Acc {
  double mx, sq, cnt, ab;
};

__device__ __forceinline__ Acc merge(Acc a, Acc b) { return {fmax(a.mx, b.mx), a.sq + b.sq, a.cnt + b.cnt, a.ab + b.ab}; }

__device__ Acc block_reduce(Acc v) {
  __shared__ double s[4][kThreads];
  const int t = threadIdx.x;
  s[0][t] = v.mx; s[1][t] = v.sq; s[2][t] = v.cnt; s[3][t] = v.ab;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (t < w) {
      s[0][t] = fmax(s[0][t], s[0][t + w]);
      s[1][t] += s[1][t + w];
      s[2][t] += s[2][t + w];
      s[3][t] += s[3][t + w];
    }
    __syncthreads();
  }
  return {s[0][0], s[1][0], s[2][0], s[3][0]};
}

__global__ __launch_bounds__(kThreads) void k_err_partial(const float* __restrict__ x, const double* __restrict__ ref,
                                                          const uint8_t* __restrict__ sel, int64_t n,
                                                          double* __restrict__ part) {
  Acc a = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)kBlocks * kThreads) {
    if (sel && !sel[i]) continue;
    const double e = (double)x[i] - ref[i];
    const double ae = fabs(e);
    a.mx = fmax(a.mx, ae != ae ? __builtin_inf() : ae);   // a NaN difference counts as infinite
    a.sq += e * e;
    a.cnt += 1.0;
    a.ab += ae;
  }
  a = block_reduce(a);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x + 0] = a.mx;
    part[4 * blockIdx.x + 1] = a.sq;
    part[4 * blockIdx.x + 2] = a.cnt;
    part[4 * blockIdx.x + 3] = a.ab;
  }
}

__global__ __launch_bounds__(kThreads) void k_err_final(const double* __restrict__ part, double* __restrict__ out) {
  Acc a = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < kBlocks; b += kThreads)
    a = merge(a, {part[4 * b], part[4 * b + 1], part[4 * b + 2], part[4 * b + 3]});
  a = block_reduce(a);
  if (threadIdx.x == 0) {
    out[0] = a.mx;
    out[1] = a.sq;
    out[2] = a.cnt;
    out[3] = a.ab;
  }
}

}  // namespace

hipError_t launch_error_stats(const float* x, const double* ref, const uint8_t* sel, int64_t n, double* part,
                              double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_err_partial, dim3(kBlocks), dim3(kThreads), 0, st, x, ref, sel, n, part);
  hipLaunchKernelGGL(k_err_final, dim3(1), dim3(kThreads), 0, st, (const double*)part, out);
  return hipGetLastError();
}

}  // namespace amn
