// Per-leaf power-of-two scales of the reduced-precision leaf operands (the
// bound is explained in scale.hpp): partial maxima of |X| per workgroup, then
// their maximum and one exponent per leaf.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "scale.hpp"

namespace rbc {
namespace {

__global__ __launch_bounds__(256) void k_maxabs(const float* __restrict__ X, int64_t ld, int64_t rows,
                                                int64_t cols, float* __restrict__ partial) {
  // a contiguous range of rows per workgroup, one partial maximum each
  const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t nr = r0 < rows ? (rows - r0 < per ? rows - r0 : per) : 0;
  const float m = scale::block_max(scale::maxabs_rows(X, ld, cols, r0, nr));
  if (threadIdx.x == 0) global_ptr(partial)[blockIdx.x] = m;
}

__global__ __launch_bounds__(256) void k_leaf_scales(const float* __restrict__ partial, int nparts,
                                                     const float* __restrict__ G, int32_t* e, int64_t n,
                                                     float target) {
  float m = 0.f;
  for (int i = threadIdx.x; i < nparts; i += 256) m = fmaxf(m, global_ptr(partial)[i]);
  const float mx = scale::block_max(m);
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n; l += (int64_t)gridDim.x * blockDim.x)
    e[l] = scale::leaf_exponent(mx, G[l], target);
}

}  // namespace

hipError_t launch_leaf_scales(const float* X, int64_t ld, int64_t rows, int64_t cols, float* partial,
                              const float* G, int32_t* e, int64_t n_leaves, float target, hipStream_t s) {
  // at least 32 KB of X per workgroup, at most kScalePartials workgroups
  int64_t blocks = (rows * cols + 8191) / 8192;
  if (blocks > kScalePartials) blocks = kScalePartials;
  if (blocks > rows) blocks = rows;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_maxabs, dim3((unsigned)blocks), dim3(256), 0, s, X, ld, rows, cols, partial);
  int64_t lb = (n_leaves + 255) / 256;
  if (lb > 1024) lb = 1024;
  hipLaunchKernelGGL(k_leaf_scales, dim3((unsigned)(lb < 1 ? 1 : lb)), dim3(256), 0, s, partial, (int)blocks, G,
                     e, n_leaves, target);
  return hipGetLastError();
}

}  // namespace rbc
