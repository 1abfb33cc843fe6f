// Per-leaf power-of-two scales of the reduced-precision leaf operands (the
// bound is explained in scale.hpp): max|X|, then one exponent per leaf.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "scale.hpp"

namespace rbc {
namespace {

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ __launch_bounds__(256) void k_maxabs(const float* __restrict__ X, int64_t ld, int64_t rows,
                                                int64_t cols, uint32_t* out) {
  // a contiguous range of rows per block
  const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t nr = r0 < rows ? (rows - r0 < per ? rows - r0 : per) : 0;
  scale::maxabs_fold(scale::maxabs_rows(X, ld, cols, r0, nr), out);
}

__global__ void k_leaf_scales(const uint32_t* maxbits, const float* __restrict__ G, int32_t* e,
                              int64_t n, float target) {
  const float mx = __uint_as_float(*maxbits);
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n; l += (int64_t)gridDim.x * blockDim.x)
    e[l] = scale::leaf_exponent(mx, G[l], target);
}

}  // namespace

hipError_t launch_leaf_scales(const float* X, int64_t ld, int64_t rows, int64_t cols, uint32_t* maxbits,
                              const float* G, int32_t* e, int64_t n_leaves, float target, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, maxbits, (int64_t)1, 0u);
  // about 16 KB of X per block, at most 2048 blocks
  int64_t blocks = (rows * cols + 4095) / 4096;
  if (blocks > 2048) blocks = 2048;
  if (blocks > rows) blocks = rows;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_maxabs, dim3((unsigned)blocks), dim3(256), 0, s, X, ld, rows, cols, maxbits);
  int64_t lb = (n_leaves + 255) / 256;
  if (lb > 1024) lb = 1024;
  hipLaunchKernelGGL(k_leaf_scales, dim3((unsigned)(lb < 1 ? 1 : lb)), dim3(256), 0, s, maxbits, G, e,
                     n_leaves, target);
  return hipGetLastError();
}

}  // namespace rbc
