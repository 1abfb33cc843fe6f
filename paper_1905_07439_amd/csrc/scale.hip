// Per-leaf power-of-two scales of the reduced-precision leaf operands (the
// bound is explained in scale.hpp): partial maxima of |X|, one per workgroup;
// the gather that writes the leaf operands reduces them and derives the
// exponents (combine.hpp, load_exponents).
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

}  // namespace

hipError_t launch_maxabs(const float* X, int64_t ld, int64_t rows, int64_t cols, float* partial, hipStream_t s) {
  const int blocks = maxabs_blocks(rows, cols);
  hipLaunchKernelGGL(k_maxabs, dim3((unsigned)blocks), dim3(256), 0, s, X, ld, rows, cols, partial);
  return hipGetLastError();
}

}  // namespace rbc
