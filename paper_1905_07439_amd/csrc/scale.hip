// Per-leaf power-of-two scales of the reduced-precision leaf operands (the
// bound is explained in scale.hpp): partial maxima of |X|, one per workgroup;
// the gather that writes the leaf operands reduces them and derives the
// exponents (combine.hpp, load_exponents).
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "scale.hpp"

namespace rbc {
namespace {

struct MaxAbsSide {
  const float* X;
  int64_t ld, rows, cols;
  float* partial;
  int32_t blocks;  // workgroups of this side = partial maxima it writes
};

__device__ __forceinline__ void maxabs_side(const MaxAbsSide& p) {
  if ((int)blockIdx.x >= p.blocks) return;  // whole workgroup
  // a contiguous range of rows per workgroup, one partial maximum each
  const int64_t per = (p.rows + p.blocks - 1) / p.blocks;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t nr = r0 < p.rows ? (p.rows - r0 < per ? p.rows - r0 : per) : 0;
  const float m = scale::block_max(scale::maxabs_rows(p.X, p.ld, p.cols, r0, nr));
  if (threadIdx.x == 0) global_ptr(p.partial)[blockIdx.x] = m;
}

// One or two matrices (blockIdx.y selects the side, each branch reading its
// own argument in place; blocks past a side's count do nothing).
__global__ __launch_bounds__(256) void k_maxabs(MaxAbsSide a, MaxAbsSide b) {
  if (blockIdx.y == 0)
    maxabs_side(a);
  else
    maxabs_side(b);
}

MaxAbsSide side(const float* X, int64_t ld, int64_t rows, int64_t cols, float* partial) {
  return MaxAbsSide{X, ld, rows, cols, partial, maxabs_blocks(rows, cols)};
}

}  // namespace

hipError_t launch_maxabs(const float* X, int64_t ld, int64_t rows, int64_t cols, float* partial, hipStream_t s) {
  const MaxAbsSide a = side(X, ld, rows, cols, partial);
  hipLaunchKernelGGL(k_maxabs, dim3((unsigned)a.blocks, 1), dim3(256), 0, s, a, a);
  return hipGetLastError();
}

hipError_t launch_maxabs2(const float* XA, int64_t lda, int64_t ra, int64_t ca, float* pa, const float* XB,
                          int64_t ldb, int64_t rb, int64_t cb, float* pb, hipStream_t s) {
  const MaxAbsSide a = side(XA, lda, ra, ca, pa), b = side(XB, ldb, rb, cb, pb);
  hipLaunchKernelGGL(k_maxabs, dim3((unsigned)(a.blocks > b.blocks ? a.blocks : b.blocks), 2), dim3(256), 0, s, a,
                     b);
  return hipGetLastError();
}

}  // namespace rbc
