// Device parts of the per-leaf power-of-two scales of reduced-precision leaf
// operands (f16, e4m3), shared by the stand-alone kernels and the batch engine.
//
// A leaf operand S_l is a chain of folded combinations of blocks of A, so
// |S_l| <= G_l max|A| with G_l the product over levels of the 1-norm of the
// coefficient column used at that level (signs and permutations leave the
// norm unchanged).  The gather writes rn_f16(2^e_l S_l) with
// e_l = floor(log2(2^15 / (G_l max|A|))): no value can exceed 2^15 < 65504,
// and the leaf kernel multiplies its f32 result by 2^-(eS_l + eT_l), exactly.
// e4m3 operands use the bound 448 (the largest finite e4m3) in place of 2^15.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "devptr.hpp"

namespace rbc {
namespace scale {

// max |X| over rows [row0, row0 + nrows) of a row-major matrix with cols
// columns and row stride ld: this thread's share (256 threads stride along
// each row).
__device__ __forceinline__ float maxabs_rows(const float* __restrict__ X, int64_t ld, int64_t cols,
                                             int64_t row0, int64_t nrows) {
  const gbl<const float>* Xg = global_ptr(X);
  float m = 0.f;
  for (int64_t r = row0; r < row0 + nrows; ++r)
    for (int64_t c = threadIdx.x; c < cols; c += 256) m = fmaxf(m, fabsf(Xg[r * ld + c]));
  return m;
}

// Fold the threads' maxima into *out as the bits of a non-negative float
// (which order like unsigned integers): one atomic max per wavefront.
__device__ __forceinline__ void maxabs_fold(float m, uint32_t* out) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// e = floor(log2(target / (G mx))), clamped to [-120, 120]; 0 when the bound is 0.
// target: 2^15 for f16 operands, 448 for e4m3.
__device__ __forceinline__ int32_t leaf_exponent(float mx, float G, float target) {
  const float bound = G * mx;
  int ex = 0;
  if (bound > 0.f && isfinite(bound)) {
    int x;
    frexpf(target / bound, &x);  // target / bound = m 2^x, m in [0.5, 1)
    ex = x - 1;
    ex = ex < -120 ? -120 : (ex > 120 ? 120 : ex);
  }
  return ex;
}

}  // namespace scale
}  // namespace rbc
