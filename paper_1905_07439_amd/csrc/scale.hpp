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
// columns and row stride ld: this thread's share.  The 256 threads walk the
// rows' elements in 16-byte chunks when the layout allows (cols and ld
// multiples of 4, X 16-byte aligned), four independent loads per step so that
// several are in flight.
__device__ __forceinline__ float maxabs_rows(const float* __restrict__ X, int64_t ld, int64_t cols,
                                             int64_t row0, int64_t nrows) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const gbl<const float>* Xg = global_ptr(X);
  float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f;
  if (cols % 4 == 0 && ld % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0) {
    const int64_t c4 = cols / 4, n = nrows * c4;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
      f4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t j = i + 256 * u < n ? i + 256 * u : i;
        const int64_t r = j / c4, c = j - r * c4;
        v[u] = *reinterpret_cast<const gbl<const f4>*>(Xg + (row0 + r) * ld + 4 * c);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        m0 = fmaxf(m0, fabsf(v[u][0]));
        m1 = fmaxf(m1, fabsf(v[u][1]));
        m2 = fmaxf(m2, fabsf(v[u][2]));
        m3 = fmaxf(m3, fabsf(v[u][3]));
      }
    }
  } else {
    const int64_t n = nrows * cols;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
      const int64_t r = i / cols, c = i - r * cols;
      m0 = fmaxf(m0, fabsf(Xg[(row0 + r) * ld + c]));
    }
  }
  return fmaxf(fmaxf(m0, m1), fmaxf(m2, m3));
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
