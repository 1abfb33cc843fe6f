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

// max |x| over the n floats at p: this thread's share of a 256-thread
// workgroup.  A few scalar loads up to the first 16-byte boundary, then
// 16-byte chunks with eight independent loads in flight per thread, then the
// scalar tail.
__device__ __forceinline__ float maxabs_run(const gbl<const float>* p, int64_t n) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f;
  const int64_t head = (int64_t)(((16u - (uint32_t)(reinterpret_cast<uintptr_t>(p) & 15u)) & 15u) >> 2);
  const int64_t h = head < n ? head : n;
  const int tid = (int)threadIdx.x;
  if (tid < h) m0 = fabsf(p[tid]);
  const gbl<const f4>* q = reinterpret_cast<const gbl<const f4>*>(p + h);
  const int64_t n4 = (n - h) >> 2;
  int64_t i = tid;
  for (; i + 7 * 256 < n4; i += 8 * 256) {
    f4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = q[i + 256 * u];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      m0 = fmaxf(m0, fabsf(v[u][0]));
      m1 = fmaxf(m1, fabsf(v[u][1]));
      m2 = fmaxf(m2, fabsf(v[u][2]));
      m3 = fmaxf(m3, fabsf(v[u][3]));
    }
  }
  for (; i < n4; i += 256) {
    const f4 v = q[i];
    m0 = fmaxf(m0, fabsf(v[0]));
    m1 = fmaxf(m1, fabsf(v[1]));
    m2 = fmaxf(m2, fabsf(v[2]));
    m3 = fmaxf(m3, fabsf(v[3]));
  }
  const int64_t t = h + 4 * n4 + tid;  // at most 3 left
  if (t < n) m1 = fmaxf(m1, fabsf(p[t]));
  return fmaxf(fmaxf(m0, m1), fmaxf(m2, m3));
}

// max |X| over rows [row0, row0 + nrows) of a row-major matrix with cols
// columns and row stride ld: this thread's share (one run when the rows are
// contiguous, else one run per row).
__device__ __forceinline__ float maxabs_rows(const float* __restrict__ X, int64_t ld, int64_t cols,
                                             int64_t row0, int64_t nrows) {
  const gbl<const float>* Xg = global_ptr(X);
  if (nrows <= 0) return 0.f;
  if (ld == cols || nrows == 1) return maxabs_run(Xg + row0 * ld, nrows * cols);
  float m = 0.f;
  for (int64_t r = 0; r < nrows; ++r) m = fmaxf(m, maxabs_run(Xg + (row0 + r) * ld, cols));
  return m;
}

// The maximum of m over the 256 threads of the workgroup, returned to every
// thread; every thread must call it.
__device__ __forceinline__ float block_max(float m) {
  __shared__ float red[4];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  __syncthreads();  // a previous call's readers are done with red
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  return fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// Fold the workgroup's maximum into *out as the bits of a non-negative float
// (which order like unsigned integers): one atomic max per workgroup.
__device__ __forceinline__ void maxabs_fold(float m, uint32_t* out) {
  const float b = block_max(m);
  if (threadIdx.x == 0) atomicMax(out, __float_as_uint(b));
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
