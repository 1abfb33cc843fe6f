// Per-leaf power-of-two scales of the f16 leaf operands.
//
// A leaf operand S_l is a chain of folded combinations of blocks of A, so
// |S_l| <= G_l max|A| with G_l the product over levels of the 1-norm of the
// coefficient column used at that level (signs and permutations leave the
// norm unchanged).  The gather writes rn_f16(2^e_l S_l) with
// e_l = floor(log2(2^15 / (G_l max|A|))): no value can exceed 2^15 < 65504,
// and the leaf kernel multiplies its f32 result by 2^-(eS_l + eT_l), exactly.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace rbc {
namespace {

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// max |X| over a rows x cols row-major matrix, as the bits of a non-negative
// float (which order like unsigned integers), folded into *out by atomic max.
__global__ __launch_bounds__(256) void k_maxabs(const float* __restrict__ X, int64_t ld, int64_t rows,
                                                int64_t cols, uint32_t* out) {
  float m = 0.f;
  const int64_t total = rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int64_t r = i / cols, c = i - r * cols;
    m = fmaxf(m, fabsf(X[r * ld + c]));
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

__global__ void k_leaf_scales(const uint32_t* maxbits, const float* __restrict__ G, int32_t* e,
                              int64_t n) {
  const float mx = __uint_as_float(*maxbits);
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n; l += (int64_t)gridDim.x * blockDim.x) {
    const float bound = G[l] * mx;
    int ex = 0;
    if (bound > 0.f && isfinite(bound)) {
      int x;
      frexpf(32768.0f / bound, &x);  // 32768 / bound = m 2^x, m in [0.5, 1)
      ex = x - 1;
      ex = ex < -120 ? -120 : (ex > 120 ? 120 : ex);
    }
    e[l] = ex;
  }
}

}  // namespace

hipError_t launch_leaf_scales(const float* X, int64_t ld, int64_t rows, int64_t cols, uint32_t* maxbits,
                              const float* G, int32_t* e, int64_t n_leaves, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, maxbits, (int64_t)1, 0u);
  const int64_t total = rows * cols;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_maxabs, dim3((unsigned)blocks), dim3(256), 0, s, X, ld, rows, cols, maxbits);
  int64_t lb = (n_leaves + 255) / 256;
  if (lb > 1024) lb = 1024;
  hipLaunchKernelGGL(k_leaf_scales, dim3((unsigned)(lb < 1 ? 1 : lb)), dim3(256), 0, s, maxbits, G, e,
                     n_leaves);
  return hipGetLastError();
}

}  // namespace rbc
