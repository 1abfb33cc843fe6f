// Averages of several products (the error-of-average quantity, Section 3):
// an f64 accumulator that adds one product at a time, elementwise, in the
// order the products are given, then one scaling by 1/K.  The same
// accumulator with a weight per product forms the approximate-to-exact
// combination sum_i alpha_i Y(eps_i) (Section 1, eq. APA-to-EBC).
#include <hip/hip_runtime.h>

#include "devptr.hpp"
#include "kernels.hpp"

namespace rbc {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_accumulate(double* __restrict__ acc, const T* __restrict__ x,
                                                    int64_t rows, int64_t cols, int64_t ldx, double w, int first) {
  gbl<double>* a = global_ptr(acc);
  const gbl<const T>* xs = global_ptr(x);
  const int64_t n = rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int64_t r = i / cols, c = i - r * cols;
    const double v = w * (double)xs[r * ldx + c];  // w = 1 for averages: exact
    a[i] = first ? v : a[i] + v;
  }
}

__global__ __launch_bounds__(256) void k_scale(double* __restrict__ acc, int64_t n, double s) {
  gbl<double>* a = global_ptr(acc);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) a[i] *= s;
}

unsigned blocks_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

}  // namespace

hipError_t launch_accumulate(double* acc, const void* x, Elt elt, int64_t rows, int64_t cols, int64_t ldx,
                             int first, hipStream_t s, double weight) {
  if (rows * cols == 0) return hipSuccess;
  const unsigned g = blocks_for(rows * cols);
  if (elt == ELT_F64)
    hipLaunchKernelGGL(k_accumulate<double>, dim3(g), dim3(256), 0, s, acc, static_cast<const double*>(x), rows,
                       cols, ldx, weight, first);
  else
    hipLaunchKernelGGL(k_accumulate<float>, dim3(g), dim3(256), 0, s, acc, static_cast<const float*>(x), rows,
                       cols, ldx, weight, first);
  return hipGetLastError();
}

hipError_t launch_scale_f64(double* acc, int64_t n, double scale, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(256), 0, s, acc, n, scale);
  return hipGetLastError();
}

}  // namespace rbc
