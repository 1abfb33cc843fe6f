// Persistent batch kernel, f16 leaves with per-leaf power-of-two scales,
// and the precision dispatch of the batch kernel launchers.
#include "batch_kernel.hpp"

namespace rbc {
namespace batch {

hipError_t occupancy_f32(int* b);
hipError_t launch_f32(const KernelArgs& a, int grid, hipStream_t s);
hipError_t occupancy_fp8c(int* b);
hipError_t launch_fp8c(const KernelArgs& a, int grid, hipStream_t s);

hipError_t batch_occupancy(int prec, int* b) {
  if (prec == RBC_PREC_F32) return occupancy_f32(b);
  if (prec == RBC_PREC_F16S) return occupancy<RBC_PREC_F16S>(b);
  if (prec == RBC_PREC_FP8C) return occupancy_fp8c(b);
  return hipErrorInvalidValue;
}

hipError_t launch_zero_words(int32_t* p, int64_t n, hipStream_t s) {
  int64_t zb = (n + 255) / 256;
  if (zb > 1024) zb = 1024;
  if (zb < 1) zb = 1;
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)zb), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_batch(int prec, const KernelArgs& a, int grid, hipStream_t s) {
  if (prec == RBC_PREC_F32) return launch_f32(a, grid, s);
  if (prec == RBC_PREC_F16S) return launch<RBC_PREC_F16S>(a, grid, s);
  if (prec == RBC_PREC_FP8C) return launch_fp8c(a, grid, s);
  return hipErrorInvalidValue;
}

}  // namespace batch
}  // namespace rbc
