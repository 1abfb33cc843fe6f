// Persistent batch kernel, fp8 leaves with one correction pass.
#include "batch_kernel.hpp"

namespace rbc {
namespace batch {
hipError_t occupancy_fp8c(int* b) { return occupancy<RBC_PREC_FP8C>(b); }
hipError_t launch_fp8c(const KernelArgs& a, int grid, hipStream_t s) { return launch<RBC_PREC_FP8C>(a, grid, s); }
}  // namespace batch
}  // namespace rbc
