// Persistent batch kernel, f32 leaves.
#include "batch_kernel.hpp"

namespace rbc {
namespace batch {
hipError_t occupancy_f32(int* b) { return occupancy<RBC_PREC_F32>(b); }
hipError_t launch_f32(const KernelArgs& a, int grid, hipStream_t s) { return launch<RBC_PREC_F32>(a, grid, s); }
}  // namespace batch
}  // namespace rbc
