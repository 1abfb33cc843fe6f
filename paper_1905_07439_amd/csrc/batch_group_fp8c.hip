// Level-synchronous batch kernels, fp8c leaves (batch_group.hpp).
#include "batch_group.hpp"

namespace rbc {
namespace batch {
hipError_t launch_group_fp8c(int kind, int variant, const GroupArgs& a, int64_t grid, hipStream_t s) {
  return launch_group_prec<RBC_PREC_FP8C>(kind, variant, a, grid, s);
}
}  // namespace batch
}  // namespace rbc
