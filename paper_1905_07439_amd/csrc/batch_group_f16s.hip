// Level-synchronous batch kernels, f16s leaves (batch_group.hpp).
#include "batch_group.hpp"

namespace rbc {
namespace batch {
hipError_t launch_group_f16s(int kind, int variant, const GroupArgs& a, int64_t grid, hipStream_t s) {
  return launch_group_prec<RBC_PREC_F16S>(kind, variant, a, grid, s);
}
}  // namespace batch
}  // namespace rbc
