// Precision dispatch of the level-synchronous batch launches.
#include "batch_group.hpp"

namespace rbc {
namespace batch {

hipError_t launch_group_f32(int kind, int variant, const GroupArgs& a, int64_t grid, hipStream_t s);
hipError_t launch_group_f16s(int kind, int variant, const GroupArgs& a, int64_t grid, hipStream_t s);
hipError_t launch_group_fp8c(int kind, int variant, const GroupArgs& a, int64_t grid, hipStream_t s);

hipError_t launch_group(int prec, int kind, int variant, const Task* tasks, const void* pieces,
                        const GatherParams* gather, const ScatterParams* scatter, const LeafDesc* leaf,
                        const ScaleDesc* scale, int64_t grid, hipStream_t s) {
  GroupArgs a{tasks, static_cast<const PieceRef*>(pieces), gather, scatter, leaf, scale};
  if (prec == RBC_PREC_F32) return launch_group_f32(kind, variant, a, grid, s);
  if (prec == RBC_PREC_F16S) return launch_group_f16s(kind, variant, a, grid, s);
  if (prec == RBC_PREC_FP8C) return launch_group_fp8c(kind, variant, a, grid, s);
  return hipErrorInvalidValue;
}

}  // namespace batch
}  // namespace rbc
