// Instantiation of the fused gather for element type float, output OUT_F16S.
#include "combine.hpp"

namespace rbc {
namespace comb {
template hipError_t gather_dispatch<float, OUT_F16S>(int, int, int, int, int, const GatherPair&, hipStream_t);
}  // namespace comb
}  // namespace rbc
