// Instantiation of the fused gather for element type double, output OUT_SAME.
#include "combine.hpp"

namespace rbc {
namespace comb {
template hipError_t gather_dispatch<double, OUT_SAME>(int, int, int, int, int, const GatherPair&, hipStream_t);
}  // namespace comb
}  // namespace rbc
