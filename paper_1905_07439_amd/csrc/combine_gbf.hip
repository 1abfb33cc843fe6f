// Instantiation of the fused gather for element type float, output OUT_BF16X2.
#include "combine.hpp"

namespace rbc {
namespace comb {
template hipError_t gather_dispatch<float, OUT_BF16X2>(int, int, int, int, int, const GatherPair&, hipStream_t);
}  // namespace comb
}  // namespace rbc
