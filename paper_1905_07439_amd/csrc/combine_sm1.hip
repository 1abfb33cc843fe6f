// Instantiation of the fused scatter: products float, accumulation double, output double.
#include "combine.hpp"

namespace rbc {
namespace comb {
template hipError_t scatter_dispatch<float, double, double>(int, int, int, int, int, const ScatterParams&, hipStream_t);
}  // namespace comb
}  // namespace rbc
