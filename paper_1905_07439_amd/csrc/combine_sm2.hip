// Instantiation of the fused scatter: products float, accumulation double, output float.
#include "combine.hpp"

namespace rbc {
namespace comb {
template hipError_t scatter_dispatch<float, double, float>(int, int, int, int, int, const ScatterParams&, hipStream_t);
}  // namespace comb
}  // namespace rbc
