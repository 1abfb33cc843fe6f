// Instantiation of the fused scatter: products double, accumulation double, output double.
#include "combine.hpp"

namespace rbc {
namespace comb {
template hipError_t scatter_dispatch<double, double, double>(int, int, int, int, int, const ScatterParams&, hipStream_t);
}  // namespace comb
}  // namespace rbc
