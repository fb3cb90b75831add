// Instantiation of the FP32 traversal kernel for 1 computed dimension
// (searches without a seed; the seeded kernels are in search_seeded_d1.hip).
#include "search_valu.hpp"

namespace knnx {
hipError_t launch_search_valu_d1(const SearchArgs &a, int K, int grid, hipStream_t s) {
    if (a.seed) return launch_search_valu_seeded_d1(a, K, grid, s);
    return launch_search_valu<1>(a, K, grid, s);
}
}  // namespace knnx
