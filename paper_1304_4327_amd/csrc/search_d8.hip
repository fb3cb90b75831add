// Instantiation of the FP32 traversal kernel for 8 computed dimensions
// (searches without a seed; the seeded kernels are in search_seeded_d8.hip).
#include "search_valu.hpp"

namespace knnx {
hipError_t launch_search_valu_d8(const SearchArgs &a, int K, int grid, hipStream_t s) {
    if (a.seed) return launch_search_valu_seeded_d8(a, K, grid, s);
    return launch_search_valu<8>(a, K, grid, s);
}
}  // namespace knnx
