// Instantiation of the FP32 traversal kernel for 16 computed dimensions,
// searches with a seed radius (second pass in the same launch).
#include "search_valu.hpp"

namespace knnx {
hipError_t launch_search_valu_seeded_d16(const SearchArgs &a, int K, int grid, hipStream_t s) {
    return launch_search_valu<16, kValuSeeded>(a, K, grid, s);
}
}  // namespace knnx
