// Instantiation of the k-furthest-neighbour kernel for stride 64.
#include "search_far.hpp"

namespace knnx {
hipError_t launch_search_far_dp64(const SearchArgs &a, int K, int grid, hipStream_t s) {
    return launch_search_far<64>(a, K, grid, s);
}
}  // namespace knnx
