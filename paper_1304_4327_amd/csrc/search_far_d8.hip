// Instantiation of the k-furthest-neighbour kernel for stride 8.
#include "search_far.hpp"

namespace knnx {
hipError_t launch_search_far_dp8(const SearchArgs &a, int K, int grid, hipStream_t s) {
    return launch_search_far<8>(a, K, grid, s);
}
}  // namespace knnx
