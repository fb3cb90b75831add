// Instantiation of the k-furthest-neighbour kernel for stride 4.
#include "search_far.hpp"

namespace knnx {
hipError_t launch_search_far_dp4(const SearchArgs &a, int K, int grid, hipStream_t s) {
    return launch_search_far<4>(a, K, grid, s);
}
}  // namespace knnx
