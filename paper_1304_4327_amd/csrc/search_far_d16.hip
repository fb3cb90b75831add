// Instantiation of the k-furthest-neighbour kernel for stride 16.
#include "search_far.hpp"

namespace knnx {
hipError_t launch_search_far_dp16(const SearchArgs &a, int K, int grid, hipStream_t s) {
    return launch_search_far<16>(a, K, grid, s);
}
}  // namespace knnx
