// Instantiation of the BF16 MFMA traversal kernel for stride 16.
#include "search_mfma.hpp"

namespace knnx {
hipError_t launch_search_mfma_dp16(const SearchArgs &a, int K, int grid, hipStream_t s) {
    return launch_search_mfma<16>(a, K, grid, s);
}
}  // namespace knnx
