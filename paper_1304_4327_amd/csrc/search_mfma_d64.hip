// Instantiation of the BF16 MFMA kernel for stride 64 (leaf sweep form).
#include "search_mfma_sweep.hpp"

namespace knnx {
hipError_t launch_search_mfma_dp64(const SearchArgs &a, int K, int grid, hipStream_t s) {
    return launch_search_mfma_sweep<64>(a, K, grid, s);
}
}  // namespace knnx
