// Instantiation of the range-search kernels for stride 8.
#include "search_range.hpp"

namespace knnx {
hipError_t launch_range_dp8(const RangeArgs &a, int lg, bool fill, int grid, hipStream_t s) {
    return launch_range<8>(a, lg, fill, grid, s);
}
}  // namespace knnx
