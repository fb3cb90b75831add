// Instantiation of the range-search kernels for stride 32.
#include "search_range.hpp"

namespace knnx {
hipError_t launch_range_dp32(const RangeArgs &a, int lg, bool fill, int grid, hipStream_t s) {
    return launch_range<32>(a, lg, fill, grid, s);
}
}  // namespace knnx
