// Instantiation of the range-search kernels for stride 16.
#include "search_range.hpp"

namespace knnx {
hipError_t launch_range_dp16(const RangeArgs &a, int lg, bool fill, int grid, hipStream_t s) {
    return launch_range<16>(a, lg, fill, grid, s);
}
}  // namespace knnx
