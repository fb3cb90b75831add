// Instantiation of the traversal kernel with BF16 matrix-core BaseCase tiles
// for 16 computed dimensions (two query leaves per wave, lists of up to 16),
// plain and seeded.
#include "search_valu.hpp"

namespace knnx {
hipError_t launch_search_mt_d16(const SearchArgs &a, int K, int grid, hipStream_t s) {
    return a.seed ? launch_search_valu_mt<16, kValuSeeded>(a, K, grid, s)
                  : launch_search_valu_mt<16, kValuPlain>(a, K, grid, s);
}
}  // namespace knnx
