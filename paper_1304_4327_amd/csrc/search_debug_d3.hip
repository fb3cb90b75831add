// The d = 3 FP32 traversal kernel in its debug form: every Score call is
// logged with the bound of each query leaf of the wave, and the walk can
// take the farther child first.  Used by knn_debug_search_log to check the
// correctness argument of the k-NN Score (the bound never falls below a
// leaf's largest true k-th distance, and a pruned node holds no true
// neighbour) and the independence of the answer from the visit order.
#include "search_valu.hpp"

namespace knnx {
hipError_t launch_search_valu_debug_d3(const SearchArgs &a, int K, int grid, hipStream_t s) {
    switch (K) {
        case 4: return launch_search_valu_k<3, 4, kValuDebug>(a, grid, s);
        case 5: return launch_search_valu_k<3, 5, kValuDebug>(a, grid, s);
        case 8: return launch_search_valu_k<3, 8, kValuDebug>(a, grid, s);
        case 10: return launch_search_valu_k<3, 10, kValuDebug>(a, grid, s);
        case 11: return launch_search_valu_k<3, 11, kValuDebug>(a, grid, s);
        case 16: return launch_search_valu_k<3, 16, kValuDebug>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace knnx
