// The pruning dual-tree traversal's reference-side walk (Algorithm 1 with a
// query node fixed per wavefront), shared by the range-search, kernel
// density and Boruvka kernels: a depth-first walk over the heap-ordered
// reference tree without a stack.  One bit per depth records which child
// was entered first; when the walk climbs back to that child, the other one
// is scored (bounds only change monotonically, so the late score can only
// prune more).  Every (query node, reference node) pair is scored at most
// once, and a pruned node's subtree is never entered.
//
// score(node, key) -> bool : Score() of a reference node, wave-uniform;
//                            key is a wave-uniform order key
// leaf(node)               : BaseCase() over a kept reference leaf
// right_first(k0, k1)      : whether to enter the right child first when
//                            both are kept
// The leaf call sits in the outer loop and the walk in the inner one, so the
// state leaf() updates is not carried through the walk's loop.
#pragma once

#include "search_valu.hpp"

namespace knnx {

template <class Score, class Leaf, class Order>
__device__ __forceinline__ void tree_walk(int first_leaf, Score &&score, Leaf &&leaf,
                                          Order &&right_first) {
    float m0, m1;
    int node = 0, depth = 0;
    uint64_t firstbits = 0;
    bool down = score(0, m0);
    if (!down) return;
    for (;;) {
        bool at_leaf = false;
        for (;;) {
            if (down) {
                if (node >= first_leaf) {
                    at_leaf = true;
                    break;
                }
                const int c0 = 2 * node + 1, c1 = c0 + 1;
                const bool k0 = score(c0, m0);
                const bool k1 = score(c1, m1);
                if (!k0 && !k1) {
                    down = false;
                    continue;
                }
                const bool right = k1 && (!k0 || right_first(m0, m1));
                if (right)
                    firstbits |= (uint64_t(1) << depth);
                else
                    firstbits &= ~(uint64_t(1) << depth);
                node = uniform_i(right ? c1 : c0);
                ++depth;
            } else {
                if (node == 0) break;
                --depth;
                const bool is_right = (node & 1) == 0;
                const bool first_right = (firstbits >> depth) & 1;
                if (is_right == first_right) {
                    const int other = is_right ? node - 1 : node + 1;
                    if (score(other, m0)) {
                        node = other;
                        ++depth;
                        down = true;
                        continue;
                    }
                }
                node = uniform_i((node - 1) >> 1);
            }
        }
        if (!at_leaf) break;
        leaf(node);
        down = false;
    }
}

// The same walk with every node scored exactly once (when its parent is
// expanded): the decision for the second child is remembered per depth
// instead of scored again on the way back.  For rules whose Score has an
// effect (kernel density's approximation adds a contribution).
template <class Score, class Leaf, class Order>
__device__ __forceinline__ void tree_walk_once(int first_leaf, Score &&score, Leaf &&leaf,
                                               Order &&right_first) {
    float m0, m1;
    if (!score(0, m0)) return;
    int node = 0, depth = 0;
    uint64_t firstbits = 0, secondbits = 0;
    bool down = true;
    for (;;) {
        bool at_leaf = false;
        for (;;) {
            if (down) {
                if (node >= first_leaf) {
                    at_leaf = true;
                    break;
                }
                const int c0 = 2 * node + 1, c1 = c0 + 1;
                const bool k0 = score(c0, m0);
                const bool k1 = score(c1, m1);
                if (!k0 && !k1) {
                    down = false;
                    continue;
                }
                const bool right = k1 && (!k0 || right_first(m0, m1));
                const bool second = right ? k0 : k1;
                const uint64_t bit = uint64_t(1) << depth;
                firstbits = right ? (firstbits | bit) : (firstbits & ~bit);
                secondbits = second ? (secondbits | bit) : (secondbits & ~bit);
                node = uniform_i(right ? c1 : c0);
                ++depth;
            } else {
                if (node == 0) break;
                --depth;
                const bool is_right = (node & 1) == 0;
                const bool first_right = (firstbits >> depth) & 1;
                if (is_right == first_right && ((secondbits >> depth) & 1)) {
                    node = uniform_i(is_right ? node - 1 : node + 1);
                    ++depth;
                    down = true;
                    continue;
                }
                node = uniform_i((node - 1) >> 1);
            }
        }
        if (!at_leaf) break;
        leaf(node);
        down = false;
    }
}

// squared distance from a point to a box: nearest (gap) and farthest point
template <int DP>
__device__ __forceinline__ void box_dist2(const float (&q)[DP], const float *b, float &dmin2,
                                          float &dmax2) {
    float lo2 = 0.f, hi2 = 0.f;
#pragma unroll
    for (int j = 0; j < DP; ++j) {
        const float lo = b[j], hi = b[DP + j];
        const float g = fmaxf(fmaxf(lo - q[j], q[j] - hi), 0.0f);
        const float f = fmaxf(fmaxf(q[j] - lo, hi - q[j]), 0.0f);
        lo2 = fmaf(g, g, lo2);
        hi2 = fmaf(f, f, hi2);
    }
    dmin2 = lo2;
    dmax2 = hi2;
}

// FP64 squared distance of FP32 coordinates with every product rounded
// (no fused multiply-add), summed in dimension order: bit for bit the value
// of a plain sequential FP64 loop, so a decision taken on it matches one
// taken by such a loop (padding dimensions add exact zeros)
template <int DP>
__device__ __forceinline__ double d2_fp64_unfused(const float (&q)[DP], const float *r) {
#pragma clang fp contract(off)
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < DP; ++j) {
        const double t = (double)q[j] - (double)r[j];
        s = s + t * t;
    }
    return s;
}

}  // namespace knnx
