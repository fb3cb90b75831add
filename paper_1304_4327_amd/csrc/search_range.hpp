// Range-search kernel (Section "Range Search", Algorithms 5 and 6): for every
// query point every reference point at a distance in [lo, hi].
//
// Mapping as in the k-NN kernel: a wavefront owns 64 / 2^LG consecutive
// query leaves (lane = query point) and walks the reference tree
// (tree_walk).  Score treats each query point as a singleton node: the lane
// keeps a reference node unless its box lies entirely nearer than lo or
// entirely farther than hi (d_max < lo or d_min > hi; the printed test on
// d_min alone would drop overlapping nodes whose farther points are in
// range), with a 2^-16 relative slack for FP32 rounding.  BaseCase filters
// with FP32 squared distances (a relative slack covers their rounding) and
// decides every surviving pair exactly in FP64: lo^2 <= s <= hi^2, with s the
// FP64 squared distance of the FP32 inputs (products rounded, summed in
// dimension order) and lo^2, hi^2 squared in FP64 -- the same decision, bit
// for bit, as a plain FP64 loop over the dimensions.
//
// Two passes over the same traversal: the count pass writes each query's
// number of neighbours (original row order); after an exclusive scan of the
// counts the fill pass writes each query's neighbours from its offset on,
// in the order the traversal meets them (the paper's lists are unordered).
#pragma once

#include "walk.hpp"

namespace knnx {

struct RangeArgs {
    const float *rpts, *rbox, *rlpts;
    const int32_t *rperm;
    const int2 *rrange;
    int r_leaf_slots, r_first_leaf;
    const float *qpts, *qbox;
    const int32_t *qperm;
    const int2 *qrange;
    int q_first_leaf, q_n_leaves;
    double lo2, hi2;      // exact decision
    float s_lo, s_hi;     // Score thresholds on squared distances (with slack)
    float t_lo, t_hi;     // BaseCase FP32 filter thresholds (with slack)
    int prune, self;
    int64_t *counts;         // count pass: per original query row
    const int64_t *offsets;  // fill pass: exclusive prefix sums of the counts
    int64_t *out_idx;
    float *out_dist;
    unsigned long long *stats;  // ST_SCORE, ST_TILES, ST_PAIRS, ST_INSERTS (results)
};

template <int DP, int LG, bool FILL>
__global__ __launch_bounds__(256) void k_range(const RangeArgs a) {
    constexpr int NG = 64 >> LG;
    const int lane = threadIdx.x & 63;
    const int wave = xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (wave * NG >= a.q_n_leaves) return;
    const int g = lane >> LG, li = lane & ((1 << LG) - 1);
    const int slot = wave * NG + g;
    const bool has_leaf = slot < a.q_n_leaves;
    const int2 qr = has_leaf ? a.qrange[a.q_first_leaf + slot] : make_int2(0, 0);
    const bool valid = has_leaf && li < qr.y;
    const int qpos = qr.x + li;
    float q[DP];
    {
        const float *qp = a.qpts + int64_t(valid ? qpos : 0) * DP;
#pragma unroll
        for (int j = 0; j < DP; ++j) q[j] = valid ? qp[j] : 0.f;
    }
    const int64_t row = valid ? int64_t(a.qperm[qpos]) : 0;
    int64_t out = 0;
    if constexpr (FILL) out = valid ? a.offsets[row] : 0;
    int found = 0;
    uint32_t n_score = 0, n_tiles = 0;
    uint64_t n_pairs = 0;
    const int n_valid = __popcll(ballot(valid));

    auto score = [&](int node, float &key) -> bool {
        ++n_score;
        float dmin2, dmax2;
        box_dist2<DP>(q, a.rbox + int64_t(node) * 2 * DP, dmin2, dmax2);
        // order key: the first lane's nearest distance (lane 0 is a point of
        // the wave's first leaf)
        key = uniform_f(dmin2);
        const bool keep = valid && (!a.prune || (!(dmin2 > a.s_hi) && !(dmax2 < a.s_lo)));
        return ballot(keep) != 0;
    };
    constexpr int CH = DP >= 32 ? 1 : 32 / DP;
    auto leaf = [&](int node) {
        ++n_tiles;
        const int2 rr = a.rrange[node];
        const int base = uniform_i(rr.x);
        const int cnt = uniform_i(rr.y);
        const float *rp = a.rlpts + int64_t(node - a.r_first_leaf) * a.r_leaf_slots * DP;
        n_pairs += uint64_t(cnt) * uint64_t(n_valid);
        for (int t0 = 0; t0 < cnt; t0 += CH) {
            // a batch of distances first, one wave-wide test: most batches
            // hold no candidate for any lane
            bool cand[CH];
            uint64_t any = 0;
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                float sd = 0.f;
#pragma unroll
                for (int j = 0; j < DP; ++j) {
                    const float df = q[j] - rp[(t0 + c) * DP + j];
                    sd = fmaf(df, df, sd);
                }
                cand[c] = valid && t0 + c < cnt && sd >= a.t_lo && sd <= a.t_hi;
                any |= ballot(cand[c]);
            }
            if (!any) continue;
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                if (cand[c]) {
                    const double x = d2_fp64_unfused<DP>(q, rp + (t0 + c) * DP);
                    const int pos = base + t0 + c;
                    if (x >= a.lo2 && x <= a.hi2 && !(a.self && pos == qpos)) {
                        if constexpr (FILL) {
                            a.out_idx[out + found] = a.rperm[pos];
                            a.out_dist[out + found] = (float)sqrt(x);
                        }
                        ++found;
                    }
                }
            }
        }
    };
    tree_walk(a.r_first_leaf, score, leaf, [](float k0, float k1) { return k1 < k0; });

    if constexpr (!FILL) {
        if (valid) a.counts[row] = found;
    }
    if (a.stats) {
        int f = found;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) f += __shfl_xor(f, off);
        if (lane == 0) {
            atomicAdd(&a.stats[ST_SCORE], (unsigned long long)n_score);
            atomicAdd(&a.stats[ST_TILES], (unsigned long long)n_tiles);
            atomicAdd(&a.stats[ST_PAIRS], (unsigned long long)n_pairs);
            atomicAdd(&a.stats[ST_INSERTS], (unsigned long long)f);
        }
    }
}

template <int DP>
hipError_t launch_range(const RangeArgs &a, int lg, bool fill, int grid, hipStream_t s) {
    if (lg == 5) {
        if (fill)
            k_range<DP, 5, true><<<grid, 256, 0, s>>>(a);
        else
            k_range<DP, 5, false><<<grid, 256, 0, s>>>(a);
    } else {
        if (fill)
            k_range<DP, 6, true><<<grid, 256, 0, s>>>(a);
        else
            k_range<DP, 6, false><<<grid, 256, 0, s>>>(a);
    }
    return hipGetLastError();
}

}  // namespace knnx
