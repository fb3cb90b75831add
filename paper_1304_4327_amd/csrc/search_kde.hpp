// Kernel density kernel (Section "Kernel Density Estimation", Algorithms 9
// and 10): f(q) = sum over references of K(||q - r||), K(d) =
// exp(-d^2 / (2 h^2)), to within eps for every query.
//
// Mapping: a wavefront owns 64 / 2^LG consecutive query leaves (lane =
// query point), an aligned group that is one node N_q of the query tree,
// and walks the reference tree with every node scored once
// (tree_walk_once).  Score is Algorithm 9 for (N_q, N_r): with d_min and
// d_max between the two boxes, B_K = K(d_min) - K(d_max); when it is below
// eps / |S_r| every query point p of N_q adds |N_r| K(||p - C_r||), C_r the
// reference box centre (a point of the box, so each pair's error is at most
// B_K and the errors over the disjoint approximated nodes sum to less than
// eps), and the pair is pruned.  (The printed Algorithm 9 has this
// comparison the other way round; the text around it, and the error bound,
// need it this way.)  Otherwise the walk descends, and at a reference leaf
// BaseCase (Algorithm 10) adds K(||p - r||) for every pair.
//
// Precision.  K values come from FP32 squared distances and the hardware
// exponential; the Score test evaluates K(d_min) from a below-rounded and
// K(d_max) from an above-rounded argument and widens both, so B_K is never
// underestimated.  Each leaf's terms are summed in FP32 and added to an
// FP64 accumulator.
#pragma once

#include <type_traits>

#include "walk.hpp"

namespace knnx {

struct KdeArgs {
    const float *rbox, *rlpts;
    const int2 *rrange;
    int r_leaf_slots, r_first_leaf;
    const float *qpts, *qbox;
    const int32_t *qperm;
    const int2 *qrange;
    int q_first_leaf, q_n_leaves;
    float c;        // 1 / (2 h^2)
    float eps_ref;  // eps / |S_r|
    int approx, self;
    double *f_out;              // per original query row
    unsigned long long *stats;  // ST_SCORE, ST_TILES, ST_PAIRS, ST_INSERTS (approximated node pairs)
};

template <int DP, int LG>
__global__ __launch_bounds__(256) void k_kde(const KdeArgs a) {
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
    // the query node of the wavefront: the ancestor of its NG leaves (the
    // query tree has at least NG leaves whenever it has more than one wave;
    // with fewer leaves than NG the root covers them all)
    int qn = a.q_first_leaf + wave * NG;
    for (int s = 1; s < NG && qn > 0; s <<= 1) qn = (qn - 1) >> 1;
    const float *qb = a.qbox + int64_t(qn) * 2 * DP;
    double f = 0.0;
    uint32_t n_score = 0, n_tiles = 0, n_appr = 0;
    uint64_t n_pairs = 0;
    const int n_valid = __popcll(ballot(valid));

    auto score = [&](int node, float &key) -> bool {
        ++n_score;
        key = 0.f;
        const int cnt = uniform_i(a.rrange[node].y);
        if (cnt == 0) return false;  // empty node: nothing to add
        const float *b = a.rbox + int64_t(node) * 2 * DP;
        float lo2 = 0.f, hi2 = 0.f;
#pragma unroll
        for (int j = 0; j < DP; ++j) {
            const float rl = b[j], rh = b[DP + j], ql = qb[j], qh = qb[DP + j];
            const float gap = fmaxf(fmaxf(rl - qh, ql - rh), 0.0f);
            const float span = fmaxf(rh - ql, qh - rl);
            lo2 = fmaf(gap, gap, lo2);
            hi2 = fmaf(span, span, hi2);
        }
        lo2 = uniform_f(lo2);
        hi2 = uniform_f(hi2);
        key = lo2;
        if (a.approx) {
            const float kmin = __expf(-lo2 * (1.0f - 0x1p-16f) * a.c) * (1.0f + 0x1p-20f);
            const float kmax = __expf(-hi2 * (1.0f + 0x1p-16f) * a.c) * (1.0f - 0x1p-20f);
            if (kmin - kmax < a.eps_ref) {
                float dc2 = 0.f;
#pragma unroll
                for (int j = 0; j < DP; ++j) {
                    const float df = q[j] - 0.5f * (b[j] + b[DP + j]);
                    dc2 = fmaf(df, df, dc2);
                }
                if (valid) f += double(cnt) * double(__expf(-dc2 * a.c));
                ++n_appr;
                return false;
            }
        }
        return true;
    };
    constexpr int CH = DP >= 32 ? 1 : 32 / DP;
    auto leaf = [&](int node) {
        ++n_tiles;
        const int2 rr = a.rrange[node];
        const int base = uniform_i(rr.x);
        const int cnt = uniform_i(rr.y);
        const float *rp = a.rlpts + int64_t(node - a.r_first_leaf) * a.r_leaf_slots * DP;
        n_pairs += uint64_t(cnt) * uint64_t(n_valid);
        // the query's own slot when it lies in this leaf (leave-one-out)
        const int own = (a.self && qpos >= base && qpos < base + cnt) ? qpos - base : -1;
        // K = 2^(-d^2 c log2 e): the hardware base-2 exponential, one multiply
        const float c2 = a.c * 1.44269504088896341f;
        float part = 0.f;
        // whole batches, no branch per pair: the slots past the leaf's points
        // hold FLT_MAX, whose squared distance is +inf and kernel value 0.
        // Only a leaf that holds one of the wave's own queries needs the
        // per-pair test of the query's own slot.
        auto batches = [&](auto skip_own) {
            for (int t0 = 0; t0 < cnt; t0 += CH) {
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    float sd = 0.f;
#pragma unroll
                    for (int j = 0; j < DP; ++j) {
                        const float df = q[j] - rp[(t0 + c) * DP + j];
                        sd = fmaf(df, df, sd);
                    }
                    const float e = __builtin_amdgcn_exp2f(-sd * c2);
                    if constexpr (decltype(skip_own)::value)
                        part += (t0 + c == own) ? 0.f : e;
                    else
                        part += e;
                }
            }
        };
        if (ballot(own >= 0))
            batches(std::true_type{});
        else
            batches(std::false_type{});
        if (valid) f += double(part);
    };
    tree_walk_once(a.r_first_leaf, score, leaf, [](float k0, float k1) { return k1 < k0; });

    if (valid) a.f_out[a.qperm[qpos]] = f;
    if (a.stats && lane == 0) {
        atomicAdd(&a.stats[ST_SCORE], (unsigned long long)n_score);
        atomicAdd(&a.stats[ST_TILES], (unsigned long long)n_tiles);
        atomicAdd(&a.stats[ST_PAIRS], (unsigned long long)n_pairs);
        atomicAdd(&a.stats[ST_INSERTS], (unsigned long long)n_appr);
    }
}

}  // namespace knnx
