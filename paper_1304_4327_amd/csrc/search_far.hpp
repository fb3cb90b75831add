// k-furthest-neighbour traversal kernel: the k-NN kernel's pruning dual-tree
// traversal (Algorithm 1) with the rules inverted as the closing remark of
// Section "k-Nearest Neighbor Search" describes -- max and min exchanged in
// the bound, lists in descending distance, the BaseCase comparison
// d > D_p[k] -- so each query keeps its k farthest references.
//
// Mapping as in k_search_valu: a wavefront owns NG = 64 / 2^LG consecutive
// query leaves, lane = query point, and walks the reference tree depth
// first without a stack, here the FARTHER child first (its d_max to the
// wave's union box is larger), since far nodes fill the lists fastest.
//
// Lists.  Each lane keeps K keys -d^2 in ascending order (so the k-th
// farthest is slot K-1, and the insertion is the k-NN one); empty slots hold
// +inf.  The paper initialises D to 0 and inserts on d > D[k], which would
// never insert a reference at distance 0 (a duplicate of the query); empty
// slots at +inf accept every reference until the list is full, and the
// bound treats them as distance 0.
//
// Bound (lower bound on every point's final k-th farthest distance):
//   L1 = min over the leaf's points of D_p[k]
//   L2 = max over the leaf's points of D_p[k] - 2 lambda(leaf)
//        (a point's k references are at least that far from every point of
//        the leaf, by the triangle inequality)
//   LP = the same L2 form over an ancestor's points and lambda
//   L  = max(L1, L2, LP)
// Score: each query point is a singleton child of its leaf, with
// d_max(p, N_r) the largest distance from p to the node's box; it keeps the
// node unless d_max^2 < max(L, D_p[k])^2 (1 - 2^-16) (strict, with slack for
// FP32 rounding).  A pair can be in a final list only if its distance is at
// least the point's final k-th farthest distance, which is >= L.
//
// Precision.  The FP32 tile only filters (with a relative slack for its
// rounding); every candidate is re-scored in FP64 before it enters a list,
// and the final list is re-scored in FP64 and ordered by (distance
// descending, original index ascending).
#pragma once

#include "search_valu.hpp"

namespace knnx {

// low dimension, short lists: six waves per SIMD fit without spills
template <int DP, int K, int LG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DP <= 4 && K <= 16 ? 6 : 1))) void
k_search_far(const SearchArgs a) {
    constexpr float kInf = __builtin_inff();
    constexpr float kShrink = 1.0f - 0x1p-16f;            // prune slack (squared)
    constexpr float kGamma = 1.0f - (DP + 6) * 0x1p-24f;  // FP32 filter slack
    constexpr int NG = 64 >> LG;
    constexpr bool WIDE = DP >= 16;
    const int lane = threadIdx.x & 63;
    const int n_list = a.q_n_leaves;
    const int wave = xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (wave * NG >= n_list) return;
    const int g = lane >> LG, li = lane & ((1 << LG) - 1);
    const int slot = wave * NG + g;
    const bool has_leaf = slot < n_list;
    const int qleaf = has_leaf ? slot : 0;
    const int qnode = a.q_first_leaf + qleaf;
    const int2 qr = has_leaf ? a.qrange[qnode] : make_int2(0, 0);
    const bool valid = has_leaf && li < qr.y;
    const int qpos = qr.x + li;
    const int kk = a.k + (a.self ? 1 : 0);

    float q[DP];
    {
        const float *qp = a.qpts + int64_t(valid ? qpos : 0) * DP;
#pragma unroll
        for (int j = 0; j < DP; ++j) q[j] = valid ? qp[j] : 0.f;
    }
    // union box of the wave's leaves for the visit-order key (low d: every
    // lane holds it; high d: lane l holds dimension l)
    constexpr int UD = WIDE ? 1 : DP;
    float ulo[UD], uhi[UD];
    if constexpr (!WIDE) {
        const float *qb = a.qbox + int64_t(has_leaf ? qnode : 0) * 2 * DP;
#pragma unroll
        for (int j = 0; j < DP; ++j) {
            float lo = has_leaf ? qb[j] : kInf;
            float hi = has_leaf ? qb[DP + j] : -kInf;
#pragma unroll
            for (int l = LG; l < 6; ++l) {
                lo = xor_level(lo, l, OpMin());
                hi = xor_level(hi, l, OpMax());
            }
            ulo[j] = lo;
            uhi[j] = hi;
        }
    } else {
        float lo = lane < DP ? kInf : 0.f, hi = lane < DP ? -kInf : 0.f;
        for (int gg = 0; gg < NG; ++gg) {
            const int sl = wave * NG + gg;
            if (sl < n_list && lane < DP) {
                const float *qb = a.qbox + int64_t(a.q_first_leaf + sl) * 2 * DP;
                lo = fminf(lo, qb[lane]);
                hi = fmaxf(hi, qb[DP + lane]);
            }
        }
        ulo[0] = lo;
        uhi[0] = hi;
    }
    const float lam2 = has_leaf ? 2.0f * a.qlam[qnode] : 0.f;
    float lam2_anc[6];
#pragma unroll
    for (int s = 1; s <= 5; ++s) {
        lam2_anc[s] = kInf;
        if (a.bound == KNN_BOUND_B && ((1 << LG) << (s - 1)) < 64 && has_leaf &&
            ((qnode + 1) >> s) >= 1)
            lam2_anc[s] = 2.0f * a.qlam[((qnode + 1) >> s) - 1];
    }

    float key[K];  // -d^2 ascending; +inf empty, -inf padding below K - kk
    int idx[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        key[j] = (j < K - kk) ? -kInf : kInf;
        idx[j] = -1;
    }
    float bound2 = 0.f;  // L^2
    uint32_t n_score = 0, n_tiles = 0, n_ins = 0;
    uint64_t n_pairs = 0;
    const int n_valid = __popcll(ballot(valid));

    // this lane's k-th farthest squared distance so far (0 until the list fills)
    auto kth2 = [&]() -> float { return key[K - 1] < kInf ? -key[K - 1] : 0.f; };
    auto point_bound2 = [&]() -> float {
        return a.bound == KNN_BOUND_NONE ? 0.f : fmaxf(bound2, kth2());
    };
    // Score of a reference node: the lane keeps it unless the farthest point
    // of its box is nearer than the lane's bound; the wave-uniform order key
    // is d_max^2 between the union box and the node's box
    auto score = [&](int node, float &key_out) -> bool {
        ++n_score;
        const float *b = a.rbox + int64_t(node) * 2 * DP;
        float sd = 0.f, u = 0.f;
#pragma unroll
        for (int j = 0; j < DP; ++j) {
            const float lo = b[j], hi = b[DP + j];
            const float s = fmaxf(fmaxf(q[j] - lo, hi - q[j]), 0.0f);
            sd = fmaf(s, s, sd);
            if constexpr (!WIDE) {
                const float us = fmaxf(fmaxf(uhi[j] - lo, hi - ulo[j]), 0.0f);
                u = fmaf(us, us, u);
            }
        }
        if constexpr (WIDE) {
            const float lo = lane < DP ? b[lane] : 0.f, hi = lane < DP ? b[DP + lane] : 0.f;
            const float us = fmaxf(fmaxf(uhi[0] - lo, hi - ulo[0]), 0.0f);
            u = us * us;
            u = sum_dim_lanes<DP>(u);
        }
        key_out = uniform_f(u);
        const bool keep = valid && !(sd < point_bound2() * kShrink);
        return ballot(keep) != 0;
    };
    auto insert = [&](float x, int id) { sorted_insert<K>(key, idx, x, id); };
    // L after a tile: min and max of the leaf's k-th distances, then the
    // ancestors whose leaves all sit in this wave (one lane level each)
    auto refresh_bound = [&]() {
        if (a.bound == KNN_BOUND_NONE) return;
        const float k2 = kth2();
        float lo = valid ? k2 : kInf;
        float hi = valid ? k2 : -kInf;
#pragma unroll
        for (int l = 0; l < LG; ++l) {
            lo = xor_level(lo, l, OpMin());
            hi = xor_level(hi, l, OpMax());
        }
        float b = lo < kInf ? lo : 0.f;  // L1^2
        if (a.bound == KNN_BOUND_B) {
            const float t = __builtin_amdgcn_sqrtf(fmaxf(hi, 0.f)) - lam2;
            b = fmaxf(b, t > 0.f ? t * t : 0.f);
#pragma unroll
            for (int s = 1; s <= 5; ++s) {
                const int l = LG + s - 1;
                if (l < 6) {
                    hi = xor_level(hi, l, OpMax());
                    const float tp = __builtin_amdgcn_sqrtf(fmaxf(hi, 0.f)) - lam2_anc[s];
                    b = fmaxf(b, tp > 0.f ? tp * tp : 0.f);
                }
            }
        }
        bound2 = b;
    };
    // BaseCase over one reference leaf (CH points per batch; slots past the
    // leaf hold FLT_MAX and are masked: their distance would be the largest)
    constexpr int CH = DP >= 32 ? 1 : 32 / DP;
    auto tile = [&](int node) {
        ++n_tiles;
        const int2 rr = a.rrange[node];
        const int base = uniform_i(rr.x);
        const int cnt = uniform_i(rr.y);
        const float *rp = a.rlpts + int64_t(node - a.r_first_leaf) * a.r_leaf_slots * DP;
        n_pairs += uint64_t(cnt) * uint64_t(n_valid);
        for (int t0 = 0; t0 < cnt; t0 += CH) {
            float sd[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                float acc = 0.f;
#pragma unroll
                for (int j = 0; j < DP; ++j) {
                    const float df = q[j] - rp[(t0 + c) * DP + j];
                    acc = fmaf(df, df, acc);
                }
                sd[c] = acc;
            }
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const float thr = point_bound2() * kGamma;
                const bool cand = valid && t0 + c < cnt && sd[c] >= thr;
                if (ballot(cand)) {
                    float x = kInf;
                    if (cand) x = -(float)d2_fp64<DP>(q, rp + (t0 + c) * DP);
                    const bool ins = cand && x < key[K - 1];
                    n_ins += ins ? 1u : 0u;
                    insert(ins ? x : kInf, base + t0 + c);
                }
            }
        }
        refresh_bound();
    };

    // ---- stackless depth-first walk, farther child first --------------------
    {
        float dm0, dm1;
        int node = 0, depth = 0;
        uint64_t firstbits = 0;
        bool down = score(0, dm0);
        if (down) {
            for (;;) {
                bool leaf = false;
                for (;;) {
                    if (down) {
                        if (node >= a.r_first_leaf) {
                            leaf = true;
                            break;
                        }
                        const int c0 = 2 * node + 1, c1 = c0 + 1;
                        const bool k0 = score(c0, dm0);
                        const bool k1 = score(c1, dm1);
                        if (!k0 && !k1) {
                            down = false;
                            continue;
                        }
                        const bool right = k1 && (!k0 || dm1 > dm0);
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
                            if (score(other, dm0)) {
                                node = other;
                                ++depth;
                                down = true;
                                continue;
                            }
                        }
                        node = uniform_i((node - 1) >> 1);
                    }
                }
                if (!leaf) break;
                tile(node);
                down = false;
            }
        }
    }

    // ---- write-out: FP64 re-score, order by (distance desc, index asc) ------
    float dist[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const bool real = valid && idx[j] >= 0 && !(a.self && idx[j] == qpos);
        const int p = real ? idx[j] : 0;
        dist[j] = real ? (float)sqrt(d2_fp64<DP>(q, a.rpts + int64_t(p) * DP)) : -kInf;
        idx[j] = real ? a.rperm[p] : 0x7fffffff - j;
    }
    if (valid) {
        const int64_t row = int64_t(a.qperm[qpos]) * a.k;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            int rank = 0;
#pragma unroll
            for (int i = 0; i < K; ++i)
                rank += (dist[i] > dist[j]) || (dist[i] == dist[j] && idx[i] < idx[j]);
            if (rank < a.k) {
                a.out_idx[row + rank] = idx[j] >= 0x7fffffff - K ? -1 : idx[j];
                a.out_dist[row + rank] = dist[j];
            }
        }
    }
    if (a.stats) {
        int ins = n_ins;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) ins += __shfl_xor(ins, off);
        if (lane == 0) {
            atomicAdd(&a.stats[ST_SCORE], (unsigned long long)n_score);
            atomicAdd(&a.stats[ST_TILES], (unsigned long long)n_tiles);
            atomicAdd(&a.stats[ST_PAIRS], (unsigned long long)n_pairs);
            atomicAdd(&a.stats[ST_INSERTS], (unsigned long long)ins);
        }
    }
}

template <int DP, int K>
hipError_t launch_search_far_k(const SearchArgs &a, int grid, hipStream_t s) {
    if (a.lpl_log2 == 5)
        k_search_far<DP, K, 5><<<grid, 256, 0, s>>>(a);
    else
        k_search_far<DP, K, 6><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

template <int DP>
hipError_t launch_search_far(const SearchArgs &a, int K, int grid, hipStream_t s) {
    switch (K) {
        case 8: return launch_search_far_k<DP, 8>(a, grid, s);
        case 16: return launch_search_far_k<DP, 16>(a, grid, s);
        case 32: return launch_search_far_k<DP, 32>(a, grid, s);
        case 64: return launch_search_far_k<DP, 64>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace knnx
