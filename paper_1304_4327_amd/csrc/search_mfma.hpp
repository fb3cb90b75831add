// BF16 matrix-core traversal kernel (strides 16 and 32; stride 64 uses the
// sweep form in search_mfma_sweep.hpp): the same pruning dual-tree traversal
// (Algorithm 1, k-NN Score of Algorithm 3 with the bound B(N_q)), with the
// BaseCase distance tiles (Algorithm 2) evaluated as a centred Gram product
// on the MFMA units and every surviving candidate re-scored in FP64.
//
// Mapping (one wavefront per query leaf of <= 32 points)
//   lane l: query j = l % 32, half h = l / 32.  A reference-leaf tile is the
//   32 x 32 block D[i][j] = ||r_i'||^2 - 2 <r_i', q_j'> computed by
//   v_mfma_f32_32x32x16_bf16 over d/16 k-steps, where x' = x - c and c is the
//   query leaf's box centre (centring keeps the BF16 error proportional to
//   the leaf size rather than to |x|).  Operand layout (gfx950): lane l holds
//   A[i = l%32][k = 8h .. 8h+7] and B[k = 8h .. 8h+7][j = l%32]; the output
//   register r of lane l is D[8(r/4) + 4h + r%4][l%32].  Rows are reference
//   slots, columns queries; the accumulator starts at ||r_i'||^2 (FP32) and
//   the query operand is -2 q' (exact scaling in BF16).
//   Each lane keeps its own k-list of the reference rows of its half; the
//   two half-lists of a query are merged at write-out.  A query's current
//   k-th distance is taken as the smaller of its two half-list k-ths (the
//   k-th of the union cannot exceed either).
//
// Filter (exactness).  The margin M_j of bf16_tile.hpp bounds the BF16
// error of each pair of the tile.  A pair is kept when D - M_j + ||q_j'||^2
// <= T_j with T_j = min(D_j[k], B)^2 (1 + 2^-16); a kept pair is re-scored
// exactly in FP64 from the FP32 inputs before it may enter a list.  So the
// BF16 value only decides which pairs are re-scored; lists hold FP64-exact
// distances.
//
// Score uses the query leaf's box (wave-uniform, lanes over dimensions) and
// B(N_q) = min(B1, min D_p[k] + 2 lambda, seed).
#pragma once

#include "bf16_tile.hpp"
#include "search_valu.hpp"

namespace knnx {

// dynamic LDS per wave: both half-lists at write-out (64 lanes x K keys +
// indices); the walk and the tiles use none
template <int DP, int K>
constexpr size_t mfma_lds_per_wave() {
    return size_t(64) * K * 8;
}

template <int DP>
__device__ inline double d2_fp64_rows(const float *x, const float *y) {
    double s2 = 0.0;
#pragma unroll 4
    for (int u = 0; u < DP; u += 4) {
        const float4 p = *reinterpret_cast<const float4 *>(x + u);
        const float4 q = *reinterpret_cast<const float4 *>(y + u);
        double df = (double)p.x - (double)q.x;
        s2 = fma(df, df, s2);
        df = (double)p.y - (double)q.y;
        s2 = fma(df, df, s2);
        df = (double)p.z - (double)q.z;
        s2 = fma(df, df, s2);
        df = (double)p.w - (double)q.w;
        s2 = fma(df, df, s2);
    }
    return s2;
}

template <int DP, int K>
__global__ __launch_bounds__(256) void k_search_mfma(const SearchArgs a) {
    static_assert(DP % 16 == 0, "MFMA tiles need the stride to be a multiple of 16");
    constexpr int S = DP / 16;  // k-steps of 16 dimensions
    constexpr float kInf = __builtin_inff();
    constexpr float kSlack = 1.0f + 0x1p-16f;
    const int lane = threadIdx.x & 63;
    const int wslot = threadIdx.x >> 6;
    const int n_list = a.q_n_leaves;
    int wave;
    if (a.order) {
        // heavy leaves first: the hardware starts workgroups in launch order
        const int raw = blockIdx.x * 4 + wslot;
        if (raw >= n_list) return;
        wave = uniform_i(a.order[raw]);
    } else {
        wave = xcd_remap(blockIdx.x, gridDim.x) * 4 + wslot;
    }
    if (wave >= n_list) return;
    if (a.active && a.active[wave] == 0) return;
    const int qleaf = uniform_i(wave);
    const int qnode = a.q_first_leaf + qleaf;
    const int2 qr = a.qrange[qnode];
    const int qcount = uniform_i(qr.y);
    if (qcount == 0) return;
    const int j = lane & 31, h = lane >> 5;
    const bool valid = j < qcount;
    const int qpos = qr.x + (valid ? j : 0);
    const int kk = a.k + (a.self ? 1 : 0);
    const float *qb = a.qbox + int64_t(qnode) * 2 * DP;

    extern __shared__ __align__(16) char smem[];
    char *wbase = smem + size_t(wslot) * mfma_lds_per_wave<DP, K>();
    float *s_key = reinterpret_cast<float *>(wbase);        // [64][K]
    int *s_ord = reinterpret_cast<int *>(s_key + 64 * K);   // [64][K]
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };

    // leaf box for Score: lane l holds dimension l (0 beyond d, as stored)
    const float qlo = lane < DP ? qb[lane] : 0.f;
    const float qhi = lane < DP ? qb[DP + lane] : 0.f;
    // leaf centre in registers (this lane's operand dimensions), query
    // operand -2 (q - c) in BF16, |q - c|^2 in FP32.  Nothing here or in the
    // tiles goes through LDS with a fence: a fence ahead of the walk would
    // turn its wave-uniform box loads into vector loads.
    float tc[S * 8];
    {
        const float cl = 0.5f * (qlo + qhi);
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int e = 0; e < 8; ++e) tc[s * 8 + e] = __shfl(cl, s * 16 + h * 8 + e);
    }
    bf16x8_t bq[S];
    float qn = bf16_query_operand_r<DP>(a.qpts + int64_t(qpos) * DP, tc, h, valid, bq);
    qn = xor32_op(qn, OpAdd());
    const float qlen = sqrtf(qn);
    const float lam2 = 2.0f * a.qlam[qnode];
    const float seed = a.seed ? fmaxf(a.seed[qleaf], 0.0f) : kInf;
    const float seed2 = seed * seed;

    float dist[K];
    int idx[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        dist[t] = (t < K - kk) ? -kInf : kInf;
        idx[t] = -1;
    }
    float bound2 = (a.bound == KNN_BOUND_NONE) ? kInf : seed2;
    // this query's k-th distance so far: the k-th smallest entry of its two
    // half-lists together (lists of exactly k entries), else the smaller of
    // the two half-list k-ths (an upper bound of it)
    float pair_kth = kInf;
    uint32_t n_score = 0, n_tiles = 0, n_ins = 0, n_pass = 0;
    uint64_t n_pairs = 0;

    // d_min^2 between the query leaf's box and a reference node's box
    auto score_box = [&](const float *b) -> float {
        const float lo = lane < DP ? b[lane] : 0.f;
        const float hi = lane < DP ? b[DP + lane] : 0.f;
        const float gap = fmaxf(fmaxf(lo - qhi, qlo - hi), 0.0f);
        float sum;
        if constexpr (DP <= 16)
            sum = reduce16(gap * gap, OpAdd());
        else if constexpr (DP <= 32)
            sum = reduce32(gap * gap, OpAdd());
        else
            sum = reduce64(gap * gap, OpAdd());
        return uniform_f(sum);
    };
    auto keep_of = [&](float dmin2) { return !(dmin2 > bound2 * kSlack); };

    auto refresh_bound = [&]() {
        if (kk == K) {
            // k-th smallest of two sorted lists A (own) and B (lane ^ 32):
            // min over i of max(A[i-1], B[k-1-i]), i entries taken from A
            float m = dist[K - 1];  // i = k
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const float y = __shfl_xor(dist[K - 1 - i], 32);
                m = fminf(m, i > 0 ? fmaxf(dist[i - 1], y) : y);
            }
            pair_kth = m;
        } else {
            pair_kth = xor32_op(dist[K - 1], OpMin());
        }
        if (a.bound == KNN_BOUND_NONE) return;
        const float hi = reduce32(valid ? pair_kth : -kInf, OpMax());
        const float lo = reduce32(valid ? pair_kth : kInf, OpMin());
        float b = hi;  // B1^2
        if (a.bound == KNN_BOUND_B) {
            // hardware square root (1 ulp): far inside the prune slack
            const float b2 = __builtin_amdgcn_sqrtf(lo) + lam2;
            b = fminf(b, b2 * b2);
        }
        bound2 = uniform_f(fminf(b, seed2));
    };

    auto insert = [&](float x, int id) { sorted_insert<K>(dist, idx, x, id); };

    auto tile = [&](int node) {
        ++n_tiles;
        const int2 rr = a.rrange[node];
        const int base = uniform_i(rr.x);
        const int cnt = uniform_i(rr.y);
        n_pairs += uint64_t(cnt) * uint64_t(qcount);
        const float *rp = a.rlpts + int64_t(node - a.r_first_leaf) * a.r_leaf_slots * DP;
        const int i = lane & 31;
        const bool vr = i < cnt;
        const int islot = vr ? i : 0;  // rows past the leaf read slot 0 (in bounds)
        // reference operand: (r - c) in BF16, |r - c|^2 in FP32
        bf16x8_t ar[S];
        float rn = bf16_ref_operand_r<DP>(rp + islot * DP, tc, h, vr, ar);
        rn = xor32_op(rn, OpAdd());
        const float rlen = bf16_tile_rlen(rn, vr);  // largest |r'| of the tile
        // accumulators start at the row norms (one more product, in lane)
        f32x16_t acc = bf16_tile_product<DP>(ar, bq, bf16_norm_init(rn, vr, h));
        // keep D < T - |q'|^2 + M (the margin is 1.25 times the proven
        // bound, so the strict test keeps every row the bound admits); T is
        // capped at FLT_MAX: rows past the leaf hold +inf and never pass,
        // valid rows always do while a list is not full
        const float lim = fminf(pair_kth, bound2) * kSlack;
        const float marg = bf16_margin<DP>(qlen, rlen);
        const float thr = valid ? fminf(lim - qn + marg, 0x1.fffffep127f) : -kInf;
        // most tiles have no candidate at all: one test on the smallest value
        // of each lane skips the per-row mask, the survivor rounds and the
        // bound refresh (the lists and so the bounds are unchanged)
        float amin = acc[0];
#pragma unroll
        for (int r = 1; r < 16; ++r) amin = fminf(amin, acc[r]);
        if (!ballot(amin < thr)) return;
        // bit r: the sign of D - thr (no per-bit constants in registers)
        uint32_t mask = 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) mask |= (__float_as_uint(acc[r] - thr) >> 31) << r;
        // survivors: one per lane per round, exact FP64 re-score, insert
        const float *qp = a.qpts + int64_t(qpos) * DP;
        // (unrolled: a loop here carried the lists and made the compiler
        // copy them on every pass; a lane holds at most 16 survivors)
#pragma unroll
        for (int pass = 0; pass < 16; ++pass) {
            if (!ballot(mask != 0)) break;
            ++n_pass;
            const bool has = mask != 0;
            const int r = has ? __builtin_ctz(mask) : 0;
            mask &= mask - 1;
            const int row = 8 * (r >> 2) + 4 * h + (r & 3);
            float x = kInf;
            if (has) x = (float)d2_fp64_rows<DP>(qp, a.rpts + int64_t(base + row) * DP);
            // every lane runs the insert (a lane without a survivor inserts
            // +inf, which moves nothing): a divergent insert made the
            // compiler copy the whole list before it
            const bool ins = has && x < dist[K - 1];
            n_ins += ins;
            insert(ins ? x : kInf, base + row);
        }
        refresh_bound();
    };

    // ---- stackless depth-first walk, nearer child first ---------------------
    {
        int node = 0, depth = 0;
        uint64_t nearbits = 0;
        ++n_score;
        bool down = keep_of(score_box(a.rbox));
        if (down) {
            // outer loop: one reference leaf per iteration; the inner walk
            // leaves the k-lists untouched, so they are not carried through
            // its loop (carried through one loop with the tile, the compiler
            // moved every list register on every walk step)
            for (;;) {
                bool leaf = false;
                for (;;) {
                    if (down) {
                        if (node >= a.r_first_leaf) {
                            leaf = true;
                            break;
                        }
                        const int c0 = 2 * node + 1, c1 = c0 + 1;
                        n_score += 2;
                        const float dm0 = score_box(a.rbox + int64_t(c0) * 2 * DP);
                        const float dm1 = score_box(a.rbox + int64_t(c1) * 2 * DP);
                        const bool k0 = keep_of(dm0), k1 = keep_of(dm1);
                        if (!k0 && !k1) {
                            down = false;
                            continue;
                        }
                        const bool right = k1 && (!k0 || dm1 < dm0);
                        if (right)
                            nearbits |= (uint64_t(1) << depth);
                        else
                            nearbits &= ~(uint64_t(1) << depth);
                        node = uniform_i(right ? c1 : c0);
                        ++depth;
                    } else {
                        if (node == 0) break;
                        --depth;
                        const bool is_right = (node & 1) == 0;
                        const bool near_right = (nearbits >> depth) & 1;
                        if (is_right == near_right) {
                            const int far = is_right ? node - 1 : node + 1;
                            ++n_score;
                            if (keep_of(score_box(a.rbox + int64_t(far) * 2 * DP))) {
                                node = far;
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

    // ---- write-out: FP64 re-score, merge the two half-lists ------------------
    // Every entry becomes its output key (FP32 distance from the FP64
    // re-score, original index), stored in LDS; each entry's rank in the
    // union of the two half-lists is counted against both, and entries of
    // rank < k are written at that rank.  Unused slots get distinct +inf
    // keys that rank after every real entry.
    const float *qp = a.qpts + int64_t(qpos) * DP;
    float *my_key = s_key + lane * K;
    int *my_ord = s_ord + lane * K;
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const bool real = valid && idx[t] >= 0 && !(a.self && idx[t] == qpos);
        const int p = real ? idx[t] : 0;
        float key = kInf;
        int o = 0x7fffffff - t - h * K;
        if (real) {
            key = (float)sqrt(d2_fp64_rows<DP>(qp, a.rpts + int64_t(p) * DP));
            o = a.rperm[p];
        }
        dist[t] = key;
        idx[t] = o;
        my_key[t] = key;
        my_ord[t] = o;
    }
    wave_sync();
    int rank[K];
#pragma unroll
    for (int t = 0; t < K; ++t) rank[t] = 0;
    const float *pk_list = s_key + (lane ^ 32) * K;
    const int *po_list = s_ord + (lane ^ 32) * K;
    for (int u = 0; u < K; ++u) {
        const float ok = my_key[u], pk = pk_list[u];
        const int oo = my_ord[u], po = po_list[u];
#pragma unroll
        for (int t = 0; t < K; ++t) {
            rank[t] += (ok < dist[t]) || (ok == dist[t] && oo < idx[t]);
            rank[t] += (pk < dist[t]) || (pk == dist[t] && po < idx[t]);
        }
    }
    float worst = -1.0f;
    if (valid) {
        const int64_t row = int64_t(a.qperm[qpos]) * a.k;
#pragma unroll
        for (int t = 0; t < K; ++t) {
            if (rank[t] < a.k) {
                a.out_idx[row + rank[t]] = idx[t] >= 0x7fffffff - 2 * K ? -1 : idx[t];
                a.out_dist[row + rank[t]] = dist[t];
                if (rank[t] == a.k - 1) worst = dist[t];
            }
        }
    }
    worst = fmaxf(worst, __shfl_xor(worst, 32));
    bool fb = false;
    if (a.seed && valid) fb = !((double)worst * worst <= (double)seed2 * (1.0 - 0x1p-20));
    float lw = worst;
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) lw = fmaxf(lw, __shfl_xor(lw, off));
    const uint64_t fbmask = ballot(fb);
    float fbb = (valid && worst < kInf) ? worst : kInf;
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) fbb = fminf(fbb, __shfl_xor(fbb, off));
    if (lane == 0) {
        if (a.leaf_kth) a.leaf_kth[qleaf] = fmaxf(lw, 0.0f);
        if (a.fallback && fbmask) {
            a.fallback[qleaf] = 1;
            if (a.fb_bound) a.fb_bound[qleaf] = fbb < kInf ? (fbb + lam2) * (1.0f + 0x1p-20f) : kInf;
        }
    }
    if (a.wave_log || a.stats) {
        int ins = n_ins;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) ins += __shfl_xor(ins, off);
        if (a.wave_log && lane == 0) {
            uint32_t *w = a.wave_log + int64_t(wave) * 8;
            w[0] = 0;
            w[1] = n_score;
            w[2] = n_tiles;
            w[3] = uint32_t(ins);
            w[4] = n_pass;
            w[5] = uint32_t(qleaf);
        }
        if (a.stats && lane == 0) {
            atomicAdd(&a.stats[ST_SCORE], (unsigned long long)n_score);
            atomicAdd(&a.stats[ST_TILES], (unsigned long long)n_tiles);
            atomicAdd(&a.stats[ST_PAIRS], (unsigned long long)n_pairs);
            atomicAdd(&a.stats[ST_INSERTS], (unsigned long long)ins);
            atomicAdd(&a.stats[ST_FB_QUERIES], (unsigned long long)(__popcll(fbmask) / 2));
        }
    }
}

template <int DP>
hipError_t launch_search_mfma(const SearchArgs &a, int K, int grid, hipStream_t s) {
    switch (K) {
#define KNN_CASE(KK)                                                  \
    case KK:                                                          \
        k_search_mfma<DP, KK><<<grid, 256, 4 * mfma_lds_per_wave<DP, KK>(), s>>>(a); \
        break;
        KNN_CASE(4)
        KNN_CASE(5)
        KNN_CASE(8)
        KNN_CASE(10)
        KNN_CASE(11)
        KNN_CASE(16)
        KNN_CASE(32)
        KNN_CASE(50)
        KNN_CASE(51)
        KNN_CASE(64)
#undef KNN_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace knnx
