// BF16 matrix-core kernel for the high-dimensional regime: the same
// BaseCase tiles, bounds and exactness argument as the per-leaf MFMA kernel
// (k_search_mfma), with the reference tree visited as a sweep over blocks of
// its leaves instead of a depth-first walk.
//
// Why a sweep.  With d = 64 and tens of thousands of reference leaves, the
// nearest-first walk enters most leaves anyway, and its cost becomes the
// chain of dependent box loads on the way down and back up.  The sweep
// scores every reference leaf against the query points' current bounds --
// still a pruning dual-tree traversal (every pair (N_q, N_r) is scored once
// and pruned when d_min exceeds the bound), only in another order -- and
// loads the next kept leaf while the current one is processed.
//
// Score.  The sweep takes blocks of 32 consecutive reference leaves (the
// leaves of one subtree), outward in tree order from the block of the leaf
// the query node's box centre falls in (neighbours in tree order are
// neighbours in space, so near blocks come first).  Each (query point p,
// reference leaf N_r) pair of a block is scored as the singleton query node
// {p} against N_r, with d_min({p}, N_r) >= ||p - C_r|| - lambda(N_r): every
// point of N_r lies within lambda of its box centre C_r.  The pair is pruned
// when that exceeds p's bound min(D_p[k], B(N_q)).  The 32 x 32 values
// ||p - C_r||^2 of a block are one BF16 MFMA tile of the queries against the
// leaf centres, with the proven margin of the distance tiles; the test takes
// the margin's low end, so it keeps every pair the exact test keeps.  In high
// dimension this prunes far more than the box-to-box distance: a 32-point
// kd-tree leaf is split on at most depth-many dimensions, and its box spans
// the leaf's whole spread in all the others.
//
// Mapping: one workgroup of four wavefronts owns four sibling query leaves
// (<= 32 points each, one leaf per wave).  Per block, all 256 threads stage
// the 32 leaf centres (centred on the centre c of the query leaves' union
// box, rounded to BF16) into LDS; each wave scores them against its 32
// queries and ORs the kept leaves into its own 32-bit mask; the union of the
// four masks is the list of leaves the workgroup stages.  A kept leaf is
// staged once into LDS by all 256 threads -- centred and rounded to BF16, its
// FP32 rows beside it for the exact re-score, and its centred row norms --
// and every wave whose own mask holds it multiplies it against its 32
// queries with v_mfma_f32_32x32x16_bf16 (layout, filter margin and FP64
// re-score as in k_search_mfma).  The staged tiles are double-buffered: one
// workgroup barrier per kept leaf publishes the tile staged last; after it
// each wave multiplies that tile, then stages the next kept leaf into the
// other buffer.  The waves exchange their bounds once per block: the query
// node above the four leaves adds the B(Par) term, min over all its queries
// of D_p[k] + 2 lambda(node).
//
// Wave-independent form (W, used whenever the reference-side operands of
// k_wsweep_prep are given).  The staged form waits at one workgroup barrier
// per kept leaf, for the slowest of four waves.  In the W form the four
// waves share only the block order; each wave then, on its own, scores a
// block's 32 leaves against its queries and multiplies its own kept leaves,
// reading their operands from global memory with the next kept leaf's loads
// in flight.  Everything is centred on the block's centre C_B: the reference
// side (rows -2 (r - C_B) in BF16, their norms, leaf centres -2 (C_L - C_B))
// is made once per search, and per block each wave forms q - C_B once for
// the block Score and all of the block's tiles.  The margin is the same
// bound with |q'| = |q - C_B| and the tile's largest |r - C_B|.
#pragma once

#include "search_mfma.hpp"

namespace knnx {

constexpr int kWgLeaves = 4;   // query leaves (one per wave) per workgroup

// LDS layout of one workgroup
template <int DP, int K>
struct SweepLds {
    static constexpr int kRowBf = DP + 8;  // bf16 per staged row (16 B pad)
    static constexpr size_t tile_f = size_t(32) * DP * 4;
    static constexpr size_t tile_bf = size_t(32) * kRowBf * 2;
    static constexpr size_t q_rows = size_t(kWgLeaves) * 32 * DP * 4;
    static constexpr size_t merge = size_t(64) * K * 8;  // one wave's half-lists
    static constexpr size_t region = q_rows > merge ? q_rows : merge;
    // two buffers of each per-tile array, one block of leaf centres
    static constexpr size_t off_tile_f = 0;
    static constexpr size_t off_tile_bf = off_tile_f + 2 * tile_f;
    static constexpr size_t off_ctr_bf = off_tile_bf + 2 * tile_bf;
    static constexpr size_t off_region = off_ctr_bf + tile_bf;
    static constexpr size_t off_cen = off_region + region;
    static constexpr size_t off_rn = off_cen + size_t(DP) * 4;
    static constexpr size_t off_ctr_n = off_rn + 2 * 32 * 4;    // centre norms
    static constexpr size_t off_ctr_lam = off_ctr_n + 32 * 4;   // leaf lambdas
    // misc words (kMisc*)
    static constexpr size_t off_misc = off_ctr_lam + 32 * 4;
    // the sorted block order and keys (the sort itself runs in the tile
    // buffers, before the sweep uses them)
    static constexpr int sort_max = int(2 * tile_f / 8) < 2048 ? int(2 * tile_f / 8) : 2048;
    static constexpr size_t off_okey = off_misc + 32 * 4;
    static constexpr size_t off_order = off_okey + size_t(sort_max) * 4;
    static constexpr size_t bytes = off_order + size_t(sort_max) * 2;
};
// misc words: each wave's bound and smallest k-th distance, the largest row
// norm of each wave's staged rows per tile buffer, the same for the block of
// centres, and each wave's block mask
constexpr int kMiscBound = 0;     // [2][kWgLeaves]
constexpr int kMiscTileMax = 8;   // [2][kWgLeaves]
constexpr int kMiscCtrMax = 16;   // [kWgLeaves]
constexpr int kMiscMask = 20;     // [kWgLeaves]
constexpr int kMiscQlen = 24;     // [kWgLeaves] largest |q - c| of each wave

// Two workgroups per CU (two waves per SIMD) where the lists allow it: each
// tile's latency chain (staging barrier, dependent MFMAs, LDS reads) is then
// covered by the other workgroup.  For K <= 50 this fits 256 registers;
// larger lists keep one workgroup.
template <int DP, int K, bool W = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(K <= 50 ? 2 : 1))) void
k_search_mfma_sweep(const SearchArgs a) {
    static_assert(DP % 16 == 0, "MFMA tiles need the stride to be a multiple of 16");
    using L = SweepLds<DP, K>;
    constexpr int S = DP / 16;  // k-steps of 16 dimensions
    constexpr int E = DP / 8;   // staged floats per thread (32 rows x DP / 256)
    constexpr int NB = kSweepBlock;
    constexpr float kInf = __builtin_inff();
    constexpr float kSlack = 1.0f + 0x1p-16f;
    __shared__ __align__(16) char smem[L::bytes];
    float *s_tf = reinterpret_cast<float *>(smem + L::off_tile_f);
    __bf16 *s_tb = reinterpret_cast<__bf16 *>(smem + L::off_tile_bf);
    __bf16 *s_cb = reinterpret_cast<__bf16 *>(smem + L::off_ctr_bf);
    float *s_q = reinterpret_cast<float *>(smem + L::off_region);
    float *s_cen = reinterpret_cast<float *>(smem + L::off_cen);
    float *s_rn = reinterpret_cast<float *>(smem + L::off_rn);
    float *s_cn = reinterpret_cast<float *>(smem + L::off_ctr_n);
    float *s_cl = reinterpret_cast<float *>(smem + L::off_ctr_lam);
    float *s_misc = reinterpret_cast<float *>(smem + L::off_misc);
    uint32_t *s_mask = reinterpret_cast<uint32_t *>(s_misc + kMiscMask);
    float *s_okey = reinterpret_cast<float *>(smem + L::off_okey);
    uint16_t *s_order = reinterpret_cast<uint16_t *>(smem + L::off_order);
    // workgroup barrier that waits for this wave's LDS traffic only: the
    // next leaf's global loads stay in flight across it
    auto lds_barrier = [] { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); };

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int n_list = a.q_n_leaves;
    const int leaf0 = blk * kWgLeaves;
    if (leaf0 >= n_list) return;  // whole workgroup
    auto leaf_on = [&](int sl) { return sl < n_list && (!a.active || a.active[sl] != 0); };
    bool any_leaf = false;
#pragma unroll
    for (int g = 0; g < kWgLeaves; ++g) any_leaf |= leaf_on(leaf0 + g);
    if (!any_leaf) return;  // whole workgroup (fallback pass)

    const int slot = leaf0 + w;
    const bool has_leaf = leaf_on(slot);
    const int qleaf = has_leaf ? slot : leaf0;
    const int qnode = a.q_first_leaf + qleaf;
    const int2 qr = has_leaf ? a.qrange[qnode] : make_int2(0, 0);
    const int qcount = uniform_i(qr.y);
    const int j = lane & 31, h = lane >> 5;
    const bool valid = j < qcount;
    const int qpos = qr.x + (valid ? j : 0);
    const int kk = a.k + (a.self ? 1 : 0);

    // union box of the workgroup's active leaves, lane l = dimension l (every
    // wave computes the same values)
    float ulo = 0.f, uhi = 0.f;
    if (lane < DP) {
        ulo = kInf;
        uhi = -kInf;
#pragma unroll
        for (int g = 0; g < kWgLeaves; ++g) {
            if (leaf_on(leaf0 + g)) {
                const float *qb = a.qbox + int64_t(a.q_first_leaf + leaf0 + g) * 2 * DP;
                ulo = fminf(ulo, qb[lane]);
                uhi = fmaxf(uhi, qb[DP + lane]);
            }
        }
    }
    if (w == 0 && lane < DP) s_cen[lane] = 0.5f * (ulo + uhi);
    // this wave's query rows (FP32) for the exact re-score; zero for idle lanes
    float *my_q = s_q + (w * 32 + j) * DP;
#pragma unroll
    for (int u = h * (DP / 2); u < (h + 1) * (DP / 2); u += 4) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (valid) v = *reinterpret_cast<const float4 *>(a.qpts + int64_t(qpos) * DP + u);
        *reinterpret_cast<float4 *>(my_q + u) = v;
    }
    __syncthreads();

    // query operand -2 (q - c) in BF16 and |q - c|^2 in FP32
    bf16x8_t bq[S];
    float qn = 0.f;
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int dim = s * 16 + h * 8 + e;
            const float qd = valid ? my_q[dim] - s_cen[dim] : 0.f;
            qn = fmaf(qd, qd, qn);
            bq[s][e] = (__bf16)(-2.0f * qd);
        }
    }
    qn = xor32_op(qn, OpAdd());
    const float qlen = sqrtf(qn);
    // centre of the staged columns of this thread
    const int trow = tid >> 3, tcol = (tid & 7) * E;
    float tc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) tc[e] = s_cen[tcol + e];

    const float lam2 = has_leaf ? 2.0f * a.qlam[qnode] : 0.f;
    // the query node two levels above the leaves (when the tree has one)
    float lam2_anc = kInf;
    if (a.bound == KNN_BOUND_B && ((a.q_first_leaf + 1) >> 2) >= 1)
        lam2_anc = 2.0f * a.qlam[((a.q_first_leaf + leaf0 + 1) >> 2) - 1];
    const float seed = (a.seed && has_leaf) ? fmaxf(a.seed[qleaf], 0.0f) : kInf;
    const float seed2 = seed * seed;

    float dist[K];
    int idx[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        dist[t] = (t < K - kk) ? -kInf : kInf;
        idx[t] = -1;
    }
    float bound2 = (a.bound == KNN_BOUND_NONE) ? kInf : seed2;  // this wave's B^2
    float lo_k = kInf;      // min over the wave's queries of D_p[k]^2
    // this query's k-th distance so far: the k-th smallest entry of its two
    // half-lists together (lists of exactly k entries), else the smaller of
    // the two half-list k-ths (an upper bound of it)
    float pair_kth = kInf;
    uint32_t n_score = 0, n_tiles = 0, n_ins = 0, n_pass = 0, n_staged = 0, n_cand = 0;
    uint64_t n_pairs = 0;

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
        lo_k = uniform_f(lo);
        float b = hi;  // B1^2
        if (a.bound == KNN_BOUND_B) {
            const float b2 = __builtin_amdgcn_sqrtf(lo) + lam2;
            b = fminf(b, b2 * b2);
        }
        bound2 = uniform_f(fminf(fminf(b, seed2), bound2));
    };

    auto insert = [&](float x, int id) { sorted_insert<K>(dist, idx, x, id); };

    // stage a leaf from prefetched rows v (this thread's E columns of row
    // trow) into tile buffer b: rows past the leaf are zero with an infinite
    // norm (never candidates)
    auto stage = [&](int b, int cnt, const float (&v)[E]) {
        __bf16 *tb = s_tb + b * 32 * L::kRowBf;
        float *tf = s_tf + b * 32 * DP;
        const bool vrow = trow < cnt;
        float rn = 0.f;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const float rd = vrow ? v[e] - tc[e] : 0.f;
            rn = fmaf(rd, rd, rn);
            tb[trow * L::kRowBf + tcol + e] = (__bf16)rd;
            tf[trow * DP + tcol + e] = v[e];
        }
        rn = reduce8(rn, OpAdd());
        if ((tid & 7) == 0) s_rn[b * 32 + trow] = vrow ? rn : kInf;
        // largest norm of this wave's eight rows (every lane of a row's
        // eight holds its norm), taken on the scalar unit: the norms are
        // non-negative, so their bit patterns order as unsigned integers
        const int rnb = __builtin_bit_cast(int, vrow ? rn : 0.f);
        uint32_t rmu = 0u;
#pragma unroll
        for (int g = 0; g < 8; ++g) rmu = max(rmu, (uint32_t)__builtin_amdgcn_readlane(rnb, 8 * g));
        if (lane == 0) s_misc[kMiscTileMax + b * kWgLeaves + w] = __builtin_bit_cast(float, rmu);
    };
    // one staged tile (buffer b, leaf rows base .. base + cnt) against this
    // wave's queries; own: the leaf is in this wave's block mask
    auto compute = [&](int b, int base, int cnt, bool own) __attribute__((always_inline)) {
        if (!own) return;
        const __bf16 *tb = s_tb + b * 32 * L::kRowBf;
        const float *tf = s_tf + b * 32 * DP;
        const float *trn = s_rn + b * 32;
        ++n_tiles;
        n_pairs += uint64_t(cnt) * uint64_t(qcount);
        // largest |r'| in the tile (hardware square root, 1 ulp, nudged up:
        // the margin only needs an upper bound)
        float rmax = 0.f;
#pragma unroll
        for (int g = 0; g < kWgLeaves; ++g) rmax = fmaxf(rmax, s_misc[kMiscTileMax + b * kWgLeaves + g]);
        const float rlen = __builtin_amdgcn_sqrtf(uniform_f(rmax)) * (1.0f + 0x1p-20f);
        f32x16_t acc;
#pragma unroll
        for (int g4 = 0; g4 < 4; ++g4) {
            const float4 v = *reinterpret_cast<const float4 *>(&trn[g4 * 8 + h * 4]);
            acc[g4 * 4 + 0] = v.x;
            acc[g4 * 4 + 1] = v.y;
            acc[g4 * 4 + 2] = v.z;
            acc[g4 * 4 + 3] = v.w;
        }
        const __bf16 *arow = tb + j * L::kRowBf + h * 8;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bf16x8_t ar = *reinterpret_cast<const bf16x8_t *>(arow + s * 16);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar, bq[s], acc, 0, 0, 0);
        }
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
        n_cand += __popc(mask);
        // survivors: one per lane per round, exact FP64 re-score, insert.
        // The round body has no divergent branch: a lane without a survivor
        // re-scores row 0 and inserts +inf (a no-op); the wave issues the
        // same instructions either way.
        // (unrolled: a loop here carried the lists and made the compiler
        // copy them on entry and exit; a lane holds at most 16 survivors)
#pragma unroll
        for (int pass = 0; pass < 16; ++pass) {
            const bool has = mask != 0;
            if (!ballot(has)) break;
            ++n_pass;
            const int r = has ? __builtin_ctz(mask) : 0;
            mask &= mask - 1u;
            const int row = 8 * (r >> 2) + 4 * h + (r & 3);
            const float x0 = (float)d2_fp64_rows<DP>(my_q, tf + row * DP);
            const float x = has ? x0 : kInf;
            n_ins += (x < dist[K - 1]) ? 1u : 0u;
            insert(x, base + row);
        }
        refresh_bound();
    };

    // ---- the sweep ---------------------------------------------------------
    // start: the reference leaf the union centre falls in (descent by box
    // distance of the centre to the two children)
    int start = 0;
    {
        const float cq = lane < DP ? 0.5f * (ulo + uhi) : 0.f;
        int node = 0;
        while (node < a.r_first_leaf) {
            const int c0 = 2 * node + 1;
            const float *b0 = a.rbox + int64_t(c0) * 2 * DP;
            const float *b1 = b0 + 2 * DP;
            const float g0 = lane < DP ? fmaxf(fmaxf(b0[lane] - cq, cq - b0[DP + lane]), 0.f) : 0.f;
            const float g1 = lane < DP ? fmaxf(fmaxf(b1[lane] - cq, cq - b1[DP + lane]), 0.f) : 0.f;
            const float d0 = uniform_f(reduce64(g0 * g0, OpAdd()));
            const float d1 = uniform_f(reduce64(g1 * g1, OpAdd()));
            node = uniform_i(d1 < d0 ? c0 + 1 : c0);
        }
        start = node - a.r_first_leaf;
    }
    const int nl = a.r_first_leaf + 1;  // reference leaves
    const int n_blocks = (nl + NB - 1) / NB;  // a power of two
    const int sblock = start / NB;
    const int bsteps = 2 * max(sblock, n_blocks - 1 - sblock) + 1;
    // Block order.  Up to sort_max blocks: nearest first by the key
    // k_b = |c - C_b| (1 - 2^-12) - lambda(b), C_b the box centre of the block's
    // subtree node, which bounds below the distance of every query within R
    // of c to every point of the block, plus R: d(q, r) >= k_b - R.  In that
    // order, once k_b exceeds R plus the largest bound of the workgroup, no
    // later block can hold a neighbour and the sweep ends.  More blocks:
    // outward in tree order from the start block, no early end.
    const bool use_sort = n_blocks <= L::sort_max;
    float R = 0.f;  // largest |q - c| of the workgroup, rounded up
    if (use_sort) {
        const float ql = reduce64(valid ? qlen : 0.f, OpMax());
        if (lane == 0) s_misc[kMiscQlen + w] = ql;
        uint64_t *s_sort = reinterpret_cast<uint64_t *>(smem + L::off_tile_f);
        const int first = n_blocks - 1;  // heap index of block 0's node
        for (int b0 = 0; b0 < n_blocks; b0 += 32) {
            const int bi = b0 + trow;
            const bool vb = bi < n_blocks;
            const float *bx = a.rbox + int64_t(first + (vb ? bi : 0)) * 2 * DP;
            float sq = 0.f;
#pragma unroll
            for (int e = 0; e < E; e += 4) {
                const float4 lo = *reinterpret_cast<const float4 *>(bx + tcol + e);
                const float4 hi = *reinterpret_cast<const float4 *>(bx + DP + tcol + e);
                const float cv[4] = {0.5f * (lo.x + hi.x), 0.5f * (lo.y + hi.y), 0.5f * (lo.z + hi.z),
                                     0.5f * (lo.w + hi.w)};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float df = cv[u] - tc[e + u];
                    sq = fmaf(df, df, sq);
                }
            }
            sq = reduce8(sq, OpAdd());
            if (vb && (tid & 7) == 0) {
                const float key = sqrtf(sq) * (1.0f - 0x1p-12f) - a.rlam[first + bi];
                s_sort[bi] = (uint64_t(f2key(key)) << 32) | uint32_t(bi);
            }
        }
        // bitonic sort of the n_blocks (key, block) words, ascending
        for (int size = 2; size <= n_blocks; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                __syncthreads();
                for (int i = tid; i < n_blocks / 2; i += 256) {
                    const int lo = 2 * stride * (i / stride) + (i & (stride - 1));
                    const int hi = lo + stride;
                    const uint64_t x = s_sort[lo], y = s_sort[hi];
                    if ((x > y) == ((lo & size) == 0)) {
                        s_sort[lo] = y;
                        s_sort[hi] = x;
                    }
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < n_blocks; i += 256) {
            const uint64_t x = s_sort[i];
            s_order[i] = uint16_t(x & 0xffffu);
            s_okey[i] = key2f(uint32_t(x >> 32));
        }
        float rq = 0.f;
#pragma unroll
        for (int g = 0; g < kWgLeaves; ++g) rq = fmaxf(rq, s_misc[kMiscQlen + g]);
        // (|q - c| is an FP32 norm: a relative error of a few 1e-6, far inside
        // this rounding up)
        // (the wave-independent form ends each wave's sweep on its own
        // queries' bounds: their largest |q - c| is enough)
        R = uniform_f(W ? ql : rq) * (1.0f + 0x1p-12f);
        __syncthreads();
    }

    // stage the box centres C = (lo + hi) / 2 of block rb's leaves (row trow =
    // leaf NB rb + trow, this thread's E columns), centred on c and rounded
    // to BF16, with their FP32 norms and lambdas; rows past the tree and
    // empty leaves get an infinite norm.  Also publishes this wave's bounds.
    auto stage_centres = [&](int rb) {
        const int leaf = rb * NB + trow;
        const int node = a.r_first_leaf + min(leaf, nl - 1);
        const bool vrow = leaf < nl && a.rrange[node].y > 0;
        const float *bx = a.rbox + int64_t(node) * 2 * DP;
        float rn = 0.f;
#pragma unroll
        for (int e = 0; e < E; e += 4) {
            const float4 lo = *reinterpret_cast<const float4 *>(bx + tcol + e);
            const float4 hi = *reinterpret_cast<const float4 *>(bx + DP + tcol + e);
            const float cv[4] = {0.5f * (lo.x + hi.x), 0.5f * (lo.y + hi.y), 0.5f * (lo.z + hi.z),
                                 0.5f * (lo.w + hi.w)};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float cd = vrow ? cv[u] - tc[e + u] : 0.f;
                rn = fmaf(cd, cd, rn);
                s_cb[trow * L::kRowBf + tcol + e + u] = (__bf16)cd;
            }
        }
        rn = reduce8(rn, OpAdd());
        if ((tid & 7) == 0) {
            s_cn[trow] = vrow ? rn : kInf;
            s_cl[trow] = vrow ? a.rlam[node] : 0.f;
        }
        const int rnb = __builtin_bit_cast(int, vrow ? rn : 0.f);
        uint32_t rmu = 0u;
#pragma unroll
        for (int g = 0; g < 8; ++g) rmu = max(rmu, (uint32_t)__builtin_amdgcn_readlane(rnb, 8 * g));
        if (lane == 0) {
            s_misc[kMiscCtrMax + w] = __builtin_bit_cast(float, rmu);
            s_misc[kMiscBound + w] = has_leaf ? bound2 : -kInf;
            s_misc[kMiscBound + kWgLeaves + w] = has_leaf ? lo_k : kInf;
        }
    };
    // after the barrier: every wave's bounds give the B(Par) term
    auto take_bounds = [&]() {
        float lo_all = kInf;
#pragma unroll
        for (int g = 0; g < kWgLeaves; ++g) lo_all = fminf(lo_all, s_misc[kMiscBound + kWgLeaves + g]);
        if (a.bound == KNN_BOUND_B && lo_all < kInf && lam2_anc < kInf) {
            // hardware square root (1 ulp): far inside the prune slack
            const float t = __builtin_amdgcn_sqrtf(lo_all) + lam2_anc;
            bound2 = uniform_f(fminf(bound2, t * t));
        }
    };
    // Score of the staged block against this wave's queries: bit i of the
    // result is set when some query p of the wave keeps leaf i, i.e. when
    // the low end of ||p - C_i||^2 does not exceed (b_p + lambda_i)^2, b_p =
    // sqrt(min(pair_kth, B^2)) rounded up (rows of invalid leaves never; with
    // KNN_BOUND_NONE every valid row)
    auto block_mask = [&]() -> uint32_t {
        float cmax = 0.f;
#pragma unroll
        for (int g = 0; g < kWgLeaves; ++g) cmax = fmaxf(cmax, s_misc[kMiscCtrMax + g]);
        const float clen = __builtin_amdgcn_sqrtf(uniform_f(cmax)) * (1.0f + 0x1p-20f);
        const uint32_t vrows = uint32_t(ballot(lane < 32 && s_cn[lane & 31] < kInf));
        f32x16_t acc;
        float lam[16];
#pragma unroll
        for (int g4 = 0; g4 < 4; ++g4) {
            const float4 v = *reinterpret_cast<const float4 *>(&s_cn[g4 * 8 + h * 4]);
            const float4 l = *reinterpret_cast<const float4 *>(&s_cl[g4 * 8 + h * 4]);
            acc[g4 * 4 + 0] = v.x;
            acc[g4 * 4 + 1] = v.y;
            acc[g4 * 4 + 2] = v.z;
            acc[g4 * 4 + 3] = v.w;
            lam[g4 * 4 + 0] = l.x;
            lam[g4 * 4 + 1] = l.y;
            lam[g4 * 4 + 2] = l.z;
            lam[g4 * 4 + 3] = l.w;
        }
        const __bf16 *arow = s_cb + j * L::kRowBf + h * 8;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bf16x8_t ar = *reinterpret_cast<const bf16x8_t *>(arow + s * 16);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar, bq[s], acc, 0, 0, 0);
        }
        const float lim = fminf(pair_kth, bound2);
        const float bp = lim < kInf ? __builtin_amdgcn_sqrtf(fmaxf(lim, 0.f)) * (1.0f + 0x1p-20f) : kInf;
        const float low0 = qn - bf16_margin<DP>(qlen, clen);
        // bit r of m16: the sign of (b_p + lambda)^2 (1 + 2^-16) - low end
        // clear (keep); then nibble g of m16 moves to rows 8 g + 4 h .. + 3
        uint32_t m16 = 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float t = bp + lam[r];
            m16 |= ((~__float_as_uint(t * t * kSlack - (acc[r] + low0))) >> 31) << r;
        }
        uint32_t m = (m16 & 0xfu) | ((m16 & 0xf0u) << 4) | ((m16 & 0xf00u) << 8) | ((m16 & 0xf000u) << 12);
        m <<= 4 * h;
        // without pruning every leaf of the block is evaluated
        m = !valid ? 0u : a.bound == KNN_BOUND_NONE ? 0xffffffffu : m;
        // OR over the wave
        float mf = __builtin_bit_cast(float, m);
        mf = reduce64(mf, OpOrBits());
        return uint32_t(uniform_i(__builtin_bit_cast(int, mf))) & vrows;
    };

    // loads of one kept leaf: range and this thread's rows (the leaf-blocked
    // copy has r_leaf_slots <= 32 rows per leaf)
    auto fetch = [&](int leaf, int2 &rr, float (&v)[E]) {
        rr = a.rrange[a.r_first_leaf + leaf];
        // unconditional loads (a clamped row; rows past the leaf are masked
        // at staging): a load under a branch makes the compiler wait for
        // every load in flight where the paths join
        const float *rp = a.rlpts + (int64_t(leaf) * a.r_leaf_slots + min(trow, a.r_leaf_slots - 1)) * DP;
#pragma unroll
        for (int e = 0; e < E; e += 2) {
            const float2 x = *reinterpret_cast<const float2 *>(rp + tcol + e);
            v[e] = x.x;
            v[e + 1] = x.y;
        }
    };
    // a kept leaf: the barrier publishes the tile staged last, which is then
    // multiplied (its LDS reads queue behind no staging writes, and this
    // leaf's loads get that much longer to land), then this leaf is staged
    // into the other buffer.
    // Every wave takes the same steps (the block's union mask is the same in
    // all of them), so the barriers match.  Safety of the two buffers: a
    // wave stages into the buffer of the tile before last, and every wave
    // finished that tile before it reached the barrier this wave has just
    // passed.
    int pend_b = 1, pend_base = 0, pend_cnt = 0;  // the staged, unmultiplied tile
    bool pend_own = false, pending = false;
    auto visit = [&](int2 rr, const float (&v)[E], bool own) {
        lds_barrier();
        ++n_staged;
        const int b = pend_b ^ 1;
        const int cnt = uniform_i(rr.y);
        if (pending) compute(pend_b, pend_base, pend_cnt, pend_own);
        stage(b, cnt, v);
        pending = true;
        pend_b = b;
        pend_base = uniform_i(rr.x);
        pend_cnt = cnt;
        pend_own = own;
    };

    const int n_steps = use_sort ? n_blocks : bsteps;
    if constexpr (!W) {
        for (int st = 0; st < n_steps; ++st) {
            int rb;
            if (use_sort) {
                rb = uniform_i(int(s_order[st]));
            } else {
                const int off = (st + 1) >> 1;
                rb = (st & 1) ? sblock + off : sblock - off;
                if (rb < 0 || rb >= n_blocks) continue;  // uniform
            }
            stage_centres(rb);
            lds_barrier();
            take_bounds();
            if (use_sort) {
                // every query's bound is at most the largest wave bound B (idle
                // waves publish -inf); the keys are ascending, so when this
                // block is out of reach, all later ones are too
                float bw = -kInf;
    #pragma unroll
                for (int g = 0; g < kWgLeaves; ++g) bw = fmaxf(bw, s_misc[kMiscBound + g]);
                const float bmax = bw < kInf ? __builtin_amdgcn_sqrtf(fmaxf(bw, 0.f)) * (1.0f + 0x1p-20f) : kInf;
                if (uniform_f(s_okey[st]) > (bmax + R) * kSlack) break;
            }
            const uint32_t own = block_mask();
            n_score += __popc(uint32_t(ballot(lane < 32 && s_cn[lane & 31] < kInf)));
            if (lane == 0) s_mask[w] = own;
            lds_barrier();
            uint32_t uni = 0;
    #pragma unroll
            for (int g = 0; g < kWgLeaves; ++g) uni |= s_mask[g];
            uni = uint32_t(uniform_i(int(uni)));
            if (!uni) continue;
            // two register sets used in turn: a leaf's loads land in the set that
            // the next visit reads, so they stay in flight while the current leaf
            // is processed (no register copy forces an early wait)
            int2 rr_a = make_int2(0, 0), rr_b = make_int2(0, 0);
            float v_a[E], v_b[E];
            int ca = __builtin_ctz(uni);
            uni &= uni - 1u;
            fetch(rb * NB + ca, rr_a, v_a);
            for (;;) {
                // past the last kept leaf the fetch repeats the current one (in
                // bounds, never visited): the loads stay unconditional
                const int cb = uni ? __builtin_ctz(uni) : ca;
                const bool more_b = uni != 0;
                uni &= uni - 1u;
                fetch(rb * NB + cb, rr_b, v_b);
                visit(rr_a, v_a, (own >> ca) & 1u);
                if (!more_b) break;
                const int cc = uni ? __builtin_ctz(uni) : cb;
                const bool more_c = uni != 0;
                uni &= uni - 1u;
                fetch(rb * NB + cc, rr_a, v_a);
                visit(rr_b, v_b, (own >> cb) & 1u);
                if (!more_c) break;
                ca = cc;
            }
        }
        if (pending) {
            lds_barrier();
            compute(pend_b, pend_base, pend_cnt, pend_own);
        }
    } else {
        // ---- wave-independent sweep: no barrier per leaf -------------------
        // Each wave scores the blocks against its own queries and multiplies
        // its own kept leaves, reading the reference side made by
        // k_wsweep_prep: per block, the query operand q - C_B (BF16) and
        // |q - C_B|^2 (FP32) serve the block Score and every tile of the
        // block.  The waves share only the block order and, through relaxed
        // LDS words, their smallest k-th distances for the B(Par) term (an
        // older value is a larger one: still a bound).
        uint32_t *s_lo = reinterpret_cast<uint32_t *>(s_misc + kMiscBound + kWgLeaves);
        auto publish = [&]() {
            if (lane == 0)
                __hip_atomic_store(&s_lo[w], __float_as_uint(lo_k), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        };
        auto par_bound = [&]() {
            if (a.bound != KNN_BOUND_B || !(lam2_anc < kInf)) return;
            float lo_all = kInf;
#pragma unroll
            for (int g = 0; g < kWgLeaves; ++g)
                lo_all = fminf(lo_all, __uint_as_float(__hip_atomic_load(&s_lo[g], __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_WORKGROUP)));
            if (lo_all < kInf) {
                const float t = __builtin_amdgcn_sqrtf(lo_all) + lam2_anc;
                bound2 = uniform_f(fminf(bound2, t * t));
            }
        };
        const __bf16 *abf = reinterpret_cast<const __bf16 *>(a.sw_abf);
        const __bf16 *cbf = reinterpret_cast<const __bf16 *>(a.sw_cbf);
        if (lane == 0) s_lo[w] = __float_as_uint(kInf);
        __syncthreads();
        for (int st = 0; st < n_steps && has_leaf; ++st) {
            int rb;
            if (use_sort) {
                rb = uniform_i(int(s_order[st]));
            } else {
                const int off = (st + 1) >> 1;
                rb = (st & 1) ? sblock + off : sblock - off;
                if (rb < 0 || rb >= n_blocks) continue;  // uniform
            }
            par_bound();
            if (use_sort) {
                // no query of this wave needs a block whose key exceeds its
                // bound plus R; the keys ascend
                const float lim = valid ? fminf(pair_kth, bound2) : -kInf;
                const float bw = uniform_f(reduce64(lim, OpMax()));
                const float bmax =
                    bw < kInf ? __builtin_amdgcn_sqrtf(fmaxf(bw, 0.f)) * (1.0f + 0x1p-20f) : kInf;
                if (uniform_f(s_okey[st]) > (bmax + R) * kSlack) break;
            }
            // query operand of the block: q - C_B at this lane's dimensions
            const float *cb = a.sw_bcen + int64_t(rb) * DP;
            bf16x8_t bqb[S];
            float qnb = 0.f;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const float4 c0 = *reinterpret_cast<const float4 *>(cb + s * 16 + h * 8);
                const float4 c1 = *reinterpret_cast<const float4 *>(cb + s * 16 + h * 8 + 4);
                const float4 x0 = *reinterpret_cast<const float4 *>(my_q + s * 16 + h * 8);
                const float4 x1 = *reinterpret_cast<const float4 *>(my_q + s * 16 + h * 8 + 4);
                const float dv[8] = {x0.x - c0.x, x0.y - c0.y, x0.z - c0.z, x0.w - c0.w,
                                     x1.x - c1.x, x1.y - c1.y, x1.z - c1.z, x1.w - c1.w};
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    qnb = fmaf(dv[e], dv[e], qnb);
                    bqb[s][e] = (__bf16)dv[e];
                }
            }
            qnb += __shfl_xor(qnb, 32);  // the query's whole |q - C_B|^2
            const float qlenb = sqrtf(qnb);
            // block Score: rows = the block's 32 leaves, value |C_L - C_B|^2
            // - 2 (q - C_B).(C_L - C_B); keep (p, L) unless the low end of
            // |p - C_L|^2 exceeds (b_p + lambda_L)^2
            const int L0 = rb * NB;
            uint32_t own;
            {
                f32x16_t acc;
                float lam[16];
#pragma unroll
                for (int g4 = 0; g4 < 4; ++g4) {
                    const float4 v = *reinterpret_cast<const float4 *>(a.sw_cn + L0 + g4 * 8 + h * 4);
                    const float4 l = *reinterpret_cast<const float4 *>(a.sw_lam + L0 + g4 * 8 + h * 4);
                    acc[g4 * 4 + 0] = v.x;
                    acc[g4 * 4 + 1] = v.y;
                    acc[g4 * 4 + 2] = v.z;
                    acc[g4 * 4 + 3] = v.w;
                    lam[g4 * 4 + 0] = l.x;
                    lam[g4 * 4 + 1] = l.y;
                    lam[g4 * 4 + 2] = l.z;
                    lam[g4 * 4 + 3] = l.w;
                }
                const __bf16 *arow = cbf + int64_t(L0 + j) * DP + h * (DP / 2);
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const bf16x8_t ar = *reinterpret_cast<const bf16x8_t *>(arow + s * 8);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar, bqb[s], acc, 0, 0, 0);
                }
                const float low0 = qnb - bf16_margin<DP>(qlenb, uniform_f(a.sw_rcb[rb]));
                const float lim = fminf(pair_kth, bound2);
                const float bp =
                    lim < kInf ? __builtin_amdgcn_sqrtf(fmaxf(lim, 0.f)) * (1.0f + 0x1p-20f) : kInf;
                uint32_t m16 = 0;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float t = bp + lam[r];
                    m16 |= ((~__float_as_uint(t * t * kSlack - (acc[r] + low0))) >> 31) << r;
                }
                uint32_t m =
                    (m16 & 0xfu) | ((m16 & 0xf0u) << 4) | ((m16 & 0xf00u) << 8) | ((m16 & 0xf000u) << 12);
                m <<= 4 * h;
                m = !valid ? 0u : a.bound == KNN_BOUND_NONE ? 0xffffffffu : m;
                float mf = reduce64(__builtin_bit_cast(float, m), OpOrBits());
                const uint32_t vrows = uint32_t(ballot(lane < 32 && a.sw_cn[L0 + j] < kInf));
                own = uint32_t(uniform_i(__builtin_bit_cast(int, mf))) & vrows;
                n_score += __popc(vrows);
            }
            // tiles of the kept leaves, software-pipelined: the next kept
            // leaf's operand rows, row norm, range and |r - C_B| bound are
            // loaded while the current one is multiplied (two register sets
            // in turn; past the last leaf the loads repeat the current one)
            struct TileIn {
                bf16x8_t ar[S];
                float rnj;  // |r_j - C_B|^2 of row j = lane % 32
                int2 rr;
                float rl;
            };
            auto tload = [&](int leaf, TileIn &t) {
                const __bf16 *arow = abf + (int64_t(leaf) * NB + j) * DP + h * (DP / 2);
#pragma unroll
                for (int s = 0; s < S; ++s) t.ar[s] = *reinterpret_cast<const bf16x8_t *>(arow + s * 8);
                t.rnj = a.sw_rn[int64_t(leaf) * NB + j];
                t.rr = a.rrange[a.r_first_leaf + leaf];
                t.rl = a.sw_rlen[leaf];
            };
            auto tile = [&](int leaf, const TileIn &t) {
                const int base = uniform_i(t.rr.x);
                const int cnt = uniform_i(t.rr.y);
                ++n_tiles;
                n_pairs += uint64_t(cnt) * uint64_t(qcount);
                // accumulators from the split-norm product (rows past the
                // leaf: +inf), then the k-steps
                f32x16_t acc = bf16_norm_init(t.rnj, t.rnj < kInf, h);
#pragma unroll
                for (int s = 0; s < S; ++s)
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(t.ar[s], bqb[s], acc, 0, 0, 0);
                // keep D < T - |q - C_B|^2 + M (strict: M is 1.25 times the
                // proven bound); T capped at FLT_MAX, rows past the leaf +inf
                const float marg = bf16_margin<DP>(qlenb, uniform_f(t.rl));
                const float lim = fminf(pair_kth, bound2) * kSlack;
                const float thr = valid ? fminf(lim - qnb + marg, 0x1.fffffep127f) : -kInf;
                float amin = acc[0];
#pragma unroll
                for (int r = 1; r < 16; ++r) amin = fminf(amin, acc[r]);
                if (!ballot(amin < thr)) return;
                uint32_t mask = 0;
#pragma unroll
                for (int r = 0; r < 16; ++r) mask |= (__float_as_uint(acc[r] - thr) >> 31) << r;
                n_cand += __popc(mask);
                const float *rows = a.rlpts + int64_t(leaf) * a.r_leaf_slots * DP;
#pragma unroll
                for (int pass = 0; pass < 16; ++pass) {
                    const bool has = mask != 0;
                    if (!ballot(has)) break;
                    ++n_pass;
                    const int r = has ? __builtin_ctz(mask) : 0;
                    mask &= mask - 1u;
                    const int row = 8 * (r >> 2) + 4 * h + (r & 3);
                    const float x0 = (float)d2_fp64_rows<DP>(my_q, rows + (has ? row : 0) * DP);
                    const float x = has ? x0 : kInf;
                    n_ins += (x < dist[K - 1]) ? 1u : 0u;
                    insert(x, base + row);
                }
                refresh_bound();
                publish();
                par_bound();
            };
            if (own) {
                auto next = [&](int prev, bool &more) -> int {
                    more = own != 0;
                    const int c = more ? __builtin_ctz(own) : prev;
                    own &= own - 1u;
                    return c;
                };
                TileIn t0, t1;
                bool m1, m2;
                int c0 = __builtin_ctz(own);
                own &= own - 1u;
                tload(L0 + c0, t0);
                for (;;) {
                    const int c1 = next(c0, m1);
                    tload(L0 + c1, t1);
                    tile(L0 + c0, t0);
                    if (!m1) break;
                    const int c2 = next(c1, m2);
                    tload(L0 + c2, t0);
                    tile(L0 + c1, t1);
                    if (!m2) break;
                    c0 = c2;
                }
            }
        }
    }

    // ---- write-out: FP64 re-score, merge the two half-lists ------------------
    // Every entry becomes its output key: the FP32 distance from the FP64
    // re-score in the high word, the original index in the low word (unused
    // slots: +inf and distinct indices that rank after every real entry).
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const bool real = valid && idx[t] >= 0 && !(a.self && idx[t] == qpos);
        const int p = real ? idx[t] : 0;
        float key = kInf;
        int o = 0x7fffffff - t - h * K;
        if (real) {
            key = (float)sqrt(d2_fp64_rows<DP>(my_q, a.rpts + int64_t(p) * DP));
            o = a.rperm[p];
        }
        dist[t] = key;
        idx[t] = o;
    }
    __syncthreads();  // the query rows are no longer read: the region holds the keys
    uint64_t *s_keys = reinterpret_cast<uint64_t *>(smem + L::off_region);
    float worst = -1.0f;
    for (int ww = 0; ww < kWgLeaves; ++ww) {
        if (w == ww) {
#pragma unroll
            for (int t = 0; t < K; ++t)
                s_keys[lane * K + t] = (uint64_t(__float_as_uint(dist[t])) << 32) | uint32_t(idx[t]);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (valid) {
                const uint64_t *mine = s_keys + lane * K;
                const uint64_t *other = s_keys + (lane ^ 32) * K;
                const int64_t row = int64_t(a.qperm[qpos]) * a.k;
#pragma unroll
                for (int t = 0; t < K; ++t) {
                    const uint64_t key = (uint64_t(__float_as_uint(dist[t])) << 32) | uint32_t(idx[t]);
                    int rank = 0;
                    for (int u = 0; u < K; ++u) rank += int(mine[u] < key) + int(other[u] < key);
                    if (rank < a.k) {
                        a.out_idx[row + rank] = idx[t] >= 0x7fffffff - 2 * K ? -1 : idx[t];
                        a.out_dist[row + rank] = dist[t];
                        if (rank == a.k - 1) worst = dist[t];
                    }
                }
            }
        }
        __syncthreads();
    }
    worst = xor32_op(worst, OpMax());
    bool fb = false;
    if (a.seed && valid) fb = !((double)worst * worst <= (double)seed2 * (1.0 - 0x1p-20));
    const float lw = reduce32(worst, OpMax());
    const uint64_t fbmask = ballot(fb);
    const float fbb = reduce32((valid && worst < kInf) ? worst : kInf, OpMin());
    if (lane == 0 && has_leaf) {
        if (a.leaf_kth) a.leaf_kth[qleaf] = fmaxf(lw, 0.0f);
        if (a.fallback && fbmask) {
            a.fallback[qleaf] = 1;
            if (a.fb_bound) a.fb_bound[qleaf] = fbb < kInf ? (fbb + lam2) * (1.0f + 0x1p-20f) : kInf;
        }
    }
    if ((a.wave_log || a.stats) && has_leaf) {
        int ins = n_ins, cand = int(n_cand);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            ins += __shfl_xor(ins, off);
            cand += __shfl_xor(cand, off);
        }
        if (a.wave_log && lane == 0) {
            uint32_t *wl = a.wave_log + int64_t(slot) * 8;
            wl[0] = 0;
            wl[1] = n_score;
            wl[2] = n_tiles;
            wl[3] = uint32_t(ins);
            wl[4] = n_pass;
            wl[5] = uint32_t(qleaf);
            wl[6] = n_staged;
            wl[7] = uint32_t(cand);
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

// the wave-independent form when the reference-side operands are given
template <int DP>
hipError_t launch_search_mfma_sweep(const SearchArgs &a, int K, int grid, hipStream_t s) {
    const bool wave_independent = a.sw_abf != nullptr;
    if (wave_independent && DP != 64) return hipErrorInvalidValue;
    switch (K) {
#define KNN_CASE(KK)                                               \
    case KK:                                                       \
        if (wave_independent)                                      \
            k_search_mfma_sweep<DP, KK, true><<<grid, 256, 0, s>>>(a); \
        else                                                       \
            k_search_mfma_sweep<DP, KK><<<grid, 256, 0, s>>>(a);   \
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
