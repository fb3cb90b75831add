// FP32 traversal kernel: the pruning dual-tree traversal (Algorithm 1) with
// the k-NN Score (Algorithm 3) and BaseCase (Algorithm 2), one wavefront per
// group of query leaves.
//
// Mapping
//   * a wavefront owns NG = 64 / LPL consecutive query leaves (LPL = lanes per
//     leaf, a power of two >= the largest leaf); lane = one query point;
//   * it walks the reference tree depth first, nearer child first (the
//     closer-of / farther-of order of Gray's AllNN, Algorithm 4), without a
//     stack: one bit per depth records which child was entered first, and the
//     farther child is re-scored when the walk climbs back (bounds only
//     tighten, so the re-score can only prune more);
//   * Score: each query point is scored as a singleton child of its leaf, so
//     N_q = {p}, d_min(N_q, N_r) = distance from p to the node's box, and
//     B(N_q) = min(D_p[k], B(leaf)) (B1({p}) = D_p[k], lambda = 0, and the
//     parent term).  The wave enters a node when any of its points would;
//   * reference nodes are wave-uniform (scalar loads); a reference leaf is the
//     BaseCase tile, read from the leaf-blocked copy of the points (fixed
//     slots per leaf, unused slots at FLT_MAX so their distance is +inf);
//   * the k-list is a sorted register array of K slots; for k < K the first
//     K-k slots hold -inf and never move, so the k-th value is always slot
//     K-1 (Algorithm 2 keeps each list sorted by distance);
//   * after each tile the leaf bound is refreshed:
//        B1 = max over the leaf's queries of D_p[k]              (B1(N_q))
//        B2 = min over the leaf's queries of D_p[k] + 2 lambda    (rho = lambda)
//        BP = min over the queries of an ancestor + 2 lambda(anc) (B(Par))
//        B  = min(B1, B2, BP)
//     and a node is pruned when d_min^2 > B^2 (1 + 2^-16).
//   * all-kNN of a set on itself keeps k+1 entries per list; the query's own
//     point (distance 0) takes one of them and is dropped at write-out, so no
//     per-pair index test is needed.
//
// Precision.  Distances are squared FP32 direct differences over the D
// computed dimensions.  For D > 8 a candidate passing the FP32 filter is
// re-scored in FP64 before it enters the list (RESCORE), because the FP32
// error (d+2) u can exceed the 1e-6 relative acceptance window at high d.
// The final k entries are always re-scored in FP64 and sorted by
// (distance, original index).
//
// Three forms of one kernel, chosen at compile time (MODE):
//   * kValuPlain: the search;
//   * kValuDebug: every Score call logged with each leaf's bound, the walk
//     optionally farther child first, and the BaseCase leaves of each wave
//     recorded or replayed without the walk;
//   * kValuSeeded: a seed radius (not in the paper; only an initial value of
//     a query leaf's pruning bound) joins the minimum of the leaf bound, and
//     a leaf whose k-th distances exceed its seed is searched again inside
//     the same wave, from empty lists, with the proven bound of the first
//     pass.
// The plain form carries none of the other two forms' state.
//
// Matrix-core tiles (MT, d = 16 or 32, two leaves of 17..32 points per wave,
// lists of up to 16): the same walk, Score and bounds; a reference leaf's
// BaseCase distances come from the BF16 tile of bf16_tile.hpp, centred on
// the union box centre c of the wave's two leaves, one product per query leaf
// (the 32 queries of leaf g are its columns).  Lane l is then both query
// l % 32 of leaf l / 32 and column l % 32 of half l / 32 of the products, so
// it holds half of its own query's 32 values and takes the other half from
// lane l ^ 32.  A row is a candidate when its value minus the proven margin
// beats min(D_p[k], B); candidates are re-scored in FP64 before they may
// enter the list, so the lists are those of the FP32 form.

#include "bf16_tile.hpp"
#include "search.hpp"

namespace knnx {

__device__ inline int xcd_remap(int b, int nblk) {
    // hardware deals consecutive workgroups round-robin over 8 XCDs; give
    // each XCD a contiguous run of logical blocks (spatially close query
    // leaves share reference nodes in that XCD's L2)
    const int q = nblk >> 3, r = nblk & 7;
    const int x = b & 7, i = b >> 3;
    return x * q + min(x, r) + i;
}

__device__ inline float uniform_f(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ inline int uniform_i(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

constexpr int stride_for(int D) { return D <= 4 ? 4 : D <= 8 ? 8 : D <= 16 ? 16 : D <= 32 ? 32 : 64; }

// FRESH: the query is converted at each call (an empty asm statement that
// also reads the row address hides its value), so that the compiler keeps no
// FP64 copy of it in registers across the walk.  The statement is not
// volatile and touches no memory: the walk's wave-uniform loads stay scalar.
template <int D, bool FRESH = false>
__device__ inline double d2_fp64(const float (&q)[D], const float *r) {
    double s = 0.0;
    const uint32_t salt = uint32_t(reinterpret_cast<uintptr_t>(r));
#pragma unroll
    for (int j = 0; j < D; ++j) {
        float qj = q[j];
        if constexpr (FRESH) asm("" : "+v"(qj) : "v"(salt));
        double t = (double)qj - (double)r[j];
        s = fma(t, t, s);
    }
    return s;
}

enum : int { kValuPlain = 0, kValuDebug = 1, kValuSeeded = 2 };

template <int D, int K, int LG, int MODE, bool MT>
__device__ __forceinline__ void search_valu_body(const SearchArgs &a) {
    constexpr bool DBG = MODE == kValuDebug;
    constexpr bool SEEDED = MODE == kValuSeeded;
    static_assert(!MT || ((D == 16 || D == 32) && LG == 5 && !DBG),
                  "matrix-core tiles: d = 16 or 32, two leaves of <= 32 points per wave");
    constexpr int DP = stride_for(D);
    constexpr bool RESCORE = D > 8;
    constexpr float kInf = __builtin_inff();
    constexpr float kSlack = 1.0f + 0x1p-16f;            // prune slack (squared)
    constexpr float kGamma = 1.0f + (D + 6) * 0x1p-24f;  // FP32 filter slack
    const int lane = threadIdx.x & 63;
    constexpr int lpl_log2 = LG;
    constexpr int NG = 64 >> lpl_log2;
    const int n_list = a.q_n_leaves;
    int wave;
    if (a.order) {
        // heavy slots first: the hardware starts workgroups in launch order
        const int raw = blockIdx.x * 4 + (threadIdx.x >> 6);
        if (raw * NG >= n_list) return;
        wave = uniform_i(a.order[raw]);
    } else {
        wave = xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    }
    if (wave * NG >= n_list) return;
    const int g = lane >> lpl_log2, li = lane & ((1 << lpl_log2) - 1);
    const int slot = wave * NG + g;
    const bool has_leaf = slot < n_list && (!a.active || a.active[slot] != 0);
    if (!ballot(has_leaf)) return;
    const int qleaf = has_leaf ? slot : 0;
    const int qnode = a.q_first_leaf + qleaf;
    const int2 qr = has_leaf ? a.qrange[qnode] : make_int2(0, 0);
    const bool valid0 = has_leaf && li < qr.y;  // this lane holds a query point
    bool valid = valid0;  // ... that the current pass searches
    const int qpos = qr.x + li;
    const int kk = a.k + (a.self ? 1 : 0);  // list length (self match included)

    float q[D];
    {
        const float *qp = a.qpts + int64_t(valid ? qpos : 0) * DP;
#pragma unroll
        for (int j = 0; j < D; ++j) q[j] = valid ? qp[j] : 0.f;
    }
    // union box of the wave's query leaves, for the wave-uniform visit-order
    // key.  Low d: every lane holds the whole box.  High d: lane l holds
    // dimension l of it (the key is then summed across lanes).
    constexpr bool WIDE = D >= 16;
    constexpr int UD = WIDE ? 1 : D;
    float ulo[UD], uhi[UD];
    if constexpr (!WIDE) {
        const float *qb = a.qbox + int64_t(has_leaf ? qnode : 0) * 2 * DP;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            float lo = has_leaf ? qb[j] : kInf;
            float hi = has_leaf ? qb[DP + j] : -kInf;
#pragma unroll
            for (int l = lpl_log2; l < 6; ++l) {
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
            if (sl < n_list && (!a.active || a.active[sl] != 0) && lane < DP) {
                const float *qb = a.qbox + int64_t(a.q_first_leaf + sl) * 2 * DP;
                lo = fminf(lo, qb[lane]);
                hi = fmaxf(hi, qb[DP + lane]);
            }
        }
        ulo[0] = lo;
        uhi[0] = hi;
    }
    // MT: the centre c (union box centre), this lane's centre values at its
    // operand dimensions, |q - c| of its own query and the query operands
    // -2 (q - c) of both leaves (column l % 32 of leaf g is the query of lane
    // 32 g + l % 32)
    constexpr int S = MT ? DP / 16 : 1;
    const int hh = lane >> 5, jj = lane & 31;
    [[maybe_unused]] float tcen[S * 8];
    [[maybe_unused]] bf16x8_t bq0[S], bq1[S];
    [[maybe_unused]] float qn_mt = 0.f, qlen_mt = 0.f;
    if constexpr (MT) {
        const float cl = lane < DP ? 0.5f * (ulo[0] + uhi[0]) : 0.f;
#pragma unroll
        for (int d0 = 0; d0 < D; ++d0) {
            const float df = q[d0] - __shfl(cl, d0);
            qn_mt = fmaf(df, df, qn_mt);
        }
        qlen_mt = sqrtf(qn_mt);
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int da = s * 16 + e, db = da + 8;
                const float ca = __shfl(cl, da), cb = __shfl(cl, db);
                const float c = hh ? cb : ca;
                tcen[s * 8 + e] = c;
                const float a0 = __shfl(q[da], jj), b0 = __shfl(q[db], jj);
                const float a1 = __shfl(q[da], 32 + jj), b1 = __shfl(q[db], 32 + jj);
                bq0[s][e] = (__bf16)(-2.0f * ((hh ? b0 : a0) - c));
                bq1[s][e] = (__bf16)(-2.0f * ((hh ? b1 : a1) - c));
            }
        }
    }
    const float lam2 = has_leaf ? 2.0f * a.qlam[qnode] : 0.f;
    // seeded form: a seed is only a pruning radius; NaN or negative values
    // prune everything and send the leaf to the second pass
    const float seed = (SEEDED && a.seed && has_leaf) ? fmaxf(a.seed[qleaf], 0.0f) : kInf;
    float seed2 = seed * seed;

    float dist[K];
    int idx[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        dist[j] = (j < K - kk) ? -kInf : kInf;
        idx[j] = -1;
    }
    float bound2 = (!SEEDED || a.bound == KNN_BOUND_NONE) ? kInf : seed2;
    uint32_t n_score = 0, n_tiles = 0, n_ins = 0, n_pass = 0;
    [[maybe_unused]] uint32_t n_cand = 0;  // MT: rows passing the BF16 filter
    uint64_t n_pairs = 0;
    int n_valid = __popcll(ballot(valid));

    // Prefetch into the scalar cache: a few scalar loads of lines that the
    // next steps will read, issued together with loads that are waited for
    // anyway.  Their values are folded into tacc one step later (a use at
    // once would make the wave wait for them) and reach a store that never
    // happens, so the compiler keeps them.
    uint32_t tacc = 0, q0 = 0, q1 = 0, q2 = 0;
    // per-point bound: min(D_p[k], B(leaf)); +inf without pruning
    auto point_bound2 = [&]() -> float {
        return a.bound == KNN_BOUND_NONE ? kInf : fminf(bound2, dist[K - 1]);
    };

    // Score a reference node from its box: keep when any point's d_min^2 to
    // the box is within its bound; the visit-order key is the wave-uniform
    // d_min^2 between the union of the wave's leaf boxes and the node's box
    auto score_box = [&](const float *b, float &key_out) -> bool {
        float sd = 0.f, u = 0.f;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const float lo = b[j], hi = b[DP + j];
            const float gap = fmaxf(fmaxf(lo - q[j], q[j] - hi), 0.0f);
            sd = fmaf(gap, gap, sd);
            if constexpr (!WIDE) {
                const float ug = fmaxf(fmaxf(lo - uhi[j], ulo[j] - hi), 0.0f);
                u = fmaf(ug, ug, u);
            }
        }
        if constexpr (WIDE) {
            const float lo = lane < DP ? b[lane] : 0.f, hi = lane < DP ? b[DP + lane] : 0.f;
            const float ug = fmaxf(fmaxf(lo - uhi[0], ulo[0] - hi), 0.0f);
            u = ug * ug;
            u = sum_dim_lanes<DP>(u);
        }
        const bool keep = valid && !(sd > point_bound2() * kSlack);
        key_out = uniform_f(u);
        return ballot(keep) != 0;
    };
    // debug form: one record per Score call with each leaf's bound
    auto log_score = [&](int node, bool keep) {
        if constexpr (DBG) {
            float bg[kDbgMaxLeaves];
#pragma unroll
            for (int g = 0; g < kDbgMaxLeaves; ++g)
                bg[g] = g < NG ? __builtin_bit_cast(float, __builtin_amdgcn_readlane(
                                                              __builtin_bit_cast(int, bound2), g << lpl_log2))
                               : 0.f;
            if (lane == 0 && a.dbg_count) {
                const unsigned r = atomicAdd(a.dbg_count, 1u);
                if (int(r) < a.dbg_cap) {
                    uint32_t *rec = a.dbg_log + int64_t(r) * kDbgWords;
                    rec[0] = uint32_t(node);
                    rec[1] = keep ? 1u : 0u;
                    rec[2] = uint32_t(wave * NG);
                    rec[3] = uint32_t(NG);
#pragma unroll
                    for (int g = 0; g < kDbgMaxLeaves; ++g) rec[4 + g] = __float_as_uint(bg[g]);
                }
            }
        }
    };
    auto score = [&](int node, float &key_out) -> bool {
        ++n_score;
        const bool keep = score_box(a.rbox + int64_t(node) * 2 * DP, key_out);
        log_score(node, keep);
        return keep;
    };
    // both children of an internal node: their boxes are adjacent
    auto score_children = [&](int c0, bool &k0, bool &k1, float &m0, float &m1) {
        n_score += 2;
        const float *b = a.rbox + int64_t(c0) * 2 * DP;
        // prefetch, issued with the children's box loads: the four
        // grandchildren's boxes (contiguous), or the first lines of both
        // leaves' tiles
        uint32_t p0 = 0, p1 = 0, p2 = 0;
        if constexpr (DP <= 4) {
            const bool inner = c0 < a.r_first_leaf;
            const float *g = inner ? a.rbox + int64_t(2 * c0 + 1) * 2 * DP
                                   : a.rlpts + int64_t(c0 - a.r_first_leaf) * a.r_leaf_slots * DP;
            const int s1 = inner ? 16 : a.r_leaf_slots * DP;
            const int s2 = inner ? 8 * DP - 1 : a.r_leaf_slots * DP + 16;
            p0 = __float_as_uint(g[0]);
            p1 = __float_as_uint(g[s1]);
            p2 = __float_as_uint(g[s2]);
        }
        k0 = score_box(b, m0);
        k1 = score_box(b + 2 * DP, m1);
        log_score(c0, k0);
        log_score(c0 + 1, k1);
        tacc ^= q0 ^ q1 ^ q2;
        q0 = p0;
        q1 = p1;
        q2 = p2;
    };

    auto insert = [&](float x, int id) { sorted_insert<K>(dist, idx, x, id); };

    // B(Par(N_q)) terms: the ancestors whose leaves all sit in this wave
    // (aligned sibling groups) contribute min D_p[k] + 2 lambda(ancestor)
    // from the live lists; ancestors reaching outside the wave are left out
    // of the minimum, which only loosens it.
    const bool par_ok = a.bound == KNN_BOUND_B;
    float lam2_anc[6];
#pragma unroll
    for (int s = 1; s <= 5; ++s) {
        // no such ancestor (shallow tree): the term is +inf
        lam2_anc[s] = kInf;
        if (par_ok && ((1 << lpl_log2) << (s - 1)) < 64 && has_leaf && ((qnode + 1) >> s) >= 1)
            lam2_anc[s] = 2.0f * a.qlam[((qnode + 1) >> s) - 1];
    }
    lam2_anc[0] = lam2;

    // refresh of B(N_q) after a tile.  The group reductions step through
    // the lane levels 0 .. lpl_log2-1 (uniform branches: DPP inside a row,
    // a shuffle across rows); the B(Par) terms continue one level per
    // ancestor.  The square root is the hardware one (about 1 ulp): its
    // error is far inside the prune slack.
    auto refresh_bound = [&]() {
        if (a.bound == KNN_BOUND_NONE) return;
        float hi = valid ? dist[K - 1] : -kInf;
        float lo = valid ? dist[K - 1] : kInf;
#pragma unroll
        for (int l = 0; l < lpl_log2; ++l) {
            hi = xor_level(hi, l, OpMax());
            lo = xor_level(lo, l, OpMin());
        }
        float b = hi;  // B1^2
        if (a.bound == KNN_BOUND_B) {
            const float b2 = __builtin_amdgcn_sqrtf(lo) + lam2;
            b = fminf(b, b2 * b2);
            if (par_ok) {
#pragma unroll
                for (int s = 1; s <= 5; ++s) {
                    const int l = lpl_log2 + s - 1;
                    if (l < 6) {
                        lo = xor_level(lo, l, OpMin());
                        const float bp = __builtin_amdgcn_sqrtf(lo) + lam2_anc[s];
                        b = fminf(b, bp * bp);
                    }
                }
            }
        }
        bound2 = SEEDED ? fminf(b, seed2) : b;
    };

    // BaseCase over one reference leaf: every lane against each reference
    // point, CH points per batch.  A candidate must beat min(D_p[k], B):
    // B bounds the point's final k-th distance, so anything farther cannot
    // enter its final list (equal distances aside).
    constexpr int CH = DP >= 32 ? 1 : 32 / DP;
    auto tile = [&](int node) {
        ++n_tiles;
        const int2 rr = a.rrange[node];
        const int base = uniform_i(rr.x);
        const int cnt = uniform_i(rr.y);
        const float *rp = a.rlpts + int64_t(node - a.r_first_leaf) * a.r_leaf_slots * DP;
        n_pairs += uint64_t(cnt) * uint64_t(n_valid);
        if constexpr (MT) {
            // reference operand: row jj, the dimensions of half hh, centred
            const bool vr = jj < cnt;
            const float *row = rp + (vr ? jj : 0) * DP + hh * 8;
            bf16x8_t ar[S];
            float rn = 0.f;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const float4 x0 = *reinterpret_cast<const float4 *>(row + s * 16);
                const float4 x1 = *reinterpret_cast<const float4 *>(row + s * 16 + 4);
                const float xv[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float rd = vr ? xv[e] - tcen[s * 8 + e] : 0.f;
                    rn = fmaf(rd, rd, rn);
                    ar[s][e] = (__bf16)rd;
                }
            }
            rn += __shfl_xor(rn, 32);  // the row's whole norm
            // largest |r - c| of the tile (hardware square root, nudged up:
            // the margin only needs an upper bound)
            const float rlen =
                __builtin_amdgcn_sqrtf(uniform_f(reduce32(vr ? rn : 0.f, OpMax()))) * (1.0f + 0x1p-20f);
            // the accumulators start at the row norms, from one more product
            // (the norms never leave their lanes: no LDS, no fence)
            const f32x16_t accn = bf16_norm_init(rn, vr, hh);
            f32x16_t acc0 = accn, acc1 = accn;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[s], bq0[s], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[s], bq1[s], acc1, 0, 0, 0);
            }
            // this lane's query: rows of half hh from its own leaf's product,
            // rows of the other half from lane ^ 32; keep D < T - |q'|^2 + M
            // (the margin is 1.25 times the proven bound, so the strict test
            // keeps every row the bound admits).  T is capped at FLT_MAX:
            // rows past the tile hold +inf and never pass, valid rows always
            // do while a list is not full.  Bit r: the sign of D - thr.
            const float marg = bf16_margin<DP>(qlen_mt, rlen);
            const float thr =
                valid ? fminf(fminf(dist[K - 1], bound2) * kSlack - qn_mt + marg, 0x1.fffffep127f) : -kInf;
            uint32_t mask = 0;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float own = hh ? acc1[r] : acc0[r];
                const float oth = __shfl_xor(hh ? acc0[r] : acc1[r], 32);
                mask |= (__float_as_uint(own - thr) >> 31) << r;
                mask |= (__float_as_uint(oth - thr) >> 31) << (16 + r);
            }
            if (!ballot(mask != 0)) return;  // lists unchanged, and so the bound
            n_cand += __popc(mask);
            // survivors: one per lane per round, FP64 re-score, insert (a lane
            // without one re-scores row 0 and inserts +inf, a no-op)
#pragma unroll 1
            for (int pass = 0; pass < 32; ++pass) {
                if (!ballot(mask != 0)) break;
                ++n_pass;
                const bool has = mask != 0;
                const int b = has ? __builtin_ctz(mask) : 0;
                mask &= mask - 1u;
                const int rb = b & 15, hb = b < 16 ? hh : 1 - hh;
                const int rw = 8 * (rb >> 2) + 4 * hb + (rb & 3);
                const float x = (float)d2_fp64<D, true>(q, rp + rw * DP);
                const bool ins = has && x < dist[K - 1];
                n_ins += ins ? 1u : 0u;
                insert(ins ? x : kInf, base + rw);
            }
            refresh_bound();
            return;
        }
        const float bnd = bound2 * kSlack;
        uint32_t r0 = 0, r1 = 0, r2 = 0;
        if constexpr (DP <= 4) {
            // the tile's later 64-byte lines, fetched with the first batch
            const int last = max(cnt * DP - 1, 0);
            r0 = __float_as_uint(rp[min(32, last)]);
            r1 = __float_as_uint(rp[min(64, last)]);
            r2 = __float_as_uint(rp[min(96, last)]);
        }
        for (int t0 = 0; t0 < cnt; t0 += CH) {
            float sd[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                float acc = 0.f;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const float df = q[j] - rp[(t0 + c) * DP + j];
                    acc = fmaf(df, df, acc);
                }
                sd[c] = acc;
            }
            // one wave-wide test per batch: most batches hold no candidate
            // for any lane once the lists have filled
            // (invalid lanes test against -inf; a plain compare ballots
            // straight into a lane mask)
            const float lim0 = fminf(dist[K - 1], bnd);
            const float thr0 = valid ? (RESCORE ? lim0 * kGamma : lim0) : -kInf;
            uint64_t any = 0;
#pragma unroll
            for (int c = 0; c < CH; ++c) any |= ballot(sd[c] < thr0);
            if (any == 0) continue;
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const float lim = fminf(dist[K - 1], bnd);
                const float thr = RESCORE ? lim * kGamma : lim;
                const bool cand = valid && sd[c] < thr;
                if (ballot(cand)) {
                    ++n_pass;
                    if (cand) {
                        float x = sd[c];
                        if (RESCORE) x = (float)d2_fp64<D, true>(q, rp + (t0 + c) * DP);
                        if (x < dist[K - 1]) {
                            insert(x, base + t0 + c);
                            ++n_ins;
                        }
                    }
                }
            }
        }
        tacc ^= r0 ^ r1 ^ r2;
        refresh_bound();
    };

    // debug form: replay of a recorded tile list instead of the walk
    bool replay = false;
    if constexpr (DBG) {
        replay = a.tile_replay != 0;
        if (replay) {
            const int nt = uniform_i(int(a.tile_cnt[wave]));
            for (int i = 0; i < nt; ++i) tile(uniform_i(int(a.tile_log[int64_t(wave) * a.tile_cap + i])));
        }
    }
    // ---- stackless depth-first walk, nearer child first ---------------------
    // Seeded form: a second pass follows in the same wave.  Leaves with a
    // query whose k-th distance exceeds its seed are searched again from empty
    // lists, with the proven B2 bound of the first pass as initial bound and
    // no seed; the other leaves' lanes sit out (their lists are final).  The
    // second pass of a few leaves then runs beside the other waves instead of
    // as a launch of its own.
    uint32_t s_score = 0, s_tiles = 0;  // first-pass counts
    uint64_t s_pairs = 0;
    int s_ins = 0;
    bool fb_q = false, fb_leaf = false;  // this lane's query / leaf missed its seed
    bool second = false;                 // a second pass ran in this wave
    // (a loop of at most two passes around the walk: as a closure called
    // twice, the walk made the kernel much slower)
    for (int pass = 0;; ++pass) {
        if (!replay) {
            float dm0, dm1;
            int node = 0, depth = 0;
            uint64_t nearbits = 0;
            bool down = score(0, dm0);
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
                            bool k0, k1;
                            score_children(c0, k0, k1, dm0, dm1);
                            if (!k0 && !k1) {
                                down = false;
                                continue;
                            }
                            bool right = k1 && (!k0 || dm1 < dm0);
                            if constexpr (DBG) {
                                // farther child first: the other visit order
                                if (a.far_first) right = k1 && (!k0 || dm1 > dm0);
                            }
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
                                if (score(far, dm0)) {
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
                    if constexpr (DBG) {
                        if (a.tile_log && lane == 0 && int(n_tiles) < a.tile_cap)
                            a.tile_log[int64_t(wave) * a.tile_cap + n_tiles] = uint32_t(node);
                    }
                    tile(node);
                    down = false;
                }
            }
            if constexpr (DBG) {
                if (a.tile_log && lane == 0) a.tile_cnt[wave] = n_tiles;
            }
        }
        if constexpr (!SEEDED) {
            break;
        } else {
            if (pass > 0) break;
            // seed check on the list (FP32 squared distances: their error is
            // far inside the check's factor)
            fb_q = valid && !(dist[K - 1] <= seed2 * (1.0f - 0x1p-18f));
            if (!ballot(fb_q)) break;
            float f = fb_q ? 1.0f : 0.0f;
            for (int l = 0; l < lpl_log2; ++l) f = xor_level(f, l, OpMax());
            fb_leaf = valid && f > 0.0f;
            // proven bound for the leaf: min over its full lists of D_p[k]
            // plus 2 lambda (the B2 argument holds whatever seed built the
            // lists)
            float kb = (valid && dist[K - 1] < kInf) ? __builtin_amdgcn_sqrtf(dist[K - 1]) : kInf;
            for (int l = 0; l < lpl_log2; ++l) kb = xor_level(kb, l, OpMin());
            const float pb = (kb + lam2) * (1.0f + 0x1p-18f);
            second = true;
            s_score = n_score;
            s_tiles = n_tiles;
            s_pairs = n_pairs;
            s_ins = n_ins;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                dist[j] = fb_leaf ? ((j < K - kk) ? -kInf : kInf) : dist[j];
                idx[j] = fb_leaf ? -1 : idx[j];
            }
            valid = fb_leaf;
            n_valid = __popcll(ballot(valid));
            // the proven bound stays in every refresh's minimum (as the seed
            // term did in the first pass): the fresh lists give B1 = +inf
            // until they fill
            seed2 = (a.bound == KNN_BOUND_NONE || !fb_leaf) ? kInf : pb * pb;
            bound2 = seed2;
        }
    }
    valid = valid0;

    // keeps the prefetch loads (k >= 1 always)
    if ((tacc ^ q0 ^ q1 ^ q2) == 0x7fc00001u && a.k < 0) a.out_idx[0] = 0;
    // ---- write-out: FP64 re-score of the final list, order by (d, index) ----
    // Each entry becomes its output key in place: the FP32 distance from the
    // FP64 re-score and the original index.  Padding slots (below K-kk),
    // unfilled slots and the query's own point get distinct +inf keys that
    // rank after every real entry, so real entries take ranks 0..k-1.
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const bool real = valid && idx[j] >= 0 && !(a.self && idx[j] == qpos);
        const int p = real ? idx[j] : 0;
        dist[j] = real ? (float)sqrt(d2_fp64<D>(q, a.rpts + int64_t(p) * DP)) : kInf;
        idx[j] = real ? a.rperm[p] : 0x7fffffff - j;
    }
    float worst = -1.0f;
    if (valid) {
        const int64_t row = int64_t(a.qperm[qpos]) * a.k;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            int rank = 0;
#pragma unroll
            for (int i = 0; i < K; ++i)
                rank += (dist[i] < dist[j]) || (dist[i] == dist[j] && idx[i] < idx[j]);
            if (rank < a.k) {
                a.out_idx[row + rank] = idx[j] >= 0x7fffffff - K ? -1 : idx[j];
                a.out_dist[row + rank] = dist[j];
                if (rank == a.k - 1) worst = dist[j];
            }
        }
    }
    // largest k-th distance of the leaf; seeded form: leaves searched a
    // second time are flagged (counted by the host)
    for (int l = 0; l < lpl_log2; ++l) worst = xor_level(worst, l, OpMax());
    if (has_leaf && li == 0) {
        if (a.leaf_kth) a.leaf_kth[qleaf] = fmaxf(worst, 0.0f);
        if (SEEDED && a.fallback && fb_leaf) a.fallback[qleaf] = 1;
    }
    if (a.wave_log || a.stats) {
        int ins = n_ins, ins1 = second ? s_ins : n_ins, cand = int(n_cand);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            ins += __shfl_xor(ins, off);
            if constexpr (SEEDED) ins1 += __shfl_xor(ins1, off);
            if constexpr (MT) cand += __shfl_xor(cand, off);
        }
        if (a.wave_log && lane == 0) {
            uint32_t *w = a.wave_log + int64_t(wave) * 8;
            w[0] = 0;  // no clock read: a side-effecting read here would
                       // turn every uniform load above into a vector load
            w[1] = n_score;
            w[2] = n_tiles;
            w[3] = uint32_t(ins);
            w[4] = n_pass;
            w[5] = uint32_t(qleaf);
            if constexpr (MT) w[7] = uint32_t(cand);
        }
        if constexpr (SEEDED) {
            const uint64_t fbmask = ballot(fb_q);
            if (a.stats && lane == 0) {
                // first-pass counts, then the second pass's in the fallback
                // block
                const uint32_t sc1 = second ? s_score : n_score, ti1 = second ? s_tiles : n_tiles;
                const uint64_t pa1 = second ? s_pairs : n_pairs;
                atomicAdd(&a.stats[ST_SCORE], (unsigned long long)sc1);
                atomicAdd(&a.stats[ST_TILES], (unsigned long long)ti1);
                atomicAdd(&a.stats[ST_PAIRS], (unsigned long long)pa1);
                atomicAdd(&a.stats[ST_INSERTS], (unsigned long long)ins1);
                atomicAdd(&a.stats[ST_FB_QUERIES], (unsigned long long)__popcll(fbmask));
                if (second) {
                    unsigned long long *f = a.stats + ST_COUNT;
                    atomicAdd(&f[ST_SCORE], (unsigned long long)(n_score - sc1));
                    atomicAdd(&f[ST_TILES], (unsigned long long)(n_tiles - ti1));
                    atomicAdd(&f[ST_PAIRS], (unsigned long long)(n_pairs - pa1));
                    atomicAdd(&f[ST_INSERTS], (unsigned long long)(ins - ins1));
                }
            }
        } else if (a.stats && lane == 0) {
            atomicAdd(&a.stats[ST_SCORE], (unsigned long long)n_score);
            atomicAdd(&a.stats[ST_TILES], (unsigned long long)n_tiles);
            atomicAdd(&a.stats[ST_PAIRS], (unsigned long long)n_pairs);
            atomicAdd(&a.stats[ST_INSERTS], (unsigned long long)ins);
        }
    }
}

// Plain form with short lists: at d = 8 seven waves per SIMD fit (one
// register fewer than the compiler's own choice, which allows six), at
// d = 16 six (instead of five, with a few spills); the seeded form carries
// more state and keeps the compiler's choice
template <int D, int K, int LG, int MODE = kValuPlain>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    MODE != kValuPlain || K > 16 ? 1 : D == 8 ? 7 : D == 16 ? 6 : 1))) void
k_search_valu(const SearchArgs a) {
    search_valu_body<D, K, LG, MODE, false>(a);
}

// matrix-core tiles; at d = 16 the register budget of three waves per SIMD
// keeps the accumulators in ordinary registers (four waves fit), at d = 32
// it would spill
template <int D, int K, int MODE = kValuPlain>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(D == 16 ? 3 : 1))) void
k_search_valu_mt(const SearchArgs a) {
    search_valu_body<D, K, 5, MODE, true>(a);
}

template <int D, int K, int MODE = kValuPlain>
hipError_t launch_search_valu_k(const SearchArgs &a, int grid, hipStream_t s) {
    switch (a.lpl_log2) {
        case 3: k_search_valu<D, K, 3, MODE><<<grid, 256, 0, s>>>(a); break;
        case 4: k_search_valu<D, K, 4, MODE><<<grid, 256, 0, s>>>(a); break;
        case 5: k_search_valu<D, K, 5, MODE><<<grid, 256, 0, s>>>(a); break;
        case 6: k_search_valu<D, K, 6, MODE><<<grid, 256, 0, s>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// MODE kValuPlain (the search) or kValuSeeded; the debug form has its own
// instantiation for d = 3
template <int D, int MODE = kValuPlain>
hipError_t launch_search_valu(const SearchArgs &a, int K, int grid, hipStream_t s) {
    switch (K) {
        case 4: return launch_search_valu_k<D, 4, MODE>(a, grid, s);
        case 5: return launch_search_valu_k<D, 5, MODE>(a, grid, s);
        case 8: return launch_search_valu_k<D, 8, MODE>(a, grid, s);
        case 10: return launch_search_valu_k<D, 10, MODE>(a, grid, s);
        case 11: return launch_search_valu_k<D, 11, MODE>(a, grid, s);
        case 16: return launch_search_valu_k<D, 16, MODE>(a, grid, s);
        case 32: return launch_search_valu_k<D, 32, MODE>(a, grid, s);
        case 50: return launch_search_valu_k<D, 50, MODE>(a, grid, s);
        case 51: return launch_search_valu_k<D, 51, MODE>(a, grid, s);
        case 64: return launch_search_valu_k<D, 64, MODE>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

// matrix-core tiles: two leaves per wave (LG = 5), lists of up to 16
template <int D, int MODE = kValuPlain>
hipError_t launch_search_valu_mt(const SearchArgs &a, int K, int grid, hipStream_t s) {
    if (a.lpl_log2 != 5 || a.r_leaf_slots > 32) return hipErrorInvalidValue;
    switch (K) {
        case 4: k_search_valu_mt<D, 4, MODE><<<grid, 256, 0, s>>>(a); break;
        case 5: k_search_valu_mt<D, 5, MODE><<<grid, 256, 0, s>>>(a); break;
        case 8: k_search_valu_mt<D, 8, MODE><<<grid, 256, 0, s>>>(a); break;
        case 10: k_search_valu_mt<D, 10, MODE><<<grid, 256, 0, s>>>(a); break;
        case 11: k_search_valu_mt<D, 11, MODE><<<grid, 256, 0, s>>>(a); break;
        case 16: k_search_valu_mt<D, 16, MODE><<<grid, 256, 0, s>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace knnx
