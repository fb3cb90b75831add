// Euclidean minimum spanning tree by dual-tree Boruvka (Section "Boruvka's
// Algorithm", Algorithms 7 and 8 with the traversal-merge loop), one
// kd-tree serving as query and reference tree.
//
// Components.  Every point carries a component label (a tree position);
// each node carries the label shared by all of its points, -1 if they lie
// in several components, -2 if it is empty.  A round:
//   1. node labels, bottom-up (leaves, then one launch per level);
//   2. every point's nearest point in another component (k_boruvka): the
//      k-NN walk with k = 1, where Score also prunes a reference node whose
//      points all lie in the query point's component, and the bound is
//      B(N_q) of the k-NN section with D_p = the component's candidate
//      distance D(F(p)), shared by all points of a component through an
//      atomic minimum.  (B2 stays a bound: a node holding two components
//      holds an edge of length <= 2 lambda between them.)  Before the walk
//      each point's nearest outside point from the previous round, when it
//      is still outside, seeds its component's D;
//   3. every component's edge: the smallest of its points' candidates under
//      the strict order (squared length, smaller index, larger index), taken
//      in three atomic-minimum passes (length, then the two endpoints), so
//      the tree is the unique minimum spanning tree under that order and no
//      merge closes a cycle (the printed BaseCase keeps the first of equal
//      lengths, which can);
//   4. merge: each component hooks onto the one its edge reaches; two
//      components that chose the same edge keep the smaller label as root
//      and the edge once; pointer jumping, relabelling.
// Rounds repeat until n - 1 edges are chosen (at most about log2 n rounds,
// as every component merges with at least one other per round).
//
// Distances: FP32 filters, every candidate decided on its FP64 squared
// length (products rounded, summed in dimension order).
#include "walk.hpp"

#include <cmath>
#include <string>
#include <vector>

namespace knnx {
namespace {

struct EmstArgs {
    const float *pts, *box, *lpts, *lam;
    const int32_t *perm;
    const int2 *range;
    int leaf_slots, first_leaf, n_leaves;
    const int32_t *comp, *node_comp;
    unsigned int *cbound;  // per label: FP32 bits of an upper bound of the
                           // component's shortest edge, squared
    double *best_d2;       // per position: nearest point in another component
    int32_t *best_r;       //   (its position, -1 if none)
    int bound;             // knn_bound
    int shared;            // 0 in the first round: every component is one
                           // point, whose own candidate is its bound
    unsigned long long *stats;
};

__device__ inline unsigned int f32_bits_up(double x) {
    // a float not below x (x >= 0): round to nearest, then one step up
    const float f = (float)x;
    return __float_as_uint(f) + ((double)f < x ? 1u : 0u);
}

// Minimum per component over a wavefront: points of a component sit mostly
// in runs of consecutive tree positions, so a segmented minimum over runs of
// lanes with the same label (Hillis-Steele steps with segment-start flags)
// leaves one atomic per run instead of one per point (device-scope atomics
// are the cost of these passes).  Returns true in the last lane of each run
// of active lanes, with the run's minimum in m.
template <class T>
__device__ inline bool run_min(int c, T v, bool act, T &m) {
    const int lane = threadIdx.x & 63;
    const int key = act ? c : -1 - lane;  // inactive lanes: a run of their own
    const int kprev = __shfl_up(key, 1);
    const int knext = __shfl_down(key, 1);
    bool f = lane == 0 || kprev != key;  // a run starts within the window
    m = v;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const T mo = __shfl_up(m, s);
        const bool fo = __shfl_up(int(f), s) != 0;
        if (lane >= s && !f) m = min(m, mo);
        if (lane >= s) f = f || fo;
    }
    return act && (lane == 63 || knext != key);
}

template <int DP, int LG>
__global__ __launch_bounds__(256) void k_boruvka(const EmstArgs a) {
    constexpr float kInf = __builtin_inff();
    constexpr float kSlack = 1.0f + 0x1p-16f;
    constexpr float kGamma = 1.0f + (DP + 6) * 0x1p-24f;
    constexpr int NG = 64 >> LG;
    const int lane = threadIdx.x & 63;
    const int wave = xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (wave * NG >= a.n_leaves) return;
    const int g = lane >> LG, li = lane & ((1 << LG) - 1);
    const int slot = wave * NG + g;
    const bool has_leaf = slot < a.n_leaves;
    const int qnode = a.first_leaf + (has_leaf ? slot : 0);
    const int2 qr = has_leaf ? a.range[qnode] : make_int2(0, 0);
    const bool valid = has_leaf && li < qr.y;
    const int qpos = qr.x + li;
    float q[DP];
    {
        const float *qp = a.pts + int64_t(valid ? qpos : 0) * DP;
#pragma unroll
        for (int j = 0; j < DP; ++j) q[j] = valid ? qp[j] : 0.f;
    }
    const int c = valid ? a.comp[qpos] : -3;
    const float lam2 = has_leaf ? 2.0f * a.lam[qnode] : 0.f;
    double best2 = __builtin_inf();
    int bpos = -1, bperm = 0x7fffffff;
    float pb = kInf;  // this point's bound, squared
    uint32_t n_score = 0, n_tiles = 0;
    uint64_t n_pairs = 0;
    const int n_valid = __popcll(ballot(valid));

    // D_p = min(own candidate, the component's shared bound); the leaf's
    // B(N_q) = min(max D_p, min D_p + 2 lambda); the point's bound is
    // min(D_p, B(leaf))
    auto refresh = [&]() {
        if (a.bound == KNN_BOUND_NONE) return;
        float dp = kInf;
        if (valid && a.shared)
            dp = __uint_as_float(
                __hip_atomic_load(&a.cbound[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (bpos >= 0) dp = fminf(dp, __uint_as_float(f32_bits_up(best2)));
        float hi = valid ? dp : -kInf, lo = valid ? dp : kInf;
#pragma unroll
        for (int l = 0; l < LG; ++l) {
            hi = xor_level(hi, l, OpMax());
            lo = xor_level(lo, l, OpMin());
        }
        float b = hi;
        if (a.bound == KNN_BOUND_B) {
            const float t = __builtin_amdgcn_sqrtf(lo) + lam2;
            b = fminf(b, t * t);
        }
        pb = fminf(dp, b);
    };
    refresh();
    auto score = [&](int node, float &key) -> bool {
        ++n_score;
        const int nc = uniform_i(a.node_comp[node]);
        float dmin2, dmax2;
        box_dist2<DP>(q, a.box + int64_t(node) * 2 * DP, dmin2, dmax2);
        key = uniform_f(dmin2);
        if (nc == -2) return false;
        const bool keep = valid && nc != c && !(dmin2 > pb * kSlack);
        return ballot(keep) != 0;
    };
    constexpr int CH = DP >= 32 ? 1 : 32 / DP;
    auto leaf = [&](int node) {
        ++n_tiles;
        const int2 rr = a.range[node];
        const int base = uniform_i(rr.x);
        const int cnt = uniform_i(rr.y);
        const float *rp = a.lpts + int64_t(node - a.first_leaf) * a.leaf_slots * DP;
        n_pairs += uint64_t(cnt) * uint64_t(n_valid);
        bool improved = false;
        // the filter follows the best candidate within the leaf too
        float thr = pb * kGamma;
        for (int t0 = 0; t0 < cnt; t0 += CH) {
#pragma unroll
            for (int cc = 0; cc < CH; ++cc) {
                const int t = t0 + cc;
                const int rc = t < cnt ? a.comp[base + t] : c;
                float sd = 0.f;
#pragma unroll
                for (int j = 0; j < DP; ++j) {
                    const float df = q[j] - rp[t * DP + j];
                    sd = fmaf(df, df, sd);
                }
                const bool cand = valid && rc != c && sd <= thr;
                if (cand) {
                    const double x = d2_fp64_unfused<DP>(q, rp + t * DP);
                    const int ro = a.perm[base + t];
                    if (x < best2 || (x == best2 && ro < bperm)) {
                        best2 = x;
                        bpos = base + t;
                        bperm = ro;
                        improved = true;
                        thr = fminf(thr, __uint_as_float(f32_bits_up(best2)) * kGamma);
                    }
                }
            }
        }
        if (a.shared && a.bound != KNN_BOUND_NONE) {
            // one atomic per run of lanes of one component
            unsigned int m;
            if (run_min(c, improved ? f32_bits_up(best2) : ~0u, improved, m)) atomicMin(&a.cbound[c], m);
        }
        refresh();
    };
    tree_walk(a.first_leaf, score, leaf, [](float k0, float k1) { return k1 < k0; });
    if (valid) {
        a.best_d2[qpos] = best2;
        a.best_r[qpos] = bpos;
    }
    if (a.stats && lane == 0) {
        atomicAdd(&a.stats[ST_SCORE], (unsigned long long)n_score);
        atomicAdd(&a.stats[ST_TILES], (unsigned long long)n_tiles);
        atomicAdd(&a.stats[ST_PAIRS], (unsigned long long)n_pairs);
    }
}

template <int DP>
hipError_t launch_boruvka(const EmstArgs &a, int lg, int grid, hipStream_t s) {
    if (lg == 5)
        k_boruvka<DP, 5><<<grid, 256, 0, s>>>(a);
    else
        k_boruvka<DP, 6><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_dp(const EmstArgs &a, int dp, int lg, int grid, hipStream_t s) {
    switch (dp) {
        case 4: return launch_boruvka<4>(a, lg, grid, s);
        case 8: return launch_boruvka<8>(a, lg, grid, s);
        case 16: return launch_boruvka<16>(a, lg, grid, s);
        case 32: return launch_boruvka<32>(a, lg, grid, s);
        default: return launch_boruvka<64>(a, lg, grid, s);
    }
}

inline int blocks(int64_t n) { return int((n + 255) / 256); }

__global__ void k_init(int32_t *comp, int64_t *flag, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        comp[i] = i;
        flag[i] = 0;
    }
}

// node labels: leaves from their points, then each level from its children
__global__ void k_leaf_comp(const int2 *range, const int32_t *comp, int first_leaf, int n_leaves,
                            int32_t *node_comp) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n_leaves) return;
    const int2 r = range[first_leaf + l];
    int lab = -2;
    for (int i = 0; i < r.y; ++i) {
        const int ci = comp[r.x + i];
        lab = lab == -2 ? ci : (lab == ci ? lab : -1);
    }
    node_comp[first_leaf + l] = lab;
}
__global__ void k_level_comp(int32_t *node_comp, int first, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int node = first + i;
    const int x = node_comp[2 * node + 1], y = node_comp[2 * node + 2];
    node_comp[node] = x == -2 ? y : (y == -2 ? x : (x == y ? x : -1));
}

__global__ void k_round_reset(unsigned int *cbound, unsigned long long *cbest, unsigned int *cmin,
                              unsigned int *cmax, int32_t *parent, int *unconverged, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *unconverged = 0;
    if (i >= n) return;
    cbound[i] = __float_as_uint(__builtin_inff());
    cbest[i] = ~0ull;
    cmin[i] = ~0u;
    cmax[i] = ~0u;
    parent[i] = i;
}

// last round's nearest outside point, when it is still outside, bounds the
// new component's shortest edge
__global__ void k_seed_bounds(const double *best_d2, const int32_t *best_r, const int32_t *comp,
                              unsigned int *cbound, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = i < n ? best_r[i] : -1;
    const int c = i < n ? comp[i] : 0;
    const bool act = r >= 0 && comp[r] != c;
    unsigned int m;
    if (run_min(c, act ? f32_bits_up(best_d2[i]) : ~0u, act, m)) atomicMin(&cbound[c], m);
}

// the component's edge: smallest (length, smaller index, larger index).
// In the first round every component is one point (labels are the points'
// own positions): a plain store
__device__ inline unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }
__global__ void k_pick_len(const double *best_d2, const int32_t *best_r, const int32_t *comp,
                           unsigned long long *cbest, int n, int singletons) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = i < n && best_r[i] >= 0;
    if (singletons) {
        if (act) cbest[i] = dbits(best_d2[i]);
        return;
    }
    const int c = i < n ? comp[i] : 0;
    unsigned long long m;
    if (run_min(c, act ? dbits(best_d2[i]) : ~0ull, act, m)) atomicMin(&cbest[c], m);
}
__global__ void k_pick_ends(const double *best_d2, const int32_t *best_r, const int32_t *comp,
                            const int32_t *perm, const unsigned long long *cbest,
                            unsigned int *cmin, unsigned int *cmax, int stage, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || best_r[i] < 0) return;
    const int c = comp[i];
    if (dbits(best_d2[i]) != cbest[c]) return;
    const unsigned int p = perm[i], r = perm[best_r[i]];
    const unsigned int lo = min(p, r), hi = max(p, r);
    if (stage == 0)
        atomicMin(&cmin[c], lo);
    else if (lo == cmin[c])
        atomicMin(&cmax[c], hi);
}
// the (unique) point holding the component's edge hooks the component onto
// the one the edge reaches and records the edge under the component's label
__global__ void k_hook(const double *best_d2, const int32_t *best_r, const int32_t *comp,
                       const int32_t *perm, const unsigned long long *cbest,
                       const unsigned int *cmin, const unsigned int *cmax, int32_t *parent,
                       int32_t *eu, int32_t *ev, float *ew, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || best_r[i] < 0) return;
    const int c = comp[i];
    const unsigned int p = perm[i], r = perm[best_r[i]];
    if (dbits(best_d2[i]) != cbest[c] || min(p, r) != cmin[c] || max(p, r) != cmax[c]) return;
    parent[c] = comp[best_r[i]];
    eu[c] = int32_t(min(p, r));
    ev[c] = int32_t(max(p, r));
    ew[c] = (float)sqrt(best_d2[i]);
}
// two components that chose the same edge: the smaller label stays root
__global__ void k_break_pairs(const unsigned long long *cbest, int32_t *parent, int n) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n || cbest[c] == ~0ull) return;
    const int o = parent[c];
    if (parent[o] == c && c < o) parent[c] = c;
}
// a component that hooked keeps its edge; one count per workgroup (all
// counts go to one word: device-scope atomics on it serialise)
__global__ __launch_bounds__(1024) void k_mark_edges(const unsigned long long *cbest,
                                                     const int32_t *parent, int64_t *flag,
                                                     int *count, int n) {
    __shared__ int total;
    if (threadIdx.x == 0) total = 0;
    __syncthreads();
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const bool m = c < n && cbest[c] != ~0ull && parent[c] != c;
    if (m) flag[c] = 1;
    const uint64_t b = ballot(m);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(&total, int(__popcll(b)));
    __syncthreads();
    if (threadIdx.x == 0 && total) atomicAdd(count, total);
}
// Path compression: every label climbs to its root, one parent per step, in
// one launch; another thread's update only shortens a path (each value read
// is an ancestor), so any interleaving is correct.  The hooks form a forest
// (the strict edge order leaves no cycle but the two-component pairs, which
// k_break_pairs removed), so each climb ends; a label still below its root
// after `steps` steps raises *unconverged and the host finishes with
// pointer jumping.
__global__ void k_compress(int32_t *parent, int *unconverged, int steps, int n) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    int p = parent[c];
    for (int it = 0; it < steps; ++it) {
        const int g = parent[p];
        if (g == p) break;
        p = g;
    }
    parent[c] = p;
    if (parent[p] != p) atomicOr(unconverged, 1);
}
__global__ void k_jump(int32_t *parent, int n) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) parent[c] = parent[parent[c]];
}
__global__ void k_relabel(int32_t *comp, const int32_t *parent, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) comp[i] = parent[comp[i]];
}
__global__ void k_compact(const int64_t *flag, const int64_t *off, const int32_t *eu,
                          const int32_t *ev, const float *ew, int64_t *ou, int64_t *ov, float *ow,
                          int n) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n || !flag[c]) return;
    const int64_t k = off[c];
    ou[k] = eu[c];
    ov[k] = ev[c];
    ow[k] = ew[c];
}

}  // namespace
}  // namespace knnx

using namespace knnx;

extern "C" knn_status knn_emst(const knn_tree *t, const knn_opts *opts_in, int64_t *edge_u,
                               int64_t *edge_v, float *edge_w, int32_t *rounds_out,
                               void *stream) {
    set_error("");
    const std::string w = "knn_emst";
    if (!t) return fail(KNN_E_INVALID_ARG, w + ": tree is NULL");
    knn_opts opts;
    knn_opts_default(&opts);
    if (opts_in) opts = *opts_in;
    if (opts.bound < 0 || opts.bound > 2 || opts.reserved != 0 || opts.exclude_self)
        return fail(KNN_E_INVALID_ARG, w + ": bad bound, reserved field or exclude_self");
    if (opts.precision != KNN_PREC_FP32 || opts.seed_radius || opts.leaf_kth_out)
        return fail(KNN_E_UNSUPPORTED, w + ": FP32 only, without seed radius or leaf k-th output");
    const int64_t n64 = t->n;
    if (n64 > kScanMax) return fail(KNN_E_INVALID_ARG, w + ": need n <= 2^24");
    if (n64 > 1 && (!edge_u || !edge_v || !edge_w))
        return fail(KNN_E_INVALID_ARG, w + ": an edge output is NULL");
    hipStream_t s = (hipStream_t)stream;
    const int n = int(n64);
    if (rounds_out) *rounds_out = 0;
    if (opts.stats) *opts.stats = knn_stats{};
    if (n == 1) return KNN_OK;

    // scratch
    std::vector<void *> held;
    struct Guard {
        hipStream_t s;
        std::vector<void *> *p;
        ~Guard() { dev_free_many(p->data(), int(p->size()), s); }
    } guard{s, &held};
    auto get = [&](auto **out, size_t count) -> hipError_t {
        hipError_t e = alloc_async(out, count, s);
        if (e == hipSuccess) held.push_back(*out);
        return e;
    };
    int32_t *comp, *node_comp, *best_r, *parent, *eu, *ev;
    unsigned int *cbound, *cmin, *cmax;
    unsigned long long *cbest, *dstats = nullptr;
    double *best_d2;
    float *ew;
    int64_t *flag, *off, *tops;
    int *count;
    KNN_HIP(get(&comp, n));
    KNN_HIP(get(&node_comp, size_t(t->n_nodes)));
    KNN_HIP(get(&best_r, n));
    KNN_HIP(get(&parent, n));
    KNN_HIP(get(&eu, n));
    KNN_HIP(get(&ev, n));
    KNN_HIP(get(&ew, n));
    KNN_HIP(get(&cbound, n));
    KNN_HIP(get(&cmin, n));
    KNN_HIP(get(&cmax, n));
    KNN_HIP(get(&cbest, n));
    KNN_HIP(get(&best_d2, n));
    KNN_HIP(get(&flag, n));
    KNN_HIP(get(&off, size_t(n) + 1));
    KNN_HIP(get(&tops, size_t(scan_scratch(n))));
    KNN_HIP(get(&count, 2));  // [0] edges chosen so far, [1] compression unfinished
    if (opts.stats) {
        KNN_HIP(get(&dstats, ST_COUNT));
        KNN_HIP(zero_words(dstats, 2 * ST_COUNT, s));
    }
    KNN_HIP(zero_words(count, 2, s));
    k_init<<<blocks(n), 256, 0, s>>>(comp, flag, n);
    KNN_HIP(hipGetLastError());

    EmstArgs a{};
    a.pts = t->pts;
    a.box = t->box;
    a.lpts = t->lpts;
    a.lam = t->lam;
    a.perm = t->perm;
    a.range = t->range;
    a.leaf_slots = t->leaf_slots;
    a.first_leaf = int(t->first_leaf);
    a.n_leaves = int(t->n_leaves);
    a.comp = comp;
    a.node_comp = node_comp;
    a.cbound = cbound;
    a.best_d2 = best_d2;
    a.best_r = best_r;
    a.bound = opts.bound;
    a.stats = dstats;
    const int max_leaf = int((t->n + t->n_leaves - 1) / t->n_leaves);
    const int lg = max_leaf <= 32 ? 5 : 6;
    const int grid = (int((t->n_leaves + (64 >> lg) - 1) / (64 >> lg)) + 3) / 4;
    int jumps = 1;
    while ((1 << jumps) < n) ++jumps;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    struct EvGuard {
        hipEvent_t *a, *b;
        ~EvGuard() {
            if (*a) (void)hipEventDestroy(*a);
            if (*b) (void)hipEventDestroy(*b);
        }
    } eg{&ev0, &ev1};
    if (opts.stats) {
        KNN_HIP(hipEventCreate(&ev0));
        KNN_HIP(hipEventCreate(&ev1));
        KNN_HIP(hipEventRecord(ev0, s));
    }
    int edges = 0, rounds = 0;
    while (edges < n - 1) {
        if (++rounds > 64) return fail(KNN_E_DEVICE, w + ": no progress after 64 rounds");
        k_leaf_comp<<<blocks(a.n_leaves), 256, 0, s>>>(t->range, comp, a.first_leaf, a.n_leaves,
                                                      node_comp);
        for (int l = t->depth - 1; l >= 0; --l)
            k_level_comp<<<blocks(1 << l), 256, 0, s>>>(node_comp, (1 << l) - 1, 1 << l);
        k_round_reset<<<blocks(n), 256, 0, s>>>(cbound, cbest, cmin, cmax, parent, count + 1, n);
        if (rounds > 1) k_seed_bounds<<<blocks(n), 256, 0, s>>>(best_d2, best_r, comp, cbound, n);
        KNN_HIP(hipGetLastError());
        a.shared = rounds > 1 ? 1 : 0;
        KNN_HIP(launch_dp(a, t->dp, lg, grid, s));
        k_pick_len<<<blocks(n), 256, 0, s>>>(best_d2, best_r, comp, cbest, n, rounds == 1 ? 1 : 0);
        k_pick_ends<<<blocks(n), 256, 0, s>>>(best_d2, best_r, comp, t->perm, cbest, cmin, cmax, 0, n);
        k_pick_ends<<<blocks(n), 256, 0, s>>>(best_d2, best_r, comp, t->perm, cbest, cmin, cmax, 1, n);
        k_hook<<<blocks(n), 256, 0, s>>>(best_d2, best_r, comp, t->perm, cbest, cmin, cmax, parent,
                                         eu, ev, ew, n);
        k_break_pairs<<<blocks(n), 256, 0, s>>>(cbest, parent, n);
        k_mark_edges<<<(n + 1023) / 1024, 1024, 0, s>>>(cbest, parent, flag, count, n);
        k_compress<<<blocks(n), 256, 0, s>>>(parent, count + 1, 64, n);
        KNN_HIP(hipGetLastError());
        int now[2] = {0, 0};
        KNN_HIP(hipMemcpyAsync(now, count, sizeof(now), hipMemcpyDeviceToHost, s));
        KNN_HIP(hipStreamSynchronize(s));
        if (now[1])
            for (int j = 0; j < jumps; ++j) k_jump<<<blocks(n), 256, 0, s>>>(parent, n);
        k_relabel<<<blocks(n), 256, 0, s>>>(comp, parent, n);
        KNN_HIP(hipGetLastError());
        if (now[0] <= edges) return fail(KNN_E_DEVICE, w + ": a round chose no edge");
        edges = now[0];
    }
    KNN_HIP(exclusive_scan(flag, n, off, tops, s));
    k_compact<<<blocks(n), 256, 0, s>>>(flag, off, eu, ev, ew, edge_u, edge_v, edge_w, n);
    KNN_HIP(hipGetLastError());
    unsigned long long hst[ST_COUNT] = {};
    if (opts.stats) {
        KNN_HIP(hipEventRecord(ev1, s));
        KNN_HIP(hipMemcpyAsync(hst, dstats, sizeof(hst), hipMemcpyDeviceToHost, s));
    }
    KNN_HIP(hipStreamSynchronize(s));
    if (edges != n - 1) return fail(KNN_E_DEVICE, w + ": chose more than n - 1 edges");
    if (rounds_out) *rounds_out = rounds;
    if (opts.stats) {
        knn_stats *st = opts.stats;
        st->score_calls = int64_t(hst[ST_SCORE]);
        st->leaf_tiles = int64_t(hst[ST_TILES]);
        st->pairs = int64_t(hst[ST_PAIRS]);
        st->n_query_leaves = a.n_leaves;
        (void)hipEventElapsedTime(&st->ms_search, ev0, ev1);
        st->ms_main_kernel = st->ms_search;
    }
    return KNN_OK;
}
