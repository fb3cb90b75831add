// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "knn.h"

// ---------------------------------------------------------------------------
// error plumbing: every C-ABI entry point returns a knn_status and records a
// message in a thread-local string.
// ---------------------------------------------------------------------------
namespace knnx {

void set_error(const std::string &msg);
const char *get_error();

struct Status {
    knn_status code = KNN_OK;
    bool ok() const { return code == KNN_OK; }
};

knn_status fail(knn_status code, const std::string &msg);
knn_status hip_fail(hipError_t e, const char *what, const char *file, int line);

}  // namespace knnx

#define KNN_HIP(expr)                                                          \
    do {                                                                       \
        hipError_t _e = (expr);                                                \
        if (_e != hipSuccess) return knnx::hip_fail(_e, #expr, __FILE__, __LINE__); \
    } while (0)

#define KNN_TRY(expr)                                                          \
    do {                                                                       \
        knn_status _s = (expr);                                                \
        if (_s != KNN_OK) return _s;                                           \
    } while (0)

// ---------------------------------------------------------------------------
// kd-tree handle.  Nodes are in heap order: children of i are 2i+1, 2i+2;
// node i at depth l covers a contiguous range of the tree-ordered points.
// ---------------------------------------------------------------------------
struct knn_tree {
    int64_t n = 0;
    int32_t d = 0, dp = 0, leaf_size = 0, depth = 0;
    int64_t n_nodes = 0, n_leaves = 0, first_leaf = 0;
    float *pts = nullptr;         // (n + kPadRows) x dp, tree order, zero padded
    float *lpts = nullptr;        // n_leaves x leaf_slots x dp: each leaf's points in a
                                  // fixed block, unused slots FLT_MAX (never a candidate)
    int32_t leaf_slots = 0;       // largest leaf, rounded up to a multiple of 8
    int32_t *perm = nullptr;      // n: original row of tree position
    int2 *range = nullptr;        // n_nodes: (start, count)
    float *box = nullptr;         // n_nodes x 2 x dp: lo, hi
    float *lam = nullptr;         // n_nodes
    int32_t *split_dim = nullptr; // n_nodes
    int device = 0;
    hipStream_t stream = nullptr;  // stream the tree was built on; its memory is
                                   // released in order on this stream
    float ms_build = 0.f;
};

namespace knnx {

constexpr int kPadRows = 64;  // zero rows after the last point: tile loops may
                              // read a whole 64-row window past any leaf start

inline int pad_dim(int d) {
    if (d <= 4) return 4;
    if (d <= 8) return 8;
    if (d <= 16) return 16;
    if (d <= 32) return 32;
    return 64;
}

inline int depth_for(int64_t n, int leaf) {
    int L = 0;
    while (((n + (int64_t(1) << L) - 1) >> L) > leaf) ++L;
    return L;
}

// FP32 -> order-preserving uint32 (after mapping -0 to +0, so that equal
// floats give equal keys).
__host__ __device__ inline uint32_t f2key(float f) {
    if (f == 0.0f) f = 0.0f;
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float key2f(uint32_t k) {
    uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}

// Cross-lane reductions: DPP row permutations within 16 lanes (no LDS
// crossbar), shuffles across rows.  Each helper returns, in
// every lane, op over the lane group; for a commutative op all lanes of the
// group hold the identical value.
template <int CTRL>
__device__ inline float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 CTRL, 0xF, 0xF, false));
}
// op of the lane's value and that of lane ^ 32 (or ^ 16): crossing rows of
// 16 lanes goes through the LDS crossbar (the gfx950 row-swap builtins are
// not used: this compiler treats both of their results as the same value)
template <class Op>
__device__ inline float xor32_op(float v, Op op) { return op(v, __shfl_xor(v, 32)); }
template <class Op>
__device__ inline float xor16_op(float v, Op op) { return op(v, __shfl_xor(v, 16)); }
template <class Op>
__device__ inline float reduce8(float v, Op op) {
    v = op(v, dpp_f<0xB1>(v));   // quad_perm [1,0,3,2]
    v = op(v, dpp_f<0x4E>(v));   // quad_perm [2,3,0,1]
    return op(v, dpp_f<0x141>(v));  // row_half_mirror
}
template <class Op>
__device__ inline float reduce16(float v, Op op) {
    const float r = reduce8(v, op);
    return op(r, dpp_f<0x140>(r));  // row_mirror
}
template <class Op>
__device__ inline float reduce32(float v, Op op) { return xor16_op(reduce16(v, op), op); }
template <class Op>
__device__ inline float reduce64(float v, Op op) { return xor32_op(reduce32(v, op), op); }
// one step of a lane-group reduction: combines each lane with its partner at
// level l (lane ^ (1 << l) for l = 0, 1, 4, 5; for l = 2, 3 the mirrored lane
// of the same 8 / 16, which is the same partner group once levels below l are
// reduced).  l is wave-uniform, so the switch is a scalar branch.
template <class Op>
__device__ inline float xor_level(float v, int l, Op op) {
    switch (l) {
        case 0: return op(v, dpp_f<0xB1>(v));
        case 1: return op(v, dpp_f<0x4E>(v));
        case 2: return op(v, dpp_f<0x141>(v));
        case 3: return op(v, dpp_f<0x140>(v));
        case 4: return op(v, __shfl_xor(v, 16));
        default: return op(v, __shfl_xor(v, 32));
    }
}
struct OpAdd {
    __device__ float operator()(float a, float b) const { return a + b; }
};
struct OpMax {
    __device__ float operator()(float a, float b) const { return fmaxf(a, b); }
};
struct OpMin {
    __device__ float operator()(float a, float b) const { return fminf(a, b); }
};
// Sum over the lanes 0 .. DP-1 that hold one dimension each (the other lanes
// hold zeros), complete in lane 0: within one row of 16 lanes by DPP alone,
// the crossbar only for the rows beyond.
template <int DP>
__device__ inline float sum_dim_lanes(float v) {
    if constexpr (DP <= 16) return reduce16(v, OpAdd());
    else if constexpr (DP <= 32) return reduce32(v, OpAdd());
    else return reduce64(v, OpAdd());
}
// Insert (x, id) into a k-list held in registers, sorted ascending, K slots,
// the largest entry dropped (Algorithm 2 keeps each list sorted).  Slot j of
// the new list is the median of (old[j-1], x, old[j]) (old[-1] = -inf): old
// slots below x stay, x lands in the first slot it beats, the rest move up
// one.  Its index follows the value: from slot j - 1 when x < old[j-1], x's
// when x < old[j], else unchanged, so equal distances keep their older entry
// first.  x = +inf changes nothing.  Every lane runs it (no divergence).
template <int K>
__device__ __forceinline__ void sorted_insert(float (&dist)[K], int (&idx)[K], float x, int id) {
#pragma unroll
    for (int j = K - 1; j > 0; --j) {
        const bool cp = x < dist[j - 1];
        const bool cj = x < dist[j];
        idx[j] = cp ? idx[j - 1] : (cj ? id : idx[j]);
        dist[j] = __builtin_amdgcn_fmed3f(dist[j - 1], x, dist[j]);
    }
    idx[0] = x < dist[0] ? id : idx[0];
    dist[0] = fminf(x, dist[0]);
}

// bitwise OR of the two values' bit patterns (a 32-bit mask carried in a float)
struct OpOrBits {
    __device__ float operator()(float a, float b) const {
        return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, a) | __builtin_bit_cast(uint32_t, b));
    }
};


// tree construction (tree_build.hip)
knn_status build_tree(const float *points, int64_t n, int d, int leaf, hipStream_t s,
                      knn_tree **out);
knn_status build_tree_pair(const float *pa, int64_t na, const float *pb, int64_t nb, int d,
                           int leaf, hipStream_t s, knn_tree **out_a, knn_tree **out_b);
void free_tree(knn_tree *t);
// builds (overlapped when query_points is given), search, frees (tree_build.hip)
knn_status all_knn(const float *ref_points, int64_t n_ref, const float *query_points,
                   int64_t n_query, int d, int leaf, int k, const knn_opts *opts,
                   int64_t *idx_out, float *dist_out, hipStream_t s);
// debug requests of knn_debug_search_log: visit order and the Score log
struct DebugReq {
    int far_first;
    uint32_t *log;       // device, cap records, or NULL
    int64_t cap;
    int64_t n_records;   // out: records the kernel produced (may exceed cap)
    uint32_t *tile_log = nullptr;  // device: the per-wave tile lists (see SearchArgs)
    uint32_t *tile_cnt = nullptr;
    int tile_cap = 0;
    int tile_replay = 0;
    float ms_kernel = 0.f;         // out: device time of the kernel launch
};
// a fixed device region the search takes its scratch from instead of the
// allocator (knn_search_noalloc)
struct ScratchArena {
    char *base;
    size_t bytes;
};
// the search of an existing pair of trees (api.hip)
knn_status search(const knn_tree *ref, const knn_tree *query, int k, const knn_opts *opts,
                  int64_t *idx_out, float *dist_out, hipStream_t s, DebugReq *dbg = nullptr,
                  const ScratchArena *arena = nullptr);

// Device memory for trees and scratch comes from the library's caching
// allocator (memory.hip): stream-ordered reuse of released blocks.
hipError_t dev_alloc(void **p, size_t bytes, hipStream_t s);
void dev_free(void *p, hipStream_t s);
void dev_free_many(void *const *ps, int n, hipStream_t s);  // one event for all
hipError_t release_cached();
size_t cached_bytes();
template <class T>
inline hipError_t alloc_async(T **p, size_t count, hipStream_t s) {
    return dev_alloc(reinterpret_cast<void **>(p), count * sizeof(T) + 256, s);
}
inline void free_async(void *p, hipStream_t s) { dev_free(p, s); }

}  // namespace knnx
