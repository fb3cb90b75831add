// C-ABI entry points (include/knn.h): argument validation, allocation of
// per-call scratch on the caller's stream, kernel dispatch, status codes.
#include "search.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

namespace knnx {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
const char *get_error() { return g_last_error.c_str(); }

knn_status fail(knn_status code, const std::string &msg) {
    set_error(msg);
    return code;
}

knn_status hip_fail(hipError_t e, const char *what, const char *file, int line) {
    std::string m = std::string(what) + " failed: " + hipGetErrorString(e) + " (" + file + ":" +
                    std::to_string(line) + ")";
    set_error(m);
    return e == hipErrorOutOfMemory ? KNN_E_OOM : KNN_E_DEVICE;
}

// zero n 32-bit words (a kernel rather than a memset node: callers may
// capture the search in a graph)
__global__ void k_zero_words(uint32_t *__restrict__ p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}
hipError_t zero_words(void *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_zero_words<<<int((n + 255) / 256), 256, 0, s>>>(static_cast<uint32_t *>(p), n);
    return hipGetLastError();
}

namespace {

hipError_t launch_valu(const SearchArgs &a, int d, int K, int grid, hipStream_t s) {
    switch (d <= 4 ? d : pad_dim(d)) {
        case 1: return launch_search_valu_d1(a, K, grid, s);
        case 2: return launch_search_valu_d2(a, K, grid, s);
        case 3: return launch_search_valu_d3(a, K, grid, s);
        case 4: return launch_search_valu_d4(a, K, grid, s);
        case 8: return launch_search_valu_d8(a, K, grid, s);
        case 16: return launch_search_valu_d16(a, K, grid, s);
        case 32: return launch_search_valu_d32(a, K, grid, s);
        default: return launch_search_valu_d64(a, K, grid, s);
    }
}

hipError_t launch_mfma(const SearchArgs &a, int dp, int K, int grid, hipStream_t s) {
    switch (dp) {
        case 16: return launch_search_mfma_dp16(a, K, grid, s);
        case 32: return launch_search_mfma_dp32(a, K, grid, s);
        default: return launch_search_mfma_dp64(a, K, grid, s);
    }
}

__global__ void k_count_flags(const int *__restrict__ flag, int n, int *__restrict__ count) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) atomicAdd(count, 1);
}

// Launch order of the wave slots, largest leaf radius first: a wave's cost
// grows with its leaves' radius (sparse regions have large k-th distances),
// and starting the heavy waves first keeps them from finishing last.
// Counting sort on 2048 buckets of the radius' float bits (exponent and
// three mantissa bits), descending, in one workgroup with the counters in
// LDS (the radii crowd into a few buckets, which made global atomics
// serialise).  The same launch clears the search's counters.
constexpr int kOrderBuckets = 2048;
__device__ inline int order_bucket(const float *__restrict__ lam, int first_leaf, int n_leaves,
                                   int ng, int w) {
    float r = 0.f;
    for (int g = 0; g < ng; ++g) {
        const int leaf = w * ng + g;
        if (leaf < n_leaves) r = fmaxf(r, lam[first_leaf + leaf]);
    }
    return kOrderBuckets - 1 - min(kOrderBuckets - 1, int(__float_as_uint(fmaxf(r, 0.f)) >> 20));
}
__global__ __launch_bounds__(1024) void k_order(const float *__restrict__ lam, int first_leaf,
                                                int n_leaves, int ng, int n_waves,
                                                int *__restrict__ order,
                                                unsigned long long *__restrict__ zero, int n_zero) {
    __shared__ int cnt[kOrderBuckets];
    __shared__ int part[1024];
    const int t = threadIdx.x;
    for (int i = t; i < kOrderBuckets; i += 1024) cnt[i] = 0;
    for (int i = t; i < n_zero; i += 1024) zero[i] = 0;
    __syncthreads();
    for (int w = t; w < n_waves; w += 1024)
        atomicAdd(&cnt[order_bucket(lam, first_leaf, n_leaves, ng, w)], 1);
    __syncthreads();
    // exclusive scan: two buckets per thread, then across threads
    const int c0 = cnt[2 * t], c1 = cnt[2 * t + 1];
    part[t] = c0 + c1;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const int excl = part[t] - c0 - c1;
    cnt[2 * t] = excl;
    cnt[2 * t + 1] = excl + c0;
    __syncthreads();
    for (int w = t; w < n_waves; w += 1024)
        order[atomicAdd(&cnt[order_bucket(lam, first_leaf, n_leaves, ng, w)], 1)] = w;
}

// Per-call scratch: blocks from the caching allocator, or consecutive
// 256-byte aligned pieces of a fixed arena (the no-alloc entry point; its
// size is checked before any device work)
struct Scratch {
    hipStream_t s;
    std::vector<void *> p;
    const ScratchArena *arena = nullptr;
    size_t used = 0;
    static size_t piece(size_t bytes) { return (bytes + 255) & ~size_t(255); }
    template <class T>
    hipError_t get(T **out, size_t n) {
        if (arena) {
            const size_t b = piece(n * sizeof(T));
            if (used + b > arena->bytes) return hipErrorOutOfMemory;
            *out = reinterpret_cast<T *>(arena->base + used);
            used += b;
            return hipSuccess;
        }
        hipError_t e = alloc_async(out, n, s);
        if (e == hipSuccess) p.push_back(*out);
        return e;
    }
    ~Scratch() {
        if (!arena) dev_free_many(p.data(), int(p.size()), s);
    }
};

knn_status validate_tree(const knn_tree *t, const char *who) {
    if (!t) return fail(KNN_E_INVALID_ARG, std::string(who) + ": tree is NULL");
    return KNN_OK;
}

}  // namespace

knn_status search(const knn_tree *ref, const knn_tree *query, int k, const knn_opts *opts_in,
                  int64_t *idx_out, float *dist_out, hipStream_t s, DebugReq *dbg,
                  const ScratchArena *arena) {
    KNN_TRY(validate_tree(ref, "knn_search"));
    knn_opts opts;
    knn_opts_default(&opts);
    if (opts_in) opts = *opts_in;
    const knn_tree *qt = query ? query : ref;
    const bool same = qt == ref;
    if (!idx_out || !dist_out) return fail(KNN_E_INVALID_ARG, "knn_search: output pointer is NULL");
    if (qt->d != ref->d) return fail(KNN_E_INVALID_ARG, "knn_search: query and reference d differ");
    if (k < 1 || k > 64) return fail(KNN_E_INVALID_ARG, "knn_search: need 1 <= k <= 64");
    if (int64_t(k) >= ref->n)
        return fail(KNN_E_INVALID_ARG, "knn_search: need k < m (number of reference points)");
    if (opts.exclude_self && !same)
        return fail(KNN_E_INVALID_ARG,
                    "knn_search: exclude_self needs the query tree to be the reference tree");
    if (opts.bound < 0 || opts.bound > 2) return fail(KNN_E_INVALID_ARG, "knn_search: bad bound");
    if (opts.precision < 0 || opts.precision > 1)
        return fail(KNN_E_INVALID_ARG, "knn_search: bad precision");
    if (opts.reserved != 0) return fail(KNN_E_INVALID_ARG, "knn_search: reserved field must be 0");

    if (opts.exclude_self && k > 63)
        return fail(KNN_E_INVALID_ARG, "knn_search: need k <= 63 with exclude_self");
    const int K = list_size_for(k + (opts.exclude_self ? 1 : 0));
    int max_leaf = int((qt->n + qt->n_leaves - 1) / qt->n_leaves);
    int lpl_log2 = 0;
    while ((1 << lpl_log2) < max_leaf) ++lpl_log2;
    if (lpl_log2 < 3) lpl_log2 = 3;  // the FP32 kernels take 8..64 lanes per leaf
    if (qt->dp >= 32) lpl_log2 = 6;
    const bool bf16 = opts.precision == KNN_PREC_BF16;
    if (bf16) {
        if (ref->dp < 16)
            return fail(KNN_E_UNSUPPORTED, "knn_search: BF16 tiles need d >= 9 (a 16-wide k-step)");
        if (max_leaf > 32 || ref->leaf_slots > 32)
            return fail(KNN_E_UNSUPPORTED, "knn_search: BF16 tiles need leaves of <= 32 points");
        lpl_log2 = 6;  // one query leaf per wave
    }
    // BF16 at stride 16 or 32 with lists of <= 16: the traversal kernel with
    // matrix-core tiles (two query leaves per wave, its own seeded pass)
    const bool mt = bf16 && !dbg && (ref->dp == 16 || ref->dp == 32) && K <= 16;
    if (mt) lpl_log2 = 5;
    const int NG = 64 >> lpl_log2;
    const int nq_leaves = int(qt->n_leaves);
    if (dbg && (ref->d != 3 || bf16 || opts.seed_radius || K > 16))
        return fail(KNN_E_UNSUPPORTED,
                    "knn_debug_search_log: the debug kernel covers d = 3, FP32, no seed, "
                    "lists of at most 16");

    const int waves = (nq_leaves + NG - 1) / NG;
    const int grid = (waves + 3) / 4;
    const bool use_order = (!bf16 || ref->dp < 64) && waves > 1;
    if (arena) {
        const size_t need = Scratch::piece(2 * ST_COUNT * sizeof(unsigned long long)) +
                            (opts.seed_radius ? Scratch::piece(size_t(nq_leaves) * 4) +
                                                    Scratch::piece(size_t(nq_leaves + 1) * 4)
                                              : 0) +
                            (use_order ? Scratch::piece(size_t(waves) * 4) : 0);
        if (dbg || need > arena->bytes)
            return fail(KNN_E_INVALID_ARG,
                        "knn_search_noalloc: the query tree needs " + std::to_string(need) +
                            " bytes of scratch, more than the fixed " +
                            std::to_string(arena->bytes));
    }

    Scratch sc{s, {}, arena};
    unsigned long long *dstats = nullptr;
    if (opts.stats) KNN_HIP(sc.get(&dstats, 2 * ST_COUNT));  // cleared before the launch
    int *fb_flag = nullptr, *fb_count = nullptr;
    float *fb_bound = nullptr;
    if (opts.seed_radius) {
        KNN_HIP(sc.get(&fb_bound, nq_leaves));
        KNN_HIP(sc.get(&fb_flag, nq_leaves + 1));  // the flags, then their count
        fb_count = fb_flag + nq_leaves;
        KNN_HIP(zero_words(fb_flag, nq_leaves + 1, s));
    }

    SearchArgs a{};
    a.rpts = ref->pts;
    a.rperm = ref->perm;
    a.rrange = ref->range;
    a.rbox = ref->box;
    a.rlam = ref->lam;
    a.rlpts = ref->lpts;
    a.r_leaf_slots = ref->leaf_slots;
    a.r_first_leaf = int(ref->first_leaf);
    a.qpts = qt->pts;
    a.qperm = qt->perm;
    a.qrange = qt->range;
    a.qbox = qt->box;
    a.qlam = qt->lam;
    a.q_first_leaf = int(qt->first_leaf);
    a.q_n_leaves = nq_leaves;
    a.active = nullptr;
    a.d = ref->d;
    a.k = k;
    a.lpl_log2 = lpl_log2;
    a.bound = opts.bound;
    a.self = opts.exclude_self ? 1 : 0;
    a.seed = opts.seed_radius;
    a.out_idx = idx_out;
    a.out_dist = dist_out;
    a.leaf_kth = opts.leaf_kth_out;
    a.fallback = fb_flag;
    a.fb_bound = fb_bound;
    a.stats = dstats;
    // debug aid: KNN_WAVE_LOG=<file> writes per-wave counters of the main launch
    const char *wlog_path = arena ? nullptr : std::getenv("KNN_WAVE_LOG");
    uint32_t *wlog = nullptr;

    if (dbg) {
        if (dbg->log) {
            unsigned int *cnt = nullptr;
            KNN_HIP(sc.get(&cnt, 1));
            KNN_HIP(zero_words(cnt, 1, s));
            a.dbg_log = dbg->log;
            a.dbg_count = cnt;
            a.dbg_cap = int(std::min<int64_t>(dbg->cap, INT32_MAX));
        }
        a.far_first = dbg->far_first;
        a.tile_log = dbg->tile_log;
        a.tile_cnt = dbg->tile_cnt;
        a.tile_cap = dbg->tile_cap;
        a.tile_replay = dbg->tile_replay;
    }
    if (wlog_path) {
        KNN_HIP(sc.get(&wlog, size_t(grid) * 4 * 8));
        KNN_HIP(zero_words(wlog, int64_t(grid) * 32, s));
        a.wave_log = wlog;
    }
    // (the stride-64 BF16 kernel sweeps reference leaves per workgroup of
    // four query leaves and takes no order)
    if (use_order) {
        int *order = nullptr;
        KNN_HIP(sc.get(&order, waves));
        k_order<<<1, 1024, 0, s>>>(qt->lam, int(qt->first_leaf), nq_leaves, NG, waves, order,
                                   dstats, dstats ? 2 * ST_COUNT : 0);
        a.order = order;
    } else if (dstats) {
        KNN_HIP(zero_words(dstats, 2 * 2 * ST_COUNT, s));
    }
    // the d = 64 sweep's wave-independent form: its reference-side operands,
    // made once per search (not in the no-alloc form, which keeps the staged
    // sweep: they take 4 KB per reference leaf)
    if (bf16 && ref->dp == 64 && !arena && !dbg) {
        const int nl = int(ref->first_leaf) + 1;
        const size_t pl = size_t((nl + kSweepBlock - 1) / kSweepBlock) * kSweepBlock;  // padded leaves
        uint16_t *abf = nullptr, *cbf = nullptr;
        float *rn = nullptr, *rlen = nullptr, *cn = nullptr, *lam = nullptr, *bcen = nullptr, *rcb = nullptr;
        KNN_HIP(sc.get(&abf, pl * 32 * 64));
        KNN_HIP(sc.get(&rn, pl * 32));
        KNN_HIP(sc.get(&rlen, pl));
        KNN_HIP(sc.get(&cbf, pl * 64));
        KNN_HIP(sc.get(&cn, pl));
        KNN_HIP(sc.get(&lam, pl));
        KNN_HIP(sc.get(&bcen, pl / kSweepBlock * 64));
        KNN_HIP(sc.get(&rcb, pl / kSweepBlock));
        KNN_HIP(launch_wsweep_prep(a, abf, rn, rlen, cbf, cn, lam, bcen, rcb, s));
        a.sw_abf = abf;
        a.sw_rn = rn;
        a.sw_rlen = rlen;
        a.sw_cbf = cbf;
        a.sw_cn = cn;
        a.sw_lam = lam;
        a.sw_bcen = bcen;
        a.sw_rcb = rcb;
    }
    // device timing (not in the no-alloc form: it creates no events)
    hipEvent_t ev[4] = {};
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            for (int i = 0; i < 4; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } eg{ev};
    const bool timing = opts.stats && !arena;
    if (timing) {
        for (auto &e : ev) KNN_HIP(hipEventCreate(&e));
        KNN_HIP(hipEventRecord(ev[0], s));
    }
    KNN_HIP(dbg    ? launch_search_valu_debug_d3(a, K, grid, s)
            : mt   ? (ref->dp == 16 ? launch_search_mt_d16(a, K, grid, s)
                                    : launch_search_mt_d32(a, K, grid, s))
            : bf16 ? launch_mfma(a, ref->dp, K, grid, s)
                   : launch_valu(a, ref->d, K, grid, s));
    if (timing) KNN_HIP(hipEventRecord(ev[1], s));
    if (opts.seed_radius) {
        k_count_flags<<<(nq_leaves + 255) / 256, 256, 0, s>>>(fb_flag, nq_leaves, fb_count);
    }
    if (opts.seed_radius && bf16 && !mt) {
        // fallback of the BF16 kernels: the listed leaves again, from empty
        // lists, with the proven bound of the first pass as their initial
        // bound (the FP32 kernel runs this second pass in the same wave)
        SearchArgs b = a;
        b.seed = fb_bound;
        b.fallback = nullptr;
        b.fb_bound = nullptr;
        b.active = fb_flag;
        b.stats = dstats ? dstats + ST_COUNT : nullptr;  // counted separately
        b.wave_log = nullptr;
        KNN_HIP(launch_mfma(b, ref->dp, K, grid, s));
    }
    if (timing) KNN_HIP(hipEventRecord(ev[2], s));
    unsigned long long hst[2 * ST_COUNT] = {};
    int hfb = 0;
    if (dstats)
        KNN_HIP(hipMemcpyAsync(hst, dstats, sizeof(hst), hipMemcpyDeviceToHost, s));
    if (fb_count) KNN_HIP(hipMemcpyAsync(&hfb, fb_count, sizeof(int), hipMemcpyDeviceToHost, s));
    unsigned int hdbg = 0;
    if (dbg && a.dbg_count)
        KNN_HIP(hipMemcpyAsync(&hdbg, a.dbg_count, sizeof(hdbg), hipMemcpyDeviceToHost, s));
    KNN_HIP(hipStreamSynchronize(s));
    if (dbg) {
        dbg->n_records = int64_t(hdbg);
        dbg->ms_kernel = 0.f;
        if (timing) (void)hipEventElapsedTime(&dbg->ms_kernel, ev[0], ev[1]);
    }
    if (wlog) {
        std::vector<uint32_t> h(size_t(grid) * 32);
        KNN_HIP(hipMemcpy(h.data(), wlog, h.size() * 4, hipMemcpyDeviceToHost));
        if (FILE *f = std::fopen(wlog_path, "wb")) {
            std::fwrite(h.data(), 4, h.size(), f);
            std::fclose(f);
        }
    }
    if (opts.stats) {
        knn_stats *st = opts.stats;
        const unsigned long long *f = hst + ST_COUNT;
        st->score_calls = int64_t(hst[ST_SCORE] + f[ST_SCORE]);
        st->leaf_tiles = int64_t(hst[ST_TILES] + f[ST_TILES]);
        st->pairs = int64_t(hst[ST_PAIRS] + f[ST_PAIRS]);
        st->inserts = int64_t(hst[ST_INSERTS] + f[ST_INSERTS]);
        st->fallback_queries = int64_t(hst[ST_FB_QUERIES]);
        st->fallback_pairs = int64_t(f[ST_PAIRS]);
        st->fallback_leaves = hfb;
        st->ms_main_kernel = st->ms_search = 0.f;
        if (timing) {
            (void)hipEventElapsedTime(&st->ms_main_kernel, ev[0], ev[1]);
            (void)hipEventElapsedTime(&st->ms_search, ev[0], ev[2]);
        }
        st->n_query_leaves = nq_leaves;
    }
    return KNN_OK;
}

// Scratch of knn_search_noalloc: one fixed array per device, resolved to
// its device address once per device (host code never uses the array's
// name as an address).  Calls that overlap on one device share it.
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

knn_status noalloc_arena(ScratchArena *out) {
    int dev = 0;
    KNN_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(KNN_E_UNSUPPORTED, "knn_search_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
        g_scratch_ptr[dev] = static_cast<char *>(p);
    }
    *out = ScratchArena{g_scratch_ptr[dev], kNoAllocScratchBytes};
    return KNN_OK;
}

}  // namespace knnx

using namespace knnx;

extern "C" {

void knn_opts_default(knn_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->bound = KNN_BOUND_B;
    o->precision = KNN_PREC_FP32;
}

const char *knn_status_string(knn_status s) {
    switch (s) {
        case KNN_OK: return "ok";
        case KNN_E_INVALID_ARG: return "invalid argument";
        case KNN_E_NONFINITE: return "non-finite input";
        case KNN_E_OOM: return "out of device memory";
        case KNN_E_DEVICE: return "device error";
        case KNN_E_MODEL: return "seed model error";
        case KNN_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *knn_last_error(void) { return get_error(); }

knn_status knn_release_cached_memory(void) {
    hipError_t e = release_cached();
    if (e != hipSuccess)
        return fail(KNN_E_DEVICE, std::string("knn_release_cached_memory: ") + hipGetErrorString(e));
    return KNN_OK;
}

int64_t knn_cached_bytes(void) { return int64_t(cached_bytes()); }

static knn_status check_build_args(const char *who, const float *points, int64_t n, int32_t d,
                                   int32_t leaf_size) {
    const std::string w(who);
    if (!points) return fail(KNN_E_INVALID_ARG, w + ": points is NULL");
    if (n < 1 || n >= (int64_t(1) << 31) - 64)
        return fail(KNN_E_INVALID_ARG, w + ": need 1 <= n < 2^31 - 64");
    if (d < 1 || d > 64) return fail(KNN_E_INVALID_ARG, w + ": need 1 <= d <= 64");
    if (leaf_size < 1 || leaf_size > 64)
        return fail(KNN_E_INVALID_ARG, w + ": need 1 <= leaf_size <= 64");
    return KNN_OK;
}

knn_status knn_build_tree(const float *points, int64_t n, int32_t d, int32_t leaf_size,
                          void *stream, knn_tree **out) {
    set_error("");
    if (!out) return fail(KNN_E_INVALID_ARG, "knn_build_tree: out is NULL");
    *out = nullptr;
    KNN_TRY(check_build_args("knn_build_tree", points, n, d, leaf_size));
    return build_tree(points, n, d, leaf_size, (hipStream_t)stream, out);
}

knn_status knn_build_tree_pair(const float *ref_points, int64_t n_ref, const float *query_points,
                               int64_t n_query, int32_t d, int32_t leaf_size, void *stream,
                               knn_tree **ref_out, knn_tree **query_out) {
    set_error("");
    if (!ref_out || !query_out)
        return fail(KNN_E_INVALID_ARG, "knn_build_tree_pair: an output pointer is NULL");
    *ref_out = nullptr;
    *query_out = nullptr;
    KNN_TRY(check_build_args("knn_build_tree_pair (reference)", ref_points, n_ref, d, leaf_size));
    KNN_TRY(check_build_args("knn_build_tree_pair (query)", query_points, n_query, d, leaf_size));
    return build_tree_pair(ref_points, n_ref, query_points, n_query, d, leaf_size,
                           (hipStream_t)stream, ref_out, query_out);
}

knn_status knn_all_knn(const float *ref_points, int64_t n_ref, const float *query_points,
                       int64_t n_query, int32_t d, int32_t leaf_size, int32_t k,
                       const knn_opts *opts, int64_t *idx_out, float *dist_out, void *stream) {
    set_error("");
    KNN_TRY(check_build_args("knn_all_knn (reference)", ref_points, n_ref, d, leaf_size));
    if (query_points)
        KNN_TRY(check_build_args("knn_all_knn (query)", query_points, n_query, d, leaf_size));
    return all_knn(ref_points, n_ref, query_points, n_query, d, leaf_size, k, opts, idx_out,
                   dist_out, (hipStream_t)stream);
}

void knn_free_tree(knn_tree *tree) { free_tree(tree); }

knn_status knn_tree_get_info(const knn_tree *t, knn_tree_info *info) {
    if (!t || !info) return fail(KNN_E_INVALID_ARG, "knn_tree_get_info: NULL argument");
    info->n = t->n;
    info->d = t->d;
    info->dp = t->dp;
    info->leaf_size = t->leaf_size;
    info->depth = t->depth;
    info->n_nodes = t->n_nodes;
    info->n_leaves = t->n_leaves;
    info->first_leaf = t->first_leaf;
    info->points = t->pts;
    info->perm = t->perm;
    info->node_range = reinterpret_cast<const int32_t *>(t->range);
    info->box = t->box;
    info->lambda = t->lam;
    info->split_dim = t->split_dim;
    info->ms_build = t->ms_build;
    return KNN_OK;
}

knn_status knn_search(const knn_tree *ref, const knn_tree *query, int32_t k,
                      const knn_opts *opts, int64_t *idx_out, float *dist_out, void *stream) {
    set_error("");
    return search(ref, query, k, opts, idx_out, dist_out, (hipStream_t)stream);
}

knn_status knn_search_noalloc(const knn_tree *ref, const knn_tree *query, int32_t k,
                              const knn_opts *opts, int64_t *idx_out, float *dist_out,
                              void *stream) {
    set_error("");
    KNN_TRY(validate_tree(ref, "knn_search_noalloc"));
    int dev = 0;
    KNN_HIP(hipGetDevice(&dev));
    if (ref->device != dev || (query && query->device != dev))
        return fail(KNN_E_INVALID_ARG,
                    "knn_search_noalloc: the trees belong to another device than the current one");
    ScratchArena arena{};
    KNN_TRY(noalloc_arena(&arena));
    return search(ref, query, k, opts, idx_out, dist_out, (hipStream_t)stream, nullptr, &arena);
}

knn_status knn_debug_search_log(const knn_tree *ref, const knn_tree *query, int32_t k,
                                const knn_opts *opts, int32_t far_first, uint32_t *log_out,
                                int64_t capacity, int64_t *n_records, int64_t *idx_out,
                                float *dist_out, void *stream) {
    set_error("");
    if (!n_records || (capacity > 0 && !log_out) || capacity < 0)
        return fail(KNN_E_INVALID_ARG, "knn_debug_search_log: bad log arguments");
    if (far_first != 0 && far_first != 1)
        return fail(KNN_E_INVALID_ARG, "knn_debug_search_log: far_first must be 0 or 1");
    DebugReq dbg{far_first, log_out, capacity, 0};
    knn_status st = search(ref, query, k, opts, idx_out, dist_out, (hipStream_t)stream, &dbg);
    *n_records = dbg.n_records;
    return st;
}

knn_status knn_debug_tile_replay(const knn_tree *ref, const knn_tree *query, int32_t k,
                                 const knn_opts *opts_in, int64_t *idx_out, float *dist_out,
                                 float *ms_search, float *ms_replay, int64_t *pairs,
                                 void *stream) {
    set_error("");
    if (!ref || !ms_search || !ms_replay || !pairs)
        return fail(KNN_E_INVALID_ARG, "knn_debug_tile_replay: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    knn_opts opts;
    knn_opts_default(&opts);
    if (opts_in) opts = *opts_in;
    knn_stats st{};
    opts.stats = &st;
    const knn_tree *qt = query ? query : ref;
    constexpr int kCap = 512;  // tiles per wave (the heaviest waves of the
                               // 1M x 1M d = 3 search take about 130)
    const size_t slots = size_t(qt->n_leaves);  // at least one per wave
    uint32_t *tlog = nullptr, *tcnt = nullptr;
    KNN_HIP(alloc_async(&tlog, slots * kCap, s));
    KNN_HIP(alloc_async(&tcnt, slots, s));
    struct Guard {
        hipStream_t s;
        void *a, *b;
        ~Guard() {
            free_async(a, s);
            free_async(b, s);
        }
    } guard{s, tlog, tcnt};
    DebugReq rec{0, nullptr, 0, 0};
    rec.tile_log = tlog;
    rec.tile_cnt = tcnt;
    rec.tile_cap = kCap;
    KNN_TRY(search(ref, query, k, &opts, idx_out, dist_out, s, &rec));
    *ms_search = rec.ms_kernel;
    *pairs = st.pairs;
    std::vector<uint32_t> cnt(slots);
    KNN_HIP(hipMemcpy(cnt.data(), tcnt, slots * sizeof(uint32_t), hipMemcpyDeviceToHost));
    // waves past the last query leaf never wrote a count: only the first
    // ceil(leaves / leaves per wave) entries are read
    const int max_leaf = int((qt->n + qt->n_leaves - 1) / qt->n_leaves);
    int lg = 3;
    while ((1 << lg) < max_leaf) ++lg;
    const size_t waves = (slots + (64 >> lg) - 1) / (64 >> lg);
    for (size_t w = 0; w < waves; ++w)
        if (cnt[w] > uint32_t(kCap))
            return fail(KNN_E_UNSUPPORTED, "knn_debug_tile_replay: a wave evaluated more than 512 tiles");
    DebugReq rep = rec;
    rep.tile_replay = 1;
    KNN_TRY(search(ref, query, k, &opts, idx_out, dist_out, s, &rep));
    *ms_replay = rep.ms_kernel;
    return KNN_OK;
}

knn_status knn_search_points(const knn_tree *ref, const float *queries, int64_t n_q, int32_t k,
                             const knn_opts *opts, int64_t *idx_out, float *dist_out,
                             void *stream) {
    set_error("");
    KNN_TRY(validate_tree(ref, "knn_search_points"));
    if (!queries) return fail(KNN_E_INVALID_ARG, "knn_search_points: queries is NULL");
    if (opts && opts->exclude_self)
        return fail(KNN_E_INVALID_ARG,
                    "knn_search_points: exclude_self needs the query tree to be the reference tree");
    knn_tree *qt = nullptr;
    knn_status st = knn_build_tree(queries, n_q, ref->d, ref->leaf_size, stream, &qt);
    if (st != KNN_OK) return st;
    st = search(ref, qt, k, opts, idx_out, dist_out, (hipStream_t)stream);
    if (st == KNN_OK && opts && opts->stats) opts->stats->ms_query_build = qt->ms_build;
    free_tree(qt);
    return st;
}

}  // extern "C"
