// C-ABI entries of the range search (include/knn.h): validation, the count
// pass, an exclusive scan of the counts into offsets, the fill pass.
#include "search_range.hpp"

#include <cmath>
#include <string>

namespace knnx {

hipError_t launch_range_dp4(const RangeArgs &a, int lg, bool fill, int grid, hipStream_t s);
hipError_t launch_range_dp8(const RangeArgs &a, int lg, bool fill, int grid, hipStream_t s);
hipError_t launch_range_dp16(const RangeArgs &a, int lg, bool fill, int grid, hipStream_t s);
hipError_t launch_range_dp32(const RangeArgs &a, int lg, bool fill, int grid, hipStream_t s);
hipError_t launch_range_dp64(const RangeArgs &a, int lg, bool fill, int grid, hipStream_t s);

namespace {

hipError_t launch_dp(const RangeArgs &a, int dp, int lg, bool fill, int grid, hipStream_t s) {
    switch (dp) {
        case 4: return launch_range_dp4(a, lg, fill, grid, s);
        case 8: return launch_range_dp8(a, lg, fill, grid, s);
        case 16: return launch_range_dp16(a, lg, fill, grid, s);
        case 32: return launch_range_dp32(a, lg, fill, grid, s);
        default: return launch_range_dp64(a, lg, fill, grid, s);
    }
}

// validation and the launch arguments shared by both passes
knn_status prepare(const char *who, const knn_tree *ref, const knn_tree *query, double lo,
                   double hi, const knn_opts *opts_in, knn_opts &opts, RangeArgs &a, int &lg,
                   int &grid) {
    const std::string w(who);
    if (!ref) return fail(KNN_E_INVALID_ARG, w + ": tree is NULL");
    knn_opts_default(&opts);
    if (opts_in) opts = *opts_in;
    const knn_tree *qt = query ? query : ref;
    if (qt->d != ref->d) return fail(KNN_E_INVALID_ARG, w + ": d differs");
    if (!(lo >= 0.0) || !(hi >= lo) || !std::isfinite(hi))
        return fail(KNN_E_INVALID_ARG, w + ": need 0 <= lo <= hi < inf");
    if (qt->n > kScanMax) return fail(KNN_E_INVALID_ARG, w + ": need n_q <= 2^24");
    if (opts.exclude_self && qt != ref)
        return fail(KNN_E_INVALID_ARG, w + ": exclude_self needs the query tree to be the reference tree");
    if (opts.bound < 0 || opts.bound > 2 || opts.reserved != 0)
        return fail(KNN_E_INVALID_ARG, w + ": bad bound or reserved field");
    if (opts.precision != KNN_PREC_FP32 || opts.seed_radius || opts.leaf_kth_out)
        return fail(KNN_E_UNSUPPORTED, w + ": FP32 only, without seed radius or leaf k-th output");
    const int max_leaf = int((qt->n + qt->n_leaves - 1) / qt->n_leaves);
    lg = max_leaf <= 32 ? 5 : 6;
    const int waves = int((qt->n_leaves + (64 >> lg) - 1) / (64 >> lg));
    grid = (waves + 3) / 4;
    const double lo2 = lo * lo, hi2 = hi * hi;
    const float g = (ref->dp + 6) * 0x1p-24f;
    a = RangeArgs{};
    a.rpts = ref->pts;
    a.rbox = ref->box;
    a.rlpts = ref->lpts;
    a.rperm = ref->perm;
    a.rrange = ref->range;
    a.r_leaf_slots = ref->leaf_slots;
    a.r_first_leaf = int(ref->first_leaf);
    a.qpts = qt->pts;
    a.qbox = qt->box;
    a.qperm = qt->perm;
    a.qrange = qt->range;
    a.q_first_leaf = int(qt->first_leaf);
    a.q_n_leaves = int(qt->n_leaves);
    a.lo2 = lo2;
    a.hi2 = hi2;
    a.s_lo = float(lo2) * (1.0f - 0x1p-16f);
    a.s_hi = float(hi2) * (1.0f + 0x1p-16f);
    a.t_lo = float(lo2) * (1.0f - 2.0f * g);
    a.t_hi = float(hi2) * (1.0f + 2.0f * g);
    a.prune = opts.bound != KNN_BOUND_NONE;
    a.self = opts.exclude_self ? 1 : 0;
    return KNN_OK;
}

// runs one pass with the optional counters and device timing
knn_status run_pass(RangeArgs &a, const knn_tree *ref, int lg, bool fill, int grid,
                    const knn_opts &opts, hipStream_t s) {
    unsigned long long *dstats = nullptr;
    hipEvent_t ev[2] = {};
    struct Guard {
        hipStream_t s;
        unsigned long long *st;
        hipEvent_t *e;
        ~Guard() {
            if (st) free_async(st, s);
            for (int i = 0; i < 2; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } guard{s, nullptr, ev};
    if (opts.stats) {
        KNN_HIP(alloc_async(&dstats, ST_COUNT, s));
        guard.st = dstats;
        KNN_HIP(zero_words(dstats, 2 * ST_COUNT, s));
        for (auto &e : ev) KNN_HIP(hipEventCreate(&e));
        KNN_HIP(hipEventRecord(ev[0], s));
    }
    a.stats = dstats;
    KNN_HIP(launch_dp(a, ref->dp, lg, fill, grid, s));
    unsigned long long hst[ST_COUNT] = {};
    if (opts.stats) {
        KNN_HIP(hipEventRecord(ev[1], s));
        KNN_HIP(hipMemcpyAsync(hst, dstats, sizeof(hst), hipMemcpyDeviceToHost, s));
    }
    KNN_HIP(hipStreamSynchronize(s));
    if (opts.stats) {
        knn_stats *st = opts.stats;
        *st = knn_stats{};
        st->score_calls = int64_t(hst[ST_SCORE]);
        st->leaf_tiles = int64_t(hst[ST_TILES]);
        st->pairs = int64_t(hst[ST_PAIRS]);
        st->inserts = int64_t(hst[ST_INSERTS]);
        st->n_query_leaves = a.q_n_leaves;
        (void)hipEventElapsedTime(&st->ms_main_kernel, ev[0], ev[1]);
        st->ms_search = st->ms_main_kernel;
    }
    return KNN_OK;
}

}  // namespace
}  // namespace knnx

using namespace knnx;

extern "C" knn_status knn_range_count(const knn_tree *ref, const knn_tree *query, double lo,
                                      double hi, const knn_opts *opts, int64_t *offsets_out,
                                      int64_t *total_out, void *stream) {
    set_error("");
    knn_opts o;
    RangeArgs a;
    int lg = 0, grid = 0;
    KNN_TRY(prepare("knn_range_count", ref, query, lo, hi, opts, o, a, lg, grid));
    if (!offsets_out || !total_out)
        return fail(KNN_E_INVALID_ARG, "knn_range_count: an output pointer is NULL");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = (query ? query : ref)->n;
    int64_t *counts = nullptr, *tops = nullptr;
    struct Guard {
        hipStream_t s;
        int64_t *c, *t;
        ~Guard() {
            if (c) free_async(c, s);
            if (t) free_async(t, s);
        }
    } guard{s, nullptr, nullptr};
    KNN_HIP(alloc_async(&counts, size_t(n), s));
    guard.c = counts;
    KNN_HIP(alloc_async(&tops, size_t(scan_scratch(n)), s));
    guard.t = tops;
    a.counts = counts;
    KNN_TRY(run_pass(a, ref, lg, false, grid, o, s));
    KNN_HIP(exclusive_scan(counts, n, offsets_out, tops, s));
    KNN_HIP(hipMemcpyAsync(total_out, offsets_out + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    KNN_HIP(hipStreamSynchronize(s));
    return KNN_OK;
}

extern "C" knn_status knn_range_fill(const knn_tree *ref, const knn_tree *query, double lo,
                                     double hi, const knn_opts *opts, const int64_t *offsets,
                                     int64_t *idx_out, float *dist_out, void *stream) {
    set_error("");
    knn_opts o;
    RangeArgs a;
    int lg = 0, grid = 0;
    KNN_TRY(prepare("knn_range_fill", ref, query, lo, hi, opts, o, a, lg, grid));
    if (!offsets || !idx_out || !dist_out)
        return fail(KNN_E_INVALID_ARG, "knn_range_fill: a pointer argument is NULL");
    a.offsets = offsets;
    a.out_idx = idx_out;
    a.out_dist = dist_out;
    return run_pass(a, ref, lg, true, grid, o, (hipStream_t)stream);
}
