// C-ABI entry of the k-furthest-neighbour search (include/knn.h): argument
// validation, per-call scratch, dispatch of k_search_far by stride.
#include "search.hpp"

#include <string>

namespace knnx {
namespace {

hipError_t launch_far(const SearchArgs &a, int dp, int K, int grid, hipStream_t s) {
    switch (dp) {
        case 4: return launch_search_far_dp4(a, K, grid, s);
        case 8: return launch_search_far_dp8(a, K, grid, s);
        case 16: return launch_search_far_dp16(a, K, grid, s);
        case 32: return launch_search_far_dp32(a, K, grid, s);
        default: return launch_search_far_dp64(a, K, grid, s);
    }
}

knn_status search_furthest(const knn_tree *ref, const knn_tree *query, int k,
                           const knn_opts *opts_in, int64_t *idx_out, float *dist_out,
                           hipStream_t s) {
    const char *who = "knn_search_furthest";
    if (!ref) return fail(KNN_E_INVALID_ARG, std::string(who) + ": tree is NULL");
    knn_opts opts;
    knn_opts_default(&opts);
    if (opts_in) opts = *opts_in;
    const knn_tree *qt = query ? query : ref;
    if (!idx_out || !dist_out) return fail(KNN_E_INVALID_ARG, std::string(who) + ": output is NULL");
    if (qt->d != ref->d) return fail(KNN_E_INVALID_ARG, std::string(who) + ": d differs");
    if (k < 1 || k > 64 || int64_t(k) >= ref->n)
        return fail(KNN_E_INVALID_ARG, std::string(who) + ": need 1 <= k <= 64 and k < m");
    if (opts.exclude_self && qt != ref)
        return fail(KNN_E_INVALID_ARG,
                    std::string(who) + ": exclude_self needs the query tree to be the reference tree");
    if (opts.exclude_self && k > 63)
        return fail(KNN_E_INVALID_ARG, std::string(who) + ": need k <= 63 with exclude_self");
    if (opts.bound < 0 || opts.bound > 2 || opts.reserved != 0)
        return fail(KNN_E_INVALID_ARG, std::string(who) + ": bad bound or reserved field");
    if (opts.precision != KNN_PREC_FP32 || opts.seed_radius || opts.leaf_kth_out)
        return fail(KNN_E_UNSUPPORTED,
                    std::string(who) + ": FP32 only, without seed radius or leaf k-th output");
    const int kk = k + (opts.exclude_self ? 1 : 0);
    const int K = kk <= 8 ? 8 : kk <= 16 ? 16 : kk <= 32 ? 32 : 64;
    const int max_leaf = int((qt->n + qt->n_leaves - 1) / qt->n_leaves);
    const int lg = max_leaf <= 32 ? 5 : 6;
    const int nq_leaves = int(qt->n_leaves);
    const int waves = (nq_leaves + (64 >> lg) - 1) / (64 >> lg);
    const int grid = (waves + 3) / 4;

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
    a.d = ref->d;
    a.k = k;
    a.lpl_log2 = lg;
    a.bound = opts.bound;
    a.self = opts.exclude_self ? 1 : 0;
    a.out_idx = idx_out;
    a.out_dist = dist_out;

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
        a.stats = dstats;
        for (auto &e : ev) KNN_HIP(hipEventCreate(&e));
        KNN_HIP(hipEventRecord(ev[0], s));
    }
    KNN_HIP(launch_far(a, ref->dp, K, grid, s));
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
        st->n_query_leaves = nq_leaves;
        (void)hipEventElapsedTime(&st->ms_main_kernel, ev[0], ev[1]);
        st->ms_search = st->ms_main_kernel;
    }
    return KNN_OK;
}

}  // namespace
}  // namespace knnx

using namespace knnx;

extern "C" knn_status knn_search_furthest(const knn_tree *ref, const knn_tree *query, int32_t k,
                                          const knn_opts *opts, int64_t *idx_out,
                                          float *dist_out, void *stream) {
    set_error("");
    return search_furthest(ref, query, k, opts, idx_out, dist_out, (hipStream_t)stream);
}
