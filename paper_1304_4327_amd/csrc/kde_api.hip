// C-ABI entry of the kernel density sums (include/knn.h): validation,
// dispatch of k_kde by stride and leaf width, counters and timing.
#include "search_kde.hpp"

#include <cmath>
#include <string>

namespace knnx {
namespace {

template <int DP>
hipError_t launch_kde(const KdeArgs &a, int lg, int grid, hipStream_t s) {
    if (lg == 5)
        k_kde<DP, 5><<<grid, 256, 0, s>>>(a);
    else
        k_kde<DP, 6><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_dp(const KdeArgs &a, int dp, int lg, int grid, hipStream_t s) {
    switch (dp) {
        case 4: return launch_kde<4>(a, lg, grid, s);
        case 8: return launch_kde<8>(a, lg, grid, s);
        case 16: return launch_kde<16>(a, lg, grid, s);
        case 32: return launch_kde<32>(a, lg, grid, s);
        default: return launch_kde<64>(a, lg, grid, s);
    }
}

}  // namespace
}  // namespace knnx

using namespace knnx;

extern "C" knn_status knn_kde(const knn_tree *ref, const knn_tree *query, double h, double eps,
                              const knn_opts *opts_in, double *f_out, void *stream) {
    set_error("");
    const std::string w = "knn_kde";
    if (!ref) return fail(KNN_E_INVALID_ARG, w + ": tree is NULL");
    if (!f_out) return fail(KNN_E_INVALID_ARG, w + ": f_out is NULL");
    knn_opts opts;
    knn_opts_default(&opts);
    if (opts_in) opts = *opts_in;
    const knn_tree *qt = query ? query : ref;
    if (qt->d != ref->d) return fail(KNN_E_INVALID_ARG, w + ": d differs");
    if (!(h > 0.0) || !std::isfinite(h) || !(eps >= 0.0) || !std::isfinite(eps))
        return fail(KNN_E_INVALID_ARG, w + ": need h > 0 and eps >= 0, both finite");
    if (opts.exclude_self && qt != ref)
        return fail(KNN_E_INVALID_ARG, w + ": exclude_self needs the query tree to be the reference tree");
    if (opts.bound < 0 || opts.bound > 2 || opts.reserved != 0)
        return fail(KNN_E_INVALID_ARG, w + ": bad bound or reserved field");
    if (opts.precision != KNN_PREC_FP32 || opts.seed_radius || opts.leaf_kth_out)
        return fail(KNN_E_UNSUPPORTED, w + ": FP32 only, without seed radius or leaf k-th output");
    hipStream_t s = (hipStream_t)stream;
    const int max_leaf = int((qt->n + qt->n_leaves - 1) / qt->n_leaves);
    const int lg = max_leaf <= 32 ? 5 : 6;
    const int waves = int((qt->n_leaves + (64 >> lg) - 1) / (64 >> lg));
    const int grid = (waves + 3) / 4;
    KdeArgs a{};
    a.rbox = ref->box;
    a.rlpts = ref->lpts;
    a.rrange = ref->range;
    a.r_leaf_slots = ref->leaf_slots;
    a.r_first_leaf = int(ref->first_leaf);
    a.qpts = qt->pts;
    a.qbox = qt->box;
    a.qperm = qt->perm;
    a.qrange = qt->range;
    a.q_first_leaf = int(qt->first_leaf);
    a.q_n_leaves = int(qt->n_leaves);
    a.c = float(1.0 / (2.0 * h * h));
    a.eps_ref = float(eps / double(ref->n));
    a.approx = opts.bound != KNN_BOUND_NONE && eps > 0.0;
    a.self = opts.exclude_self ? 1 : 0;
    a.f_out = f_out;

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
    KNN_HIP(launch_dp(a, ref->dp, lg, grid, s));
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
