/*
 * knn.h -- exact k-nearest-neighbour search by a pruning dual-tree traversal
 * over kd-trees, on AMD MI355X (gfx950).  C ABI.
 *
 * The method is the dual-tree meta-algorithm of Curtin et al.,
 * "Tree-Independent Dual-Tree Algorithms" (ICML 2013): a space tree (here a
 * kd-tree, Section "Space Trees"), a pruning dual-tree traversal (Section
 * "Tree Traversals", Algorithm 1), the k-NN BaseCase (Algorithm 2) and the
 * k-NN Score with the node bound B(N_q) (Algorithm 3 and the bound
 * equations of Section "k-Nearest Neighbor Search").
 *
 * Conventions for every entry point
 *   - Point arrays are row-major FP32, n rows of d values, in DEVICE memory
 *     unless the argument says "host".  The caller owns every buffer it
 *     passes; the library never frees or retains caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; every call synchronises that stream before it
 *     returns, so the status reflects device-side errors.
 *   - Nothing is thrown across the ABI.  Arguments are validated before any
 *     device work; on error the outputs are unspecified and
 *     knn_last_error() describes the failure (thread-local string).
 *   - Opaque handles (knn_tree, knn_mlp) own device memory on the device that
 *     was current when they were created; free them with the matching
 *     *_free call.
 *   - Trees and per-call scratch use a caching allocator: released blocks
 *     stay with the process and are reused in stream order (a block released
 *     on one stream and taken on another makes the new stream wait for the
 *     release).  knn_release_cached_memory() hands them back to the device.
 */
#ifndef KNN_DUALTREE_H
#define KNN_DUALTREE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum knn_status {
    KNN_OK = 0,
    KNN_E_INVALID_ARG = 1, /* argument outside the documented domain        */
    KNN_E_NONFINITE = 2,   /* NaN or Inf in an input coordinate             */
    KNN_E_OOM = 3,         /* device allocation failed                      */
    KNN_E_DEVICE = 4,      /* HIP runtime error (no device, launch failure) */
    KNN_E_MODEL = 5,       /* seed-network file unreadable or inconsistent  */
    KNN_E_UNSUPPORTED = 6  /* valid request the library does not implement  */
} knn_status;

/* Pruning bound used by Score() (Section "k-Nearest Neighbor Search").
 * KNN_BOUND_B    combined bound B(N_q) = min{ B1(N_q),
 *                min_{p in D^p_q} D_p[k] + rho + lambda, B(Par(N_q)) }; at a
 *                kd-tree leaf rho = lambda, so the middle term is
 *                min D_p[k] + 2 lambda(N_q).  The printed child term
 *                B(N_c) + 2(lambda_q - lambda_c) is not used: it is not an
 *                upper bound when B(N_c) is attained by its max term.
 * KNN_BOUND_B1   B1(N_q) = max_{p in D^p_q} D_p[k] (Gray's AllNN rule,
 *                Algorithm 4, generalised to k).
 * KNN_BOUND_NONE no pruning: every (query leaf, reference leaf) pair is
 *                evaluated (the non-pruning traversal of the correctness
 *                argument; brute force through the same kernels).
 * Every mode prunes only when d_min exceeds the bound strictly (with a
 * relative slack of 2^-16 for FP32 rounding), never at equality. */
typedef enum knn_bound { KNN_BOUND_B = 0, KNN_BOUND_B1 = 1, KNN_BOUND_NONE = 2 } knn_bound;

/* Arithmetic of BaseCase() distance evaluation.
 * KNN_PREC_FP32  FP32 direct difference ||p_q - p_r||^2 on the vector ALUs;
 *                for d > 8 every candidate that passes the FP32 filter is
 *                re-scored in FP64 before it enters a k-list.
 * KNN_PREC_BF16  BF16 matrix-core (MFMA) tiles, FP32 accumulation, of the
 *                centred Gram form ||q||^2 + ||r||^2 - 2 q.r; a candidate is
 *                kept when the BF16 value minus a proven error margin beats
 *                the current k-th distance, and is then re-scored in FP64.
 * Both modes return the same exact answer (see knn_search). */
typedef enum knn_precision { KNN_PREC_FP32 = 0, KNN_PREC_BF16 = 1 } knn_precision;

/* Counters of one knn_search call (filled when knn_opts.stats != NULL). */
typedef struct knn_stats {
    int64_t score_calls;      /* Score() evaluations (reference nodes tested)   */
    int64_t leaf_tiles;       /* (query-leaf group, reference leaf) tiles       */
    int64_t pairs;            /* BaseCase() point pairs evaluated                */
    int64_t inserts;          /* candidates inserted into a k-list               */
    int64_t fallback_leaves;  /* query leaves searched again without their seed  */
    int64_t fallback_queries; /* queries whose k-th distance exceeded the seed   */
    float ms_query_build;     /* device time, query-tree build (0 if reused)     */
    float ms_search;          /* device time, traversal incl. fallback           */
    float ms_main_kernel;     /* device time of the main traversal launch (FP32
                                 with a seed: the second pass of the leaves
                                 that missed their seed runs in this launch)    */
    int32_t n_query_leaves;   /* leaves of the query tree                        */
    int64_t fallback_pairs;   /* pairs evaluated by the fallback pass (included
                                 in `pairs`)                                     */
    float ms_ref_build;       /* device time, reference-tree build (knn_all_knn
                                 only; 0 otherwise)                              */
} knn_stats;

typedef struct knn_opts {
    int32_t bound;              /* knn_bound                                       */
    int32_t precision;          /* knn_precision                                   */
    int32_t exclude_self;       /* 1: skip reference i for query i (footnote to
                                   Algorithm 2); only with query tree == ref tree  */
    int32_t reserved;           /* must be 0                                       */
    const float *seed_radius;   /* device, one per query leaf (distance units), or
                                   NULL.  Initial bound of that leaf; a leaf with a
                                   query whose k-th distance exceeds it is searched
                                   again without it, so any values keep the answer
                                   exact.                                          */
    float *leaf_kth_out;        /* device, one per query leaf, or NULL: largest
                                   final k-th distance in the leaf (the final
                                   B1 of the leaf)                                 */
    knn_stats *stats;           /* host, or NULL                                   */
} knn_opts;

/* Fill *opts with the defaults: bound B, FP32, no self exclusion, no seed. */
void knn_opts_default(knn_opts *opts);

const char *knn_status_string(knn_status s);
/* Description of the last error on the calling thread ("" if none). */
const char *knn_last_error(void);

/* Returns every cached (released, unused) device block of every device to
 * the runtime.  Waits for the work queued before each block's release.
 * Blocks still owned by live trees are not affected.  Errors: KNN_E_DEVICE. */
knn_status knn_release_cached_memory(void);
/* Bytes currently held in the cache (released, not yet reused). */
int64_t knn_cached_bytes(void);

/* ------------------------------------------------------------------------
 * kd-tree (Section "Space Trees", Definition 1; kd-tree bounds paragraph).
 * ------------------------------------------------------------------------ */
typedef struct knn_tree knn_tree;

/* Build a kd-tree over `points` (device, n x d FP32 row-major).
 * Split rule: complete tree of depth L = smallest L with
 * ceil(n / 2^L) <= leaf_size, heap-ordered nodes; a node splits on the
 * dimension of largest FP32 box extent (ties: lowest), the left child takes
 * the floor(n/2) smallest points by (coordinate, original index), both
 * children keep ascending original-index order; points live only in leaves.
 * Node data: tight FP32 box, centre fl(0.5 fl(lo+hi)), lambda = max distance
 * from the centre to a descendant point (leaves: exact, rounded up to FP32;
 * internal nodes: an upper bound from the children).
 * The tree copies the points (permuted); the caller may free `points` after
 * the call.  Domain: n >= 1 (n < 2^31), 1 <= d <= 64, 1 <= leaf_size <= 64.
 * Errors: KNN_E_INVALID_ARG, KNN_E_NONFINITE, KNN_E_OOM, KNN_E_DEVICE. */
knn_status knn_build_tree(const float *points, int64_t n, int32_t d, int32_t leaf_size,
                          void *stream, knn_tree **out);
/* Builds a reference tree and a query tree (same d and leaf size) as two
 * knn_build_tree calls would, but lets the two builds overlap on the device:
 * the query build runs on a library-owned stream of the current device
 * (created on first use, default priority), which first waits for the work
 * already queued on `stream`.  On return both builds have completed and both
 * trees belong to `stream` (knn_free_tree releases them in its order).  On
 * any error neither tree is returned.  Domain and errors as knn_build_tree;
 * each of the two point sets is checked. */
knn_status knn_build_tree_pair(const float *ref_points, int64_t n_ref, const float *query_points,
                               int64_t n_query, int32_t d, int32_t leaf_size, void *stream,
                               knn_tree **ref_out, knn_tree **query_out);
void knn_free_tree(knn_tree *tree);

/* Read-only view of a tree's device arrays (for tests and tools).
 * Layout: dp = d rounded up to 4, 8, 16, 32 or 64 (padding coordinates are 0).
 *   points     (n + 64) x dp FP32, tree order (last 64 rows zero padding)
 *   perm       n int32: original row of tree position i
 *   node_range n_nodes x 2 int32: start, count (heap order)
 *   box        n_nodes x 2 x dp FP32: lo[dp] then hi[dp]
 *   lambda     n_nodes FP32
 *   split_dim  n_nodes int32 (-1 at leaves) */
typedef struct knn_tree_info {
    int64_t n;
    int32_t d, dp, leaf_size, depth;
    int64_t n_nodes, n_leaves, first_leaf;
    const float *points;
    const int32_t *perm;
    const int32_t *node_range;
    const float *box;
    const float *lambda;
    const int32_t *split_dim;
    float ms_build; /* device time of the build */
} knn_tree_info;
knn_status knn_tree_get_info(const knn_tree *tree, knn_tree_info *info);

/* ------------------------------------------------------------------------
 * Search (Section "k-Nearest Neighbor Search": for each query point the k
 * nearest reference points and their distances, 0 < k < m).
 * ------------------------------------------------------------------------ */

/* All k nearest neighbours of every point of `query` among the points of
 * `ref`.  query == NULL or query == ref: all-kNN of ref on itself (set
 * opts->exclude_self to skip each point's own index).
 * Outputs (device, caller-owned, n_q x k row-major, rows in original query
 * order): idx_out = original reference row, dist_out = Euclidean distance
 * (FP32, from an FP64 evaluation), ascending; equal distances are ordered by
 * reference index.  The answer is exact: the index set equals the FP64
 * brute-force set except where FP64 distances tie within 1e-6 relative at
 * the k-th place.  Domain: 1 <= k <= 64 and k < m; with exclude_self the
 * m - 1 other points are the candidates (the same condition) and k <= 63.
 * Same d in both trees.  opts == NULL means the defaults. */
knn_status knn_search(const knn_tree *ref, const knn_tree *query, int32_t k,
                      const knn_opts *opts, int64_t *idx_out, float *dist_out,
                      void *stream);

/* knn_search for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same search, kernels and answer as knn_search on trees built beforehand,
 * with the per-call scratch (launch order, counters, fallback flags and
 * bounds) in a fixed 4 MiB device array that the library holds on every
 * device it runs on until the process ends.  It calls no device allocation
 * or free and records no memset node (clears are kernels).  Limits: query
 * trees of up to 2^18 leaves always fit; a larger tree whose scratch
 * (12 bytes per query leaf with a seed, 4 per wavefront of leaves without)
 * exceeds the array is rejected with KNN_E_INVALID_ARG before any device
 * work; the trees must belong to the current device.  Every call on a device shares that device's array, so
 * calls that overlap on one device (other threads, other streams) race and
 * must be serialised by the caller.  With opts->stats the counters are
 * filled and the ms_* timing fields are 0 (no events are created).  Other
 * arguments, errors and outputs as knn_search. */
knn_status knn_search_noalloc(const knn_tree *ref, const knn_tree *query, int32_t k,
                              const knn_opts *opts, int64_t *idx_out, float *dist_out,
                              void *stream);

/* Convenience: builds the query tree from `queries` (device, n_q x d) with
 * the reference tree's leaf size, searches, frees it.  The query-tree build
 * time is reported in stats->ms_query_build. */
knn_status knn_search_points(const knn_tree *ref, const float *queries, int64_t n_q,
                             int32_t k, const knn_opts *opts, int64_t *idx_out,
                             float *dist_out, void *stream);

/* The whole path in one call: builds the reference tree and (unless
 * query_points is NULL) the query tree, the two builds overlapped as in
 * knn_build_tree_pair, searches as knn_search, and frees both trees.  The
 * result equals that of the separate calls; the difference is that the
 * search is enqueued behind the builds without a host wait in between, so
 * the stream is synchronised once, at the end, where the builds' input
 * checks are read.  query_points == NULL: all-kNN of ref_points on itself
 * (opts->exclude_self as in knn_search).  Argument domains and errors are
 * those of knn_build_tree (for each point set) and knn_search; after an
 * error the contents of idx_out and dist_out are undefined.  With
 * opts->stats, ms_ref_build and ms_query_build report the two builds. */
knn_status knn_all_knn(const float *ref_points, int64_t n_ref, const float *query_points,
                       int64_t n_query, int32_t d, int32_t leaf_size, int32_t k,
                       const knn_opts *opts, int64_t *idx_out, float *dist_out, void *stream);


/* k-furthest neighbours (the closing remark of Section "k-Nearest Neighbor
 * Search": the same meta-algorithm with the bound inverted -- max and min
 * exchanged -- lists in descending distance and the BaseCase comparison
 * d > D_p[k]).  For every query point the k reference points at the
 * LARGEST distances.  The bound is L(N_q) = max{ min_p D_p[k],
 * max_p D_p[k] - 2 lambda(N_q), L(Par(N_q)) }, a lower bound on every
 * point's final k-th farthest distance, and Score prunes a node whose box
 * lies entirely nearer than it (strictly, with a 2^-16 relative slack).
 * opts: bound (KNN_BOUND_B all three terms, KNN_BOUND_B1 the first and the
 * parent's, KNN_BOUND_NONE no pruning), exclude_self, stats; precision must
 * be FP32 and seed_radius, leaf_kth_out NULL (else KNN_E_UNSUPPORTED).
 * Outputs (device, n_q x k, original query order): idx_out = original
 * reference row, dist_out = FP32 of the FP64 distance, DESCENDING; equal
 * distances are ordered by reference index.  Lists start empty (the paper
 * starts them at distance 0), so a reference at distance 0 from the query
 * (a duplicate) is still returned when fewer than k others are farther.
 * Domain as knn_search (1 <= k <= 64, k < m; k <= 63 with exclude_self).
 * Errors: KNN_E_INVALID_ARG, KNN_E_UNSUPPORTED, KNN_E_OOM, KNN_E_DEVICE. */
knn_status knn_search_furthest(const knn_tree *ref, const knn_tree *query, int32_t k,
                               const knn_opts *opts, int64_t *idx_out, float *dist_out,
                               void *stream);

/* Range search (Section "Range Search", Algorithms 5 and 6): for every query
 * point, every reference point at a distance in [lo, hi] (both ends
 * included), decided exactly: lo*lo <= s <= hi*hi in FP64, with s the FP64
 * squared distance of the FP32 inputs.  Score prunes a node pair only when
 * every distance misses the range (d_min > hi or d_max < lo, with a 2^-16
 * slack); the printed test on d_min alone is not used because it drops
 * overlapping nodes whose farther points are in range.
 * Two calls with the same trees, range and opts:
 *   knn_range_count writes offsets_out (device, n_q + 1 int64): exclusive
 *     prefix sums of the per-query neighbour counts in original query order
 *     (offsets_out[0] = 0), and *total_out (host) = offsets_out[n_q];
 *   knn_range_fill writes the neighbours of query i at
 *     idx_out[offsets[i] .. offsets[i+1]-1] (device int64, original
 *     reference rows) and their distances at the same places of dist_out
 *     (device FP32 of the FP64 distance); the caller allocates both with
 *     total entries.  Within a query the order is the traversal's
 *     (deterministic; the paper's lists are unordered).
 * opts: bound (KNN_BOUND_NONE: no pruning, anything else: the range test),
 * exclude_self; precision FP32 and no seed or leaf output (else
 * KNN_E_UNSUPPORTED); stats (per call; inserts = neighbours found).
 * Domain: 0 <= lo <= hi < inf, n_q <= 2^24.  Errors: KNN_E_INVALID_ARG,
 * KNN_E_UNSUPPORTED, KNN_E_OOM, KNN_E_DEVICE. */
knn_status knn_range_count(const knn_tree *ref, const knn_tree *query, double lo, double hi,
                           const knn_opts *opts, int64_t *offsets_out, int64_t *total_out,
                           void *stream);
knn_status knn_range_fill(const knn_tree *ref, const knn_tree *query, double lo, double hi,
                          const knn_opts *opts, const int64_t *offsets, int64_t *idx_out,
                          float *dist_out, void *stream);

/* Kernel density sums (Section "Kernel Density Estimation", Algorithms 9 and
 * 10): f_out[i] (device, n_q FP64, original query order) estimates
 * f(q_i) = sum over reference points r of K(||q_i - r||) with the Gaussian
 * kernel K(d) = exp(-d^2 / (2 h^2)) (no normalising constant), such that
 * |f_out[i] - f(q_i)| <= eps for every query, plus FP32 evaluation error of
 * the kernel values (relative about 1e-6 per term).  For a query node N_q
 * (a group of query leaves) and a reference node N_r whose kernel values
 * vary by less than eps / |S_r| (K(d_min) - K(d_max) between their boxes),
 * each query point q of N_q adds |N_r| K(||q - C||), C the reference box
 * centre, instead of N_r's points (the printed Algorithm 9 compares the
 * other way round; the text and the error bound need this way).  opts: bound
 * KNN_BOUND_NONE (or eps = 0) sums every pair exactly, anything else
 * approximates as described; exclude_self (leave-one-out: skip each point's
 * own term); stats (inserts = approximated (query point, node) pairs);
 * precision FP32, no seed or leaf output (else KNN_E_UNSUPPORTED).
 * Domain: h > 0, eps >= 0, both finite.  Errors: KNN_E_INVALID_ARG,
 * KNN_E_UNSUPPORTED, KNN_E_OOM, KNN_E_DEVICE. */
knn_status knn_kde(const knn_tree *ref, const knn_tree *query, double h, double eps,
                   const knn_opts *opts, double *f_out, void *stream);

/* Euclidean minimum spanning tree of a tree's points by dual-tree Boruvka
 * (Section "Boruvka's Algorithm", Algorithms 7 and 8 and the
 * traversal-merge loop), with the tree as both query and reference tree.
 * Each round finds, for every component, its shortest edge to another
 * component (the k = 1 traversal with the bound B(N_q) and a Score that
 * prunes node pairs inside one component), then merges.  Edges are
 * compared by the strict order (FP64 squared length of the FP32 points,
 * smaller index, larger index), so the result is the unique minimum
 * spanning tree under that order, edge for edge.
 * Outputs (device, caller-owned, n - 1 entries each): edge_u[i] < edge_v[i]
 * original point rows, edge_w[i] = FP32 of the FP64 length; the order is
 * deterministic (by the tree position of the component that chose the
 * edge), not sorted.  *rounds_out (host, optional): Boruvka rounds.
 * opts: bound (KNN_BOUND_B, KNN_BOUND_B1, or KNN_BOUND_NONE: prune only
 * pairs inside one component), stats (summed over rounds; ms_search is the
 * whole computation); precision FP32, no seed or leaf output, no
 * exclude_self (else KNN_E_UNSUPPORTED / KNN_E_INVALID_ARG).
 * Domain: n <= 2^24.  Errors: KNN_E_INVALID_ARG, KNN_E_UNSUPPORTED,
 * KNN_E_OOM, KNN_E_DEVICE. */
knn_status knn_emst(const knn_tree *tree, const knn_opts *opts, int64_t *edge_u, int64_t *edge_v,
                    float *edge_w, int32_t *rounds_out, void *stream);

/* ------------------------------------------------------------------------
 * Learned seed radius (not part of the paper; it only supplies the initial
 * value of a query leaf's bound, see knn_opts.seed_radius).
 * Network: n_in -> 64 -> 64 -> 1, ReLU, FP32 weights, inputs standardised
 * inside the network as (x - mu) * inv_sd.  Parameters travel as one flat
 * FP32 vector: W1 (64 x n_in, row-major), b1 (64), W2 (64 x 64), b2 (64),
 * w3 (64), b3 (1).  All compute runs in the library's kernels; every call
 * synchronises its stream.
 * ------------------------------------------------------------------------ */
typedef struct knn_mlp knn_mlp;

/* New network with all parameters 0, mu = 0, inv_sd = 1, y_mu = 0, y_sd = 1.
 * Domain: 1 <= n_in <= 72; hidden must be 64 (else KNN_E_UNSUPPORTED). */
knn_status knn_mlp_create(int32_t n_in, int32_t hidden, knn_mlp **out);
void knn_mlp_free(knn_mlp *mlp);
knn_status knn_mlp_num_params(const knn_mlp *mlp, int64_t *n);
/* host <-> device parameter copies (n must equal the parameter count);
 * set_params also clears the Adam moments and step counter */
knn_status knn_mlp_set_params(knn_mlp *mlp, const float *host, int64_t n);
knn_status knn_mlp_get_params(const knn_mlp *mlp, float *host, int64_t n);
/* gradient of the last knn_mlp_loss_grad call */
knn_status knn_mlp_get_grads(const knn_mlp *mlp, float *host, int64_t n);
/* input standardisation (host arrays of n_in) and the output scale used by
 * knn_seed_radius: log radius = y * y_sd + y_mu */
knn_status knn_mlp_set_norm(knn_mlp *mlp, const float *mu_host, const float *inv_sd_host,
                            float y_mu, float y_sd);
/* y[i] = network output for x[i] (device, x: n x n_in, y: n) */
knn_status knn_mlp_forward(const knn_mlp *mlp, const float *x, int64_t n, float *y, void *stream);
/* L = (1/n) sum (y_i - t_i)^2 over the batch (device x: n x n_in, t: n);
 * stores dL/dparams in the network and *loss_host = L (if not NULL) */
knn_status knn_mlp_loss_grad(knn_mlp *mlp, const float *x, const float *t, int64_t n,
                             float *loss_host, void *stream);
/* one Adam step (bias-corrected) with the stored gradient */
knn_status knn_mlp_adam_step(knn_mlp *mlp, float lr, float beta1, float beta2, float eps,
                             void *stream);
/* versioned binary file: magic, sizes, output scale, mu, inv_sd, params */
knn_status knn_mlp_save(const knn_mlp *mlp, const char *path);
knn_status knn_mlp_load(const char *path, knn_mlp **out);

/* Per query leaf (n_leaves x (d + 3), device): its box centre (d values),
 * lambda, point count, and log(count / volume) of the reference leaf reached
 * by descending from the root toward that centre (volume of the tight box,
 * each extent clamped below at 1e-6 of the root's extent).  query == NULL:
 * the reference tree's own leaves. */
knn_status knn_seed_features(const knn_tree *ref, const knn_tree *query, float *feats,
                             void *stream);
/* radius[i] = exp(net(feats[i]) * y_sd + y_mu + log_margin), device arrays */
knn_status knn_seed_radius(const knn_mlp *mlp, const float *feats, int64_t n, float log_margin,
                           float *radius, void *stream);

/* Options of knn_seed_train. */
typedef struct knn_train_opts {
    int32_t epochs;        /* passes over the training rows, >= 1               */
    int32_t batch;         /* rows per Adam step, >= 1                          */
    float lr;              /* Adam step size, > 0 (beta1 0.9, beta2 0.999,
                              eps 1e-8)                                         */
    float val_frac;        /* held-out fraction for the margin, in (0, 1)       */
    float target_fallback; /* fraction of held-out leaves whose target may
                              exceed the calibrated radius, in [0, 1)           */
    uint64_t seed;         /* random streams of the split, the initial
                              weights and the batch orders                      */
} knn_train_opts;

/* Trains a new seed network on the GPU from n (features, target) rows, the
 * targets being each query leaf's largest k-th neighbour distance from a
 * plain search (knn_search's leaf_kth_out; the network learns its log).
 * feats: device, n x n_in (knn_seed_features rows); kth: device, n.
 * Steps, all on the device except the two sorts of random keys and the
 * quantile of the held-out residuals (host, O(n log n)):
 *   1. split: the rows ordered by random key; the first
 *      max(1, floor(n * val_frac)) are held out, the rest train;
 *   2. standardisation: mean and (population) deviation of every training
 *      column in FP64 (a deviation below 1e-12 counts as 1); targets
 *      t = (log max(kth, 1e-30) - y_mu) / y_sd;
 *   3. weights uniform in +-sqrt(6 / fan_in), biases 0;
 *   4. each epoch: the training rows in a fresh random-key order, cut into
 *      batches of `batch` rows (the last one shorter); per batch the mean
 *      squared error gradient (knn_mlp_loss_grad) and one Adam step;
 *   5. log_margin: the (1 - target_fallback) quantile (linear between order
 *      statistics) of the held-out residuals log kth - (y * y_sd + y_mu).
 * Random numbers: SplitMix64 (Steele, Lea and Flood, 2014) in counter form,
 * value(s, i) = mix(s + (i + 1) * 0x9E3779B97F4A7C15) mod 2^64; stream p
 * (0 weights, 1 split, 2 + e epoch e) has seed value(seed, p); a key is the
 * stream's i-th value (ties broken by row), a uniform is its top 53 bits
 * times 2^-53.
 * Outputs: *out a new network (free with knn_mlp_free) with the
 * standardisation set; *log_margin_out (host); loss_out (host, optional,
 * `epochs` floats): mean batch loss of each epoch.
 * Domain: n >= 2, 1 <= n_in <= 72, kth finite and >= 0 (else
 * KNN_E_INVALID_ARG, checked on the device copy before training).
 * Errors: KNN_E_INVALID_ARG, KNN_E_OOM, KNN_E_DEVICE. */
knn_status knn_seed_train(const float *feats, const float *kth, int64_t n, int32_t n_in,
                          const knn_train_opts *opts, knn_mlp **out, float *log_margin_out,
                          float *loss_out, void *stream);

/* ------------------------------------------------------------------------
 * Test exports.  They run pieces of the search kernels on inputs the caller
 * chooses, so that tests can check them against the paper's definitions.
 * ------------------------------------------------------------------------ */

/* The BF16 distance tile of the matrix-core BaseCase (Algorithm 2 distance
 * evaluation; BF16 tiles themselves are this library's addition), computed by
 * the same device code as the search kernels, for n_tiles independent tiles.
 * Tile t: query rows q[t*32 .. t*32+31] and reference rows r[t*32 .. +31]
 * (device, row-major, d FP32 values per row), centre[t*d .. +d-1] (device).
 * Outputs (device, caller-owned):
 *   acc_out    n_tiles x 32 x 32, [t][i][j] = ||r_i - c||^2 - 2 <r_i - c, q_j - c>
 *              as the matrix unit computed it (BF16 operands, FP32 sums);
 *   qnorm_out  n_tiles x 32, ||q_j - c||^2 in FP32;
 *   margin_out n_tiles x 32, the margin M_j the kernels subtract: the tile's
 *              estimate acc + qnorm of ||q_j - r_i||^2 is claimed to lie within
 *              M_j of the exact value for every row i of the tile.
 * Domain: 9 <= d <= 64, 1 <= n_tiles <= 2^24.  Errors: KNN_E_INVALID_ARG,
 * KNN_E_DEVICE. */
knn_status knn_debug_bf16_tiles(const float *q, const float *r, const float *centre,
                                int64_t n_tiles, int32_t d, float *acc_out, float *qnorm_out,
                                float *margin_out, void *stream);

/* The BaseCase tiles of a search, timed on their own: the d = 3 FP32 debug
 * kernel first runs the search while each wavefront records the reference
 * leaves it evaluates (BaseCase, Algorithm 2, with the k-list inserts and
 * bound refreshes), then a second launch evaluates exactly those leaves in
 * the same order without the walk and Score, and returns the same answer.
 * *ms_search / *ms_replay (host): device time of the two launches;
 * *pairs (host): point pairs evaluated (the same in both).  idx_out,
 * dist_out as knn_search (from the replay).  Domain as knn_debug_search_log;
 * KNN_E_UNSUPPORTED if a wavefront evaluates more than 512 leaves. */
knn_status knn_debug_tile_replay(const knn_tree *ref, const knn_tree *query, int32_t k,
                                 const knn_opts *opts, int64_t *idx_out, float *dist_out,
                                 float *ms_search, float *ms_replay, int64_t *pairs,
                                 void *stream);

/* knn_search with its traversal instrumented, for checking the correctness
 * argument of the k-NN Score (Section "k-Nearest Neighbor Search", the
 * argument after Algorithm 3: the bound B(N_q) never falls below the largest
 * true k-th distance of the node's points, so a pruned node pair holds no
 * true neighbour) and the independence of the answer from the visit order
 * (Algorithm 4 takes the closer child first; any order gives the same
 * answer).  Runs the FP32 kernel built with a Score log, for d = 3, no seed,
 * k-lists of at most 16 entries (k <= 16, or k <= 15 with exclude_self).
 * far_first: 0 enters the nearer reference child first (as knn_search), 1
 * the farther one.  log_out (device, capacity x 12 uint32): one record per
 * Score call, in the order the kernel wrote them:
 *   [0] reference node (heap order)   [1] 1 if kept, 0 if pruned
 *   [2] first query leaf of the wavefront  [3] number of query leaves g of
 *       the wavefront (consecutive leaves)
 *   [4 .. 4+g-1] FP32 bits of B(N_q)^2 of each of those leaves at that call
 *       (+inf before the first tile; the per-point bound is min(D_p[k]^2, it))
 * *n_records (host) receives the number of Score calls; records beyond
 * capacity are dropped.  Outputs idx_out, dist_out as knn_search.  Errors as
 * knn_search, KNN_E_UNSUPPORTED outside the covered domain. */
knn_status knn_debug_search_log(const knn_tree *ref, const knn_tree *query, int32_t k,
                                const knn_opts *opts, int32_t far_first, uint32_t *log_out,
                                int64_t capacity, int64_t *n_records, int64_t *idx_out,
                                float *dist_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* KNN_DUALTREE_H */
