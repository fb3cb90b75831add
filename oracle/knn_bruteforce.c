/*
 * Oracle (test infrastructure only): exact k-nearest-neighbour search by brute
 * force, in FP64, on the CPU.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The GPU search never calls it and shares no code,
 * header or table with it.
 *
 * What it computes (Section "k-Nearest Neighbor Search", problem statement
 * and brute-force remark): for every query q in S_q (n rows of d FP32
 * values) it compares q with every reference r in S_r (m rows) and keeps the
 * k smallest distances, in ascending order.  Distances are Euclidean
 * (Section "Space Trees", minimum-distance definition, which uses the 2-norm).
 *
 * Readings where the paper is silent:
 *   - coordinates are FP32 inputs, upcast to FP64 before subtraction, so the
 *     squared distance is computed with ~1e-16 relative error;
 *   - equal distances are ordered by reference index (lower first);
 *   - with exclude_self != 0 (query set identical to reference set, footnote
 *     to the k-NN BaseCase), reference i is skipped for query i, by index
 *     identity only: an exact duplicate with another index is kept.
 *
 * Outputs: idx_out[i*k + j] = reference row of the j-th neighbour of query i,
 * d2_out[i*k + j] = its squared distance (FP64).  Returns 0 on success, -1
 * on invalid arguments (0 < k < m violated, or k > m - 1 with exclusion).
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int knn_oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* lexicographic order on (squared distance, reference index) */
static int before(double da, int64_t ia, double db, int64_t ib)
{
    return (da < db) || (da == db && ia < ib);
}

int knn_oracle_bruteforce(const float *q, int64_t n, const float *r, int64_t m,
                          int32_t d, int32_t k, int32_t exclude_self,
                          int64_t *idx_out, double *d2_out)
{
    if (!q || !r || !idx_out || !d2_out || n < 0 || m <= 0 || d <= 0 || k <= 0)
        return -1;
    if (k >= m) return -1;                     /* 0 < k < m */
    if (exclude_self && n != m) return -1;     /* identical sets only */

    int64_t i;
#pragma omp parallel for schedule(dynamic, 16)
    for (i = 0; i < n; ++i) {
        /* the list of the k best so far, ascending; slots beyond `len` are
         * treated as +infinity (empty-list initialisation of the k-NN rule) */
        double *bd = d2_out + i * (int64_t)k;
        int64_t *bi = idx_out + i * (int64_t)k;
        int len = 0;
        const float *qi = q + i * (int64_t)d;
        for (int64_t j = 0; j < m; ++j) {
            if (exclude_self && j == i) continue;
            const float *rj = r + j * (int64_t)d;
            double s = 0.0;
            for (int t = 0; t < d; ++t) {
                double diff = (double)qi[t] - (double)rj[t];
                s += diff * diff;
            }
            if (len == k && !before(s, j, bd[k - 1], bi[k - 1])) continue;
            /* ordered insert, truncating the list to length k */
            int pos = (len < k) ? len : k - 1;
            while (pos > 0 && before(s, j, bd[pos - 1], bi[pos - 1])) {
                bd[pos] = bd[pos - 1];
                bi[pos] = bi[pos - 1];
                --pos;
            }
            bd[pos] = s;
            bi[pos] = j;
            if (len < k) ++len;
        }
    }
    return 0;
}

/*
 * Same definition, for a subset of the queries: rows listed in qsel (so a
 * benchmark can time the oracle on a bounded sample).  Row t of the outputs
 * belongs to query qsel[t].  exclude_self compares qsel[t] with j.
 */
int knn_oracle_bruteforce_rows(const float *q, const int64_t *qsel, int64_t nsel,
                               const float *r, int64_t m, int32_t d, int32_t k,
                               int32_t exclude_self, int64_t *idx_out,
                               double *d2_out)
{
    if (!q || !qsel || !r || !idx_out || !d2_out || nsel < 0 || m <= 0 || d <= 0 ||
        k <= 0 || k >= m)
        return -1;
    int64_t t;
#pragma omp parallel for schedule(dynamic, 4)
    for (t = 0; t < nsel; ++t) {
        int64_t i = qsel[t];
        double *bd = d2_out + t * (int64_t)k;
        int64_t *bi = idx_out + t * (int64_t)k;
        int len = 0;
        const float *qi = q + i * (int64_t)d;
        for (int64_t j = 0; j < m; ++j) {
            if (exclude_self && j == i) continue;
            const float *rj = r + j * (int64_t)d;
            double s = 0.0;
            for (int u = 0; u < d; ++u) {
                double diff = (double)qi[u] - (double)rj[u];
                s += diff * diff;
            }
            if (len == k && !before(s, j, bd[k - 1], bi[k - 1])) continue;
            int pos = (len < k) ? len : k - 1;
            while (pos > 0 && before(s, j, bd[pos - 1], bi[pos - 1])) {
                bd[pos] = bd[pos - 1];
                bi[pos] = bi[pos - 1];
                --pos;
            }
            bd[pos] = s;
            bi[pos] = j;
            if (len < k) ++len;
        }
    }
    return 0;
}

/*
 * Squared distances in FP64 for explicit (query row, reference row) pairs.
 * The parity predicate uses it to price any index the GPU returns.
 */
int knn_oracle_pair_d2(const float *q, const float *r, int32_t d,
                       const int64_t *qi, const int64_t *ri, int64_t npairs,
                       double *d2_out)
{
    if (!q || !r || !qi || !ri || !d2_out || d <= 0 || npairs < 0) return -1;
    int64_t t;
#pragma omp parallel for schedule(static)
    for (t = 0; t < npairs; ++t) {
        const float *a = q + qi[t] * (int64_t)d;
        const float *b = r + ri[t] * (int64_t)d;
        double s = 0.0;
        for (int u = 0; u < d; ++u) {
            double diff = (double)a[u] - (double)b[u];
            s += diff * diff;
        }
        d2_out[t] = s;
    }
    return 0;
}

/*
 * k-furthest neighbours (the closing remark of Section "k-Nearest Neighbor
 * Search": the same problem with the order reversed): for each selected
 * query the k references at the LARGEST distances, in descending order of
 * distance; equal distances are ordered by reference index (lower first).
 * exclude_self as above.  Same argument conventions as
 * knn_oracle_bruteforce_rows; d2_out holds squared FP64 distances.
 */
static int after(double da, int64_t ia, double db, int64_t ib)
{
    return (da > db) || (da == db && ia < ib);
}

int knn_oracle_furthest_rows(const float *q, const int64_t *qsel, int64_t nsel,
                             const float *r, int64_t m, int32_t d, int32_t k,
                             int32_t exclude_self, int64_t *idx_out, double *d2_out)
{
    if (!q || !qsel || !r || !idx_out || !d2_out || nsel < 0 || m <= 0 || d <= 0 ||
        k <= 0 || k >= m)
        return -1;
    int64_t t;
#pragma omp parallel for schedule(dynamic, 4)
    for (t = 0; t < nsel; ++t) {
        int64_t i = qsel[t];
        double *bd = d2_out + t * (int64_t)k;
        int64_t *bi = idx_out + t * (int64_t)k;
        int len = 0;
        const float *qi = q + i * (int64_t)d;
        for (int64_t j = 0; j < m; ++j) {
            if (exclude_self && j == i) continue;
            const float *rj = r + j * (int64_t)d;
            double s = 0.0;
            for (int u = 0; u < d; ++u) {
                double diff = (double)qi[u] - (double)rj[u];
                s += diff * diff;
            }
            if (len == k && !after(s, j, bd[k - 1], bi[k - 1])) continue;
            int pos = (len < k) ? len : k - 1;
            while (pos > 0 && after(s, j, bd[pos - 1], bi[pos - 1])) {
                bd[pos] = bd[pos - 1];
                bi[pos] = bi[pos - 1];
                --pos;
            }
            bd[pos] = s;
            bi[pos] = j;
            if (len < k) ++len;
        }
    }
    return 0;
}

/*
 * Range search (Section "Range Search", problem statement): for each
 * selected query every reference at a distance in [lo, hi], both ends
 * included.  The decision is taken on squared distances in FP64:
 * lo*lo <= s <= hi*hi with s the FP64 squared distance of the FP32 inputs.
 * exclude_self skips reference qsel[t] for query row t.
 *
 * knn_oracle_range_rows fills counts_out[t] (the number of neighbours of
 * row t); with idx_out != NULL it also writes them, in increasing reference
 * index, at idx_out[offsets[t] ..] with squared distances in d2_out
 * (offsets: exclusive prefix sums of the counts, supplied by the caller).
 */
int knn_oracle_range_rows(const float *q, const int64_t *qsel, int64_t nsel,
                          const float *r, int64_t m, int32_t d, double lo, double hi,
                          int32_t exclude_self, int64_t *counts_out,
                          const int64_t *offsets, int64_t *idx_out, double *d2_out)
{
    if (!q || !qsel || !r || !counts_out || nsel < 0 || m <= 0 || d <= 0 || !(lo >= 0.0) ||
        !(hi >= lo) || (idx_out && (!offsets || !d2_out)))
        return -1;
    const double lo2 = lo * lo, hi2 = hi * hi;
    int64_t t;
#pragma omp parallel for schedule(dynamic, 4)
    for (t = 0; t < nsel; ++t) {
        int64_t i = qsel[t];
        const float *qi = q + i * (int64_t)d;
        int64_t c = 0;
        for (int64_t j = 0; j < m; ++j) {
            if (exclude_self && j == i) continue;
            const float *rj = r + j * (int64_t)d;
            double s = 0.0;
            for (int u = 0; u < d; ++u) {
                double diff = (double)qi[u] - (double)rj[u];
                s += diff * diff;
            }
            if (s >= lo2 && s <= hi2) {
                if (idx_out) {
                    idx_out[offsets[t] + c] = j;
                    d2_out[offsets[t] + c] = s;
                }
                ++c;
            }
        }
        counts_out[t] = c;
    }
    return 0;
}

/*
 * Kernel density sums (Section "Kernel Density Estimation"): for each
 * selected query f = sum over references of K(||q - r||) with the Gaussian
 * kernel K(d) = exp(-d^2 / (2 h^2)) (no normalising constant), in FP64.
 * budget_out (optional) receives sum of K(d) (1 + d^2 / (2 h^2)), the scale
 * of the FP32 rounding of a sum whose terms are evaluated from FP32 squared
 * distances.  exclude_self skips reference qsel[t] for row t.
 */
int knn_oracle_kde_rows(const float *q, const int64_t *qsel, int64_t nsel, const float *r,
                        int64_t m, int32_t d, double h, int32_t exclude_self, double *f_out,
                        double *budget_out)
{
    if (!q || !qsel || !r || !f_out || nsel < 0 || m <= 0 || d <= 0 || !(h > 0.0))
        return -1;
    const double c = 1.0 / (2.0 * h * h);
    int64_t t;
#pragma omp parallel for schedule(dynamic, 4)
    for (t = 0; t < nsel; ++t) {
        int64_t i = qsel[t];
        const float *qi = q + i * (int64_t)d;
        double f = 0.0, b = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            if (exclude_self && j == i) continue;
            const float *rj = r + j * (int64_t)d;
            double s = 0.0;
            for (int u = 0; u < d; ++u) {
                double diff = (double)qi[u] - (double)rj[u];
                s += diff * diff;
            }
            const double x = s * c, k = exp(-x);
            f += k;
            b += k * (1.0 + x);
        }
        f_out[t] = f;
        if (budget_out) budget_out[t] = b;
    }
    return 0;
}

/*
 * Euclidean minimum spanning tree (Section "Boruvka's Algorithm": the tree
 * the dual-tree Boruvka iteration ends with) by Prim's algorithm on the
 * complete graph, FP64 squared distances of the FP32 points.  Edges are
 * compared by the strict total order (squared length, smaller endpoint
 * index, larger endpoint index), under which the tree is unique.
 * Outputs n - 1 edges in the order Prim adds them: edge_u < edge_v
 * (point indices) and the squared length in edge_d2.  Returns 0, or -1 on
 * invalid arguments.
 */
static int edge_before(double da, int64_t ua, int64_t va, double db, int64_t ub, int64_t vb)
{
    if (da != db) return da < db;
    if (ua != ub) return ua < ub;
    return va < vb;
}

int knn_oracle_emst(const float *x, int64_t n, int32_t d, int64_t *edge_u, int64_t *edge_v,
                    double *edge_d2)
{
    if (!x || n < 1 || d <= 0 || (n > 1 && (!edge_u || !edge_v || !edge_d2))) return -1;
    char *in = (char *)calloc((size_t)n, 1);
    double *key = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t *from = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!in || !key || !from) {
        free(in); free(key); free(from);
        return -1;
    }
    for (int64_t j = 0; j < n; ++j) { key[j] = INFINITY; from[j] = -1; }
    int64_t cur = 0;
    in[0] = 1;
    for (int64_t step = 0; step + 1 < n; ++step) {
        /* the new tree vertex updates every outside vertex's best edge */
        const float *xc = x + cur * (int64_t)d;
        int64_t j;
#pragma omp parallel for schedule(static)
        for (j = 0; j < n; ++j) {
            if (in[j]) continue;
            const float *xj = x + j * (int64_t)d;
            double s = 0.0;
            for (int u = 0; u < d; ++u) {
                double diff = (double)xc[u] - (double)xj[u];
                s += diff * diff;
            }
            int64_t a = cur < j ? cur : j, b = cur < j ? j : cur;
            int64_t fa = from[j] < 0 ? 0 : (from[j] < j ? from[j] : j);
            int64_t fb = from[j] < 0 ? 0 : (from[j] < j ? j : from[j]);
            if (from[j] < 0 || edge_before(s, a, b, key[j], fa, fb)) {
                key[j] = s;
                from[j] = cur;
            }
        }
        /* the outside vertex with the smallest best edge joins */
        int64_t best = -1;
        for (j = 0; j < n; ++j) {
            if (in[j]) continue;
            if (best < 0) { best = j; continue; }
            int64_t a = from[j] < j ? from[j] : j, b = from[j] < j ? j : from[j];
            int64_t ba = from[best] < best ? from[best] : best;
            int64_t bb = from[best] < best ? best : from[best];
            if (edge_before(key[j], a, b, key[best], ba, bb)) best = j;
        }
        in[best] = 1;
        edge_u[step] = from[best] < best ? from[best] : best;
        edge_v[step] = from[best] < best ? best : from[best];
        edge_d2[step] = key[best];
        cur = best;
    }
    free(in); free(key); free(from);
    return 0;
}
