// Learned seed radius: a small MLP (n_in -> H -> H -> 1, ReLU) whose output
// is an initial value of a query leaf's pruning bound.  Not in the paper: it
// only feeds min(B(N_q), seed) and every leaf whose k-th distances exceed
// its seed is searched again without it, so the network can never change
// the answer, only the amount of work.
//
// Kernels (FP32, deterministic):
//   k_mlp_forward   one thread per sample, weights staged in LDS
//   k_mlp_grad      32 samples per block: per-sample forward/backward, then
//                   block-level reductions of the weight gradients into a
//                   per-block partial vector (fixed order)
//   k_mlp_reduce    sums the partials over blocks in block order
//   k_mlp_adam      Adam with bias correction
//   k_seed_features per query leaf: box centre, lambda, point count, log
//                   density of the reference leaf reached from the centre
//   k_seed_radius   exp(y * y_sd + y_mu + log_margin)
//   k_train_*       training-set preparation for knn_seed_train: log
//                   targets, row gathers, FP64 column mean and deviation,
//                   standardised targets
// Parameter layout: W1 (H x n_in, row-major), b1, W2 (H x H), b2, w3 (H), b3.
#include "search.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <utility>
#include <vector>

namespace knnx {

constexpr int kH = 64;         // hidden width (fixed)
constexpr int kMaxIn = 72;     // d + 3 <= 67
constexpr int kGradBlock = 32;  // samples (and threads) per gradient block

struct MlpDev {
    const float *p;
    const float *mu, *isd;
    int n_in;
};

__device__ inline int off_b1(int n_in) { return kH * n_in; }
__device__ inline int off_W2(int n_in) { return kH * n_in + kH; }
__device__ inline int off_b2(int n_in) { return kH * n_in + kH + kH * kH; }
__device__ inline int off_w3(int n_in) { return kH * n_in + 2 * kH + kH * kH; }
__device__ inline int off_b3(int n_in) { return kH * n_in + 3 * kH + kH * kH; }
__host__ __device__ inline int64_t n_params_of(int n_in) { return int64_t(kH) * n_in + 3 * kH + kH * kH + 1; }

// ---- forward -----------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_forward(MlpDev m, const float *__restrict__ x,
                                                     int64_t n, float *__restrict__ y) {
    extern __shared__ float sw[];
    const int n_in = m.n_in;
    const int P = int(n_params_of(n_in));
    for (int i = threadIdx.x; i < P; i += blockDim.x) sw[i] = m.p[i];
    __syncthreads();
    const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= n) return;
    float a1[kH];
#pragma unroll
    for (int hh = 0; hh < kH; ++hh) a1[hh] = sw[off_b1(n_in) + hh];
    for (int i = 0; i < n_in; ++i) {
        const float xh = (x[b * n_in + i] - m.mu[i]) * m.isd[i];
#pragma unroll
        for (int hh = 0; hh < kH; ++hh) a1[hh] = fmaf(sw[hh * n_in + i], xh, a1[hh]);
    }
#pragma unroll
    for (int hh = 0; hh < kH; ++hh) a1[hh] = fmaxf(a1[hh], 0.f);
    float out = sw[off_b3(n_in)];
#pragma unroll 4
    for (int o = 0; o < kH; ++o) {
        float acc = sw[off_b2(n_in) + o];
#pragma unroll
        for (int i = 0; i < kH; ++i) acc = fmaf(sw[off_W2(n_in) + o * kH + i], a1[i], acc);
        out = fmaf(sw[off_w3(n_in) + o], fmaxf(acc, 0.f), out);
    }
    y[b] = out;
}

// ---- loss and gradient ---------------------------------------------------------
// Block of 32 threads = 32 samples.  LDS: x_hat, h1, relu(a2), da2, da1 per
// sample; the weights are read from global memory (broadcast loads).
__global__ __launch_bounds__(kGradBlock) void k_mlp_grad(MlpDev m, const float *__restrict__ x,
                                                        const float *__restrict__ t, int64_t n,
                                                        float *__restrict__ partial,
                                                        float *__restrict__ loss_partial) {
    const int n_in = m.n_in;
    const int P = int(n_params_of(n_in));
    __shared__ float s_x[kGradBlock][kMaxIn];
    __shared__ float s_h1[kGradBlock][kH + 1];
    __shared__ float s_d2[kGradBlock][kH + 1];
    __shared__ float s_d1[kGradBlock][kH + 1];
    __shared__ float s_dy[kGradBlock];
    const float *p = m.p;
    const int tid = threadIdx.x;
    const int64_t b = int64_t(blockIdx.x) * kGradBlock + tid;
    const bool live = b < n;
    const float inv_n = 1.0f / float(n);

    // per-sample forward, keeping h1 and the ReLU masks
    for (int i = 0; i < n_in; ++i) s_x[tid][i] = live ? (x[b * n_in + i] - m.mu[i]) * m.isd[i] : 0.f;
    float a1[kH];
#pragma unroll
    for (int hh = 0; hh < kH; ++hh) a1[hh] = p[off_b1(n_in) + hh];
    for (int i = 0; i < n_in; ++i) {
        const float xh = s_x[tid][i];
#pragma unroll
        for (int hh = 0; hh < kH; ++hh) a1[hh] = fmaf(p[hh * n_in + i], xh, a1[hh]);
    }
    uint64_t m1 = 0;
#pragma unroll
    for (int hh = 0; hh < kH; ++hh) {
        if (a1[hh] > 0.f) m1 |= 1ull << hh;
        a1[hh] = fmaxf(a1[hh], 0.f);
        s_h1[tid][hh] = a1[hh];
    }
    float a2v[kH];
    float y = p[off_b3(n_in)];
#pragma unroll
    for (int o = 0; o < kH; ++o) {
        float acc = p[off_b2(n_in) + o];
#pragma unroll
        for (int i = 0; i < kH; ++i) acc = fmaf(p[off_W2(n_in) + o * kH + i], a1[i], acc);
        a2v[o] = acc;
        y = fmaf(p[off_w3(n_in) + o], fmaxf(acc, 0.f), y);
    }
    const float r = live ? y - t[b] : 0.f;
    const float dy = 2.0f * r * inv_n;
    s_dy[tid] = dy;
    // backward to layer 2 pre-activations, then to layer 1
    float dh1[kH];
#pragma unroll
    for (int i = 0; i < kH; ++i) dh1[i] = 0.f;
#pragma unroll
    for (int o = 0; o < kH; ++o) {
        const float d2 = a2v[o] > 0.f ? dy * p[off_w3(n_in) + o] : 0.f;
        s_d2[tid][o] = d2;
#pragma unroll
        for (int i = 0; i < kH; ++i) dh1[i] = fmaf(p[off_W2(n_in) + o * kH + i], d2, dh1[i]);
    }
#pragma unroll
    for (int i = 0; i < kH; ++i) s_d1[tid][i] = ((m1 >> i) & 1ull) ? dh1[i] : 0.f;
    __shared__ float s_h2[kGradBlock][kH + 1];
#pragma unroll
    for (int o = 0; o < kH; ++o) s_h2[tid][o] = fmaxf(a2v[o], 0.f);
    // loss partial
    float lsum = r * r;
#pragma unroll
    for (int off = kGradBlock / 2; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
    __syncthreads();

    float *out = partial + int64_t(blockIdx.x) * P;
    // W1 (H x n_in) and b1
    for (int e = tid; e < kH * n_in; e += kGradBlock) {
        const int hh = e / n_in, i = e % n_in;
        float acc = 0.f;
        for (int s = 0; s < kGradBlock; ++s) acc = fmaf(s_d1[s][hh], s_x[s][i], acc);
        out[e] = acc;
    }
    for (int hh = tid; hh < kH; hh += kGradBlock) {
        float acc = 0.f;
        for (int s = 0; s < kGradBlock; ++s) acc += s_d1[s][hh];
        out[off_b1(n_in) + hh] = acc;
    }
    // W2 (H x H) and b2
    for (int e = tid; e < kH * kH; e += kGradBlock) {
        const int o = e / kH, i = e % kH;
        float acc = 0.f;
        for (int s = 0; s < kGradBlock; ++s) acc = fmaf(s_d2[s][o], s_h1[s][i], acc);
        out[off_W2(n_in) + e] = acc;
    }
    for (int o = tid; o < kH; o += kGradBlock) {
        float acc = 0.f, acc3 = 0.f;
        for (int s = 0; s < kGradBlock; ++s) {
            acc += s_d2[s][o];
            acc3 = fmaf(s_dy[s], s_h2[s][o], acc3);
        }
        out[off_b2(n_in) + o] = acc;
        out[off_w3(n_in) + o] = acc3;
    }
    if (tid == 0) {
        float acc = 0.f;
        for (int s = 0; s < kGradBlock; ++s) acc += s_dy[s];
        out[off_b3(n_in)] = acc;
        loss_partial[blockIdx.x] = lsum;
    }
}

__global__ void k_mlp_reduce(const float *__restrict__ partial, int nblk, int P,
                             float *__restrict__ grad, const float *__restrict__ loss_partial,
                             float *__restrict__ loss, float inv_n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P) {
        float acc = 0.f;
        for (int b = 0; b < nblk; ++b) acc += partial[int64_t(b) * P + i];
        grad[i] = acc;
    }
    if (i == 0) {
        float acc = 0.f;
        for (int b = 0; b < nblk; ++b) acc += loss_partial[b];
        *loss = acc * inv_n;
    }
}

__global__ void k_mlp_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                           float *__restrict__ v, int P, float lr, float b1, float b2, float eps,
                           float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---- seed features and radii --------------------------------------------------
template <int DP>
__global__ void k_seed_features(const float *__restrict__ rbox, const int2 *__restrict__ rrange,
                                int r_first_leaf, const float *__restrict__ qbox,
                                const int2 *__restrict__ qrange, const float *__restrict__ qlam,
                                int q_first_leaf, int nq_leaves, int d, float *__restrict__ feats) {
    const int leaf = blockIdx.x * blockDim.x + threadIdx.x;
    if (leaf >= nq_leaves) return;
    const int qn = q_first_leaf + leaf;
    const float *qb = qbox + int64_t(qn) * 2 * DP;
    const int nf = d + 3;
    float *f = feats + int64_t(leaf) * nf;
    const int cnt = qrange[qn].y;
    float c[DP];
#pragma unroll
    for (int j = 0; j < DP; ++j) c[j] = cnt > 0 ? 0.5f * (qb[j] + qb[DP + j]) : 0.f;
    for (int j = 0; j < d; ++j) f[j] = c[j];
    f[d] = qlam[qn];
    f[d + 1] = float(cnt);
    // descend the reference tree toward the centre (nearer child, left on ties)
    int node = 0;
    while (node < r_first_leaf) {
        float dm[2];
        for (int q = 0; q < 2; ++q) {
            const float *b = rbox + int64_t(2 * node + 1 + q) * 2 * DP;
            // plain IEEE products and sums (no contraction): the branch taken
            // is a documented function of the FP32 inputs
            float s = 0.f;
            for (int j = 0; j < d; ++j) {
                const float gap = fmaxf(fmaxf(b[j] - c[j], c[j] - b[DP + j]), 0.f);
                s = __fadd_rn(s, __fmul_rn(gap, gap));
            }
            dm[q] = s;
        }
        node = 2 * node + 1 + ((dm[1] < dm[0]) ? 1 : 0);
    }
    const float *rb = rbox + int64_t(node) * 2 * DP;
    const float *root = rbox;
    float logvol = 0.f;
    for (int j = 0; j < d; ++j) {
        const float eps = 1e-6f * (root[DP + j] - root[j]) + 1e-30f;
        logvol += logf(fmaxf(rb[DP + j] - rb[j], eps));
    }
    f[d + 2] = logf(fmaxf(float(rrange[node].y), 1.0f)) - logvol;
}

__global__ void k_seed_radius(const float *__restrict__ yraw, int64_t n, float y_mu, float y_sd,
                              float log_margin, float *__restrict__ radius) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) radius[i] = expf(yraw[i] * y_sd + y_mu + log_margin);
}

// ---- training-set preparation ---------------------------------------------
// y[i] = log max(kth[i], 1e-30); bad = 1 when kth[i] is negative or not finite
__global__ void k_train_log_targets(const float *__restrict__ kth, int64_t n, float *__restrict__ y,
                                    int *__restrict__ bad) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = kth[i];
    if (!(v >= 0.f) || !isfinite(v)) *bad = 1;
    y[i] = float(log(fmax(double(v), 1e-30)));
}

// rows idx[0 .. n) of x (n_in columns) and of y, in that order
__global__ void k_train_gather(const float *__restrict__ x, const float *__restrict__ y,
                               const int32_t *__restrict__ idx, int64_t n, int n_in,
                               float *__restrict__ xo, float *__restrict__ yo) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t r = idx[i];
    for (int j = 0; j < n_in; ++j) xo[i * n_in + j] = x[r * n_in + j];
    yo[i] = y[r];
}

// FP64 sum of a block's values (fixed order: strided per thread, then a tree)
__device__ inline double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// one block per column c of x (n rows, row stride ld): out[2c] = mean,
// out[2c + 1] = population deviation, both in FP64 (two passes)
__global__ __launch_bounds__(256) void k_train_column_stats(const float *__restrict__ x, int64_t n,
                                                            int ld, double *__restrict__ out) {
    __shared__ double red[256];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += double(x[i * ld + c]);
    const double mean = block_sum(s, red) / double(n);
    double q = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double t = double(x[i * ld + c]) - mean;
        q = fma(t, t, q);
    }
    const double var = block_sum(q, red) / double(n);
    if (threadIdx.x == 0) {
        out[2 * c] = mean;
        out[2 * c + 1] = sqrt(var);
    }
}

// t[i] = (y[i] - mu) / sd
__global__ void k_train_standardise(const float *__restrict__ y, int64_t n, double mu, double sd,
                                    float *__restrict__ t) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) t[i] = float((double(y[i]) - mu) / sd);
}

}  // namespace knnx

// ---------------------------------------------------------------------------
// handle and C ABI
// ---------------------------------------------------------------------------
struct knn_mlp {
    int n_in = 0, hidden = 0;
    int64_t P = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    float *mu = nullptr, *isd = nullptr;
    float *partial = nullptr;
    int64_t partial_blocks = 0;
    float *lossbuf = nullptr;  // [0] loss, [1..] per-block partials
    int64_t loss_cap = 0;
    float y_mu = 0.f, y_sd = 1.f;
    int64_t step = 0;
};

using namespace knnx;

namespace {

knn_status ensure_grad_scratch(knn_mlp *m, int64_t nblk) {
    if (nblk > m->partial_blocks) {
        (void)hipFree(m->partial);
        (void)hipFree(m->lossbuf);
        m->partial = nullptr;
        m->lossbuf = nullptr;
        KNN_HIP(hipMalloc(&m->partial, size_t(nblk) * m->P * sizeof(float)));
        KNN_HIP(hipMalloc(&m->lossbuf, size_t(nblk + 1) * sizeof(float)));
        m->partial_blocks = nblk;
    }
    return KNN_OK;
}

MlpDev dev_of(const knn_mlp *m) { return MlpDev{m->p, m->mu, m->isd, m->n_in}; }

// gradient of the mean squared error over n rows into m->g, the loss into
// m->lossbuf[0] (no synchronisation)
knn_status launch_loss_grad(knn_mlp *m, const float *x, const float *t, int64_t n, hipStream_t s) {
    const int64_t nblk = (n + kGradBlock - 1) / kGradBlock;
    KNN_TRY(ensure_grad_scratch(m, nblk));
    k_mlp_grad<<<int(nblk), kGradBlock, 0, s>>>(dev_of(m), x, t, n, m->partial, m->lossbuf + 1);
    k_mlp_reduce<<<int((m->P + 255) / 256), 256, 0, s>>>(m->partial, int(nblk), int(m->P), m->g,
                                                         m->lossbuf + 1, m->lossbuf,
                                                         1.0f / float(n));
    KNN_HIP(hipGetLastError());
    return KNN_OK;
}

// one Adam step with the stored gradient (no synchronisation)
knn_status launch_adam(knn_mlp *m, float lr, float beta1, float beta2, float eps, hipStream_t s) {
    m->step += 1;
    const float c1 = float(1.0 - std::pow(double(beta1), double(m->step)));
    const float c2 = float(1.0 - std::pow(double(beta2), double(m->step)));
    k_mlp_adam<<<int((m->P + 255) / 256), 256, 0, s>>>(m->p, m->g, m->m, m->v, int(m->P), lr, beta1,
                                                       beta2, eps, c1, c2);
    KNN_HIP(hipGetLastError());
    return KNN_OK;
}

// device buffers of one call, released in stream order on every return
struct CallBufs {
    hipStream_t s;
    std::vector<void *> ps;
    ~CallBufs() {
        for (void *p : ps) free_async(p, s);
    }
    template <class T>
    hipError_t get(T **p, size_t count) {
        const hipError_t e = alloc_async(p, count, s);
        if (e == hipSuccess) ps.push_back(*p);
        return e;
    }
};

// SplitMix64 (Steele, Lea and Flood, 2014) in counter form: the i-th value of
// the sequence started at state s
uint64_t splitmix_value(uint64_t s, uint64_t i) {
    uint64_t z = s + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// rows 0 .. n-1 ordered by (key, row), key i = value i of stream s
std::vector<int32_t> key_order(uint64_t s, int64_t n) {
    std::vector<std::pair<uint64_t, int32_t>> kv(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) kv[size_t(i)] = {splitmix_value(s, uint64_t(i)), int32_t(i)};
    std::sort(kv.begin(), kv.end());
    std::vector<int32_t> o(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) o[size_t(i)] = kv[size_t(i)].second;
    return o;
}

}  // namespace

extern "C" {

knn_status knn_mlp_create(int32_t n_in, int32_t hidden, knn_mlp **out) {
    set_error("");
    if (!out) return fail(KNN_E_INVALID_ARG, "knn_mlp_create: out is NULL");
    *out = nullptr;
    if (n_in < 1 || n_in > kMaxIn)
        return fail(KNN_E_INVALID_ARG, "knn_mlp_create: need 1 <= n_in <= 72");
    if (hidden != kH) return fail(KNN_E_UNSUPPORTED, "knn_mlp_create: hidden width must be 64");
    knn_mlp *m = new knn_mlp();
    m->n_in = n_in;
    m->hidden = hidden;
    m->P = n_params_of(n_in);
    hipError_t e = hipSuccess;
    e = e ? e : hipMalloc(&m->p, m->P * sizeof(float));
    e = e ? e : hipMalloc(&m->g, m->P * sizeof(float));
    e = e ? e : hipMalloc(&m->m, m->P * sizeof(float));
    e = e ? e : hipMalloc(&m->v, m->P * sizeof(float));
    e = e ? e : hipMalloc(&m->mu, n_in * sizeof(float));
    e = e ? e : hipMalloc(&m->isd, n_in * sizeof(float));
    e = e ? e : hipMemset(m->p, 0, m->P * sizeof(float));
    e = e ? e : hipMemset(m->g, 0, m->P * sizeof(float));
    e = e ? e : hipMemset(m->m, 0, m->P * sizeof(float));
    e = e ? e : hipMemset(m->v, 0, m->P * sizeof(float));
    if (e == hipSuccess) {
        std::vector<float> z(n_in, 0.f), o(n_in, 1.f);
        e = hipMemcpy(m->mu, z.data(), n_in * 4, hipMemcpyHostToDevice);
        e = e ? e : hipMemcpy(m->isd, o.data(), n_in * 4, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        knn_mlp_free(m);
        return fail(e == hipErrorOutOfMemory ? KNN_E_OOM : KNN_E_DEVICE,
                    std::string("knn_mlp_create: ") + hipGetErrorString(e));
    }
    *out = m;
    return KNN_OK;
}

void knn_mlp_free(knn_mlp *m) {
    if (!m) return;
    hipFree(m->p);
    hipFree(m->g);
    hipFree(m->m);
    hipFree(m->v);
    hipFree(m->mu);
    hipFree(m->isd);
    hipFree(m->partial);
    hipFree(m->lossbuf);
    delete m;
}

knn_status knn_mlp_num_params(const knn_mlp *m, int64_t *n) {
    if (!m || !n) return fail(KNN_E_INVALID_ARG, "knn_mlp_num_params: NULL argument");
    *n = m->P;
    return KNN_OK;
}

knn_status knn_mlp_set_params(knn_mlp *m, const float *host, int64_t n) {
    set_error("");
    if (!m || !host) return fail(KNN_E_INVALID_ARG, "knn_mlp_set_params: NULL argument");
    if (n != m->P) return fail(KNN_E_INVALID_ARG, "knn_mlp_set_params: wrong parameter count");
    KNN_HIP(hipMemcpy(m->p, host, n * sizeof(float), hipMemcpyHostToDevice));
    KNN_HIP(hipMemset(m->m, 0, n * sizeof(float)));
    KNN_HIP(hipMemset(m->v, 0, n * sizeof(float)));
    m->step = 0;
    return KNN_OK;
}

knn_status knn_mlp_get_params(const knn_mlp *m, float *host, int64_t n) {
    if (!m || !host) return fail(KNN_E_INVALID_ARG, "knn_mlp_get_params: NULL argument");
    if (n != m->P) return fail(KNN_E_INVALID_ARG, "knn_mlp_get_params: wrong parameter count");
    KNN_HIP(hipMemcpy(host, m->p, n * sizeof(float), hipMemcpyDeviceToHost));
    return KNN_OK;
}

knn_status knn_mlp_get_grads(const knn_mlp *m, float *host, int64_t n) {
    if (!m || !host) return fail(KNN_E_INVALID_ARG, "knn_mlp_get_grads: NULL argument");
    if (n != m->P) return fail(KNN_E_INVALID_ARG, "knn_mlp_get_grads: wrong parameter count");
    KNN_HIP(hipMemcpy(host, m->g, n * sizeof(float), hipMemcpyDeviceToHost));
    return KNN_OK;
}

knn_status knn_mlp_set_norm(knn_mlp *m, const float *mu_host, const float *inv_sd_host,
                            float y_mu, float y_sd) {
    set_error("");
    if (!m || !mu_host || !inv_sd_host) return fail(KNN_E_INVALID_ARG, "knn_mlp_set_norm: NULL argument");
    for (int i = 0; i < m->n_in; ++i)
        if (!std::isfinite(mu_host[i]) || !std::isfinite(inv_sd_host[i]))
            return fail(KNN_E_INVALID_ARG, "knn_mlp_set_norm: non-finite normalisation");
    if (!std::isfinite(y_mu) || !std::isfinite(y_sd))
        return fail(KNN_E_INVALID_ARG, "knn_mlp_set_norm: non-finite output scale");
    KNN_HIP(hipMemcpy(m->mu, mu_host, m->n_in * 4, hipMemcpyHostToDevice));
    KNN_HIP(hipMemcpy(m->isd, inv_sd_host, m->n_in * 4, hipMemcpyHostToDevice));
    m->y_mu = y_mu;
    m->y_sd = y_sd;
    return KNN_OK;
}

knn_status knn_mlp_forward(const knn_mlp *m, const float *x, int64_t n, float *y, void *stream) {
    set_error("");
    if (!m || !x || !y || n < 0) return fail(KNN_E_INVALID_ARG, "knn_mlp_forward: bad argument");
    if (n == 0) return KNN_OK;
    hipStream_t s = (hipStream_t)stream;
    const size_t lds = size_t(m->P) * sizeof(float);
    k_mlp_forward<<<int((n + 255) / 256), 256, lds, s>>>(dev_of(m), x, n, y);
    KNN_HIP(hipGetLastError());
    KNN_HIP(hipStreamSynchronize(s));
    return KNN_OK;
}

knn_status knn_mlp_loss_grad(knn_mlp *m, const float *x, const float *t, int64_t n,
                             float *loss_host, void *stream) {
    set_error("");
    if (!m || !x || !t || n <= 0) return fail(KNN_E_INVALID_ARG, "knn_mlp_loss_grad: bad argument");
    hipStream_t s = (hipStream_t)stream;
    KNN_TRY(launch_loss_grad(m, x, t, n, s));
    if (loss_host) KNN_HIP(hipMemcpyAsync(loss_host, m->lossbuf, 4, hipMemcpyDeviceToHost, s));
    KNN_HIP(hipStreamSynchronize(s));
    return KNN_OK;
}

knn_status knn_mlp_adam_step(knn_mlp *m, float lr, float beta1, float beta2, float eps,
                             void *stream) {
    set_error("");
    if (!m) return fail(KNN_E_INVALID_ARG, "knn_mlp_adam_step: NULL model");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return fail(KNN_E_INVALID_ARG, "knn_mlp_adam_step: bad hyper-parameters");
    hipStream_t s = (hipStream_t)stream;
    KNN_TRY(launch_adam(m, lr, beta1, beta2, eps, s));
    KNN_HIP(hipStreamSynchronize(s));
    return KNN_OK;
}

knn_status knn_mlp_save(const knn_mlp *m, const char *path) {
    set_error("");
    if (!m || !path) return fail(KNN_E_INVALID_ARG, "knn_mlp_save: NULL argument");
    std::vector<float> p(m->P), mu(m->n_in), isd(m->n_in);
    KNN_HIP(hipMemcpy(p.data(), m->p, m->P * 4, hipMemcpyDeviceToHost));
    KNN_HIP(hipMemcpy(mu.data(), m->mu, m->n_in * 4, hipMemcpyDeviceToHost));
    KNN_HIP(hipMemcpy(isd.data(), m->isd, m->n_in * 4, hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(KNN_E_MODEL, std::string("knn_mlp_save: cannot open ") + path);
    const char magic[8] = {'K', 'N', 'N', 'S', 'E', 'E', 'D', '1'};
    const int32_t hdr[2] = {m->n_in, m->hidden};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, 4, 2, f) == 2 &&
              std::fwrite(&m->y_mu, 4, 1, f) == 1 && std::fwrite(&m->y_sd, 4, 1, f) == 1 &&
              std::fwrite(mu.data(), 4, m->n_in, f) == size_t(m->n_in) &&
              std::fwrite(isd.data(), 4, m->n_in, f) == size_t(m->n_in) &&
              std::fwrite(p.data(), 4, m->P, f) == size_t(m->P);
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(KNN_E_MODEL, "knn_mlp_save: write failed");
    return KNN_OK;
}

knn_status knn_mlp_load(const char *path, knn_mlp **out) {
    set_error("");
    if (!path || !out) return fail(KNN_E_INVALID_ARG, "knn_mlp_load: NULL argument");
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(KNN_E_MODEL, std::string("knn_mlp_load: cannot open ") + path);
    char magic[8];
    int32_t hdr[2];
    float ym, ys;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "KNNSEED1", 8) == 0 &&
              std::fread(hdr, 4, 2, f) == 2 && std::fread(&ym, 4, 1, f) == 1 &&
              std::fread(&ys, 4, 1, f) == 1 && hdr[0] >= 1 && hdr[0] <= kMaxIn && hdr[1] == kH;
    std::vector<float> mu, isd, p;
    if (ok) {
        mu.resize(hdr[0]);
        isd.resize(hdr[0]);
        p.resize(n_params_of(hdr[0]));
        ok = std::fread(mu.data(), 4, mu.size(), f) == mu.size() &&
             std::fread(isd.data(), 4, isd.size(), f) == isd.size() &&
             std::fread(p.data(), 4, p.size(), f) == p.size();
        char extra;
        ok = ok && std::fread(&extra, 1, 1, f) == 0;
    }
    std::fclose(f);
    if (!ok) return fail(KNN_E_MODEL, "knn_mlp_load: not a seed-network file or truncated");
    knn_mlp *m = nullptr;
    KNN_TRY(knn_mlp_create(hdr[0], hdr[1], &m));
    knn_status st = knn_mlp_set_params(m, p.data(), int64_t(p.size()));
    if (st == KNN_OK) st = knn_mlp_set_norm(m, mu.data(), isd.data(), ym, ys);
    if (st != KNN_OK) {
        knn_mlp_free(m);
        return st;
    }
    *out = m;
    return KNN_OK;
}

knn_status knn_seed_features(const knn_tree *ref, const knn_tree *query, float *feats,
                             void *stream) {
    set_error("");
    if (!ref || !feats) return fail(KNN_E_INVALID_ARG, "knn_seed_features: NULL argument");
    const knn_tree *qt = query ? query : ref;
    if (qt->d != ref->d) return fail(KNN_E_INVALID_ARG, "knn_seed_features: d differs");
    hipStream_t s = (hipStream_t)stream;
    const int nq = int(qt->n_leaves);
    const int grid = (nq + 127) / 128;
#define KNN_FEAT(DP)                                                                          \
    k_seed_features<DP><<<grid, 128, 0, s>>>(ref->box, ref->range, int(ref->first_leaf),      \
                                             qt->box, qt->range, qt->lam, int(qt->first_leaf), \
                                             nq, ref->d, feats)
    switch (ref->dp) {
        case 4: KNN_FEAT(4); break;
        case 8: KNN_FEAT(8); break;
        case 16: KNN_FEAT(16); break;
        case 32: KNN_FEAT(32); break;
        default: KNN_FEAT(64); break;
    }
#undef KNN_FEAT
    KNN_HIP(hipGetLastError());
    KNN_HIP(hipStreamSynchronize(s));
    return KNN_OK;
}

knn_status knn_seed_radius(const knn_mlp *m, const float *feats, int64_t n, float log_margin,
                           float *radius, void *stream) {
    set_error("");
    if (!m || !feats || !radius || n < 0) return fail(KNN_E_INVALID_ARG, "knn_seed_radius: bad argument");
    if (n == 0) return KNN_OK;
    hipStream_t s = (hipStream_t)stream;
    float *y = nullptr;
    KNN_HIP(alloc_async(&y, size_t(n), s));
    const size_t lds = size_t(m->P) * sizeof(float);
    k_mlp_forward<<<int((n + 255) / 256), 256, lds, s>>>(dev_of(m), feats, n, y);
    k_seed_radius<<<int((n + 255) / 256), 256, 0, s>>>(y, n, m->y_mu, m->y_sd, log_margin, radius);
    hipError_t e = hipGetLastError();
    free_async(y, s);
    if (e != hipSuccess) return hip_fail(e, "knn_seed_radius launch", __FILE__, __LINE__);
    KNN_HIP(hipStreamSynchronize(s));
    return KNN_OK;
}

knn_status knn_seed_train(const float *feats, const float *kth, int64_t n, int32_t n_in,
                          const knn_train_opts *opts, knn_mlp **out, float *log_margin_out,
                          float *loss_out, void *stream) {
    set_error("");
    if (!feats || !kth || !opts || !out || !log_margin_out)
        return fail(KNN_E_INVALID_ARG, "knn_seed_train: NULL argument");
    *out = nullptr;
    if (n < 2 || n > INT32_MAX) return fail(KNN_E_INVALID_ARG, "knn_seed_train: need 2 <= n < 2^31");
    if (n_in < 1 || n_in > kMaxIn) return fail(KNN_E_INVALID_ARG, "knn_seed_train: need 1 <= n_in <= 72");
    const knn_train_opts o = *opts;
    if (o.epochs < 1 || o.batch < 1 || !(o.lr > 0.f) || !std::isfinite(o.lr) || !(o.val_frac > 0.f) ||
        !(o.val_frac < 1.f) || !(o.target_fallback >= 0.f) || !(o.target_fallback < 1.f))
        return fail(KNN_E_INVALID_ARG, "knn_seed_train: option outside its domain");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n_val = std::max<int64_t>(1, int64_t(std::floor(double(n) * double(o.val_frac))));
    const int64_t n_tr = n - n_val;
    const int64_t bmax = std::min<int64_t>(o.batch, n_tr);

    CallBufs B{s, {}};
    float *ylog, *xtr, *ytr, *ttr, *xva, *yva, *xb, *tb, *pred, *hist;
    int32_t *idx, *ord;
    double *st;
    int *bad;
    const int64_t steps = int64_t(o.epochs) * ((n_tr + bmax - 1) / bmax);
    KNN_HIP(B.get(&ylog, size_t(n)));
    KNN_HIP(B.get(&xtr, size_t(n_tr) * n_in));
    KNN_HIP(B.get(&ytr, size_t(n_tr)));
    KNN_HIP(B.get(&ttr, size_t(n_tr)));
    KNN_HIP(B.get(&xva, size_t(n_val) * n_in));
    KNN_HIP(B.get(&yva, size_t(n_val)));
    KNN_HIP(B.get(&xb, size_t(bmax) * n_in));
    KNN_HIP(B.get(&tb, size_t(bmax)));
    KNN_HIP(B.get(&pred, size_t(n_val)));
    KNN_HIP(B.get(&hist, size_t(steps)));
    KNN_HIP(B.get(&idx, size_t(n)));
    KNN_HIP(B.get(&ord, size_t(n_tr)));
    KNN_HIP(B.get(&st, size_t(2 * (n_in + 1))));
    KNN_HIP(B.get(&bad, size_t(1)));
    const int T = 256;
    auto blocks = [&](int64_t m) { return int((m + T - 1) / T); };

    // targets, checked
    KNN_HIP(zero_words(bad, 1, s));
    k_train_log_targets<<<blocks(n), T, 0, s>>>(kth, n, ylog, bad);
    KNN_HIP(hipGetLastError());
    int bad_h = 0;
    KNN_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    KNN_HIP(hipStreamSynchronize(s));
    if (bad_h) return fail(KNN_E_INVALID_ARG, "knn_seed_train: a target is negative or not finite");

    // 1. split (stream 1)
    const std::vector<int32_t> split = key_order(splitmix_value(o.seed, 1), n);
    KNN_HIP(hipMemcpyAsync(idx, split.data(), size_t(n) * 4, hipMemcpyHostToDevice, s));
    k_train_gather<<<blocks(n_val), T, 0, s>>>(feats, ylog, idx, n_val, n_in, xva, yva);
    k_train_gather<<<blocks(n_tr), T, 0, s>>>(feats, ylog, idx + n_val, n_tr, n_in, xtr, ytr);
    // 2. standardisation
    k_train_column_stats<<<n_in, T, 0, s>>>(xtr, n_tr, n_in, st);
    k_train_column_stats<<<1, T, 0, s>>>(ytr, n_tr, 1, st + 2 * n_in);
    KNN_HIP(hipGetLastError());
    std::vector<double> sth(size_t(2 * (n_in + 1)));
    KNN_HIP(hipMemcpyAsync(sth.data(), st, sth.size() * 8, hipMemcpyDeviceToHost, s));
    KNN_HIP(hipStreamSynchronize(s));
    std::vector<float> mu(static_cast<size_t>(n_in)), isd(static_cast<size_t>(n_in));
    for (int j = 0; j < n_in; ++j) {
        const double sd = sth[2 * j + 1] < 1e-12 ? 1.0 : sth[2 * j + 1];
        mu[j] = float(sth[2 * j]);
        isd[j] = float(1.0 / sd);
    }
    const double y_mu = sth[2 * n_in], y_sd = std::max(sth[2 * n_in + 1], 1e-12);
    k_train_standardise<<<blocks(n_tr), T, 0, s>>>(ytr, n_tr, y_mu, y_sd, ttr);
    KNN_HIP(hipGetLastError());

    // 3. network and initial weights (stream 0)
    knn_mlp *m = nullptr;
    KNN_TRY(knn_mlp_create(n_in, kH, &m));
    std::unique_ptr<knn_mlp, void (*)(knn_mlp *)> guard(m, knn_mlp_free);
    {
        std::vector<float> p(size_t(m->P), 0.f);
        const uint64_t s0 = splitmix_value(o.seed, 0);
        uint64_t c = 0;
        size_t at = 0;
        const int shapes[3][2] = {{kH, n_in}, {kH, kH}, {1, kH}};
        for (const auto &sh : shapes) {
            const double a = std::sqrt(6.0 / double(sh[1]));
            for (int64_t w = 0; w < int64_t(sh[0]) * sh[1]; ++w) {
                const double u = double(splitmix_value(s0, c++) >> 11) * 0x1p-53;
                p[at++] = float(-a + 2.0 * a * u);
            }
            at += size_t(sh[0]);  // biases stay 0
        }
        KNN_TRY(knn_mlp_set_params(m, p.data(), m->P));
        KNN_TRY(knn_mlp_set_norm(m, mu.data(), isd.data(), float(y_mu), float(y_sd)));
    }

    // 4. epochs (stream 2 + e)
    int64_t step = 0;
    std::vector<int64_t> per_epoch(static_cast<size_t>(o.epochs));
    for (int e = 0; e < o.epochs; ++e) {
        const std::vector<int32_t> order = key_order(splitmix_value(o.seed, 2 + uint64_t(e)), n_tr);
        KNN_HIP(hipMemcpyAsync(ord, order.data(), size_t(n_tr) * 4, hipMemcpyHostToDevice, s));
        int64_t nb = 0;
        for (int64_t b0 = 0; b0 < n_tr; b0 += bmax, ++nb, ++step) {
            const int64_t bn = std::min(bmax, n_tr - b0);
            k_train_gather<<<blocks(bn), T, 0, s>>>(xtr, ttr, ord + b0, bn, n_in, xb, tb);
            KNN_HIP(hipGetLastError());
            KNN_TRY(launch_loss_grad(m, xb, tb, bn, s));
            KNN_HIP(hipMemcpyAsync(hist + step, m->lossbuf, sizeof(float), hipMemcpyDeviceToDevice, s));
            KNN_TRY(launch_adam(m, o.lr, 0.9f, 0.999f, 1e-8f, s));
        }
        per_epoch[size_t(e)] = nb;
        // the host copy of this epoch's order must outlive its upload
        KNN_HIP(hipStreamSynchronize(s));
    }

    // 5. calibration on the held-out rows
    const size_t lds = size_t(m->P) * sizeof(float);
    k_mlp_forward<<<blocks(n_val), T, lds, s>>>(dev_of(m), xva, n_val, pred);
    KNN_HIP(hipGetLastError());
    std::vector<float> ph(static_cast<size_t>(n_val)), yh(static_cast<size_t>(n_val)),
        hh(static_cast<size_t>(steps));
    KNN_HIP(hipMemcpyAsync(ph.data(), pred, size_t(n_val) * 4, hipMemcpyDeviceToHost, s));
    KNN_HIP(hipMemcpyAsync(yh.data(), yva, size_t(n_val) * 4, hipMemcpyDeviceToHost, s));
    KNN_HIP(hipMemcpyAsync(hh.data(), hist, size_t(steps) * 4, hipMemcpyDeviceToHost, s));
    KNN_HIP(hipStreamSynchronize(s));
    std::vector<double> r(static_cast<size_t>(n_val));
    for (int64_t i = 0; i < n_val; ++i) r[size_t(i)] = double(yh[size_t(i)]) - (double(ph[size_t(i)]) * y_sd + y_mu);
    std::sort(r.begin(), r.end());
    const double h = double(n_val - 1) * (1.0 - double(o.target_fallback));
    const int64_t lo = std::min<int64_t>(int64_t(std::floor(h)), n_val - 1);
    const int64_t hi = std::min<int64_t>(lo + 1, n_val - 1);
    const double margin = r[size_t(lo)] + (h - double(lo)) * (r[size_t(hi)] - r[size_t(lo)]);
    if (!std::isfinite(margin)) return fail(KNN_E_DEVICE, "knn_seed_train: non-finite margin (training diverged)");
    if (loss_out) {
        int64_t at = 0;
        for (int e = 0; e < o.epochs; ++e) {
            double acc = 0.0;
            for (int64_t b = 0; b < per_epoch[size_t(e)]; ++b) acc += double(hh[size_t(at++)]);
            loss_out[e] = float(acc / double(per_epoch[size_t(e)]));
        }
    }
    *log_margin_out = float(margin);
    *out = guard.release();
    return KNN_OK;
}


}  // extern "C"
