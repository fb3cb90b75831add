// Exclusive prefix sums of int64 values (range-search offsets, the
// compaction of spanning-tree edges): one pass of workgroup-local scans,
// one workgroup scanning the block totals, one pass adding them.
#include "search.hpp"

namespace knnx {
namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;                          // per thread
constexpr int kScanBlock = kScanThreads * kScanItems;  // per workgroup

// inclusive scan of one workgroup's values (one per thread) in LDS
__device__ int64_t block_inclusive(int64_t v, int64_t *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int64_t u = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += u;
        __syncthreads();
    }
    return sh[t];
}

// out[i + 1] = sum of in[block start .. i] (within the block); tops[b] = the
// block's total
__global__ __launch_bounds__(kScanThreads) void k_scan_local(const int64_t *__restrict__ in,
                                                             int64_t n, int64_t *__restrict__ out,
                                                             int64_t *__restrict__ tops) {
    __shared__ int64_t sh[kScanThreads];
    const int64_t b0 = int64_t(blockIdx.x) * kScanBlock + int64_t(threadIdx.x) * kScanItems;
    int64_t v[kScanItems], s = 0;
#pragma unroll
    for (int e = 0; e < kScanItems; ++e) {
        v[e] = b0 + e < n ? in[b0 + e] : 0;
        s += v[e];
    }
    int64_t run = block_inclusive(s, sh) - s;
#pragma unroll
    for (int e = 0; e < kScanItems; ++e) {
        run += v[e];
        if (b0 + e < n) out[b0 + e + 1] = run;
    }
    if (threadIdx.x == kScanThreads - 1) tops[blockIdx.x] = sh[kScanThreads - 1];
}

// exclusive scan of the block totals (one workgroup: at most kScanBlock)
__global__ __launch_bounds__(kScanThreads) void k_scan_tops(int64_t *__restrict__ tops, int nb,
                                                            int64_t *__restrict__ out) {
    __shared__ int64_t sh[kScanThreads];
    const int b0 = threadIdx.x * kScanItems;
    int64_t v[kScanItems], s = 0;
#pragma unroll
    for (int e = 0; e < kScanItems; ++e) {
        v[e] = b0 + e < nb ? tops[b0 + e] : 0;
        s += v[e];
    }
    int64_t run = block_inclusive(s, sh) - s;
#pragma unroll
    for (int e = 0; e < kScanItems; ++e) {
        if (b0 + e < nb) tops[b0 + e] = run;
        run += v[e];
    }
    if (threadIdx.x == 0) out[0] = 0;
}

__global__ void k_scan_add(int64_t *__restrict__ out, int64_t n, const int64_t *__restrict__ tops) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i + 1] += tops[i / kScanBlock];
}

}  // namespace

int64_t scan_scratch(int64_t n) { return (n + kScanBlock - 1) / kScanBlock; }

hipError_t exclusive_scan(const int64_t *in, int64_t n, int64_t *out, int64_t *tops,
                          hipStream_t s) {
    if (n < 1 || n > kScanMax) return hipErrorInvalidValue;
    const int nb = int(scan_scratch(n));
    k_scan_local<<<nb, kScanThreads, 0, s>>>(in, n, out, tops);
    k_scan_tops<<<1, kScanThreads, 0, s>>>(tops, nb, out);
    k_scan_add<<<int((n + 255) / 256), 256, 0, s>>>(out, n, tops);
    return hipGetLastError();
}

}  // namespace knnx
