// Instantiation of the BF16 MFMA kernel for stride 64 (leaf sweep form), and
// the reference-side operands of its wave-independent form.
#include "search_mfma_sweep.hpp"

namespace knnx {

namespace {

// One workgroup per block of 32 reference leaves (the subtree whose leaves
// the sweep scores together); thread (li, i) = row i of leaf 32 rb + li.
// Everything is centred on the block's box centre C_B = (lo + hi) / 2 of the
// block's subtree node, the same FP32 value the search reads back from bcen.
// The norms are FP32 sums of the FP32 differences (dimension order for rows,
// a fixed lane tree for leaf centres): the tile margin counts that error.
template <int DP>
__global__ __launch_bounds__(1024) void k_wsweep_prep(const SearchArgs a, uint16_t *__restrict__ abf,
                                                      float *__restrict__ rn, float *__restrict__ rlen,
                                                      uint16_t *__restrict__ cbf, float *__restrict__ cn,
                                                      float *__restrict__ lam, float *__restrict__ bcen,
                                                      float *__restrict__ rcb) {
    constexpr int NB = kSweepBlock;
    constexpr float kInf = __builtin_inff();
    __shared__ float s_cb[DP];
    __shared__ uint32_t s_max;
    const int rb = blockIdx.x;
    const int tid = threadIdx.x;
    const int li = tid >> 5, i = tid & 31;
    const int nl = a.r_first_leaf + 1;
    const int n_blocks = (nl + NB - 1) / NB;
    const int bnode = n_blocks - 1 + rb;  // heap index of the block's subtree node
    if (tid < DP) {
        const float *bx = a.rbox + int64_t(bnode) * 2 * DP;
        const float c = 0.5f * (bx[tid] + bx[DP + tid]);
        s_cb[tid] = c;
        bcen[int64_t(rb) * DP + tid] = c;
    }
    if (tid == 0) s_max = 0u;
    __syncthreads();
    const int L = rb * NB + li;
    const bool leaf_ok = L < nl;
    const int node = a.r_first_leaf + (leaf_ok ? L : 0);
    const int cnt = leaf_ok ? a.rrange[node].y : 0;
    const bool vr = i < cnt;
    // row i: -2 (r - C_B) in BF16 at [h][s][e] for dimension 16 s + 8 h + e
    {
        const float *row = a.rlpts + (int64_t(L < nl ? L : 0) * a.r_leaf_slots + (vr ? i : 0)) * DP;
        uint16_t *dst = abf + (int64_t(L) * NB + i) * DP;
        float n2 = 0.f;
#pragma unroll
        for (int dd = 0; dd < DP; ++dd) {
            const float df = vr ? row[dd] - s_cb[dd] : 0.f;
            n2 = fmaf(df, df, n2);
            const int s = dd >> 4, h = (dd >> 3) & 1, e = dd & 7;
            dst[h * (DP / 2) + s * 8 + e] = __builtin_bit_cast(uint16_t, (__bf16)(-2.0f * df));
        }
        rn[int64_t(L) * NB + i] = vr ? n2 : kInf;
        const float m = reduce32(vr ? n2 : 0.f, OpMax());
        if (i == 0) rlen[L] = __builtin_amdgcn_sqrtf(m) * (1.0f + 0x1p-20f);
    }
    // the leaf's box centre C_L - C_B: this thread's dimensions i and i + 32
    {
        const bool has = leaf_ok && cnt > 0;
        const float *bx = a.rbox + int64_t(node) * 2 * DP;
        float c2 = 0.f;
#pragma unroll
        for (int u = 0; u < DP / 32; ++u) {
            const int dd = i + 32 * u;
            const float df = has ? 0.5f * (bx[dd] + bx[DP + dd]) - s_cb[dd] : 0.f;
            c2 = fmaf(df, df, c2);
            const int s = dd >> 4, h = (dd >> 3) & 1, e = dd & 7;
            cbf[int64_t(L) * DP + h * (DP / 2) + s * 8 + e] = __builtin_bit_cast(uint16_t, (__bf16)(-2.0f * df));
        }
        c2 = reduce32(c2, OpAdd());
        if (i == 0) {
            cn[L] = has ? c2 : kInf;
            lam[L] = has ? a.rlam[node] : 0.f;
            // non-negative floats order as unsigned integers
            if (has) atomicMax(&s_max, __float_as_uint(c2));
        }
    }
    __syncthreads();
    if (tid == 0) rcb[rb] = __builtin_amdgcn_sqrtf(__uint_as_float(s_max)) * (1.0f + 0x1p-20f);
}

}  // namespace

hipError_t launch_search_mfma_dp64(const SearchArgs &a, int K, int grid, hipStream_t s) {
    return launch_search_mfma_sweep<64>(a, K, grid, s);
}

hipError_t launch_wsweep_prep(const SearchArgs &a, uint16_t *abf, float *rn, float *rlen, uint16_t *cbf,
                              float *cn, float *lam, float *bcen, float *rcb, hipStream_t s) {
    const int nl = a.r_first_leaf + 1;
    const int n_blocks = (nl + kSweepBlock - 1) / kSweepBlock;
    if (a.r_leaf_slots > 32) return hipErrorInvalidValue;
    k_wsweep_prep<64><<<n_blocks, 1024, 0, s>>>(a, abf, rn, rlen, cbf, cn, lam, bcen, rcb);
    return hipGetLastError();
}

}  // namespace knnx
