// Instantiation of the BF16 MFMA kernel for stride 64 (leaf sweep form), and
// the reference-side operands of its wave-independent form.
#include "search_mfma_sweep.hpp"

namespace knnx {

namespace {

// One workgroup per block of 32 reference leaves (the subtree whose leaves
// the sweep scores together), four leaves at a time: thread t of a leaf's
// 256 takes row t / 8, dimensions 8 (t % 8) .. + 7 (chunk c = 2 s + h of the
// operand layout), so that reads and writes are whole 16-byte pieces.
// Everything is centred on the block's box centre C_B = (lo + hi) / 2 of the
// block's subtree node, the same FP32 value the search reads back from bcen.
// Norms are FP32 sums of the FP32 differences in a fixed order (chunk, then
// a lane tree): the tile margin counts that error.
constexpr int kMebSteps = 32;  // enclosing-ball steps per leaf

template <int DP>
__global__ __launch_bounds__(1024) void k_wsweep_prep(const SearchArgs a, uint16_t *__restrict__ abf,
                                                      float *__restrict__ rn, float *__restrict__ rlen,
                                                      uint16_t *__restrict__ cbf, float *__restrict__ cn,
                                                      float *__restrict__ lam, float *__restrict__ bcen,
                                                      float *__restrict__ rcb) {
    static_assert(DP == 64, "the operand layout below assumes 64 dimensions (8 chunks of 8)");
    constexpr int NB = kSweepBlock;
    constexpr float kInf = __builtin_inff();
    __shared__ float s_cb[DP];
    // per leaf slot: its rows (padded by 4 floats: a lane per row reads
    // them without bank conflicts)
    __shared__ __align__(16) float s_rows[4][32][DP + 4];
    __shared__ __align__(16) float s_c[4][DP];         // per leaf slot: the ball's centre
    __shared__ uint32_t s_rmax[4];  // per leaf slot: largest row norm (bits)
    __shared__ uint32_t s_max;      // the block: largest centre norm (bits)
    const int rb = blockIdx.x;
    const int tid = threadIdx.x;
    const int ls = tid >> 8, t = tid & 255;
    const int i = t >> 3, c = t & 7, h = c & 1, s = c >> 1;
    const int nl = a.r_first_leaf + 1;
    const int n_blocks = (nl + NB - 1) / NB;
    const int bnode = n_blocks - 1 + rb;  // heap index of the block's subtree node
    if (tid < DP) {
        const float *bx = a.rbox + int64_t(bnode) * 2 * DP;
        const float cc = 0.5f * (bx[tid] + bx[DP + tid]);
        s_cb[tid] = cc;
        bcen[int64_t(rb) * DP + tid] = cc;
    }
    if (tid < 4) s_rmax[tid] = 0u;
    if (tid == 0) s_max = 0u;
    __syncthreads();
    for (int l0 = 0; l0 < NB; l0 += 4) {
        const int L = rb * NB + l0 + ls;
        const bool leaf_ok = L < nl;
        const int node = a.r_first_leaf + (leaf_ok ? L : 0);
        const int cnt = leaf_ok ? a.rrange[node].y : 0;
        const bool vr = i < cnt;
        // row i, dimensions 8c .. 8c+7: -2 (r - C_B) in BF16 (one 16-byte store)
        {
            const float4 *src = reinterpret_cast<const float4 *>(
                a.rlpts + (int64_t(leaf_ok ? L : 0) * a.r_leaf_slots + (vr ? i : 0)) * DP + 8 * c);
            const float4 x0 = src[0], x1 = src[1];
            const float xv[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
            bf16x8_t out;
            float n2 = 0.f;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float df = vr ? xv[e] - s_cb[8 * c + e] : 0.f;
                n2 = fmaf(df, df, n2);
                out[e] = (__bf16)(-2.0f * df);
            }
            *reinterpret_cast<bf16x8_t *>(abf + (int64_t(L) * NB + i) * DP + h * (DP / 2) + s * 8) = out;
            n2 = reduce8(n2, OpAdd());  // the row's whole norm, in all 8 lanes
            if (c == 0) {
                rn[int64_t(L) * NB + i] = vr ? n2 : kInf;
                // non-negative floats order as unsigned integers
                if (vr) atomicMax(&s_rmax[ls], __float_as_uint(n2));
            }
        }
        // the leaf's ball for the block Score, a small enclosing ball: from
        // the box centre, steps of Badoiu and Clarkson (move the centre 1/(i+1)
        // of the way to the farthest point), keeping the centre whose largest
        // distance was smallest; the radius is that largest distance (FP32,
        // rounded up by 2^-12: far above the sum's rounding).  Then C_L - C_B.
        // The slot's first wave: lane = dimension, or lane = row for the
        // distances.
        if (t < DP) {
            const bool has = leaf_ok && cnt > 0;
            const float *bx = a.rbox + int64_t(node) * 2 * DP;
            const float *rows = a.rlpts + int64_t(leaf_ok ? L : 0) * a.r_leaf_slots * DP;
            for (int r = 0; r < cnt; ++r) s_rows[ls][r][t] = rows[r * DP + t];
            float cl = has ? 0.5f * (bx[t] + bx[DP + t]) : 0.f;
            float best_c = cl, best_r2 = kInf;
            for (int it = 0; it < kMebSteps && has; ++it) {
                s_c[ls][t] = cl;
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
                // lane r < cnt: squared distance of row r to the centre
                float d2 = -1.0f;
                if (t < cnt) {
                    d2 = 0.f;
#pragma unroll 4
                    for (int u = 0; u < DP; u += 4) {
                        const float4 x = *reinterpret_cast<const float4 *>(&s_rows[ls][t][u]);
                        const float4 cc = *reinterpret_cast<const float4 *>(&s_c[ls][u]);
                        const float g0 = x.x - cc.x, g1 = x.y - cc.y, g2 = x.z - cc.z, g3 = x.w - cc.w;
                        d2 = fmaf(g0, g0, d2);
                        d2 = fmaf(g1, g1, d2);
                        d2 = fmaf(g2, g2, d2);
                        d2 = fmaf(g3, g3, d2);
                    }
                }
                const float m = __builtin_bit_cast(
                    float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, reduce64(d2, OpMax()))));
                if (m < best_r2) {
                    best_r2 = m;
                    best_c = cl;
                }
                const int f = __builtin_ctzll(ballot(d2 == m));
                // (any centre is valid: the step needs no exact division)
                cl += (s_rows[ls][f][t] - cl) * __builtin_amdgcn_rcpf(float(it + 2));
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            }
            const float df = has ? best_c - s_cb[t] : 0.f;
            const int ps = t >> 4, ph = (t >> 3) & 1, pe = t & 7;
            cbf[int64_t(L) * DP + ph * (DP / 2) + ps * 8 + pe] =
                __builtin_bit_cast(uint16_t, (__bf16)(-2.0f * df));
            const float c2 = reduce64(df * df, OpAdd());
            if (t == 0) {
                cn[L] = has ? c2 : kInf;
                lam[L] = has ? __builtin_amdgcn_sqrtf(best_r2) * (1.0f + 0x1p-12f) : 0.f;
                if (has) atomicMax(&s_max, __float_as_uint(c2));
            }
        }
        __syncthreads();
        if (t == 0) {
            rlen[L] = __builtin_amdgcn_sqrtf(__uint_as_float(s_rmax[ls])) * (1.0f + 0x1p-20f);
            s_rmax[ls] = 0u;
        }
        __syncthreads();
    }
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
