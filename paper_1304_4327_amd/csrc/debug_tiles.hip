// Export of the BF16 distance tile (bf16_tile.hpp) for tests: the values the
// matrix-core kernels filter on and the margin they subtract, for tiles the
// caller chooses, so that the error bound can be checked on every pair.
#include "bf16_tile.hpp"

#include <string>

namespace knnx {
namespace {

// One wavefront per tile: 32 query rows, 32 reference rows, one centre.
// The rows are staged into LDS with the stride the search kernels use (DP,
// zero padding past d); operands, product, row norms and margin then come
// from the same helpers as the search kernels.
template <int DP>
__global__ __launch_bounds__(64) void k_debug_bf16_tiles(const float *__restrict__ q,
                                                         const float *__restrict__ r,
                                                         const float *__restrict__ cen,
                                                         int d, float *__restrict__ acc_out,
                                                         float *__restrict__ qn_out,
                                                         float *__restrict__ marg_out) {
    __shared__ __align__(16) float s_q[32 * DP];
    __shared__ __align__(16) float s_r[32 * DP];
    __shared__ __align__(16) float s_c[DP];
    __shared__ __align__(16) float s_rn[32];
    const int t = blockIdx.x;
    const int lane = threadIdx.x;
    const float *qt = q + int64_t(t) * 32 * d;
    const float *rt = r + int64_t(t) * 32 * d;
    for (int e = lane; e < 32 * DP; e += 64) {
        const int row = e / DP, dim = e % DP;
        s_q[e] = dim < d ? qt[row * d + dim] : 0.f;
        s_r[e] = dim < d ? rt[row * d + dim] : 0.f;
    }
    for (int e = lane; e < DP; e += 64) s_c[e] = e < d ? cen[int64_t(t) * d + e] : 0.f;
    __syncthreads();
    const int j = lane & 31, h = lane >> 5;
    bf16x8_t bq[DP / 16], ar[DP / 16];
    float qn = bf16_query_operand<DP>(s_q + j * DP, s_c, h, true, bq);
    qn = xor32_op(qn, OpAdd());
    float rn = bf16_ref_operand<DP>(s_r + j * DP, s_c, h, true, ar);
    rn = xor32_op(rn, OpAdd());
    const float rlen = bf16_tile_rlen(rn, true);
    if (h == 0) s_rn[j] = rn;
    __syncthreads();
    f32x16_t acc;
#pragma unroll
    for (int g4 = 0; g4 < 4; ++g4) {
        const float4 v = *reinterpret_cast<const float4 *>(&s_rn[g4 * 8 + h * 4]);
        acc[g4 * 4 + 0] = v.x;
        acc[g4 * 4 + 1] = v.y;
        acc[g4 * 4 + 2] = v.z;
        acc[g4 * 4 + 3] = v.w;
    }
    acc = bf16_tile_product<DP>(ar, bq, acc);
    float *ao = acc_out + int64_t(t) * 32 * 32;
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
        const int row = 8 * (rr / 4) + 4 * h + (rr % 4);
        ao[row * 32 + j] = acc[rr];
    }
    if (h == 0) {
        qn_out[int64_t(t) * 32 + j] = qn;
        marg_out[int64_t(t) * 32 + j] = bf16_margin<DP>(sqrtf(qn), rlen);
    }
}

template <int DP>
hipError_t launch(const float *q, const float *r, const float *c, int64_t n, int d, float *acc,
                  float *qn, float *marg, hipStream_t s) {
    k_debug_bf16_tiles<DP><<<int(n), 64, 0, s>>>(q, r, c, d, acc, qn, marg);
    return hipGetLastError();
}

}  // namespace
}  // namespace knnx

using namespace knnx;

extern "C" knn_status knn_debug_bf16_tiles(const float *q, const float *r, const float *centre,
                                           int64_t n_tiles, int32_t d, float *acc_out,
                                           float *qnorm_out, float *margin_out, void *stream) {
    set_error("");
    if (!q || !r || !centre || !acc_out || !qnorm_out || !margin_out)
        return fail(KNN_E_INVALID_ARG, "knn_debug_bf16_tiles: NULL pointer");
    if (n_tiles < 1 || n_tiles > (int64_t(1) << 24))
        return fail(KNN_E_INVALID_ARG, "knn_debug_bf16_tiles: need 1 <= n_tiles <= 2^24");
    if (d < 9 || d > 64)
        return fail(KNN_E_INVALID_ARG, "knn_debug_bf16_tiles: need 9 <= d <= 64");
    hipStream_t s = (hipStream_t)stream;
    const int dp = pad_dim(d);
    hipError_t e = dp == 16   ? launch<16>(q, r, centre, n_tiles, d, acc_out, qnorm_out, margin_out, s)
                   : dp == 32 ? launch<32>(q, r, centre, n_tiles, d, acc_out, qnorm_out, margin_out, s)
                              : launch<64>(q, r, centre, n_tiles, d, acc_out, qnorm_out, margin_out, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "knn_debug_bf16_tiles", __FILE__, __LINE__);
    return KNN_OK;
}
