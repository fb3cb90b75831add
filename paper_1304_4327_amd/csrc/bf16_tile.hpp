// The BF16 distance tile of the matrix-core kernels: operand construction,
// the MFMA product and the proven error margin, shared by the per-leaf
// kernel (search_mfma.hpp), the leaf sweep (search_mfma_sweep.hpp) and the
// tile export that tests the margin (debug_tiles.hip).
//
// A tile is the 32 x 32 block D[i][j] = ||r_i'||^2 - 2 <r_i', q_j'> of the
// BaseCase distances (Algorithm 2) of 32 reference rows i and 32 queries j,
// with x' = x - c for a centre c (a query box centre), so that the squared
// distance estimate is D[i][j] + ||q_j'||^2.  v_mfma_f32_32x32x16_bf16
// computes it over DP/16 k-steps of 16 dimensions.  Operand layout (gfx950):
// lane l holds A[i = l%32][k = 8h .. 8h+7] and B[k = 8h .. 8h+7][j = l%32]
// with h = l/32; output register r of lane l is
// D[8(r/4) + 4h + r%4][l%32].  The accumulator starts at ||r_i'||^2 (FP32)
// and the query operand is -2 q' (an exact scaling in BF16).
//
// Error bound.  With u_b = 2^-8 (BF16 round to nearest) and u = 2^-24,
//   |D + ||q'||^2 - ||q - r||^2| <= 2 (2 u_b + u_b^2) |q'| |r'|
//                                   + (DP + 8) u (|q'| + |r'|)^2 :
// products of BF16 values are exact in FP32, the rounding of both operands
// gives the first term, the FP32 centring, norms and accumulation the
// second.  The margin takes |r'| <= R, the largest row of the tile, and
// multiplies the bound by 1.25 against unspecified rounding inside the
// matrix unit.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace knnx {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

template <int DP>
struct Bf16Margin {
    static constexpr float ub = 0x1p-8f;
    static constexpr float C1 = 1.25f * 2.0f * (2.0f * ub + ub * ub);
    static constexpr float C2 = 1.25f * (DP + 8) * 0x1p-24f;
};

// margin M(q, tile) for |q'| = qlen and the tile's largest |r'| <= rlen
template <int DP>
__device__ __forceinline__ float bf16_margin(float qlen, float rlen) {
    return Bf16Margin<DP>::C1 * qlen * rlen +
           Bf16Margin<DP>::C2 * (qlen + rlen) * (qlen + rlen);
}

// This lane's query operand: -2 (q - c) in BF16 over dimensions
// 16 s + 8 h .. + 7 of each k-step s; returns the lane's part of |q - c|^2
// (the two halves of a query sum to the whole).  qrow and cen are DP-strided
// and 16-byte aligned; invalid lanes contribute zeros.
template <int DP>
__device__ __forceinline__ float bf16_query_operand(const float *qrow, const float *cen, int h,
                                                    bool valid, bf16x8_t (&bq)[DP / 16]) {
    float qn = 0.f;
#pragma unroll
    for (int s = 0; s < DP / 16; ++s) {
        const float4 *cp = reinterpret_cast<const float4 *>(cen + s * 16 + h * 8);
        const float4 *xp = reinterpret_cast<const float4 *>(qrow + s * 16 + h * 8);
        const float4 c0 = cp[0], c1 = cp[1], x0 = xp[0], x1 = xp[1];
        const float cv[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
        const float xv[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float qd = valid ? xv[e] - cv[e] : 0.f;
            qn = fmaf(qd, qd, qn);
            bq[s][e] = (__bf16)(-2.0f * qd);
        }
    }
    return qn;
}

// This lane's reference operand (row i = lane % 32): (r - c) in BF16;
// returns the lane's part of |r - c|^2.  Invalid rows contribute zeros.
template <int DP>
__device__ __forceinline__ float bf16_ref_operand(const float *rrow, const float *cen, int h,
                                                  bool valid, bf16x8_t (&ar)[DP / 16]) {
    float rn = 0.f;
#pragma unroll
    for (int s = 0; s < DP / 16; ++s) {
        const float4 *src = reinterpret_cast<const float4 *>(rrow + s * 16 + h * 8);
        const float4 *cp = reinterpret_cast<const float4 *>(cen + s * 16 + h * 8);
        const float4 v0 = src[0], v1 = src[1], c0 = cp[0], c1 = cp[1];
        const float rv[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
        const float cv[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float rd = valid ? rv[e] - cv[e] : 0.f;
            rn = fmaf(rd, rd, rn);
            ar[s][e] = (__bf16)rd;
        }
    }
    return rn;
}

// The same two operands with the centre held in registers: tc[8 s + e] is
// the centre at dimension 16 s + 8 h + e of this lane's half h.
template <int DP>
__device__ __forceinline__ float bf16_query_operand_r(const float *qrow, const float (&tc)[DP / 2], int h,
                                                      bool valid, bf16x8_t (&bq)[DP / 16]) {
    float qn = 0.f;
#pragma unroll
    for (int s = 0; s < DP / 16; ++s) {
        const float4 *xp = reinterpret_cast<const float4 *>(qrow + s * 16 + h * 8);
        const float4 x0 = xp[0], x1 = xp[1];
        const float xv[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float qd = valid ? xv[e] - tc[s * 8 + e] : 0.f;
            qn = fmaf(qd, qd, qn);
            bq[s][e] = (__bf16)(-2.0f * qd);
        }
    }
    return qn;
}
template <int DP>
__device__ __forceinline__ float bf16_ref_operand_r(const float *rrow, const float (&tc)[DP / 2], int h,
                                                    bool valid, bf16x8_t (&ar)[DP / 16]) {
    float rn = 0.f;
#pragma unroll
    for (int s = 0; s < DP / 16; ++s) {
        const float4 *src = reinterpret_cast<const float4 *>(rrow + s * 16 + h * 8);
        const float4 v0 = src[0], v1 = src[1];
        const float rv[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float rd = valid ? rv[e] - tc[s * 8 + e] : 0.f;
            rn = fmaf(rd, rd, rn);
            ar[s][e] = (__bf16)rd;
        }
    }
    return rn;
}

// The accumulators' initial values ||r_i'||^2 without leaving the lanes: a
// product of each row's norm split into three BF16 parts (their sum is the
// FP32 norm exactly: 3 x 8 significand bits) against ones.  rn is the full
// norm of row lane % 32 (+inf for rows past the tile: then the other parts
// are 0 and no product is 0 x inf); the result's register r of lane l holds
// the norm of row 8(r/4) + 4h + r%4, as the tile product expects.
__device__ __forceinline__ f32x16_t bf16_norm_init(float rn, bool vr, int h) {
    const float nr = vr ? rn : __builtin_inff();
    const __bf16 n0 = (__bf16)nr;
    const float r1 = vr ? rn - float(n0) : 0.f;
    const __bf16 n1 = (__bf16)r1;
    const __bf16 n2 = (__bf16)(r1 - float(n1));
    bf16x8_t an = {}, ones = {};
    if (h == 0) {
        an[0] = n0;
        an[1] = n1;
        an[2] = n2;
        ones[0] = ones[1] = ones[2] = (__bf16)1.0f;
    }
    const f32x16_t zero = {};
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(an, ones, zero, 0, 0, 0);
}

// Largest |r'| of a tile from each lane's full row norm rn (rows past the
// tile invalid): a DPP maximum over each 16 rows, then the two halves on the
// scalar unit (non-negative floats order as unsigned integers); hardware
// square root (1 ulp) nudged up, since the margin only needs an upper bound.
__device__ __forceinline__ float bf16_tile_rlen(float rn, bool vr) {
    const float r16 = reduce16(vr ? rn : 0.f, OpMax());
    const float rmax = __builtin_bit_cast(
        float, max((uint32_t)__builtin_amdgcn_readlane(__builtin_bit_cast(int, r16), 0),
                   (uint32_t)__builtin_amdgcn_readlane(__builtin_bit_cast(int, r16), 16)));
    const float u = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(rmax)));
    return __builtin_amdgcn_sqrtf(u) * (1.0f + 0x1p-20f);
}

// acc += A B over the DP/16 k-steps
template <int DP>
__device__ __forceinline__ f32x16_t bf16_tile_product(const bf16x8_t (&ar)[DP / 16],
                                                      const bf16x8_t (&bq)[DP / 16],
                                                      f32x16_t acc) {
#pragma unroll
    for (int s = 0; s < DP / 16; ++s)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[s], bq[s], acc, 0, 0, 0);
    return acc;
}

}  // namespace knnx
