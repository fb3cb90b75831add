// kd-tree construction on the GPU (Section "Space Trees": Definition 1 and the
// kd-tree bounds paragraph; points live only in leaves, as in the discussion of
// Gray's AllNN).
//
// Split rule (the paper fixes none; this is the library's):
//   complete tree of depth L = smallest L with ceil(n / 2^L) <= leaf_size,
//   heap-ordered nodes; node ranges are data independent (left child gets
//   floor(c/2) of its parent's c points).  A node splits on the dimension of
//   largest FP32 box extent (ties -> lowest); its left child receives the
//   floor(c/2) smallest points under (coordinate, original index); both
//   children keep ascending original-index order (stable partition).
//
// Level-synchronous construction:
//   * levels whose segments exceed kLocalMax points run as grid-wide passes:
//     segmented box reduction, radix select (4 x 8-bit digits of an
//     order-preserving uint32 key) of the median key per segment, and a
//     stable partition by a segmented scan of (less, equal) counts;
//   * the remaining levels of every segment of <= kLocalMax points are built
//     by one wavefront in LDS (same select/partition, wave ballots instead of
//     block scans).
// Then the points are gathered into tree order (FP32, padded to dp), leaf
// boxes and lambda are computed exactly (FP64, rounded up), and internal
// lambda gets an upper bound from the children.
#include "common.hpp"

#include <algorithm>
#include <vector>

namespace knnx {
namespace {

constexpr int kLocalMax = 1024;  // segments this small finish in one wave
constexpr int kChunk = 4096;     // elements per block in grid-wide levels
constexpr int kBlock = 256;

struct Sel {
    uint32_t prefix, mask;
    int32_t rank, pad;
};

__device__ inline uint64_t lanemask_lt() {
    return (uint64_t(1) << (threadIdx.x & 63)) - 1;
}

__global__ void k_ranges(int2 *range, int n, int n_nodes) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    unsigned v = unsigned(i) + 1u;
    int depth = 31 - __clz(v);
    int start = 0, cnt = n;
    for (int l = depth - 1; l >= 0; --l) {
        int half = cnt >> 1;
        if ((v >> l) & 1u) {
            start += half;
            cnt -= half;
        } else {
            cnt = half;
        }
    }
    range[i] = make_int2(start, cnt);
}

__global__ void k_iota(int *a, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = i;
}

__global__ void k_fill_u32(uint32_t *a, int n, uint32_t lo_val, uint32_t hi_val, int dp) {
    // boxu layout: [seg][2][dp]; first half of each seg = lo (init lo_val)
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = ((i / dp) & 1) ? hi_val : lo_val;
}

// ---- grid-wide level: box ---------------------------------------------------
template <int DP>
__global__ __launch_bounds__(kBlock) void k_box_level(const float *__restrict__ P, int d,
                                                      const int *__restrict__ idx,
                                                      const int2 *__restrict__ range,
                                                      int node0, int bps,
                                                      uint32_t *__restrict__ boxu) {
    const int seg = blockIdx.x / bps, chunk = blockIdx.x % bps;
    const int2 r = range[node0 + seg];
    const int e0 = chunk * kChunk, e1 = min(r.y, e0 + kChunk);
    const int t = threadIdx.x, j = t % DP, grp = t / DP;
    constexpr int NG = kBlock / DP;
    uint32_t lo = 0xffffffffu, hi = 0u;
    if (j < d) {
        for (int e = e0 + grp; e < e1; e += NG) {
            uint32_t k = f2key(P[int64_t(idx[r.x + e]) * d + j]);
            lo = min(lo, k);
            hi = max(hi, k);
        }
    }
#pragma unroll
    for (int off = DP; off < 64; off <<= 1) {
        lo = min(lo, (uint32_t)__shfl_xor((int)lo, off));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, off));
    }
    __shared__ uint32_t slo[kBlock / 64][DP], shi[kBlock / 64][DP];
    const int w = t >> 6, lane = t & 63;
    if (lane < DP) {
        slo[w][lane] = lo;
        shi[w][lane] = hi;
    }
    __syncthreads();
    if (t < DP && t < d) {
        for (int q = 1; q < kBlock / 64; ++q) {
            lo = min(lo, slo[q][t]);
            hi = max(hi, shi[q][t]);
        }
        if (lo != 0xffffffffu) atomicMin(&boxu[(seg * 2) * DP + t], lo);
        if (hi != 0u) atomicMax(&boxu[(seg * 2 + 1) * DP + t], hi);
    }
}

template <int DP>
__global__ void k_box_finalize(const uint32_t *__restrict__ boxu, const int2 *__restrict__ range,
                               int node0, int nseg, int d, float *__restrict__ box,
                               int *__restrict__ split_dim, Sel *__restrict__ sel) {
    int seg = blockIdx.x * blockDim.x + threadIdx.x;
    if (seg >= nseg) return;
    const int node = node0 + seg;
    const int2 r = range[node];
    float *b = box + int64_t(node) * 2 * DP;
    int best = 0;
    float bestext = -1.0f;
    for (int j = 0; j < DP; ++j) {
        float lo = 0.f, hi = 0.f;
        if (j < d) {
            if (r.y > 0) {
                lo = key2f(boxu[(seg * 2) * DP + j]);
                hi = key2f(boxu[(seg * 2 + 1) * DP + j]);
                float ext = hi - lo;
                if (ext > bestext) {
                    bestext = ext;
                    best = j;
                }
            } else {
                lo = __builtin_inff();
                hi = -__builtin_inff();
            }
        }
        b[j] = lo;
        b[DP + j] = hi;
    }
    split_dim[node] = best;
    sel[seg] = Sel{0u, 0u, r.y / 2, 0};
}

// ---- grid-wide level: radix select of the median key ----------------------
template <int DP>
__global__ __launch_bounds__(kBlock) void k_hist(const float *__restrict__ P, int d,
                                                 const int *__restrict__ idx,
                                                 const int2 *__restrict__ range, int node0,
                                                 int bps, const int *__restrict__ split_dim,
                                                 uint32_t *__restrict__ keys,
                                                 const Sel *__restrict__ sel,
                                                 int *__restrict__ hist, int pass) {
    const int seg = blockIdx.x / bps, chunk = blockIdx.x % bps;
    const int node = node0 + seg;
    const int2 r = range[node];
    const int e0 = chunk * kChunk, e1 = min(r.y, e0 + kChunk);
    const int j = split_dim[node];
    const Sel s = sel[seg];
    const int shift = 24 - 8 * pass;
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    for (int e = e0 + threadIdx.x; e < e1; e += kBlock) {
        uint32_t key;
        if (pass == 0) {
            key = f2key(P[int64_t(idx[r.x + e]) * d + j]);
            keys[r.x + e] = key;
        } else {
            key = keys[r.x + e];
        }
        if ((key & s.mask) == s.prefix) atomicAdd(&h[(key >> shift) & 255u], 1);
    }
    __syncthreads();
    int c = h[threadIdx.x];
    if (c) atomicAdd(&hist[seg * 256 + threadIdx.x], c);
}

// one wave per segment: pick the digit holding the wanted rank
__global__ __launch_bounds__(64) void k_select(int *__restrict__ hist, Sel *__restrict__ sel,
                                               const int2 *__restrict__ range, int node0,
                                               int pass) {
    const int seg = blockIdx.x, lane = threadIdx.x;
    const int shift = 24 - 8 * pass;
    int *h = hist + seg * 256;
    int h0 = h[lane * 4 + 0], h1 = h[lane * 4 + 1], h2 = h[lane * 4 + 2], h3 = h[lane * 4 + 3];
    int s = h0 + h1 + h2 + h3;
    int incl = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    const int excl = incl - s;
    Sel st = sel[seg];
    const bool live = range[node0 + seg].y > 0;
    const bool mine = live && excl <= st.rank && st.rank < incl;
    if (mine) {
        int rem = st.rank - excl, bin = lane * 4;
        if (rem >= h0) {
            rem -= h0;
            ++bin;
            if (rem >= h1) {
                rem -= h1;
                ++bin;
                if (rem >= h2) {
                    rem -= h2;
                    ++bin;
                }
            }
        }
        st.prefix |= uint32_t(bin) << shift;
        st.mask |= 255u << shift;
        st.rank = rem;
        sel[seg] = st;
    }
    h[lane * 4 + 0] = 0;
    h[lane * 4 + 1] = 0;
    h[lane * 4 + 2] = 0;
    h[lane * 4 + 3] = 0;
}

// ---- grid-wide level: stable partition ---------------------------------------
__global__ __launch_bounds__(kBlock) void k_part_count(const uint32_t *__restrict__ keys,
                                                       const int2 *__restrict__ range,
                                                       int node0, int bps,
                                                       const Sel *__restrict__ sel,
                                                       int2 *__restrict__ counts) {
    const int seg = blockIdx.x / bps, chunk = blockIdx.x % bps;
    const int2 r = range[node0 + seg];
    const int e0 = chunk * kChunk, e1 = min(r.y, e0 + kChunk);
    const uint32_t v = sel[seg].prefix;
    int nl = 0, ne = 0;
    for (int e = e0 + threadIdx.x; e < e1; e += kBlock) {
        uint32_t key = keys[r.x + e];
        nl += key < v;
        ne += key == v;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        nl += __shfl_xor(nl, off);
        ne += __shfl_xor(ne, off);
    }
    __shared__ int sl[kBlock / 64], se[kBlock / 64];
    if ((threadIdx.x & 63) == 0) {
        sl[threadIdx.x >> 6] = nl;
        se[threadIdx.x >> 6] = ne;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = 0, b = 0;
        for (int q = 0; q < kBlock / 64; ++q) {
            a += sl[q];
            b += se[q];
        }
        counts[blockIdx.x] = make_int2(a, b);
    }
}

__global__ void k_part_scan(int2 *counts, int nseg, int bps) {
    int seg = blockIdx.x * blockDim.x + threadIdx.x;
    if (seg >= nseg) return;
    int a = 0, b = 0;
    for (int c = 0; c < bps; ++c) {
        int2 v = counts[seg * bps + c];
        counts[seg * bps + c] = make_int2(a, b);
        a += v.x;
        b += v.y;
    }
}

__global__ __launch_bounds__(kBlock) void k_part_scatter(const uint32_t *__restrict__ keys,
                                                         const int *__restrict__ idx_in,
                                                         int *__restrict__ idx_out,
                                                         const int2 *__restrict__ range,
                                                         int node0, int bps,
                                                         const Sel *__restrict__ sel,
                                                         const int2 *__restrict__ counts,
                                                         int *__restrict__ err) {
    const int seg = blockIdx.x / bps, chunk = blockIdx.x % bps;
    const int2 r = range[node0 + seg];
    const int e0 = chunk * kChunk, e1 = min(r.y, e0 + kChunk);
    const Sel s = sel[seg];
    const uint32_t v = s.prefix;
    const int req = s.rank;  // equal keys that go left
    const int m = r.y / 2;
    const int2 off = counts[blockIdx.x];
    const int w = threadIdx.x >> 6;
    __shared__ int wl[kBlock / 64], we[kBlock / 64];
    int run_l = off.x, run_e = off.y;
    for (int base = e0; base < e1; base += kBlock) {
        const int e = base + threadIdx.x;
        const bool valid = e < e1;
        const uint32_t key = valid ? keys[r.x + e] : 0u;
        const bool less = valid && key < v, eq = valid && key == v;
        const uint64_t bl = __ballot(less), be = __ballot(eq);
        const int pl = __popcll(bl & lanemask_lt()), pe = __popcll(be & lanemask_lt());
        if ((threadIdx.x & 63) == 0) {
            wl[w] = __popcll(bl);
            we[w] = __popcll(be);
        }
        __syncthreads();
        int ol = 0, oe = 0, tl = 0, te = 0;
        for (int q = 0; q < kBlock / 64; ++q) {
            if (q < w) {
                ol += wl[q];
                oe += we[q];
            }
            tl += wl[q];
            te += we[q];
        }
        __syncthreads();
        if (valid) {
            const int less_before = run_l + ol + pl;
            const int eq_before = run_e + oe + pe;
            const bool left = less || (eq && eq_before < req);
            const int left_before = less_before + min(eq_before, req);
            int pos = left ? left_before : m + (e - left_before);
            if (pos < 0 || pos >= r.y) {  // cannot happen for a correct select
                atomicOr(err, 2);
                pos = min(max(pos, 0), r.y - 1);
            }
            idx_out[r.x + pos] = idx_in[r.x + e];
        }
        run_l += tl;
        run_e += te;
    }
}

// ---- one wave finishes a segment's subtree in LDS -------------------------
template <int DP>
__global__ __launch_bounds__(64) void k_local_build(const float *__restrict__ P, int d,
                                                    int *__restrict__ idx,
                                                    const int2 *__restrict__ range, int l0,
                                                    int L, float *__restrict__ box,
                                                    int *__restrict__ split_dim,
                                                    int *__restrict__ err) {
    const int seg = blockIdx.x, lane = threadIdx.x;
    const int2 rr = range[(1 << l0) - 1 + seg];
    const int base = rr.x, c = rr.y;
    __shared__ int sidx[2][kLocalMax];
    __shared__ uint32_t skey[kLocalMax];
    __shared__ int hist[256];
    for (int e = lane; e < c; e += 64) sidx[0][e] = idx[base + e];
    __syncthreads();
    int cur = 0;
    const int j_l = lane % DP, grp = lane / DP;
    constexpr int NG = 64 / DP;
    for (int lv = l0; lv < L; ++lv) {
        const int nsub = 1 << (lv - l0);
        for (int sub = 0; sub < nsub; ++sub) {
            const int node = (1 << lv) - 1 + seg * nsub + sub;
            const int2 nr = range[node];
            const int o = nr.x - base, cc = nr.y;
            const int *src = sidx[cur] + o;
            // box over the node's points
            uint32_t lo = 0xffffffffu, hi = 0u;
            if (j_l < d) {
                for (int e = grp; e < cc; e += NG) {
                    uint32_t k = f2key(P[int64_t(src[e]) * d + j_l]);
                    lo = min(lo, k);
                    hi = max(hi, k);
                }
            }
#pragma unroll
            for (int off = DP; off < 64; off <<= 1) {
                lo = min(lo, (uint32_t)__shfl_xor((int)lo, off));
                hi = max(hi, (uint32_t)__shfl_xor((int)hi, off));
            }
            float flo = 0.f, fhi = 0.f, ext = -1.0f;
            if (lane < d) {
                if (cc > 0) {
                    flo = key2f(lo);
                    fhi = key2f(hi);
                    ext = fhi - flo;
                } else {
                    flo = __builtin_inff();
                    fhi = -__builtin_inff();
                }
            }
            if (lane < DP) {
                box[int64_t(node) * 2 * DP + lane] = flo;
                box[int64_t(node) * 2 * DP + DP + lane] = fhi;
            }
            // widest dimension, lowest on ties
            float mx = ext;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
            const uint64_t cand = __ballot(lane < d && ext == mx);
            const int jsplit = cand ? (__ffsll((unsigned long long)cand) - 1) : 0;
            if (lane == 0) split_dim[node] = jsplit;
            // keys
            for (int e = lane; e < cc; e += 64) skey[o + e] = f2key(P[int64_t(src[e]) * d + jsplit]);
            __syncthreads();
            // radix select of the key at rank floor(cc/2)
            const int m = cc / 2;
            uint32_t prefix = 0u, mask = 0u;
            int rank = m;
            for (int pass = 0; pass < 4; ++pass) {
                const int shift = 24 - 8 * pass;
                hist[lane * 4 + 0] = 0;
                hist[lane * 4 + 1] = 0;
                hist[lane * 4 + 2] = 0;
                hist[lane * 4 + 3] = 0;
                __syncthreads();
                for (int e = lane; e < cc; e += 64) {
                    uint32_t key = skey[o + e];
                    if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1);
                }
                __syncthreads();
                const int h0 = hist[lane * 4 + 0], h1 = hist[lane * 4 + 1];
                const int h2 = hist[lane * 4 + 2], h3 = hist[lane * 4 + 3];
                const int sum = h0 + h1 + h2 + h3;
                int incl = sum;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    int v = __shfl_up(incl, off);
                    if (lane >= off) incl += v;
                }
                const int excl = incl - sum;
                const bool mine = cc > 0 && excl <= rank && rank < incl;
                int bin = 0, rem = 0;
                if (mine) {
                    rem = rank - excl;
                    bin = lane * 4;
                    if (rem >= h0) {
                        rem -= h0;
                        ++bin;
                        if (rem >= h1) {
                            rem -= h1;
                            ++bin;
                            if (rem >= h2) {
                                rem -= h2;
                                ++bin;
                            }
                        }
                    }
                }
                const uint64_t who = __ballot(mine);
                const int owner = who ? (__ffsll((unsigned long long)who) - 1) : 0;
                bin = __shfl(bin, owner);
                rem = __shfl(rem, owner);
                prefix |= uint32_t(bin) << shift;
                mask |= 255u << shift;
                rank = rem;
                __syncthreads();
            }
            // stable partition into the other buffer
            int *dst = sidx[cur ^ 1] + o;
            int run_l = 0, run_e = 0;
            for (int b0 = 0; b0 < cc; b0 += 64) {
                const int e = b0 + lane;
                const bool valid = e < cc;
                const uint32_t key = valid ? skey[o + e] : 0u;
                const bool less = valid && key < prefix, eq = valid && key == prefix;
                const uint64_t bl = __ballot(less), be = __ballot(eq);
                const int less_before = run_l + __popcll(bl & lanemask_lt());
                const int eq_before = run_e + __popcll(be & lanemask_lt());
                if (valid) {
                    const bool left = less || (eq && eq_before < rank);
                    const int left_before = less_before + min(eq_before, rank);
                    int pos = left ? left_before : m + (e - left_before);
                    if (pos < 0 || pos >= cc) {  // cannot happen for a correct select
                        atomicOr(err, 2);
                        pos = min(max(pos, 0), cc - 1);
                    }
                    dst[pos] = src[e];
                }
                run_l += __popcll(bl);
                run_e += __popcll(be);
            }
            __syncthreads();
        }
        cur ^= 1;
    }
    for (int e = lane; e < c; e += 64) idx[base + e] = sidx[cur][e];
}

// ---- gather into tree order, non-finite check ------------------------------
template <int DP>
__global__ void k_gather(const float *__restrict__ P, int64_t n, int d, const int *__restrict__ idx,
                         float *__restrict__ pts, int32_t *__restrict__ perm,
                         int *__restrict__ nonfinite) {
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t p = t / DP;
    int j = int(t % DP);
    if (p >= n + kPadRows) return;
    float v = 0.f;
    if (p < n) {
        int src = idx[p];
        if (j == 0) perm[p] = src;
        if (j < d) {
            v = P[int64_t(src) * d + j];
            if (!isfinite(v)) atomicOr(nonfinite, 1);
        }
    }
    pts[p * DP + j] = v;
}

// leaf-blocked copy of the tree-ordered points for the BaseCase tiles
template <int DP>
__global__ void k_leaf_pad(const float *__restrict__ pts, const int2 *__restrict__ range,
                           int first_leaf, int64_t n_leaves, int slots, float *__restrict__ lpts) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t row = t / DP;
    const int j = int(t % DP);
    const int64_t leaf = row / slots;
    const int slot = int(row % slots);
    if (leaf >= n_leaves) return;
    const int2 r = range[first_leaf + leaf];
    lpts[t] = slot < r.y ? pts[int64_t(r.x + slot) * DP + j] : 3.402823466e38f;
}

__device__ inline float round_up_f(double x) {
    x *= 1.0 + 0x1p-46;  // covers the FP64 evaluation error
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, __builtin_inff());
    return f;
}

// ---- leaves: tight box and exact lambda (one wave per leaf) ----------------
template <int DP>
__global__ __launch_bounds__(64) void k_leaf_stats(const float *__restrict__ pts,
                                                   const int2 *__restrict__ range, int first_leaf,
                                                   int n_leaves, int d, float *__restrict__ box,
                                                   float *__restrict__ lam,
                                                   int *__restrict__ split_dim) {
    const int leaf = blockIdx.x, lane = threadIdx.x;
    if (leaf >= n_leaves) return;
    const int node = first_leaf + leaf;
    const int2 r = range[node];
    const int j = lane % DP, grp = lane / DP;
    constexpr int NG = 64 / DP;
    float lo = __builtin_inff(), hi = -__builtin_inff();
    for (int e = grp; e < r.y; e += NG) {
        float v = pts[int64_t(r.x + e) * DP + j];
        if (v == 0.0f) v = 0.0f;
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
    }
#pragma unroll
    for (int off = DP; off < 64; off <<= 1) {
        lo = fminf(lo, __shfl_xor(lo, off));
        hi = fmaxf(hi, __shfl_xor(hi, off));
    }
    __shared__ float cen[DP];
    if (lane < DP) {
        float blo = lane < d ? lo : 0.f, bhi = lane < d ? hi : 0.f;
        box[int64_t(node) * 2 * DP + lane] = blo;
        box[int64_t(node) * 2 * DP + DP + lane] = bhi;
        cen[lane] = lane < d ? 0.5f * (blo + bhi) : 0.f;
        if (lane == 0) split_dim[node] = -1;
    }
    __syncthreads();
    double s = -1.0;
    if (lane < r.y) {
        s = 0.0;
        for (int q = 0; q < d; ++q) {
            double diff = (double)pts[int64_t(r.x + lane) * DP + q] - (double)cen[q];
            s = fma(diff, diff, s);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s = fmax(s, __shfl_xor(s, off));
    if (lane == 0) lam[node] = r.y > 0 ? round_up_f(sqrt(s)) : 0.f;
}

// ---- internal nodes: lambda <= max_c (|C - C_c| + lambda_c), and <= the
//      distance from C to the farthest box corner ------------------------------
template <int DP>
__global__ void k_internal_lambda(const int2 *__restrict__ range, int node0, int nnodes, int d,
                                  const float *__restrict__ box, float *__restrict__ lam) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nnodes) return;
    const int node = node0 + i;
    if (range[node].y == 0) {
        lam[node] = 0.f;
        return;
    }
    const float *b = box + int64_t(node) * 2 * DP;
    double corner = 0.0;
    double viakids = 0.0;
    double dc[2] = {0.0, 0.0};
    for (int j = 0; j < d; ++j) {
        float c = 0.5f * (b[j] + b[DP + j]);
        double h = fmax((double)b[DP + j] - c, (double)c - b[j]);
        corner += h * h;
        for (int q = 0; q < 2; ++q) {
            const int ch = 2 * node + 1 + q;
            if (range[ch].y == 0) continue;
            const float *cb = box + int64_t(ch) * 2 * DP;
            float cc = 0.5f * (cb[j] + cb[DP + j]);
            double diff = (double)c - (double)cc;
            dc[q] += diff * diff;
        }
    }
    for (int q = 0; q < 2; ++q) {
        const int ch = 2 * node + 1 + q;
        if (range[ch].y == 0) continue;
        viakids = fmax(viakids, sqrt(dc[q]) + (double)lam[ch]);
    }
    lam[node] = round_up_f(fmin(sqrt(corner), viakids));
}

template <int DP>
knn_status build_impl(const float *points, int64_t n, int d, int leaf, hipStream_t s,
                      knn_tree *t) {
    const int L = t->depth;
    const int n_nodes = int(t->n_nodes);
    const int nn = int(n);
    int *idxA = nullptr, *idxB = nullptr, *flag = nullptr, *hist = nullptr;
    uint32_t *keys = nullptr, *boxu = nullptr;
    Sel *sel = nullptr;
    int2 *counts = nullptr;
    struct Guard {
        hipStream_t s;
        std::vector<void *> p;
        ~Guard() {
            for (void *q : p) free_async(q, s);
        }
    } g{s, {}};
    KNN_HIP(alloc_async(&idxA, n, s));
    g.p.push_back(idxA);
    KNN_HIP(alloc_async(&idxB, n, s));
    g.p.push_back(idxB);
    KNN_HIP(alloc_async(&keys, n, s));
    g.p.push_back(keys);
    KNN_HIP(alloc_async(&flag, 1, s));
    g.p.push_back(flag);
    KNN_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));

    k_ranges<<<(n_nodes + 255) / 256, 256, 0, s>>>(t->range, nn, n_nodes);
    k_iota<<<(nn + 255) / 256, 256, 0, s>>>(idxA, nn);

    int l = 0;
    auto cmax = [&](int lv) { return int((n + (int64_t(1) << lv) - 1) >> lv); };
    while (l < L && cmax(l) > kLocalMax) {
        const int nseg = 1 << l, node0 = nseg - 1;
        const int bps = (cmax(l) + kChunk - 1) / kChunk;
        const int nblk = nseg * bps;
        if (!boxu) {
            // sized for the largest grid-wide level (segments and blocks)
            int maxseg = 1, maxblk = 1;
            for (int q = 0; q < L && cmax(q) > kLocalMax; ++q) {
                maxseg = std::max(maxseg, 1 << q);
                maxblk = std::max(maxblk, (1 << q) * ((cmax(q) + kChunk - 1) / kChunk));
            }
            KNN_HIP(alloc_async(&boxu, size_t(maxseg) * 2 * DP, s));
            g.p.push_back(boxu);
            KNN_HIP(alloc_async(&sel, maxseg, s));
            g.p.push_back(sel);
            KNN_HIP(alloc_async(&hist, size_t(maxseg) * 256, s));
            g.p.push_back(hist);
            KNN_HIP(alloc_async(&counts, size_t(maxblk), s));
            g.p.push_back(counts);
        }
        const int nbox = nseg * 2 * DP;
        k_fill_u32<<<(nbox + 255) / 256, 256, 0, s>>>(boxu, nbox, 0xffffffffu, 0u, DP);
        k_box_level<DP><<<nblk, kBlock, 0, s>>>(points, d, idxA, t->range, node0, bps, boxu);
        k_box_finalize<DP><<<(nseg + 63) / 64, 64, 0, s>>>(boxu, t->range, node0, nseg, d, t->box,
                                                          t->split_dim, sel);
        KNN_HIP(hipMemsetAsync(hist, 0, size_t(nseg) * 256 * sizeof(int), s));
        for (int pass = 0; pass < 4; ++pass) {
            k_hist<DP><<<nblk, kBlock, 0, s>>>(points, d, idxA, t->range, node0, bps, t->split_dim,
                                              keys, sel, hist, pass);
            k_select<<<nseg, 64, 0, s>>>(hist, sel, t->range, node0, pass);
        }
        k_part_count<<<nblk, kBlock, 0, s>>>(keys, t->range, node0, bps, sel, counts);
        k_part_scan<<<(nseg + 63) / 64, 64, 0, s>>>(counts, nseg, bps);
        k_part_scatter<<<nblk, kBlock, 0, s>>>(keys, idxA, idxB, t->range, node0, bps, sel, counts,
                                               flag);
        std::swap(idxA, idxB);
        ++l;
    }
    if (l < L) {
        k_local_build<DP><<<1 << l, 64, 0, s>>>(points, d, idxA, t->range, l, L, t->box,
                                               t->split_dim, flag);
    }
    const int64_t tot = (n + kPadRows) * DP;
    k_gather<DP><<<int((tot + 255) / 256), 256, 0, s>>>(points, n, d, idxA, t->pts, t->perm, flag);
    k_leaf_stats<DP><<<int(t->n_leaves), 64, 0, s>>>(t->pts, t->range, int(t->first_leaf),
                                                     int(t->n_leaves), d, t->box, t->lam,
                                                     t->split_dim);
    {
        const int64_t tot_l = t->n_leaves * t->leaf_slots * DP;
        k_leaf_pad<DP><<<int((tot_l + 255) / 256), 256, 0, s>>>(t->pts, t->range,
                                                                int(t->first_leaf), t->n_leaves,
                                                                t->leaf_slots, t->lpts);
    }
    for (int lv = L - 1; lv >= 0; --lv) {
        const int cnt = 1 << lv;
        k_internal_lambda<DP><<<(cnt + 63) / 64, 64, 0, s>>>(t->range, cnt - 1, cnt, d, t->box,
                                                            t->lam);
    }
    KNN_HIP(hipGetLastError());
    int hflag = 0;
    KNN_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    KNN_HIP(hipStreamSynchronize(s));
    if (hflag & 1) return fail(KNN_E_NONFINITE, "knn_build_tree: non-finite coordinate in input");
    if (hflag & 2) return fail(KNN_E_DEVICE, "knn_build_tree: internal partition inconsistency");
    return KNN_OK;
}

}  // namespace

void free_tree(knn_tree *t) {
    if (!t) return;
    hipFree(t->pts);
    hipFree(t->lpts);
    hipFree(t->perm);
    hipFree(t->range);
    hipFree(t->box);
    hipFree(t->lam);
    hipFree(t->split_dim);
    delete t;
}

knn_status build_tree(const float *points, int64_t n, int d, int leaf, hipStream_t s,
                      knn_tree **out) {
    knn_tree *t = new knn_tree();
    t->n = n;
    t->d = d;
    t->dp = pad_dim(d);
    t->leaf_size = leaf;
    t->depth = depth_for(n, leaf);
    t->n_nodes = (int64_t(2) << t->depth) - 1;
    t->n_leaves = int64_t(1) << t->depth;
    t->first_leaf = t->n_leaves - 1;
    {
        const int64_t max_leaf = (n + t->n_leaves - 1) / t->n_leaves;
        t->leaf_slots = int32_t((max_leaf + 7) / 8 * 8);
    }
    KNN_HIP(hipGetDevice(&t->device));
    const int dp = t->dp;
    auto cleanup_fail = [&](knn_status st) {
        free_tree(t);
        return st;
    };
    hipError_t e = hipSuccess;
    e = e ? e : hipMalloc(&t->pts, size_t(n + kPadRows) * dp * sizeof(float));
    e = e ? e : hipMalloc(&t->lpts, size_t(t->n_leaves) * t->leaf_slots * dp * sizeof(float));
    e = e ? e : hipMalloc(&t->perm, size_t(n) * sizeof(int32_t));
    e = e ? e : hipMalloc(&t->range, size_t(t->n_nodes) * sizeof(int2));
    e = e ? e : hipMalloc(&t->box, size_t(t->n_nodes) * 2 * dp * sizeof(float));
    e = e ? e : hipMalloc(&t->lam, size_t(t->n_nodes) * sizeof(float));
    e = e ? e : hipMalloc(&t->split_dim, size_t(t->n_nodes) * sizeof(int32_t));
    if (e != hipSuccess) {
        cleanup_fail(KNN_OK);
        return fail(e == hipErrorOutOfMemory ? KNN_E_OOM : KNN_E_DEVICE,
                    std::string("knn_build_tree: allocation failed: ") + hipGetErrorString(e));
    }
    hipEvent_t ev0, ev1;
    KNN_HIP(hipEventCreate(&ev0));
    KNN_HIP(hipEventCreate(&ev1));
    KNN_HIP(hipEventRecord(ev0, s));
    knn_status st;
    switch (dp) {
        case 4: st = build_impl<4>(points, n, d, leaf, s, t); break;
        case 8: st = build_impl<8>(points, n, d, leaf, s, t); break;
        case 16: st = build_impl<16>(points, n, d, leaf, s, t); break;
        case 32: st = build_impl<32>(points, n, d, leaf, s, t); break;
        default: st = build_impl<64>(points, n, d, leaf, s, t); break;
    }
    if (st == KNN_OK) {
        (void)hipEventRecord(ev1, s);
        (void)hipEventSynchronize(ev1);
        (void)hipEventElapsedTime(&t->ms_build, ev0, ev1);
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (st != KNN_OK) return cleanup_fail(st);
    *out = t;
    return KNN_OK;
}

}  // namespace knnx
