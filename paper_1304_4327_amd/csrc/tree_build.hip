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
//   * levels whose segments exceed kLocalMax points run as grid-wide passes
//     over a copy of the points kept in the current order (coalesced reads;
//     each partition moves the rows along with their indices): segmented box
//     reduction, radix select (11 + 11 + 10-bit digits of an order-preserving
//     uint32 key) of the median key per segment, and a stable partition by a
//     segmented scan of (less, equal) counts;
//   * the remaining levels of every segment of <= kLocalMax points are built
//     by one wavefront in LDS (same select/partition, wave ballots instead of
//     block scans).
// Then the points are gathered into tree order (FP32, padded to dp), leaf
// boxes and lambda are computed exactly (FP64, rounded up), and internal
// lambda gets an upper bound from the children.
#include "common.hpp"

#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>

#include <algorithm>
#include <vector>

namespace knnx {
namespace {

constexpr int kLocalMax = 1024;  // segments this small finish in one wave
// elements per block in grid-wide levels: larger chunks for short rows
// (fewer blocks, so fewer histogram flushes and block-level selection
// steps per level); long rows keep blocks short for the scatter
constexpr int chunk_for(int DP) { return DP <= 8 ? 2048 : 1024; }
constexpr int kBlock = 256;

struct Sel {
    uint32_t prefix, mask;  // key bits fixed so far
    int32_t rank;           // rank still wanted among keys matching the prefix
    int32_t bits;           // low bits not yet fixed (0: the median key is known)
};

__device__ inline uint64_t lanemask_lt() {
    return (uint64_t(1) << (threadIdx.x & 63)) - 1;
}

// Set-up of one build in a single launch: node ranges (heap order, the left
// child takes floor(c/2) of a node's c points), the error flag, the
// histogram and padding buffers cleared, the box accumulators initialised.
struct PrepArgs {
    int2 *range;
    int n, n_nodes;
    int *flag;
    int *hist;
    int64_t n_hist;
    float *pad0, *pad1;  // padding rows to zero (either may be NULL)
    int n_pad;
    uint32_t *boxu;  // [seg][2][dp]: lo words all-ones, hi words zero
    int n_box, dp;
};
__global__ void k_prep(const PrepArgs p) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i == 0) *p.flag = 0;
    if (i < p.n_hist) p.hist[i] = 0;
    if (i < p.n_pad) {
        if (p.pad0) p.pad0[i] = 0.f;
        if (p.pad1) p.pad1[i] = 0.f;
    }
    if (i < p.n_box) p.boxu[i] = ((i / p.dp) & 1) ? 0u : 0xffffffffu;
    if (i < p.n_nodes) {
        const unsigned v = unsigned(i) + 1u;
        const int depth = 31 - __clz(v);
        int start = 0, cnt = p.n;
        for (int l = depth - 1; l >= 0; --l) {
            const int half = cnt >> 1;
            if ((v >> l) & 1u) {
                start += half;
                cnt -= half;
            } else {
                cnt = half;
            }
        }
        p.range[i] = make_int2(start, cnt);
    }
}

// ---- initial copy: padded rows in input order, non-finite check -------------
template <int DP>
__global__ void k_init(const float *__restrict__ P, int64_t n, int d, float *__restrict__ cur,
                       int *__restrict__ idx, int *__restrict__ flag) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t row = t / DP;
    const int j = int(t % DP);
    if (row >= n + kPadRows) return;
    float v = 0.f;
    if (row < n) {
        if (j == 0) idx[row] = int(row);
        if (j < d) {
            v = P[row * d + j];
            if (!isfinite(v)) atomicOr(flag, 1);
        }
    }
    cur[t] = v;
}

// ---- grid-wide level: box -----------------------------------------------------
template <int DP, int CH>
__global__ __launch_bounds__(kBlock) void k_box_level(const float *__restrict__ cur, int d,
                                                      const int2 *__restrict__ range, int node0,
                                                      int bps, uint32_t *__restrict__ boxu) {
    const int seg = blockIdx.x / bps, chunk = blockIdx.x % bps;
    const int2 r = range[node0 + seg];
    const int e0 = chunk * CH, e1 = min(r.y, e0 + CH);
    const int t = threadIdx.x, j = t % DP, grp = t / DP;
    constexpr int NG = kBlock / DP;
    constexpr int IT = CH / NG;  // elements per thread
    constexpr int BATCH = IT < 16 ? IT : 16;  // loads issued together
    uint32_t lo = 0xffffffffu, hi = 0u;
    if (j < d) {
        for (int q0 = 0; q0 < IT; q0 += BATCH) {
            float v[BATCH];
#pragma unroll
            for (int q = 0; q < BATCH; ++q) {
                const int e = e0 + grp + (q0 + q) * NG;
                v[q] = e < e1 ? cur[int64_t(r.x + e) * DP + j] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < BATCH; ++q) {
                if (e0 + grp + (q0 + q) * NG < e1) {
                    const uint32_t k = f2key(v[q]);
                    lo = min(lo, k);
                    hi = max(hi, k);
                }
            }
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

// ---- grid-wide level: five launches ------------------------------------------
//   A  split dimension and box of each segment from the accumulated box keys,
//      first digit histogram (keys stored);
//   B  selection step on digit 0, second digit histogram, box accumulators
//      cleared;
//   C  selection step on digit 1, third digit histogram;
//   D  selection step on digit 2 (the median key is known), per-block counts
//      of keys below / equal to it;
//   E  stable partition (each block sums the counts of the blocks before it)
//      with the children's box keys accumulated for the next level.
// A selection step is a block-wide scan of the segment's histogram; every
// block of the segment takes the same step, the first block stores it.
// Digits are up to 11 bits wide, starting below the bits that the whole
// segment shares (the bits above the highest bit where its extremes differ);
// three digits always suffice, and a segment whose median key is known skips
// the remaining histograms.  Histograms are cleared by the kernel after the
// one that reads them.
constexpr int kDigitBits = 11, kBins = 1 << kDigitBits;
__device__ inline int digit_width(int bits) { return bits < kDigitBits ? bits : kDigitBits; }

// block-wide: the selection after one more digit (all threads return it)
__device__ Sel select_step(const int *__restrict__ H, Sel s) {
    __shared__ int wsum[kBlock / 64];
    __shared__ int sbin[2];
    if (s.bits == 0) return s;  // uniform: the same Sel in the whole block
    const int width = digit_width(s.bits), shift = s.bits - width;
    const uint32_t dm = (1u << width) - 1u;
    constexpr int PER = kBins / kBlock;
    static_assert(PER == 8, "two 16-byte loads per thread");
    int c[PER], sum = 0;
    {
        const int4 *h4 = reinterpret_cast<const int4 *>(H + threadIdx.x * PER);
        const int4 x = h4[0], y = h4[1];
        c[0] = x.x, c[1] = x.y, c[2] = x.z, c[3] = x.w;
        c[4] = y.x, c[5] = y.y, c[6] = y.z, c[7] = y.w;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) sum += c[q];
    // inclusive prefix of the threads' sums: within each wave by shuffles,
    // then the sums of the waves before
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    for (int q = 0; q < wv; ++q) incl += wsum[q];
    const int excl = incl - sum;
    if (excl <= s.rank && s.rank < incl) {
        int rem = s.rank - excl, bin = threadIdx.x * PER;
#pragma unroll
        for (int q = 0; q < PER - 1; ++q) {
            if (rem >= c[q] && bin == threadIdx.x * PER + q) {
                rem -= c[q];
                ++bin;
            }
        }
        sbin[0] = bin;
        sbin[1] = rem;
    }
    __syncthreads();
    Sel r = s;
    r.prefix |= uint32_t(sbin[0]) << shift;
    r.mask |= dm << shift;
    r.rank = sbin[1];
    r.bits = shift;
    __syncthreads();  // wsum / sbin are reused by the next step
    return r;
}

// histogram of the current digit of the keys matching the selection prefix;
// PASS 0 also makes and stores the keys (coordinate of the split dimension)
template <int DP, int PASS, int CH>
__device__ void hist_digit(const float *__restrict__ cur, int2 r, int e0, int e1, int jsplit,
                           uint32_t *__restrict__ keys, Sel s, int *__restrict__ gh) {
    __shared__ int h[kBins];
    const bool count = s.bits > 0;
    const int width = digit_width(s.bits), shift = count ? s.bits - width : 0;
    const uint32_t dm = (1u << width) - 1u;
    if (count)
        for (int i = threadIdx.x; i < kBins; i += kBlock) h[i] = 0;
    __syncthreads();
    constexpr int IT = CH / kBlock;
    uint32_t kv[IT];
#pragma unroll
    for (int q = 0; q < IT; ++q) {
        const int e = e0 + threadIdx.x + q * kBlock;
        if constexpr (PASS == 0)
            kv[q] = e < e1 ? f2key(cur[int64_t(r.x + e) * DP + jsplit]) : 0u;
        else
            kv[q] = (count && e < e1) ? keys[r.x + e] : 0u;
    }
#pragma unroll
    for (int q = 0; q < IT; ++q) {
        const int e = e0 + threadIdx.x + q * kBlock;
        if (e < e1) {
            if constexpr (PASS == 0) keys[r.x + e] = kv[q];
            if (count && (kv[q] & s.mask) == s.prefix) atomicAdd(&h[(kv[q] >> shift) & dm], 1);
        }
    }
    __syncthreads();
    if (count)
        for (int i = threadIdx.x; i < kBins; i += kBlock)
            if (h[i]) atomicAdd(&gh[i], h[i]);
}

// this block's share of a segment's histogram bins, cleared
__device__ inline void clear_share(int *__restrict__ gh, int chunk, int bps) {
    const int per = (kBins + bps - 1) / bps;
    const int b0 = chunk * per, b1 = min(kBins, b0 + per);
    for (int i = b0 + threadIdx.x; i < b1; i += kBlock) gh[i] = 0;
}

// A: split dimension, box, first selection state, digit-0 histogram
template <int DP, int CH>
__global__ __launch_bounds__(kBlock) void k_level_a(const float *__restrict__ cur, int d,
                                                    const int2 *__restrict__ range, int node0,
                                                    int bps, const uint32_t *__restrict__ boxu,
                                                    float *__restrict__ box,
                                                    int *__restrict__ split_dim,
                                                    Sel *__restrict__ sel0,
                                                    uint32_t *__restrict__ keys,
                                                    int *__restrict__ hist0) {
    const int seg = blockIdx.x / bps, chunk = blockIdx.x % bps;
    const int node = node0 + seg;
    const int2 r = range[node];
    __shared__ uint32_t slo[DP], shi[DP];
    __shared__ int sbest;
    if (threadIdx.x < DP) {
        slo[threadIdx.x] = boxu[(seg * 2) * DP + threadIdx.x];
        shi[threadIdx.x] = boxu[(seg * 2 + 1) * DP + threadIdx.x];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // widest extent, lowest dimension on ties
        int best = 0;
        float bestext = -1.0f;
        if (r.y > 0)
            for (int j = 0; j < d; ++j) {
                const float ext = key2f(shi[j]) - key2f(slo[j]);
                if (ext > bestext) {
                    bestext = ext;
                    best = j;
                }
            }
        sbest = best;
    }
    __syncthreads();
    const int best = sbest;
    const uint32_t klo = slo[best], khi = shi[best];
    // every key of the segment shares the bits above the highest bit where
    // the extremes differ: the digits start below them
    const uint32_t diff = klo ^ khi;
    const int bits = r.y > 0 && diff ? 32 - __clz(diff) : 0;
    const uint32_t mask = bits >= 32 ? 0u : ~((1u << bits) - 1u);
    const Sel s0 = Sel{klo & mask, mask, r.y / 2, r.y > 0 ? bits : 0};
    if (chunk == 0) {
        if (threadIdx.x < DP) {
            const int j = threadIdx.x;
            float lo = 0.f, hi = 0.f;
            if (j < d) {
                lo = r.y > 0 ? key2f(slo[j]) : __builtin_inff();
                hi = r.y > 0 ? key2f(shi[j]) : -__builtin_inff();
            }
            box[int64_t(node) * 2 * DP + j] = lo;
            box[int64_t(node) * 2 * DP + DP + j] = hi;
        }
        if (threadIdx.x == 0) {
            split_dim[node] = best;
            sel0[seg] = s0;
        }
    }
    const int e0 = chunk * CH, e1 = min(r.y, e0 + CH);
    hist_digit<DP, 0, CH>(cur, r, e0, e1, best, keys, s0, hist0 + int64_t(seg) * kBins);
}

// B, C: selection step on the previous digit, next digit's histogram.
// B also restores the box accumulators the level has read; C clears the
// digit-0 histogram.
template <int PASS, int CH>
__global__ __launch_bounds__(kBlock) void k_level_bc(const int2 *__restrict__ range, int node0,
                                                     int bps, uint32_t *__restrict__ keys,
                                                     const Sel *__restrict__ sel_in,
                                                     Sel *__restrict__ sel_out,
                                                     const int *__restrict__ hist_in,
                                                     int *__restrict__ hist_out,
                                                     int *__restrict__ hist_clear,
                                                     uint32_t *__restrict__ boxu_reset, int dp) {
    const int seg = blockIdx.x / bps, chunk = blockIdx.x % bps;
    const int2 r = range[node0 + seg];
    const Sel s = select_step(hist_in + int64_t(seg) * kBins, sel_in[seg]);
    if (chunk == 0 && threadIdx.x == 0) sel_out[seg] = s;
    if (boxu_reset && chunk == 0 && threadIdx.x < 2 * dp)
        boxu_reset[seg * 2 * dp + threadIdx.x] = threadIdx.x < dp ? 0xffffffffu : 0u;
    if (hist_clear) clear_share(hist_clear + int64_t(seg) * kBins, chunk, bps);
    const int e0 = chunk * CH, e1 = min(r.y, e0 + CH);
    hist_digit<4, PASS, CH>(nullptr, r, e0, e1, 0, keys, s, hist_out + int64_t(seg) * kBins);
}

// D: last selection step; counts of keys below / equal to the median key
template <int CH>
__global__ __launch_bounds__(kBlock) void k_level_count(const uint32_t *__restrict__ keys,
                                                        const int2 *__restrict__ range,
                                                        int node0, int bps,
                                                        const Sel *__restrict__ sel_in,
                                                        Sel *__restrict__ sel_out,
                                                        const int *__restrict__ hist_in,
                                                        int *__restrict__ hist_clear,
                                                        int2 *__restrict__ counts) {
    const int seg = blockIdx.x / bps, chunk = blockIdx.x % bps;
    const int2 r = range[node0 + seg];
    const Sel s = select_step(hist_in + int64_t(seg) * kBins, sel_in[seg]);
    if (chunk == 0 && threadIdx.x == 0) sel_out[seg] = s;
    clear_share(hist_clear + int64_t(seg) * kBins, chunk, bps);
    const int e0 = chunk * CH, e1 = min(r.y, e0 + CH);
    const uint32_t v = s.prefix;
    int nl = 0, ne = 0;
    constexpr int IT = CH / kBlock;
#pragma unroll
    for (int q = 0; q < IT; ++q) {
        const int e = e0 + threadIdx.x + q * kBlock;
        if (e < e1) {
            const uint32_t key = keys[r.x + e];
            nl += key < v;
            ne += key == v;
        }
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

// E: stable partition; for strides <= 8 the two children's box keys are
// accumulated for the next level (boxu_next != NULL)
template <int DP, int CH>
__global__ __launch_bounds__(kBlock) void k_level_scatter(const uint32_t *__restrict__ keys,
                                                          const int *__restrict__ idx_in,
                                                          int *__restrict__ idx_out,
                                                          const float *__restrict__ cur,
                                                          float *__restrict__ nxt,
                                                          const int2 *__restrict__ range,
                                                          int node0, int bps,
                                                          const Sel *__restrict__ sel,
                                                          const int2 *__restrict__ counts,
                                                          int *__restrict__ hist_clear,
                                                          int *__restrict__ err, int d,
                                                          uint32_t *__restrict__ boxu_next) {
    constexpr bool kBox = DP <= 8;
    const int seg = blockIdx.x / bps, chunk = blockIdx.x % bps;
    const int2 r = range[node0 + seg];
    const int e0 = chunk * CH, e1 = min(r.y, e0 + CH);
    const Sel s = sel[seg];
    const uint32_t v = s.prefix;
    const int req = s.rank;  // equal keys that go left
    const int m = r.y / 2;
    clear_share(hist_clear + int64_t(seg) * kBins, chunk, bps);
    // counts of the segment's blocks before this one
    __shared__ int wl[kBlock / 64], we[kBlock / 64];
    int2 off;
    {
        int a = 0, b = 0;
        for (int c = threadIdx.x; c < chunk; c += kBlock) {
            const int2 q = counts[seg * bps + c];
            a += q.x;
            b += q.y;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            a += __shfl_xor(a, o);
            b += __shfl_xor(b, o);
        }
        if ((threadIdx.x & 63) == 0) {
            wl[threadIdx.x >> 6] = a;
            we[threadIdx.x >> 6] = b;
        }
        __syncthreads();
        a = b = 0;
        for (int q = 0; q < kBlock / 64; ++q) {
            a += wl[q];
            b += we[q];
        }
        off = make_int2(a, b);
        __syncthreads();
    }
    const int w = threadIdx.x >> 6;
    float blo[2][kBox ? DP : 1], bhi[2][kBox ? DP : 1];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int j = 0; j < (kBox ? DP : 1); ++j) {
            blo[q][j] = __builtin_inff();
            bhi[q][j] = -__builtin_inff();
        }
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
            const float4 *src = reinterpret_cast<const float4 *>(cur + int64_t(r.x + e) * DP);
            float4 *dst = reinterpret_cast<float4 *>(nxt + int64_t(r.x + pos) * DP);
#pragma unroll
            for (int q = 0; q < DP / 4; ++q) {
                const float4 x = src[q];
                dst[q] = x;
                if constexpr (kBox) {
                    const float xv[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int j = 4 * q + c;
                        if (j < d) {
                            blo[left ? 0 : 1][j] = fminf(blo[left ? 0 : 1][j], xv[c]);
                            bhi[left ? 0 : 1][j] = fmaxf(bhi[left ? 0 : 1][j], xv[c]);
                        }
                    }
                }
            }
        }
        run_l += tl;
        run_e += te;
    }
    if constexpr (kBox) {
        if (boxu_next) {
            // wave reduction, one atomic per wave into the block's copy, one
            // per block into the next level's box keys
            __shared__ uint32_t sb[2][2][DP];
            if (threadIdx.x < 4 * DP)
                (&sb[0][0][0])[threadIdx.x] = ((threadIdx.x / DP) & 1) ? 0u : 0xffffffffu;
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int j = 0; j < DP; ++j) {
                    if (j >= d) continue;
                    // float min / max (-0 and +0 map to one key below)
                    const float a = reduce64(blo[q][j], OpMin());
                    const float b = reduce64(bhi[q][j], OpMax());
                    if ((threadIdx.x & 63) == 0 && a <= b) {
                        atomicMin(&sb[q][0][j], f2key(a));
                        atomicMax(&sb[q][1][j], f2key(b));
                    }
                }
            __syncthreads();
            if (threadIdx.x < 2 * DP) {
                const int q = threadIdx.x / DP, j = threadIdx.x % DP;
                const int child = 2 * seg + q;
                if (j < d) {
                    if (sb[q][0][j] != 0xffffffffu)
                        atomicMin(&boxu_next[(child * 2) * DP + j], sb[q][0][j]);
                    if (sb[q][1][j] != 0u) atomicMax(&boxu_next[(child * 2 + 1) * DP + j], sb[q][1][j]);
                }
            }
        }
    }
}

// ---- one workgroup finishes a segment's subtree ---------------------------------
// The segment's rows are contiguous in `cur`; for small strides they are
// staged in LDS.  sidx holds local row numbers in the current order.  Each
// of the four waves takes every fourth node of a level (a node is one wave's
// work; its waits are wave-level), and the workgroup meets between levels.
// At the end the rows are written in final (tree) order to `out_pts` and
// their original indices to `out_perm`.
constexpr int kLocalWaves = 4;
__device__ inline void wave_lds_sync() {
    // LDS writes of this wave visible to its other lanes; no workgroup wait
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
template <int DP>
__global__ __launch_bounds__(64 * kLocalWaves) void k_local_build(const float *__restrict__ cur, int d,
                                                    const int *__restrict__ idx_glob,
                                                    const int2 *__restrict__ range, int l0,
                                                    int L, float *__restrict__ box,
                                                    int *__restrict__ split_dim,
                                                    int *__restrict__ err,
                                                    float *__restrict__ out_pts,
                                                    int *__restrict__ out_perm) {
    constexpr bool kLds = DP <= 8;
    const int seg = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int kThreads = 64 * kLocalWaves;
    const int2 rr = range[(1 << l0) - 1 + seg];
    const int base = rr.x, c = rr.y;
    __shared__ int sidx[2][kLocalMax];
    __shared__ uint32_t skey[kLocalMax];
    __shared__ int hist_all[kLocalWaves][256];
    int *hist = hist_all[wave];
    __shared__ float spts[kLds ? kLocalMax * DP : 4];
    const float *gpts = cur + int64_t(base) * DP;
    if constexpr (kLds) {
        for (int t = threadIdx.x; t < c * DP; t += kThreads) spts[t] = gpts[t];
    }
    auto X = [&](int row, int j) -> float {
        if constexpr (kLds)
            return spts[row * DP + j];
        else
            return gpts[int64_t(row) * DP + j];
    };
    for (int e = threadIdx.x; e < c; e += kThreads) sidx[0][e] = e;
    __syncthreads();
    int cb = 0;
    const int j_l = lane % DP, grp = lane / DP;
    constexpr int NG = 64 / DP;
    for (int lv = l0; lv < L; ++lv) {
        const int nsub = 1 << (lv - l0);
        for (int sub = wave; sub < nsub; sub += kLocalWaves) {
            const int node = (1 << lv) - 1 + seg * nsub + sub;
            const int2 nr = range[node];
            const int o = nr.x - base, cc = nr.y;
            const int *src = sidx[cb] + o;
            // box over the node's points
            uint32_t lo = 0xffffffffu, hi = 0u;
            if (j_l < d) {
                for (int e = grp; e < cc; e += NG) {
                    uint32_t k = f2key(X(src[e], j_l));
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
            for (int e = lane; e < cc; e += 64) skey[o + e] = f2key(X(src[e], jsplit));
            wave_lds_sync();
            const int m = cc / 2;
            int *dst = sidx[cb ^ 1] + o;
            // radix select of the key at rank floor(cc/2), 8-bit digits from
            // the first bit where the node's smallest and largest keys differ
            // (the bits above are shared by every key of the node)
            const uint32_t klo = (uint32_t)__shfl((int)lo, jsplit);
            const uint32_t khi = (uint32_t)__shfl((int)hi, jsplit);
            const uint32_t diff = klo ^ khi;
            int bits = diff ? 32 - __clz(diff) : 0;  // bits still to resolve
            uint32_t mask = bits >= 32 ? 0u : ~((1u << bits) - 1u);
            uint32_t prefix = klo & mask;
            int rank = m;
            while (bits > 0) {
                const int width = bits < 8 ? bits : 8;
                const int shift = bits - width;
                const uint32_t dmask = (1u << width) - 1u;
                hist[lane * 4 + 0] = 0;
                hist[lane * 4 + 1] = 0;
                hist[lane * 4 + 2] = 0;
                hist[lane * 4 + 3] = 0;
                wave_lds_sync();
                for (int e = lane; e < cc; e += 64) {
                    uint32_t key = skey[o + e];
                    if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & dmask], 1);
                }
                wave_lds_sync();
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
                mask |= dmask << shift;
                rank = rem;
                bits = shift;
                wave_lds_sync();
            }
            // stable partition into the other buffer
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
            wave_lds_sync();
        }
        __syncthreads();  // the next level reads every node's partition
        cb ^= 1;
    }
    // final order: rows and original indices
    for (int e = threadIdx.x; e < c; e += kThreads) out_perm[base + e] = idx_glob[base + sidx[cb][e]];
    for (int t = threadIdx.x; t < c * DP; t += kThreads) {
        const int e = t / DP, j = t % DP;
        out_pts[int64_t(base + e) * DP + j] = X(sidx[cb][e], j);
    }
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
__device__ void internal_lambda(const int2 *__restrict__ range, int node, int d,
                                const float *__restrict__ box, float *__restrict__ lam) {
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

// levels [L - H, L - 1]: block b finishes the subtree under node b of level
// L - H, bottom up (2^H - 1 nodes, a barrier between levels)
template <int DP>
__global__ __launch_bounds__(64) void k_lambda_subtrees(const int2 *__restrict__ range, int L,
                                                        int H, int d,
                                                        const float *__restrict__ box,
                                                        float *__restrict__ lam) {
    const int b = blockIdx.x;
    for (int t = H - 1; t >= 0; --t) {
        const int lv = L - H + t;
        const int cnt = 1 << t;
        for (int i = threadIdx.x; i < cnt; i += blockDim.x)
            internal_lambda<DP>(range, (1 << lv) - 1 + b * cnt + i, d, box, lam);
        __syncthreads();
    }
}

// levels [0, top - 1] in one block, bottom up
template <int DP>
__global__ __launch_bounds__(1024) void k_lambda_top(const int2 *__restrict__ range, int top,
                                                     int d, const float *__restrict__ box,
                                                     float *__restrict__ lam) {
    for (int lv = top - 1; lv >= 0; --lv) {
        const int cnt = 1 << lv;
        for (int i = threadIdx.x; i < cnt; i += blockDim.x)
            internal_lambda<DP>(range, (1 << lv) - 1 + i, d, box, lam);
        __syncthreads();
    }
}

template <int DP>
knn_status build_impl(const float *points, int64_t n, int d, int leaf, hipStream_t s,
                      knn_tree *t, int *flag, hipEvent_t done) {
    const int L = t->depth;
    const int n_nodes = int(t->n_nodes);
    const int nn = int(n);
    int *idxA = nullptr, *idxB = nullptr, *hist = nullptr;
    uint32_t *keys = nullptr, *boxu = nullptr;
    float *cur = nullptr, *nxt = nullptr;
    Sel *sel = nullptr;
    int2 *counts = nullptr;
    struct Guard {
        hipStream_t s;
        std::vector<void *> p;
        ~Guard() {
            dev_free_many(p.data(), int(p.size()), s);
        }
    } g{s, {}};
    auto get = [&](auto **ptr, size_t cnt) -> hipError_t {
        hipError_t e = alloc_async(ptr, cnt, s);
        if (e == hipSuccess) g.p.push_back(*ptr);
        return e;
    };
    const size_t rows = size_t(n) + kPadRows;
    KNN_HIP(get(&idxA, n));
    KNN_HIP(get(&cur, rows * DP));

    auto cmax = [&](int lv) { return int((n + (int64_t(1) << lv) - 1) >> lv); };
    constexpr int CH = chunk_for(DP);
    int n_global = 0, maxseg = 1, maxblk = 1;
    for (int q = 0; q < L && cmax(q) > kLocalMax; ++q) {
        n_global = q + 1;
        maxseg = std::max(maxseg, 1 << q);
        maxblk = std::max(maxblk, (1 << q) * ((cmax(q) + CH - 1) / CH));
    }
    if (n_global > 0) {
        KNN_HIP(get(&idxB, n));
        KNN_HIP(get(&keys, n));
        KNN_HIP(get(&nxt, rows * DP));
        KNN_HIP(get(&boxu, size_t(maxseg) * 2 * DP));
        KNN_HIP(get(&sel, 4 * size_t(maxseg)));
        KNN_HIP(get(&hist, 3 * size_t(maxseg) * kBins));
        KNN_HIP(get(&counts, size_t(maxblk)));
    }
    {
        PrepArgs p{};
        p.range = t->range;
        p.n = nn;
        p.n_nodes = n_nodes;
        p.flag = flag;
        p.hist = hist;
        p.n_hist = n_global > 0 ? 3 * int64_t(maxseg) * kBins : 0;
        p.pad0 = t->pts + size_t(n) * DP;
        p.pad1 = n_global > 0 ? nxt + size_t(n) * DP : nullptr;
        p.n_pad = kPadRows * DP;
        p.boxu = boxu;
        p.n_box = n_global > 0 ? maxseg * 2 * DP : 0;
        p.dp = DP;
        const int64_t tot = std::max<int64_t>({p.n_hist, int64_t(p.n_pad), int64_t(p.n_box),
                                              int64_t(n_nodes), 1});
        k_prep<<<int((tot + 255) / 256), 256, 0, s>>>(p);
        const int64_t tot_init = int64_t(rows) * DP;
        k_init<DP><<<int((tot_init + 255) / 256), 256, 0, s>>>(points, n, d, cur, idxA, flag);
    }
    int *H[3] = {hist, hist + size_t(maxseg) * kBins, hist + 2 * size_t(maxseg) * kBins};
    Sel *S[4] = {sel, sel + maxseg, sel + 2 * maxseg, sel + 3 * maxseg};
    for (int l = 0; l < n_global; ++l) {
        const int nseg = 1 << l, node0 = nseg - 1;
        const int bps = (cmax(l) + CH - 1) / CH;
        const int nblk = nseg * bps;
        // the box pass runs at level 0, and at every level for strides > 8
        // (for strides <= 8 the previous level's scatter accumulated it)
        if (l == 0 || DP > 8) k_box_level<DP, CH><<<nblk, kBlock, 0, s>>>(cur, d, t->range, node0, bps, boxu);
        k_level_a<DP, CH><<<nblk, kBlock, 0, s>>>(cur, d, t->range, node0, bps, boxu, t->box, t->split_dim,
                                             S[0], keys, H[0]);
        k_level_bc<1, CH><<<nblk, kBlock, 0, s>>>(t->range, node0, bps, keys, S[0], S[1], H[0], H[1],
                                              nullptr, boxu, DP);
        k_level_bc<2, CH><<<nblk, kBlock, 0, s>>>(t->range, node0, bps, keys, S[1], S[2], H[1], H[2],
                                              H[0], nullptr, DP);
        k_level_count<CH><<<nblk, kBlock, 0, s>>>(keys, t->range, node0, bps, S[2], S[3], H[2], H[1],
                                              counts);
        k_level_scatter<DP, CH><<<nblk, kBlock, 0, s>>>(keys, idxA, idxB, cur, nxt, t->range, node0, bps,
                                                    S[3], counts, H[2], flag, d,
                                                    (DP <= 8 && l + 1 < n_global) ? boxu : nullptr);
        std::swap(idxA, idxB);
        std::swap(cur, nxt);
    }
    if (n_global < L) {
        k_local_build<DP><<<1 << n_global, 64 * kLocalWaves, 0, s>>>(cur, d, idxA, t->range, n_global, L, t->box,
                                                       t->split_dim, flag, t->pts, t->perm);
    } else {
        // no split below the root (n <= leaf size): tree order = input order
        KNN_HIP(hipMemcpyAsync(t->pts, cur, rows * DP * sizeof(float), hipMemcpyDeviceToDevice, s));
        KNN_HIP(hipMemcpyAsync(t->perm, idxA, size_t(n) * sizeof(int), hipMemcpyDeviceToDevice, s));
    }
    k_leaf_stats<DP><<<int(t->n_leaves), 64, 0, s>>>(t->pts, t->range, int(t->first_leaf),
                                                     int(t->n_leaves), d, t->box, t->lam,
                                                     t->split_dim);
    {
        const int64_t tot_l = t->n_leaves * t->leaf_slots * DP;
        k_leaf_pad<DP><<<int((tot_l + 255) / 256), 256, 0, s>>>(t->pts, t->range,
                                                                int(t->first_leaf), t->n_leaves,
                                                                t->leaf_slots, t->lpts);
    }
    {
        // internal levels: subtrees of up to 6 levels per block, then the rest
        // of the tree in one block
        const int H = L < 6 ? L : 6;
        if (H > 0)
            k_lambda_subtrees<DP><<<1 << (L - H), 64, 0, s>>>(t->range, L, H, d, t->box, t->lam);
        if (L - H > 0) k_lambda_top<DP><<<1, 1024, 0, s>>>(t->range, L - H, d, t->box, t->lam);
    }
    KNN_HIP(hipGetLastError());
    KNN_HIP(hipEventRecord(done, s));
    return KNN_OK;
}

}  // namespace

void free_tree(knn_tree *t) {
    if (!t) return;
    int cur = 0;
    const bool switch_dev = hipGetDevice(&cur) == hipSuccess && cur != t->device;
    if (switch_dev) (void)hipSetDevice(t->device);
    void *blocks[] = {t->pts, t->lpts, t->perm, t->range, t->box, t->lam, t->split_dim};
    dev_free_many(blocks, 7, t->stream);
    if (switch_dev) (void)hipSetDevice(cur);
    delete t;
}

namespace {

// one build in flight: its tree, stream, error flag and timing events
struct BuildJob {
    knn_tree *t = nullptr;
    hipStream_t s = nullptr;
    int *flag = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

void drop_job(BuildJob &job) {
    free_async(job.flag, job.s);
    if (job.ev0) (void)hipEventDestroy(job.ev0);
    if (job.ev1) (void)hipEventDestroy(job.ev1);
    free_tree(job.t);
    job = BuildJob{};
}

// allocations and every launch of one build on stream s; no host wait
knn_status build_enqueue(const float *points, int64_t n, int d, int leaf, hipStream_t s,
                         BuildJob &job) {
    knn_tree *t = new knn_tree();
    job.t = t;
    job.s = s;
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
    t->stream = s;
    const int dp = t->dp;
    hipError_t e = hipGetDevice(&t->device);
    e = e ? e : alloc_async(&t->pts, size_t(n + kPadRows) * dp, s);
    e = e ? e : alloc_async(&t->lpts, size_t(t->n_leaves) * t->leaf_slots * dp, s);
    e = e ? e : alloc_async(&t->perm, size_t(n), s);
    e = e ? e : alloc_async(&t->range, size_t(t->n_nodes), s);
    e = e ? e : alloc_async(&t->box, size_t(t->n_nodes) * 2 * dp, s);
    e = e ? e : alloc_async(&t->lam, size_t(t->n_nodes), s);
    e = e ? e : alloc_async(&t->split_dim, size_t(t->n_nodes), s);
    e = e ? e : alloc_async(&job.flag, 1, s);
    if (e != hipSuccess) {
        drop_job(job);
        return fail(e == hipErrorOutOfMemory ? KNN_E_OOM : KNN_E_DEVICE,
                    std::string("knn_build_tree: allocation failed: ") + hipGetErrorString(e));
    }
    e = hipEventCreate(&job.ev0);
    e = e ? e : hipEventCreate(&job.ev1);
    e = e ? e : hipEventRecord(job.ev0, s);
    if (e != hipSuccess) {
        drop_job(job);
        return hip_fail(e, "knn_build_tree: set-up", __FILE__, __LINE__);
    }
    knn_status st;
    switch (dp) {
        case 4: st = build_impl<4>(points, n, d, leaf, s, t, job.flag, job.ev1); break;
        case 8: st = build_impl<8>(points, n, d, leaf, s, t, job.flag, job.ev1); break;
        case 16: st = build_impl<16>(points, n, d, leaf, s, t, job.flag, job.ev1); break;
        case 32: st = build_impl<32>(points, n, d, leaf, s, t, job.flag, job.ev1); break;
        default: st = build_impl<64>(points, n, d, leaf, s, t, job.flag, job.ev1); break;
    }
    if (st != KNN_OK) {
        (void)hipStreamSynchronize(s);  // the launches already queued must end first
        drop_job(job);
    }
    return st;
}

// wait for a build, check its flag; the tree is handed out or freed
knn_status build_finish(BuildJob &job, knn_tree **out) {
    int hflag = 0;
    hipError_t e = hipMemcpyAsync(&hflag, job.flag, sizeof(int), hipMemcpyDeviceToHost, job.s);
    e = e ? e : hipStreamSynchronize(job.s);
    if (e != hipSuccess) {
        drop_job(job);
        return hip_fail(e, "knn_build_tree: device work", __FILE__, __LINE__);
    }
    if (hflag & 1) {
        drop_job(job);
        return fail(KNN_E_NONFINITE, "knn_build_tree: non-finite coordinate in input");
    }
    if (hflag & 2) {
        drop_job(job);
        return fail(KNN_E_DEVICE, "knn_build_tree: internal partition inconsistency");
    }
    (void)hipEventElapsedTime(&job.t->ms_build, job.ev0, job.ev1);
    free_async(job.flag, job.s);
    (void)hipEventDestroy(job.ev0);
    (void)hipEventDestroy(job.ev1);
    *out = job.t;
    job = BuildJob{};
    return KNN_OK;
}

// A helper thread that issues the second build of a pair.  It lives for the
// whole process (never joined: it waits for work on a condition variable),
// so a pair build costs no thread start.  One pair build uses it at a time;
// a concurrent caller starts a thread of its own.
class BuildHelper {
  public:
    static BuildHelper &get() {
        static BuildHelper *h = new BuildHelper();  // never destroyed
        return *h;
    }
    std::mutex use;  // held by the pair build that owns the helper
    void run(std::function<void()> f) {
        std::lock_guard<std::mutex> lock(mu_);
        task_ = std::move(f);
        pending_ = true;
        cv_.notify_all();
    }
    void wait() {
        std::unique_lock<std::mutex> lock(mu_);
        cv_.wait(lock, [&] { return !pending_; });
    }

  private:
    BuildHelper() { std::thread([this] { loop(); }).detach(); }
    void loop() {
        for (;;) {
            std::function<void()> f;
            {
                std::unique_lock<std::mutex> lock(mu_);
                cv_.wait(lock, [&] { return pending_; });
                f = std::move(task_);
            }
            f();
            std::lock_guard<std::mutex> lock(mu_);
            pending_ = false;
            cv_.notify_all();
        }
    }
    std::mutex mu_;
    std::condition_variable cv_;
    std::function<void()> task_;
    bool pending_ = false;
};

// a second stream per device (default priority) for the pair build
hipError_t aux_stream(hipStream_t *out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static hipStream_t streams[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[dev]) {
        e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    *out = streams[dev];
    return hipSuccess;
}

}  // namespace

knn_status build_tree(const float *points, int64_t n, int d, int leaf, hipStream_t s,
                      knn_tree **out) {
    BuildJob job;
    KNN_TRY(build_enqueue(points, n, d, leaf, s, job));
    return build_finish(job, out);
}

namespace {

// enqueues the builds of a and (when pb is not NULL) b, b on the second
// stream from the helper thread; on error nothing is left queued or held
knn_status pair_enqueue(const float *pa, int64_t na, const float *pb, int64_t nb, int d, int leaf,
                        hipStream_t s, BuildJob &ja, BuildJob &jb) {
    if (!pb) return build_enqueue(pa, na, d, leaf, s, ja);
    hipStream_t s2;
    KNN_HIP(aux_stream(&s2));
    // the second build may only start once the caller's stream has produced
    // its inputs
    hipEvent_t ready;
    KNN_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ready, s);
    e = e ? e : hipStreamWaitEvent(s2, ready, 0);
    (void)hipEventDestroy(ready);
    if (e != hipSuccess) return hip_fail(e, "knn_build_tree_pair: stream join", __FILE__, __LINE__);
    // the launches of one build take about as long to issue as to run, so
    // the second build is issued from a second host thread
    int dev = 0;
    KNN_HIP(hipGetDevice(&dev));
    knn_status sb = KNN_OK;
    std::string msg_b;
    auto second = [&] {
        if (hipSetDevice(dev) != hipSuccess) {
            sb = KNN_E_DEVICE;
            msg_b = "knn_build_tree_pair: hipSetDevice failed in the build thread";
            return;
        }
        sb = build_enqueue(pb, nb, d, leaf, s2, jb);
        if (sb != KNN_OK) msg_b = get_error();
    };
    BuildHelper &helper = BuildHelper::get();
    std::unique_lock<std::mutex> owner(helper.use, std::try_to_lock);
    std::thread own;
    if (owner.owns_lock())
        helper.run(second);
    else
        own = std::thread(second);
    const knn_status sa = build_enqueue(pa, na, d, leaf, s, ja);
    const std::string msg_a = get_error();
    if (owner.owns_lock())
        helper.wait();
    else
        own.join();
    if (sa != KNN_OK || sb != KNN_OK) {
        knn_tree *tmp = nullptr;
        if (sa == KNN_OK && build_finish(ja, &tmp) == KNN_OK) free_tree(tmp);
        tmp = nullptr;
        if (sb == KNN_OK && build_finish(jb, &tmp) == KNN_OK) free_tree(tmp);
        return sa != KNN_OK ? fail(sa, msg_a) : fail(sb, msg_b);
    }
    return KNN_OK;
}

// waits for both builds; on error neither tree is returned
knn_status pair_finish(BuildJob &ja, BuildJob &jb, hipStream_t s, knn_tree **ta, knn_tree **tb) {
    const bool two = jb.t != nullptr;
    knn_tree *a = nullptr, *b = nullptr;
    const knn_status sa = build_finish(ja, &a);
    const std::string msg_a = get_error();
    const knn_status sb = two ? build_finish(jb, &b) : KNN_OK;
    if (sa != KNN_OK || sb != KNN_OK) {
        if (a) free_tree(a);
        if (b) free_tree(b);
        return sa != KNN_OK ? fail(sa, msg_a) : sb;
    }
    // both builds have completed (finish waited for each stream); the second
    // tree belongs to the caller's stream from now on
    if (b) b->stream = s;
    *ta = a;
    if (tb) *tb = b;
    return KNN_OK;
}

}  // namespace

knn_status build_tree_pair(const float *pa, int64_t na, const float *pb, int64_t nb, int d,
                           int leaf, hipStream_t s, knn_tree **out_a, knn_tree **out_b) {
    BuildJob ja, jb;
    KNN_TRY(pair_enqueue(pa, na, pb, nb, d, leaf, s, ja, jb));
    return pair_finish(ja, jb, s, out_a, out_b);
}

knn_status all_knn(const float *ref_points, int64_t n_ref, const float *query_points,
                   int64_t n_query, int d, int leaf, int k, const knn_opts *opts,
                   int64_t *idx_out, float *dist_out, hipStream_t s) {
    BuildJob ja, jb;
    KNN_TRY(pair_enqueue(ref_points, n_ref, query_points, n_query, d, leaf, s, ja, jb));
    // the search reads the query tree built on the second stream
    hipError_t e = jb.t ? hipStreamWaitEvent(s, jb.ev1, 0) : hipSuccess;
    knn_status st = e == hipSuccess
                        ? search(ja.t, jb.t, k, opts, idx_out, dist_out, s)
                        : hip_fail(e, "knn_all_knn: stream join", __FILE__, __LINE__);
    const std::string msg = get_error();
    knn_tree *ta = nullptr, *tb = nullptr;
    const knn_status sf = pair_finish(ja, jb, s, &ta, &tb);  // input checks of the builds
    if (sf != KNN_OK) return sf;
    if (st == KNN_OK && opts && opts->stats) {
        opts->stats->ms_ref_build = ta->ms_build;
        opts->stats->ms_query_build = tb ? tb->ms_build : 0.f;
    }
    free_tree(ta);
    if (tb) free_tree(tb);
    return st == KNN_OK ? KNN_OK : fail(st, msg);
}

}  // namespace knnx
