// Search-side declarations shared by the traversal kernels and the host code.
#pragma once

#include "common.hpp"

namespace knnx {

// counters accumulated by the traversal kernels (uint64 each)
enum StatSlot {
    ST_SCORE = 0,
    ST_TILES = 1,
    ST_PAIRS = 2,
    ST_INSERTS = 3,
    ST_FB_QUERIES = 4,
    ST_COUNT = 8
};

struct SearchArgs {
    // reference tree
    const float *rpts;
    const int32_t *rperm;
    const int2 *rrange;
    const float *rbox;
    const float *rlam;
    const float *rlpts;  // leaf-blocked points (r_leaf_slots per leaf)
    int r_leaf_slots;
    int r_first_leaf;
    // query tree
    const float *qpts;
    const int32_t *qperm;
    const int2 *qrange;
    const float *qbox;
    const float *qlam;
    int q_first_leaf;
    int q_n_leaves;
    // leaves to process: active == NULL means all; otherwise only leaves
    // with active[leaf] != 0 (the waves keep their sibling-aligned leaves)
    const int *active;
    // launch order of the wave slots (largest leaf radius first), or NULL:
    // wave i of the launch takes slot order[i]
    const int *order;
    int d, k, lpl_log2;
    int bound;          // knn_bound
    int self;           // exclude reference position == query position
    const float *seed;  // per query leaf, or NULL
    int64_t *out_idx;
    float *out_dist;
    float *leaf_kth;    // per query leaf, or NULL
    int *fallback;      // per query leaf flag (seeded runs), or NULL
    float *fb_bound;    // per query leaf (seeded runs): a proven bound for the
                        // fallback pass, min D_p[k] + 2 lambda over the leaf's
                        // queries with a full list (+inf if none), or NULL
    unsigned long long *stats;  // ST_COUNT counters, or NULL; the FP32 kernel with a
                                // seed adds its second pass's counts to the next
                                // ST_COUNT
    // wave-independent d = 64 sweep (k_search_mfma_sweep with W): the
    // reference side of every tile and block Score, centred on the centre
    // C_B of the leaf's block (subtree of 32 leaves), made once per search
    // by k_wsweep_prep; sw_abf == NULL selects the staged sweep.  Leaves are
    // padded to whole blocks.
    const uint16_t *sw_abf;  // [leaf][32 rows][h][s][8] bf16(-2 (r - C_B)), 0 past the leaf
    const float *sw_rn;      // [leaf][32] |r - C_B|^2 (FP32), +inf past the leaf
    const float *sw_rlen;    // [leaf] largest |r - C_B|, rounded up
    const uint16_t *sw_cbf;  // [leaf][h][s][8] bf16(-2 (C_L - C_B)), C_L the leaf's box centre
    const float *sw_cn;      // [leaf] |C_L - C_B|^2, +inf for empty or padding leaves
    const float *sw_lam;     // [leaf] lambda of the leaf, 0 for padding
    const float *sw_bcen;    // [block][DP] C_B
    const float *sw_rcb;     // [block] largest |C_L - C_B| of the block, rounded up
    uint32_t *wave_log;         // debug: 8 words per wave (ticks, scores, tiles, inserts, passes, leaf,
                                // staged tiles of the d = 64 sweep, candidates of the BF16 filters)
    // Score log of the debug kernel (launch_search_valu_debug_d3): one
    // record of kDbgWords words per Score call, or NULL; and the visit order
    // (0: nearer child first, 1: farther child first)
    uint32_t *dbg_log;
    unsigned int *dbg_count;  // records written (may exceed dbg_cap: then truncated)
    int dbg_cap;              // capacity in records
    int far_first;
    // tile list of the debug kernel: with tile_replay == 0 each wave records
    // the reference leaves it evaluates (tile_log[wave * tile_cap + i], the
    // count in tile_cnt[wave]); with tile_replay == 1 it evaluates exactly
    // those leaves in that order, without the walk
    uint32_t *tile_log;
    uint32_t *tile_cnt;
    int tile_cap;
    int tile_replay;
};

// Score-log record: node, kept (1/0), first query leaf of the wave, number
// of leaves of the wave, then the squared bound B(N_q)^2 of each leaf (as
// FP32 bits) at the time of the call
constexpr int kDbgWords = 12;
constexpr int kDbgMaxLeaves = kDbgWords - 4;

// per-dimension launchers (search_d*.hip): D computed dimensions (d for
// d <= 4, else d rounded up to 8, 16, 32 or 64 with zero padding); K is
// the compile-time list length
hipError_t launch_search_valu_d1(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_valu_d2(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_valu_d3(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_valu_d4(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_valu_d8(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_valu_d16(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_valu_d32(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_valu_d64(const SearchArgs &a, int K, int grid, hipStream_t s);
// the same with a seed radius (search_seeded_d*.hip)
hipError_t launch_search_valu_seeded_d1(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_valu_seeded_d2(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_valu_seeded_d3(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_valu_seeded_d4(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_valu_seeded_d8(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_valu_seeded_d16(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_valu_seeded_d32(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_valu_seeded_d64(const SearchArgs &a, int K, int grid, hipStream_t s);

// the d = 3 FP32 kernel with the Score log and the visit-order switch
// (search_debug_d3.hip); lists up to 16
hipError_t launch_search_valu_debug_d3(const SearchArgs &a, int K, int grid, hipStream_t s);

// the traversal kernel with BF16 matrix-core BaseCase tiles
// (search_mt_d*.hip): 16 or 32 computed dimensions, two query leaves per wave
// (lpl_log2 = 5), reference leaves of <= 32 points, K <= 16; the seeded form
// when a.seed is set
hipError_t launch_search_mt_d16(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_mt_d32(const SearchArgs &a, int K, int grid, hipStream_t s);

// reference leaves the d = 64 sweep scores together (one subtree)
constexpr int kSweepBlock = 32;

// reference-side operands of the wave-independent d = 64 sweep (see the
// sw_* fields): fills them for the n_blocks * 32 (padded) leaves of the
// reference tree in args
hipError_t launch_wsweep_prep(const SearchArgs &args, uint16_t *abf, float *rn, float *rlen,
                              uint16_t *cbf, float *cn, float *lam, float *bcen, float *rcb,
                              hipStream_t s);

// BF16 MFMA kernels (search_mfma_d*.hip), stride 16, 32 or 64
hipError_t launch_search_mfma_dp16(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_mfma_dp32(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_mfma_dp64(const SearchArgs &a, int K, int grid, hipStream_t s);

// zero n 32-bit words with a kernel (api.hip)
hipError_t zero_words(void *p, int64_t n, hipStream_t s);

// exclusive prefix sums (scan.hip): out[0] = 0, out[i + 1] = in[0] + ... +
// in[i] for 1 <= n <= kScanMax; tops is scratch of scan_scratch(n) values
constexpr int64_t kScanMax = int64_t(1) << 24;
int64_t scan_scratch(int64_t n);
hipError_t exclusive_scan(const int64_t *in, int64_t n, int64_t *out, int64_t *tops,
                          hipStream_t s);

// k-furthest-neighbour kernels (search_far_d*.hip), stride 4 .. 64, lists of
// 8, 16, 32 or 64
hipError_t launch_search_far_dp4(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_far_dp8(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_far_dp16(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_far_dp32(const SearchArgs &a, int K, int grid, hipStream_t s);
hipError_t launch_search_far_dp64(const SearchArgs &a, int K, int grid, hipStream_t s);

// compile-time list lengths; a request for a list of kk entries (k, or k+1
// when the query's own point shares the list) uses the smallest K >= kk
constexpr int kListSizes[] = {4, 5, 8, 10, 11, 16, 32, 50, 51, 64};
inline int list_size_for(int kk) {
    for (int K : kListSizes)
        if (K >= kk) return K;
    return -1;
}

}  // namespace knnx
