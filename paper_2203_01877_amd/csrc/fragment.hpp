// Workspace layouts of the fused fragments (shared by the single-fragment
// entry points and the batch runner).
#pragma once
#include "host.hpp"
#include "join.hpp"
#include "radix.hpp"
#include "segreduce.hpp"
#include "topk.hpp"

namespace tqp {

using JCfgFrag = JoinCfg<256, 8, 2048>;
using SCfgFrag = SegCfg<256, 16>;

// Join scratch: the R window of every left tile, the dynamic tile counter
// (aggregating emitters), and the per-tile and per-block output counts of
// the two-kernel join.
struct JoinBufs {
    int64_t tiles = 0;
    int64_t* win = nullptr;
    int64_t* tile_cnt = nullptr;
    int64_t* blk_total = nullptr;
    uint32_t* counter = nullptr;
};

template <class Cfg>
JoinBufs join_reserve(Arena& a, int64_t nl_upper) {
    JoinBufs b;
    b.tiles = (nl_upper + Cfg::TILE - 1) / Cfg::TILE;
    const int64_t t = b.tiles > 0 ? b.tiles : 1;
    b.counter = a.zero<uint32_t>(1);
    b.win = a.scratch<int64_t>(2 * b.tiles);
    b.tile_cnt = a.scratch<int64_t>(t);
    b.blk_total = a.scratch<int64_t>(t);       // the grid never exceeds the tile count
    return b;
}

// Emitters that write at output positions run the two-kernel join (per-tile
// counts, then the expansion, each block over the same contiguous range of
// tiles); aggregating emitters need only the join size and run the expansion
// directly.  Either way *d_count ends up holding the join size; for the
// aggregating form it must be zero on entry.
template <class Cfg, class LP, class RP, class Emit, int KIND = JOIN_INNER>
tqp_status join_launch(tqp_ctx* ctx, hipStream_t s, const char* name, const JoinBufs& b, const uint32_t* lkey,
                       const LP* lpay, int64_t nl, const int64_t* d_nl, const uint32_t* rkey, const RP* rpay,
                       int64_t nr, const int64_t* d_nr, int64_t* d_count, int64_t cap, const Emit& e,
                       int lowb = 0, int64_t* d_count_out = nullptr, const int64_t* rbstart = nullptr,
                       int64_t nbkt = 0) {
    const int64_t tiles = b.tiles;
    if (tiles > 0) {
        TQP_LAUNCH(ctx, s, "join_windows",
                   k_join_windows<<<grid_for(tiles, 256, 0), 256, 0, s>>>(lkey, nl, d_nl, rkey, nr, d_nr,
                                                                            Cfg::TILE, b.win, lowb, rbstart,
                                                                            nbkt));
    }
    // persistent blocks: as many as fit on the chip at once (both kernels
    // split the tiles over the same grid)
    static const int per_cu = [] {
        int a = 8, b = 8;
        if (Emit::ORDERED &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_join_count<Cfg, KIND>, Cfg::BLOCK, 0) != hipSuccess)
            a = 4;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_join<Cfg, LP, RP, Emit, KIND>, Cfg::BLOCK, 0) != hipSuccess)
            b = 4;
        const int m = a < b ? a : b;
        return m < 1 ? 1 : m > 8 ? 8 : m;
    }();
    const int grid = grid_for(tiles, 1, (int64_t)ctx->num_cus * per_cu);
    if (Emit::ORDERED && tiles > 0) {
        TQP_LAUNCH(ctx, s, "join_count",
                   k_join_count<Cfg, KIND><<<grid, Cfg::BLOCK, 0, s>>>(lkey, nl, d_nl, rkey, b.win, b.tile_cnt,
                                                                 b.blk_total, lowb));
    }
    TQP_LAUNCH(ctx, s, name,
               (k_join<Cfg, LP, RP, Emit, KIND><<<grid, Cfg::BLOCK, 0, s>>>(
                   lkey, lpay, nl, d_nl, rkey, rpay, b.win, b.counter, b.tile_cnt, b.blk_total, d_count,
                   d_count_out, cap, e, ctx->d_err, lowb)));
    return TQP_OK;
}

template <class Cfg>
struct FlagsBufs {
    RadixBufs<Cfg, uint32_t> fact, dim;
    int lowb = 0;              // fact key bits the fact sort leaves to the join tiles
    JoinBufs join;
    int64_t* d_join = nullptr;
    int64_t* acc = nullptr;
    uint32_t *fkeys = nullptr, *fvals = nullptr, *dkeys = nullptr, *dvals = nullptr;
};

// Top-k scratch: the sample threshold, the filtered candidates and their
// count, and the chunk levels over the candidates.  Each level keeps k of
// every CH candidates (k <= CH / 2, so a level at least halves the set); 32
// levels cover 2^30 groups.
struct TopkBufs {
    int levels = 0;            // chunk levels planned for the worst case
    int64_t n_upper = 0;
    int64_t blocks[TOPK_MAX_LEVELS] = {0};
    TopkLevels lvl = {};
    TopCand* filtered = nullptr;
    int64_t* d_nf = nullptr;
    int64_t* thr = nullptr;
};

TopkBufs topk_reserve(Arena& a, int64_t n_upper, int k);
tqp_status topk_launch(const TopkBufs& t, const int32_t* key, const int64_t* sum, const int64_t* cnt,
                       const int64_t* d_n, int k, int32_t* out_key, int64_t* out_sum, int64_t* out_cnt,
                       int32_t* d_k, hipStream_t s, tqp_ctx* ctx);
// Steps 3-4 only, over candidates already in t.filtered (count in *t.d_nf,
// at most t.n_upper), e.g. each group bucket's own first k.
tqp_status topk_launch_candidates(const TopkBufs& t, const int64_t* cnt, int k, int32_t* out_key,
                                  int64_t* out_sum, int64_t* out_cnt, int32_t* d_k, hipStream_t s, tqp_ctx* ctx);

template <class Cfg, class VT>
struct CustBufs {
    // VT: the revenue payload, uint64_t (int64 bits) or uint32_t (declared 32-bit revenue)
    RadixBufs<Cfg, VT> fact;
    int fact_lowb = 0;         // fact key bits left unsorted (the join resolves them)
    RadixBufs<Cfg, uint32_t> mid;
    RadixBufs<Cfg, VT> grp;
    int lowb = 0;              // group-key bits resolved in LDS by the bucket kernel
    int64_t nbuckets = 0;
    int64_t* bstarts = nullptr;    // start of every bucket, nbuckets + 1
    JoinBufs join;
    int64_t* d_join = nullptr;
    uint64_t* sstatus = nullptr;
    uint32_t* scounter = nullptr;
    uint32_t *fkeys = nullptr, *mkeys = nullptr, *mvals = nullptr, *gkeys_in = nullptr, *gkeys = nullptr;
    uint32_t *mkeys_full = nullptr, *mvals_full = nullptr;   // mid after the finishing pass (fact_lowb > 0)
    int64_t nspans = 0;                                       // 4096-key spans of the finishing pass
    int64_t* mbstart = nullptr;    // start of every 2^fact_lowb-key bucket in the finished mid keys
    int64_t nmbkt = 0;             // buckets (mbstart holds nmbkt + 1 entries)
    VT *fvals = nullptr, *gvals_in = nullptr, *gvals = nullptr;
    uint64_t* fmask = nullptr;     // date < D of every fact row, one bit each
    TopkBufs topk;
};

tqp_status check_flags(const tqp_flags_fragment* f, const tqp_flags_out* o);
// Low key bits a join's left sort may leave unsorted (the join resolves them
// in LDS) for n left rows of kb-bit keys, tiles of `tile` rows and LDS tables
// of `rwin` keys; the right side then needs the same high-bit passes plus the
// finishing pass.
int join_low_bits(int64_t n, int kb, int rb, int tile, int rwin);
// Group-key bits left to the bucket-aggregation kernel for cb-bit keys and
// rb-bit radix digits (the bits above them take one pass when cb <= rb + 13).
int bucket_low_bits(int cb, int rb);

// Batch preparation without any allocation: descriptor tables go into the
// workspace, uploaded on `stream` (or synchronously); only the configurations
// in cand_mask are planned.  Used by tqp_batch_create and by the server.
tqp_status batch_prepare(tqp_ctx* ctx, const tqp_flags_fragment* frags, const tqp_flags_out* outs, int nf,
                         int cand_mask, int chosen, void* ws, size_t* ws_bytes, hipStream_t stream, bool sync,
                         tqp_batch** out);
tqp_status batch_launch(tqp_batch* b, hipStream_t stream);
void batch_free(tqp_batch* b);
constexpr int BATCH_CONFIG_DEFAULT = 2;
__global__ void k_flags_finalize(const int64_t* acc, const int64_t* d_join_in, tqp_flags_out o);

}  // namespace tqp
