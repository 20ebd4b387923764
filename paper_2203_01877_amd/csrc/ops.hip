// C ABI of the single operators: filter, sort, join, group-by, top-k.
#include "filter.hpp"
#include "fragment.hpp"
#include "host.hpp"
#include "join.hpp"
#include "radix.hpp"
#include "segreduce.hpp"
#include "topk.hpp"

namespace tqp {

// The sort-based group-by's bucket form: keys of at least this many bits,
// and buckets of this many rows on average (or at most 256 buckets).
constexpr int GB_BUCKET_MIN_BITS = 16;
constexpr int64_t GB_BUCKET_MIN_ROWS = 2048;

using JCfg = JoinCfg<256, 8, 4096>;
using SCfg = SegCfg<256, 16>;
constexpr int FILTER_BLOCK = 256, FILTER_ITEMS = 16;

// ---------------------------------------------------------------- top-k plan
// Chunk levels for the worst case (every group survives the filter): level l
// runs while its input n_l exceeds TOPK_DIRECT and leaves k per chunk of CH.
TopkBufs topk_reserve(Arena& a, int64_t n_upper, int k) {
    TopkBufs t;
    t.n_upper = n_upper;
    t.d_nf = a.zero<int64_t>(1);
    t.thr = a.scratch<int64_t>(1);
    t.filtered = a.scratch<TopCand>(n_upper > 0 ? n_upper : 1);
    int64_t n = n_upper;
    while (n > TOPK_DIRECT && t.levels < TOPK_MAX_LEVELS) {
        const int64_t b = (n + TOPK_CH - 1) / TOPK_CH;
        t.blocks[t.levels] = b;
        t.lvl.out[t.levels] = a.scratch<TopCand>(b * k);
        ++t.levels;
        n = b * k;
    }
    return t;
}

tqp_status topk_launch(const TopkBufs& t, const int32_t* key, const int64_t* sum, const int64_t* cnt,
                       const int64_t* d_n, int k, int32_t* out_key, int64_t* out_sum, int64_t* out_cnt,
                       int32_t* d_k, hipStream_t s, tqp_ctx* ctx) {
    TQP_LAUNCH(ctx, s, "topk_thresh",
               (k_topk_thresh<TOPK_BLOCK, TOPK_SAMPLE_PER><<<1, TOPK_BLOCK, 0, s>>>(sum, t.n_upper, d_n, k, t.thr)));
    TQP_LAUNCH(ctx, s, "topk_filter",
               k_topk_filter<<<grid_for(t.n_upper, 256 * 8, (int64_t)ctx->num_cus * 4), 256, 0, s>>>(
                   key, sum, t.n_upper, d_n, t.thr, t.filtered, t.d_nf));
    return topk_launch_candidates(t, cnt, k, out_key, out_sum, out_cnt, d_k, s, ctx);
}

tqp_status topk_launch_candidates(const TopkBufs& t, const int64_t* cnt, int k, int32_t* out_key,
                                  int64_t* out_sum, int64_t* out_cnt, int32_t* d_k, hipStream_t s, tqp_ctx* ctx) {
    for (int l = 0; l < t.levels; ++l) {
        TQP_LAUNCH(ctx, s, "topk_level",
                   (k_topk_level<TOPK_BLOCK, TOPK_CH><<<(unsigned)t.blocks[l], TOPK_BLOCK, 0, s>>>(
                       t.d_nf, l == 0 ? t.filtered : t.lvl.out[l - 1], t.lvl.out[l], k, l)));
    }
    TQP_LAUNCH(ctx, s, "topk_final",
               (k_topk_final<TOPK_BLOCK, TOPK_FINAL_PER><<<1, TOPK_BLOCK, 0, s>>>(t.d_nf, t.filtered, t.lvl, t.levels, k,
                                                                         cnt, out_key, out_sum, out_cnt, d_k)));
    return TQP_OK;
}

// Composite keys: the columns packed into one key, the first column most
// significant (Section 5.4 concatenates the group-by columns before the
// sort; Algorithm 3 compares several join-key columns).
constexpr int PACK_MAX_COLS = 4;
struct PackCols {
    const int32_t* col[PACK_MAX_COLS];
    int32_t bits[PACK_MAX_COLS];
    int32_t n;
};

__global__ void k_pack_keys(PackCols pc, int64_t n_upper, const int64_t* d_n, int32_t* out, uint32_t* flags) {
    int64_t n = n_upper;
    if (d_n) { const int64_t t = *d_n; n = t < n ? t : n; }
    uint32_t bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t v = 0;
#pragma unroll
        for (int c = 0; c < PACK_MAX_COLS; ++c) {
            if (c < pc.n) {
                const uint32_t x = (uint32_t)pc.col[c][i];
                const uint32_t lim_mask = (1u << pc.bits[c]) - 1;
                bad |= x & ~lim_mask;                        // negative values have the sign bit
                v = (v << pc.bits[c]) | (x & lim_mask);
            }
        }
        out[i] = (int32_t)v;
    }
    if (__any(bad != 0) && lane_id() == 0) set_flag(flags, FLAG_KEY_RANGE);
}

}  // namespace tqp

using namespace tqp;

extern "C" {

tqp_status tqp_filter(tqp_ctx* ctx, const tqp_column* cols, int ncols, int64_t n, const tqp_pred* preds,
                      int npreds, const int32_t* carry, int32_t* out_rowid, int32_t* out_carry, int64_t cap,
                      int64_t* d_count, void* ws, size_t* ws_bytes, hipStream_t stream) {
    clear_error();
    if (!ctx || !d_count || (cap > 0 && !out_rowid) || n < 0 || cap < 0 || npreds < 0 || ncols < 0)
        return fail(TQP_ERR_INVALID, "tqp_filter: null pointer or negative size");
    if (n > MAX_ELEMS) return fail(TQP_ERR_UNSUPPORTED, "tqp_filter: n = %lld", (long long)n);
    if (npreds > FILTER_MAX_PREDS) return fail(TQP_ERR_UNSUPPORTED, "tqp_filter: %d predicates", npreds);
    if (n > 0 && cap > 0 && (carry == nullptr) != (out_carry == nullptr))
        return fail(TQP_ERR_INVALID, "tqp_filter: carry and out_carry must both be given or both null");
    if (n == 0 || cap == 0) { carry = nullptr; out_carry = nullptr; }
    FilterPreds fp{};
    fp.np = npreds;
    for (int p = 0; p < npreds; ++p) {
        const tqp_pred& q = preds[p];
        if (q.col < 0 || q.col >= ncols || !cols || (n > 0 && !cols[q.col].data))
            return fail(TQP_ERR_INVALID, "tqp_filter: predicate %d names column %d", p, q.col);
        if (q.op < TQP_LT || q.op > TQP_NE) return fail(TQP_ERR_INVALID, "tqp_filter: op %d", q.op);
        const int t = cols[q.col].type;
        if (t != TQP_I8 && t != TQP_I32 && t != TQP_I64) return fail(TQP_ERR_INVALID, "tqp_filter: type %d", t);
        fp.col[p] = cols[q.col].data;
        fp.type[p] = t;
        fp.op[p] = q.op;
        fp.k[p] = q.k;
    }
    constexpr int TILE = FILTER_BLOCK * FILTER_ITEMS;
    const int64_t tiles = (n + TILE - 1) / TILE;
    uint64_t* status = nullptr;
    uint32_t* counter = nullptr;
    Arena a;
    auto plan = [&](Arena& ar) {
        status = ar.zero<uint64_t>(tiles);
        counter = ar.zero<uint32_t>(1);
    };
    tqp_status st = with_workspace(ctx, ws, ws_bytes, stream, plan, a);
    if (st != TQP_OK || !ws) return st;
    if ((st = fill_zero(a.base, a.zsize, stream, ctx)) != TQP_OK) return st;
    TQP_LAUNCH(ctx, stream, "filter",
               k_filter<FILTER_BLOCK, FILTER_ITEMS><<<grid_for(n, TILE, 0), FILTER_BLOCK, 0, stream>>>(
                   fp, n, carry, out_rowid, out_carry, cap, d_count, status, counter, ctx->d_err));
    return TQP_OK;
}

tqp_status tqp_sort(tqp_ctx* ctx, const int32_t* keys, const int32_t* vals, int64_t n, const int64_t* d_n,
                    int key_bits, int32_t* keys_out, int32_t* vals_out, void* ws, size_t* ws_bytes,
                    hipStream_t stream) {
    clear_error();
    if (!ctx || n < 0 || (n > 0 && (!keys || !keys_out)))
        return fail(TQP_ERR_INVALID, "tqp_sort: null pointer or n < 0");
    if (n > 0 && vals && !vals_out) return fail(TQP_ERR_INVALID, "tqp_sort: vals given without vals_out");
    if (n > MAX_ELEMS) return fail(TQP_ERR_UNSUPPORTED, "tqp_sort: n = %lld", (long long)n);
    const int kb = norm_key_bits(key_bits);
    const uint32_t mask = key_mask_for(kb);
    return with_radix_cfg(ctx->digit_bits, [&](auto cfg) -> tqp_status {
        using Cfg = decltype(cfg);
        Arena a;
        tqp_status st;
        if (vals_out) {
            RadixBufs<Cfg, uint32_t> b;
            auto plan = [&](Arena& ar) { b = radix_reserve<Cfg, uint32_t>(ar, n, kb); };
            st = with_workspace(ctx, ws, ws_bytes, stream, plan, a);
            if (st != TQP_OK || !ws) return st;
            if ((st = fill_zero(a.base, a.zsize, stream, ctx)) != TQP_OK) return st;
            if (!vals) {       // payload = input position
                SrcKeysIndex src{reinterpret_cast<const uint32_t*>(keys), n, d_n};
                return radix_launch<Cfg, uint32_t>(b, src, n, true, nullptr, mask,
                                                   reinterpret_cast<uint32_t*>(keys_out),
                                                   reinterpret_cast<uint32_t*>(vals_out), ctx, stream);
            }
            SrcPairs<uint32_t> src{reinterpret_cast<const uint32_t*>(keys),
                                   reinterpret_cast<const uint32_t*>(vals), n, d_n};
            return radix_launch<Cfg, uint32_t>(b, src, n, true, nullptr, mask,
                                               reinterpret_cast<uint32_t*>(keys_out),
                                               reinterpret_cast<uint32_t*>(vals_out), ctx, stream);
        }
        RadixBufs<Cfg, NoVal> b;
        auto plan = [&](Arena& ar) { b = radix_reserve<Cfg, NoVal>(ar, n, kb); };
        st = with_workspace(ctx, ws, ws_bytes, stream, plan, a);
        if (st != TQP_OK || !ws) return st;
        if ((st = fill_zero(a.base, a.zsize, stream, ctx)) != TQP_OK) return st;
        SrcPairs<NoVal> src{reinterpret_cast<const uint32_t*>(keys), nullptr, n, d_n};
        return radix_launch<Cfg, NoVal>(b, src, n, true, nullptr, mask, reinterpret_cast<uint32_t*>(keys_out),
                                        nullptr, ctx, stream);
    });
}

tqp_status tqp_join_kind(tqp_ctx* ctx, int kind, const int32_t* lkey, const int32_t* lrow, int64_t nl,
                         const int64_t* d_nl, const int32_t* rkey, const int32_t* rrow, int64_t nr,
                         const int64_t* d_nr, int32_t* out_l, int32_t* out_r, int64_t cap, int64_t* d_count,
                         void* ws, size_t* ws_bytes, hipStream_t stream) {
    clear_error();
    if (kind < TQP_JOIN_INNER || kind > TQP_JOIN_LEFT_OUTER)
        return fail(TQP_ERR_INVALID, "tqp_join_kind: kind %d", kind);
    const bool need_r = kind == TQP_JOIN_INNER || kind == TQP_JOIN_LEFT_OUTER;
    if (!ctx || !d_count || nl < 0 || nr < 0 || cap < 0 || (nl > 0 && !lkey) || (nr > 0 && !rkey) ||
        (cap > 0 && (!out_l || (need_r && !out_r))))
        return fail(TQP_ERR_INVALID, "tqp_join: null pointer or negative size");
    if (nl > MAX_ELEMS || nr > MAX_ELEMS) return fail(TQP_ERR_UNSUPPORTED, "tqp_join: input too large");
    JoinBufs b;
    Arena a;
    auto plan = [&](Arena& ar) { b = join_reserve<JCfg>(ar, nl); };
    tqp_status st = with_workspace(ctx, ws, ws_bytes, stream, plan, a);
    if (st != TQP_OK || !ws) return st;
    if ((st = fill_zero(a.base, a.zsize, stream, ctx)) != TQP_OK) return st;
    EmitPairs e{out_l, out_r, cap};
    const uint32_t* lk = reinterpret_cast<const uint32_t*>(lkey);
    const uint32_t* lp = reinterpret_cast<const uint32_t*>(lrow);
    const uint32_t* rk = reinterpret_cast<const uint32_t*>(rkey);
    const uint32_t* rp = reinterpret_cast<const uint32_t*>(rrow);
    auto run = [&](auto kc, const char* name) {
        return join_launch<JCfg, uint32_t, uint32_t, EmitPairs, decltype(kc)::value>(
            ctx, stream, name, b, lk, lp, nl, d_nl, rk, rp, nr, d_nr, d_count, cap, e);
    };
    switch (kind) {
        case TQP_JOIN_LEFT_SEMI: return run(std::integral_constant<int, JOIN_SEMI>{}, "join_semi");
        case TQP_JOIN_LEFT_ANTI: return run(std::integral_constant<int, JOIN_ANTI>{}, "join_anti");
        case TQP_JOIN_LEFT_OUTER: return run(std::integral_constant<int, JOIN_OUTER>{}, "join_outer");
        default: return run(std::integral_constant<int, JOIN_INNER>{}, "join_pairs");
    }
}

tqp_status tqp_join(tqp_ctx* ctx, const int32_t* lkey, const int32_t* lrow, int64_t nl, const int64_t* d_nl,
                    const int32_t* rkey, const int32_t* rrow, int64_t nr, const int64_t* d_nr, int32_t* out_l,
                    int32_t* out_r, int64_t cap, int64_t* d_count, void* ws, size_t* ws_bytes,
                    hipStream_t stream) {
    return tqp_join_kind(ctx, TQP_JOIN_INNER, lkey, lrow, nl, d_nl, rkey, rrow, nr, d_nr, out_l, out_r, cap,
                         d_count, ws, ws_bytes, stream);
}

tqp_status tqp_groupby_agg(tqp_ctx* ctx, const int32_t* gkey, int64_t n, const int64_t* d_n, int key_bits,
                           const int64_t* sum_in, const int64_t* avg_in, int32_t* out_key, int64_t* out_sum,
                           int64_t* out_cnt, double* out_avg, int64_t gcap, int64_t* d_ngroups, void* ws,
                           size_t* ws_bytes, hipStream_t stream) {
    clear_error();
    if (!ctx || !d_ngroups || n < 0 || gcap < 0 || (n > 0 && (!gkey || !sum_in)) ||
        (gcap > 0 && (!out_key || !out_sum || !out_cnt)))
        return fail(TQP_ERR_INVALID, "tqp_groupby_agg: null pointer or negative size");
    if (n == 0 && out_avg) avg_in = nullptr, out_avg = nullptr;
    if ((avg_in == nullptr) != (out_avg == nullptr))
        return fail(TQP_ERR_INVALID, "tqp_groupby_agg: avg_in and out_avg must both be given or both null");
    if (n > MAX_ELEMS) return fail(TQP_ERR_UNSUPPORTED, "tqp_groupby_agg: n = %lld", (long long)n);
    const int kb = norm_key_bits(key_bits);
    const uint32_t mask = key_mask_for(kb);
    if (!avg_in) {
        // Wide keys over many rows: Algorithm 2 with the last key bits
        // resolved in LDS (as the custkey fragment's group-by): the sort
        // covers the key bits above lowb, and one block per bucket of 2^lowb
        // keys sums and counts its rows in LDS and writes its groups in key
        // order.  Taken when the buckets hold enough rows to fill a block.
        const bool bucket = n > 0 && kb >= GB_BUCKET_MIN_BITS && [&] {
            const int lowb = bucket_low_bits(kb, ctx->digit_bits == 4 ? 4 : ctx->digit_bits == 11 ? 11 : 8);
            const int64_t nb = int64_t(1) << (kb - lowb);
            return nb <= 256 || nb * GB_BUCKET_MIN_ROWS <= n;
        }();
        if (bucket)
            return with_radix_cfg(ctx->digit_bits, [&](auto cfg) -> tqp_status {
                using Cfg = decltype(cfg);
                const int lowb = bucket_low_bits(kb, Cfg::RADIX_BITS);
                const int64_t nb = int64_t(1) << (kb - lowb);
                RadixBufs<Cfg, uint64_t> b;
                uint32_t* skeys = nullptr;
                uint64_t* svals = nullptr;
                int64_t* bstarts = nullptr;
                uint64_t* bstatus = nullptr;
                uint32_t* bcounter = nullptr;
                Arena a;
                auto plan = [&](Arena& ar) {
                    b = radix_reserve<Cfg, uint64_t>(ar, n, kb, lowb);
                    bstatus = ar.zero<uint64_t>(nb);
                    bcounter = ar.zero<uint32_t>(1);
                    bstarts = ar.scratch<int64_t>(nb + 1);
                    skeys = ar.scratch<uint32_t>(n);
                    svals = ar.scratch<uint64_t>(n);
                };
                tqp_status st = with_workspace(ctx, ws, ws_bytes, stream, plan, a);
                if (st != TQP_OK || !ws) return st;
                if ((st = fill_zero(a.base, a.zsize, stream, ctx)) != TQP_OK) return st;
                SrcPairs<uint64_t> src{reinterpret_cast<const uint32_t*>(gkey),
                                       reinterpret_cast<const uint64_t*>(sum_in), n, d_n};
                st = radix_launch<Cfg, uint64_t>(b, src, n, true, nullptr, mask, skeys, svals, ctx, stream);
                if (st != TQP_OK) return st;
                const uint32_t* bhist = b.pd.npass == 1 ? b.hist : nullptr;
                if (!bhist)
                    TQP_LAUNCH(ctx, stream, "groupby_bucket_bounds",
                               k_bucket_bounds<<<grid_for(nb + 1, 256, 0), 256, 0, stream>>>(skeys, n, b.d_cnt, lowb, nb,
                                                                                            bstarts));
                SegOut o{out_key, out_sum, out_cnt, nullptr, gcap, d_ngroups};
                TQP_LAUNCH(ctx, stream, "groupby_bucket_agg",
                           (k_bucket_agg<1024, 1 << BUCKET_LOWB_MAX, int64_t><<<(unsigned)nb, 1024, 0, stream>>>(
                               skeys, reinterpret_cast<const int64_t*>(svals), bstarts, bhist, lowb, nb, bstatus,
                               bcounter, o, ctx->d_err)));
                return TQP_OK;
            });
        // One value column: sort it alongside the keys (8-byte payload), so
        // the run reduction reads the values in order instead of gathering
        // them through the permutation.
        return with_radix_cfg(ctx->digit_bits, [&](auto cfg) -> tqp_status {
            using Cfg = decltype(cfg);
            RadixBufs<Cfg, uint64_t> b;
            uint32_t* skeys = nullptr;
            uint64_t* svals = nullptr;
            uint64_t* sstatus = nullptr;
            uint32_t* scounter = nullptr;
            const int64_t stiles = (n + SCfg::TILE - 1) / SCfg::TILE;
            Arena a;
            auto plan = [&](Arena& ar) {
                b = radix_reserve<Cfg, uint64_t>(ar, n, kb);
                sstatus = ar.zero<uint64_t>(stiles);
                scounter = ar.zero<uint32_t>(1);
                skeys = ar.scratch<uint32_t>(n);
                svals = ar.scratch<uint64_t>(n);
            };
            tqp_status st = with_workspace(ctx, ws, ws_bytes, stream, plan, a);
            if (st != TQP_OK || !ws) return st;
            if ((st = fill_zero(a.base, a.zsize, stream, ctx)) != TQP_OK) return st;
            if ((st = fill_zero(out_sum, gcap * 8, stream, ctx)) != TQP_OK) return st;
            if ((st = fill_zero(out_cnt, gcap * 8, stream, ctx)) != TQP_OK) return st;
            SrcPairs<uint64_t> src{reinterpret_cast<const uint32_t*>(gkey), reinterpret_cast<const uint64_t*>(sum_in),
                                   n, d_n};
            st = radix_launch<Cfg, uint64_t>(b, src, n, true, nullptr, mask, skeys, svals, ctx, stream);
            if (st != TQP_OK) return st;
            ValsDirect vs{reinterpret_cast<const int64_t*>(svals), nullptr};
            SegOut o{out_key, out_sum, out_cnt, nullptr, gcap, d_ngroups};
            TQP_LAUNCH(ctx, stream, "segreduce",
                       k_segreduce<SCfg, ValsDirect, false><<<grid_for(n, SCfg::TILE, 0), SCfg::BLOCK, 0, stream>>>(
                           skeys, vs, n, b.d_cnt, sstatus, scounter, o, ctx->d_err));
            return TQP_OK;
        });
    }
    return with_radix_cfg(ctx->digit_bits, [&](auto cfg) -> tqp_status {
        using Cfg = decltype(cfg);
        RadixBufs<Cfg, uint32_t> b;
        uint32_t* skeys = nullptr;
        uint32_t* perm = nullptr;
        int64_t* sa = nullptr;
        uint64_t* sstatus = nullptr;
        uint32_t* scounter = nullptr;
        const int64_t stiles = (n + SCfg::TILE - 1) / SCfg::TILE;
        Arena a;
        auto plan = [&](Arena& ar) {
            b = radix_reserve<Cfg, uint32_t>(ar, n, kb);
            sstatus = ar.zero<uint64_t>(stiles);
            scounter = ar.zero<uint32_t>(1);
            skeys = ar.scratch<uint32_t>(n);
            perm = ar.scratch<uint32_t>(n);
            sa = avg_in ? ar.scratch<int64_t>(gcap) : nullptr;
        };
        tqp_status st = with_workspace(ctx, ws, ws_bytes, stream, plan, a);
        if (st != TQP_OK || !ws) return st;
        if ((st = fill_zero(a.base, a.zsize, stream, ctx)) != TQP_OK) return st;
        if ((st = fill_zero(out_sum, gcap * 8, stream, ctx)) != TQP_OK) return st;
        if ((st = fill_zero(out_cnt, gcap * 8, stream, ctx)) != TQP_OK) return st;
        if (sa && (st = fill_zero(sa, gcap * 8, stream, ctx)) != TQP_OK) return st;
        // Algorithm 2: sort the keys and obtain the permutation (grpsInvIdx) ...
        SrcKeysIndex src{reinterpret_cast<const uint32_t*>(gkey), n, d_n};
        st = radix_launch<Cfg, uint32_t>(b, src, n, true, nullptr, mask, skeys, perm, ctx, stream);
        if (st != TQP_OK) return st;
        // ... then runs of equal keys and their aggregates, values read through the permutation.
        ValsGather vs{reinterpret_cast<const int32_t*>(perm), sum_in, avg_in};
        SegOut o{out_key, out_sum, out_cnt, sa, gcap, d_ngroups};
        TQP_LAUNCH(ctx, stream, "segreduce_gather",
                   k_segreduce<SCfg, ValsGather, true><<<grid_for(n, SCfg::TILE, 0), SCfg::BLOCK, 0, stream>>>(
                       skeys, vs, n, b.d_cnt, sstatus, scounter, o, ctx->d_err));
        if (avg_in) {
            TQP_LAUNCH(ctx, stream, "avg",
                       k_avg<<<grid_for(gcap, 256 * 4, 1024), 256, 0, stream>>>(sa, out_cnt, out_avg, d_ngroups,
                                                                                 gcap));
        }
        return TQP_OK;
    });
}

tqp_status tqp_topk(tqp_ctx* ctx, const int32_t* key, const int64_t* sum, const int64_t* cnt, int64_t n,
                    const int64_t* d_n, int k, int32_t* out_key, int64_t* out_sum, int64_t* out_cnt,
                    int32_t* d_k, void* ws, size_t* ws_bytes, hipStream_t stream) {
    clear_error();
    if (!ctx || !out_key || !out_sum || !out_cnt || !d_k || n < 0 || (n > 0 && (!key || !sum || !cnt)))
        return fail(TQP_ERR_INVALID, "tqp_topk: null pointer or n < 0");
    if (k < 1 || k > TOPK_K_MAX) return fail(TQP_ERR_UNSUPPORTED, "tqp_topk: k = %d", k);
    if (n > MAX_ELEMS) return fail(TQP_ERR_UNSUPPORTED, "tqp_topk: n = %lld", (long long)n);
    TopkBufs t;
    Arena a;
    auto plan = [&](Arena& ar) { t = topk_reserve(ar, n, k); };
    tqp_status st = with_workspace(ctx, ws, ws_bytes, stream, plan, a);
    if (st != TQP_OK || !ws) return st;
    if ((st = fill_zero(a.base, a.zsize, stream, ctx)) != TQP_OK) return st;
    return topk_launch(t, key, sum, cnt, d_n, k, out_key, out_sum, out_cnt, d_k, stream, ctx);
}

tqp_status tqp_pack_keys(tqp_ctx* ctx, const int32_t* const* cols, const int32_t* bits, int ncols, int64_t n,
                         const int64_t* d_n, int32_t* out, hipStream_t stream) {
    clear_error();
    if (!ctx || n < 0 || (n > 0 && (!cols || !bits || !out)))
        return fail(TQP_ERR_INVALID, "tqp_pack_keys: null pointer or negative size");
    if (ncols < 1 || ncols > PACK_MAX_COLS) return fail(TQP_ERR_UNSUPPORTED, "tqp_pack_keys: %d columns", ncols);
    PackCols pc{};
    pc.n = ncols;
    int total = 0;
    for (int c = 0; c < ncols; ++c) {
        if (bits[c] < 1 || bits[c] > 31) return fail(TQP_ERR_INVALID, "tqp_pack_keys: bits[%d] = %d", c, bits[c]);
        if (n > 0 && !cols[c]) return fail(TQP_ERR_INVALID, "tqp_pack_keys: column %d is null", c);
        pc.col[c] = cols[c];
        pc.bits[c] = bits[c];
        total += bits[c];
    }
    if (total > 31) return fail(TQP_ERR_UNSUPPORTED, "tqp_pack_keys: %d key bits (at most 31)", total);
    if (n > MAX_ELEMS) return fail(TQP_ERR_UNSUPPORTED, "tqp_pack_keys: n = %lld", (long long)n);
    if (n == 0) return TQP_OK;
    TQP_LAUNCH(ctx, stream, "pack_keys",
               k_pack_keys<<<grid_for(n, 256 * 4, (int64_t)ctx->num_cus * 8), 256, 0, stream>>>(pc, n, d_n, out,
                                                                                            ctx->d_err));
    return TQP_OK;
}

}  // extern "C"
