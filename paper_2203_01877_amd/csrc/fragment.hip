// Whole fragments: filter -> sort-based join -> group-by in one launch
// sequence, every intermediate in the workspace, no host synchronisation.
#include <cmath>
#include <type_traits>

#include "fragment.hpp"

namespace tqp {

// Group-key bits left to the bucket kernel: enough that the bits above them
// take one radix pass (a digit's worth of buckets), at most BUCKET_LOWB_MAX.
// Small slot tables go to 256-thread blocks, large ones to one 1024-thread
// block per CU.
int bucket_low_bits(int cb, int rb) {
    int lowb = cb - rb;
    if (lowb < 0) lowb = 0;
    if (lowb > BUCKET_LOWB_MAX) lowb = BUCKET_LOWB_MAX;
    return lowb;
}
constexpr int BUCKET_SMALL_LOWB = 9;
constexpr int64_t FLAGS_SIDE_MIN_DIM = 32768;   // dim rows from which the flags fragment's dim sort forks
// profile tags of the custkey fragment's three sorts
constexpr int SORT_TAG_FACT = 1, SORT_TAG_MID = 2, SORT_TAG_GROUP = 3;

// Low key bits the left sort of a join may leave out.  A join tile of TILE left rows
// over keys spread evenly on [0, 2^kb) spans about TILE * 2^kb / n key values
// plus one bucket of 2^s; both must fit the join's LDS table (RWIN), and the
// sorted high bits should fill whole radix passes.  Tiles that do not fit
// fall back to binary searches, so this is a cost choice, not a correctness
// condition.
int join_low_bits(int64_t n, int kb, int rb, int tile, int rwin) {
    if (n <= 0) return 0;
    const double spread = (double)tile * std::ldexp(1.0, kb) / (double)n;
    const double room = 0.85 * rwin - spread;
    if (room < 64) return 0;
    int smax = 0;
    while (smax + 1 <= kb && std::ldexp(1.0, smax + 1) <= room) ++smax;
    const int passes = (kb - smax + rb - 1) / rb;
    int s = kb - passes * rb;
    return s < 0 ? 0 : s;
}
int fact_low_bits(int64_t n, int kb, int rb) { return join_low_bits(n, kb, rb, JCfgFrag::TILE, JCfgFrag::RWIN); }

// Groups of the flags fragment in ascending packed-key order, skipping
// packed keys no row reached (SQL emits no empty group).
__global__ void k_flags_finalize(const int64_t* acc, const int64_t* d_join_in, tqp_flags_out o) {
    if (threadIdx.x != 0) return;
    int64_t g = 0;
    for (int k = 0; k < 6; ++k) {
        const int64_t s = acc[k * 3], c = acc[k * 3 + 1], p = acc[k * 3 + 2];
        if (c == 0) continue;
        o.key[g] = k;
        o.sum[g] = s;
        o.cnt[g] = c;
        o.avg[g] = (double)p / (double)c;
        ++g;
    }
    *o.d_ngroups = g;
    if (o.d_join) *o.d_join = *d_join_in;
}

template <class Cfg>
void flags_reserve(Arena& a, const tqp_flags_fragment& f, FlagsBufs<Cfg>& b) {
    const int kb = norm_key_bits(f.key_bits);
    // the fact sort covers the key bits above lowb (the join tiles resolve
    // the rest in LDS; at least one pass stays, which also drops the filtered
    // rows), the dim sort all of them
    b.lowb = join_low_bits(f.n_fact, kb, Cfg::RADIX_BITS, JCfgFrag::TILE, JCfgFrag::RWIN);
    b.lowb = b.lowb < kb - 1 ? b.lowb : kb - 1;
    b.fact = radix_reserve<Cfg, uint32_t>(a, f.n_fact, kb, b.lowb);
    b.dim = radix_reserve<Cfg, uint32_t>(a, f.n_dim, kb);
    b.join = join_reserve<JCfgFrag>(a, f.n_fact);
    b.d_join = a.zero<int64_t>(1);
    b.acc = a.zero<int64_t>(24);
    b.fkeys = a.scratch<uint32_t>(f.n_fact);
    b.fvals = a.scratch<uint32_t>(f.n_fact);
    b.dkeys = a.scratch<uint32_t>(f.n_dim);
    b.dvals = a.scratch<uint32_t>(f.n_dim);
}

template <class Cfg>
tqp_status flags_launch(tqp_ctx* ctx, const tqp_flags_fragment& f, const tqp_flags_out& o,
                        const FlagsBufs<Cfg>& b, hipStream_t s) {
    const int kb = norm_key_bits(f.key_bits);
    const uint32_t mask = key_mask_for(kb);
    tqp_status st;
    // dim side (seg == c fused into the sort, payload = dim row id) on the
    // side stream beside the fact side when it is big enough for the overlap
    // to outweigh the two stream events
    const bool fork = f.n_dim >= FLAGS_SIDE_MIN_DIM;
    const hipStream_t sd = fork ? ctx->side : s;
    if (fork && (st = side_fork(ctx, s)) != TQP_OK) return st;
    SrcFilterRowid<int8_t> dsrc{f.pk, f.seg, CMP_EQ, f.c, f.n_dim, 0};
    if ((st = radix_launch<Cfg, uint32_t>(b.dim, dsrc, f.n_dim, true, nullptr, mask, b.dkeys, b.dvals, ctx, sd)) !=
        TQP_OK)
        return st;
    // fact side: date < D fused into the sort, payload = global fact row id
    SrcFilterRowid<int32_t> fsrc{f.fk + f.row0, f.date + f.row0, CMP_LT, f.D, f.n_fact, f.row0};
    if ((st = radix_launch<Cfg, uint32_t>(b.fact, fsrc, f.n_fact, true, nullptr, mask, b.fkeys, b.fvals, ctx,
                                          s)) != TQP_OK)
        return st;
    if (fork && (st = side_join(ctx, s)) != TQP_OK) return st;
    // join + gather + direct aggregation over the six packed groups
    EmitFlagsAgg<JCfgFrag::BLOCK> e{};
    e.price = f.price;
    e.disc = f.disc;
    e.flagA = f.flagA;
    e.flagB = f.flagB;
    e.acc = b.acc;
    e.flags = ctx->d_err;
    if ((st = join_launch<JCfgFrag, uint32_t, uint32_t>(ctx, s, "join_flags_agg", b.join, b.fkeys, b.fvals, f.n_fact,
                                                        b.fact.d_cnt, b.dkeys, (const uint32_t*)nullptr, f.n_dim,
                                                        b.dim.d_cnt, b.d_join, INT64_MAX, e, b.lowb)) != TQP_OK)
        return st;
    TQP_LAUNCH(ctx, s, "flags_finalize", k_flags_finalize<<<1, 64, 0, s>>>(b.acc, b.d_join, o));
    return TQP_OK;
}

tqp_status check_flags(const tqp_flags_fragment* f, const tqp_flags_out* o) {
    if (!f || !o) return fail(TQP_ERR_INVALID, "null fragment or output");
    if (f->n_fact < 0 || f->n_dim < 0 || f->row0 < 0) return fail(TQP_ERR_INVALID, "negative size");
    if (f->n_fact > MAX_ELEMS || f->n_dim > MAX_ELEMS) return fail(TQP_ERR_UNSUPPORTED, "fragment too large");
    if (f->row0 + f->n_fact > (int64_t(1) << 31)) return fail(TQP_ERR_UNSUPPORTED, "fact row ids beyond int32");
    if ((f->n_fact && (!f->fk || !f->date || !f->price || !f->disc || !f->flagA || !f->flagB)) ||
        (f->n_dim && (!f->pk || !f->seg)))
        return fail(TQP_ERR_INVALID, "null column");
    if (!o->key || !o->sum || !o->cnt || !o->avg || !o->d_ngroups) return fail(TQP_ERR_INVALID, "null output");
    return TQP_OK;
}

template <class Cfg, class VT>
void cust_reserve(Arena& a, const tqp_cust_fragment& f, const tqp_cust_out& o, CustBufs<Cfg, VT>& b) {
    const int kb = norm_key_bits(f.key_bits);
    const int cb = norm_key_bits(f.cust_bits);
    // The join needs the fact keys sorted only on their bits above fact_lowb
    // when a join tile still spans a small key range: then the low digits are
    // never sorted.
    b.fact_lowb = fact_low_bits(f.n_fact, kb, Cfg::RADIX_BITS);
    if (b.fact_lowb > FINISH_LOG2) b.fact_lowb = FINISH_LOG2;      // the mid finishing pass covers at most this
    // the fused first pass keeps its look-back: pre-counting it costs the
    // histogram kernel more than the pass saves while the mid sort shares HBM
    b.fact = radix_reserve<Cfg, VT>(a, f.n_fact, kb, b.fact_lowb, false);
    // the mid keys: radix passes over the same high bits, then one finishing
    // pass sorts each span of 4096 keys in LDS (the join's binary-search
    // fallback needs them fully sorted) and records where each bucket of
    // 2^fact_lowb keys starts (the join tiles' windows)
    if (f.mid_sorted) {
        // the caller's mid keys are in order already: only the bucket starts
        // of the join windows are needed
        if (b.fact_lowb > 0) {
            b.nmbkt = ((int64_t(1) << kb) + (int64_t(1) << b.fact_lowb) - 1) >> b.fact_lowb;
            b.mbstart = a.scratch<int64_t>(b.nmbkt + 1);
        }
    } else {
        b.mid = radix_reserve<Cfg, uint32_t>(a, f.n_mid, kb, b.fact_lowb);
        if (b.fact_lowb > 0) {
            b.mkeys_full = a.scratch<uint32_t>(f.n_mid);
            b.mvals_full = a.scratch<uint32_t>(f.n_mid);
            b.nspans = ((int64_t(1) << kb) + FINISH_SPAN - 1) >> FINISH_LOG2;
            b.nmbkt = b.nspans << (FINISH_LOG2 - b.fact_lowb);
            b.mbstart = a.scratch<int64_t>(b.nmbkt + 1);
        }
        b.mkeys = a.scratch<uint32_t>(f.n_mid);
        b.mvals = a.scratch<uint32_t>(f.n_mid);
    }
    b.join = join_reserve<JCfgFrag>(a, f.n_fact);
    b.d_join = a.zero<int64_t>(1);
    // group-by: radix passes over the custkey bits above lowb, then one
    // bucket-aggregation block per value of those bits
    b.lowb = bucket_low_bits(cb, Cfg::RADIX_BITS);
    b.nbuckets = int64_t(1) << (cb - b.lowb);
    b.grp = radix_reserve<Cfg, VT>(a, f.join_cap, cb, b.lowb, false);
    b.sstatus = a.zero<uint64_t>(b.nbuckets);
    b.bstarts = a.scratch<int64_t>(b.nbuckets + 1);
    b.scounter = a.zero<uint32_t>(1);
    b.fkeys = a.scratch<uint32_t>(f.n_fact);
    b.fvals = a.scratch<VT>(f.n_fact);
    b.fmask = a.scratch<uint64_t>((f.n_fact + 63) / 64 + 1);
    b.gkeys_in = a.scratch<uint32_t>(f.join_cap);
    b.gvals_in = a.scratch<VT>(f.join_cap);
    b.gkeys = a.scratch<uint32_t>(f.join_cap);
    b.gvals = a.scratch<VT>(f.join_cap);
    // top-k candidates: the first k groups of every bucket (at most the groups)
    b.topk = topk_reserve(a, std::min<int64_t>(o.gcap, b.nbuckets * f.k), f.k);
}

template <class Cfg, class VT>
tqp_status cust_launch(tqp_ctx* ctx, const tqp_cust_fragment& f, const tqp_cust_out& o, const CustBufs<Cfg, VT>& b,
                       hipStream_t s) {
    const int kb = norm_key_bits(f.key_bits);
    const int cb = norm_key_bits(f.cust_bits);
    tqp_status st;
    const uint32_t* mk = reinterpret_cast<const uint32_t*>(f.pk);
    const uint32_t* mv = reinterpret_cast<const uint32_t*>(f.custkey);
    SrcKeyCol msrc{f.pk, f.custkey, f.n_mid};
    // fact side: date < D fused into the sort; the payload is the revenue
    // price * (100 - disc), evaluated while the row is read
    SrcFilterRevenue<VT, true> fsrc{f.fk, f.date, f.price, f.disc, CMP_LT, f.D, f.n_fact, b.fmask};
    // Two streams.  The mid sort's histogram and first pass run on the side
    // stream beside the fact histogram; the fused fact pass then runs alone
    // (it is the longest kernel, and sharing HBM cost it a third of its
    // speed); the mid's remaining passes and its finishing sort run beside
    // the second fact pass.
    if (f.mid_sorted) {
        // sorted by the caller: the start of every 2^fact_lowb-key bucket, one
        // search each, for the join windows
        if (b.fact_lowb > 0)
            TQP_LAUNCH(ctx, s, "mid_bucket_bounds",
                       k_bucket_bounds<<<grid_for(b.nmbkt + 1, 256, 0), 256, 0, s>>>(mk, f.n_mid, nullptr,
                                                                                     b.fact_lowb, b.nmbkt,
                                                                                     b.mbstart));
    } else {
        if ((st = side_fork(ctx, s)) != TQP_OK) return st;
        if ((st = radix_launch<Cfg, uint32_t, SORT_TAG_MID>(b.mid, msrc, f.n_mid, true, nullptr, key_mask_for(kb),
                                                            b.mkeys, b.mvals, ctx, ctx->side, "mid_pass_first",
                                                            "mid_pass", 0, 1)) != TQP_OK)
            return st;
    }
    if (b.fact.ntiles > 0) {
        // the fact histogram of every pass, and the filter as one bit per row
        using FC = typename Cfg::template ForVal<VT>;
        const int g = grid_for(f.n_fact, (int64_t)FC::BLOCK * HIST_ITEMS * 4, (int64_t)ctx->num_cus * 2);
        TQP_LAUNCH(ctx, s, "radix_hist",
                   (k_radix_hist<FC, SrcFilterRevenue<VT, true>><<<g, FC::BLOCK, 0, s>>>(
                       fsrc, b.fact.pd, key_mask_for(kb), b.fact.hist, b.fact.d_cnt, ctx->d_err)));
    }
    if (!f.mid_sorted && (st = side_join(ctx, s)) != TQP_OK) return st;
    if ((st = radix_launch<Cfg, VT, SORT_TAG_FACT>(b.fact, fsrc, f.n_fact, false, b.fact.d_cnt, key_mask_for(kb),
                                                   b.fkeys, b.fvals, ctx, s, "fact_pass_fused", "fact_pass", 0,
                                                   1)) != TQP_OK)
        return st;
    if (!f.mid_sorted) {
        if ((st = side_fork(ctx, s)) != TQP_OK) return st;
        if ((st = radix_launch<Cfg, uint32_t, SORT_TAG_MID>(b.mid, msrc, f.n_mid, true, nullptr, key_mask_for(kb),
                                                            b.mkeys, b.mvals, ctx, ctx->side, "mid_pass_first",
                                                            "mid_pass", 1)) != TQP_OK)
            return st;
        mk = b.mkeys;
        mv = b.mvals;
        if (b.fact_lowb > 0 && f.n_mid > 0) {
            // the join's fallback searches need the mid keys fully sorted:
            // finish the low bits span by span
            TQP_LAUNCH(ctx, ctx->side, "finish_sort",
                       k_finish_sort<<<(unsigned)b.nspans, FINISH_BLOCK, 0, ctx->side>>>(
                           b.mkeys, b.mvals, f.n_mid, b.mkeys_full, b.mvals_full, b.fact_lowb, b.mbstart));
            mk = b.mkeys_full;
            mv = b.mvals_full;
        }
    }
    if ((st = radix_launch<Cfg, VT, SORT_TAG_FACT>(b.fact, fsrc, f.n_fact, false, b.fact.d_cnt, key_mask_for(kb),
                                                   b.fkeys, b.fvals, ctx, s, "fact_pass_fused", "fact_pass",
                                                   1)) != TQP_OK)
        return st;
    if (!f.mid_sorted && (st = side_join(ctx, s)) != TQP_OK) return st;
    // join: emits (custkey, revenue); the bucket starts exist only for a
    // non-empty mid (an empty one gives empty windows by search)
    using Emit = EmitKeyVal<JCfgFrag::BLOCK, Cfg::RADIX_BITS, VT>;
    Emit e{};
    e.out_key = b.gkeys_in;
    e.out_val = b.gvals_in;
    e.cap = f.join_cap;
    e.key_mask = key_mask_for(cb);
    e.flags = ctx->d_err;
    e.hist = b.grp.hist;       // digit counts of the group-key sort, taken on the way out
    e.npass = b.grp.pd.npass;
    for (int p = 0; p < b.grp.pd.npass && p < Emit::NP; ++p) {
        e.shift[p] = b.grp.pd.shift[p];
        e.bits[p] = b.grp.pd.bits[p];
    }
    if ((st = join_launch<JCfgFrag, VT, uint32_t>(ctx, s, "join_keyval", b.join, b.fkeys, b.fvals, f.n_fact,
                                                  b.fact.d_cnt, mk, mv, f.n_mid, (const int64_t*)nullptr, b.d_join,
                                                  f.join_cap, e, b.fact_lowb, o.d_join,
                                                  f.n_mid > 0 ? b.mbstart : nullptr, b.nmbkt)) !=
        TQP_OK)
        return st;
    // group-by: sort (custkey, revenue) on the custkey bits above lowb (the
    // histogram came from the join), then aggregate each bucket
    SrcPairs<VT> gsrc{b.gkeys_in, b.gvals_in, f.join_cap, b.d_join};
    if ((st = radix_launch<Cfg, VT, SORT_TAG_GROUP>(b.grp, gsrc, f.join_cap, false, b.d_join, key_mask_for(cb),
                                                    b.gkeys, b.gvals, ctx, s, "group_pass", "group_pass")) !=
        TQP_OK)
        return st;
    SegOut so{o.key, o.sum, o.cnt, nullptr, o.gcap, o.d_ngroups};
    // bucket starts: with one group pass the buckets are its digits, so the
    // pass's histogram gives them; otherwise one search per bucket
    const uint32_t* bhist = b.grp.pd.npass == 1 ? b.grp.hist : nullptr;
    if (!bhist) {
        TQP_LAUNCH(ctx, s, "bucket_bounds",
                   k_bucket_bounds<<<grid_for(b.nbuckets + 1, 256, 0), 256, 0, s>>>(b.gkeys, f.join_cap, b.d_join,
                                                                                      b.lowb, b.nbuckets, b.bstarts));
    }
    // the aggregation reads int64 values, or 32-bit values known to be in [0, 2^32)
    using AV = typename std::conditional<sizeof(VT) == 8, int64_t, uint32_t>::type;
    const AV* gv = reinterpret_cast<const AV*>(b.gvals);
    if (b.lowb <= BUCKET_SMALL_LOWB) {
        TQP_LAUNCH(ctx, s, "bucket_agg",
                   (k_bucket_agg<256, 1 << BUCKET_SMALL_LOWB, AV><<<(unsigned)b.nbuckets, 256, 0, s>>>(
                       b.gkeys, gv, b.bstarts, bhist, b.lowb, b.nbuckets, b.sstatus, b.scounter, so, ctx->d_err,
                       b.topk.filtered, b.topk.d_nf, f.k)));
    } else {
        TQP_LAUNCH(ctx, s, "bucket_agg",
                   (k_bucket_agg<1024, 1 << BUCKET_LOWB_MAX, AV><<<(unsigned)b.nbuckets, 1024, 0, s>>>(
                       b.gkeys, gv, b.bstarts, bhist, b.lowb, b.nbuckets, b.sstatus, b.scounter, so, ctx->d_err,
                       b.topk.filtered, b.topk.d_nf, f.k)));
    }
    // ORDER BY sum DESC, custkey ASC LIMIT k, over the buckets' candidates
    if ((st = topk_launch_candidates(b.topk, o.cnt, f.k, o.top_key, o.top_sum, o.top_cnt, o.d_topk, s, ctx)) !=
        TQP_OK)
        return st;
    return TQP_OK;
}

tqp_status check_cust(const tqp_cust_fragment* f, const tqp_cust_out* o) {
    if (!f || !o) return fail(TQP_ERR_INVALID, "null fragment or output");
    if (f->n_fact < 0 || f->n_mid < 0 || f->join_cap < 0 || o->gcap < 0) return fail(TQP_ERR_INVALID, "negative size");
    if (f->n_fact > MAX_ELEMS || f->n_mid > MAX_ELEMS || f->join_cap > MAX_ELEMS || o->gcap > MAX_ELEMS)
        return fail(TQP_ERR_UNSUPPORTED, "fragment too large");
    if (f->k < 1 || f->k > 1024) return fail(TQP_ERR_UNSUPPORTED, "k = %d", f->k);
    if (f->revenue_bits != 0 && f->revenue_bits != 32 && f->revenue_bits != 64)
        return fail(TQP_ERR_UNSUPPORTED, "revenue_bits = %d (0, 32 or 64)", f->revenue_bits);
    if ((f->n_fact && (!f->fk || !f->date || !f->price || !f->disc)) || (f->n_mid && (!f->pk || !f->custkey)))
        return fail(TQP_ERR_INVALID, "null column");
    if (!o->key || !o->sum || !o->cnt || !o->d_ngroups || !o->top_key || !o->top_sum || !o->top_cnt || !o->d_topk)
        return fail(TQP_ERR_INVALID, "null output");
    return TQP_OK;
}

}  // namespace tqp

using namespace tqp;

extern "C" {

tqp_status tqp_fragment_flags(tqp_ctx* ctx, const tqp_flags_fragment* f, const tqp_flags_out* o, void* ws,
                              size_t* ws_bytes, hipStream_t stream) {
    clear_error();
    if (!ctx) return fail(TQP_ERR_INVALID, "null context");
    tqp_status st = check_flags(f, o);
    if (st != TQP_OK) return st;
    return with_radix_cfg(ctx->digit_bits, [&](auto cfg) -> tqp_status {
        using Cfg = decltype(cfg);
        FlagsBufs<Cfg> b;
        Arena a;
        auto plan = [&](Arena& ar) { flags_reserve<Cfg>(ar, *f, b); };
        tqp_status s2 = with_workspace(ctx, ws, ws_bytes, stream, plan, a);
        if (s2 != TQP_OK || !ws) return s2;
        if ((s2 = fill_zero(a.base, a.zsize, stream, ctx)) != TQP_OK) return s2;
        return flags_launch<Cfg>(ctx, *f, *o, b, stream);
    });
}

tqp_status tqp_fragment_cust_plan(tqp_ctx* ctx, const tqp_cust_fragment* f, int* fact_passes, int* fact_lowb,
                                  int* mid_passes, int* group_passes, int* group_lowb) {
    clear_error();
    if (!ctx || !f) return fail(TQP_ERR_INVALID, "null argument");
    return with_radix_cfg(ctx->digit_bits, [&](auto cfg) -> tqp_status {
        using Cfg = decltype(cfg);
        tqp_cust_out o{};
        CustBufs<Cfg, uint64_t> b;
        Arena a;
        cust_reserve<Cfg, uint64_t>(a, *f, o, b);
        if (fact_passes) *fact_passes = b.fact.pd.npass;
        if (fact_lowb) *fact_lowb = b.fact_lowb;
        if (mid_passes) *mid_passes = b.mid.pd.npass;
        if (group_passes) *group_passes = b.grp.pd.npass;
        if (group_lowb) *group_lowb = b.lowb;
        return TQP_OK;
    });
}

tqp_status tqp_fragment_cust(tqp_ctx* ctx, const tqp_cust_fragment* f, const tqp_cust_out* o, void* ws,
                             size_t* ws_bytes, hipStream_t stream) {
    clear_error();
    if (!ctx) return fail(TQP_ERR_INVALID, "null context");
    tqp_status st = check_cust(f, o);
    if (st != TQP_OK) return st;
    return with_radix_cfg(ctx->digit_bits, [&](auto cfg) -> tqp_status {
        using Cfg = decltype(cfg);
        auto run = [&](auto vt) -> tqp_status {
            using VT = decltype(vt);
            CustBufs<Cfg, VT> b;
            Arena a;
            auto plan = [&](Arena& ar) { cust_reserve<Cfg, VT>(ar, *f, *o, b); };
            tqp_status s2 = with_workspace(ctx, ws, ws_bytes, stream, plan, a);
            if (s2 != TQP_OK || !ws) return s2;
            if ((s2 = fill_zero(a.base, a.zsize, stream, ctx)) != TQP_OK) return s2;
            return cust_launch<Cfg, VT>(ctx, *f, *o, b, stream);
        };
        return f->revenue_bits == 32 ? run(uint32_t{}) : run(uint64_t{});
    });
}

}  // extern "C"
