// Chains of sort-based equi-joins: multi-join plans such as the six-join
// query of Section 6.3, with the plan rules of Section 6.6 (the sort of a key
// column that is already in order is skipped; a key column that is exactly
// 0..M-1 in row order turns its join into a filter).
//
// Table 0's key column joins table 1's key, table 1's next key column joins
// table 2's, and so on.  A tuple is one row position per table joined so far.
// Hop t (t >= 1) joins the current tuples to table t:
//   1. the tuples' keys into table t are sorted with the tuple index as the
//      payload (radix sort at the hop's key width; as in the fused
//      fragments, the low key bits a join tile resolves in LDS are left
//      unsorted when that saves a pass);
//   2. table t's key column is sorted with its row positions, unless the
//      caller declares it sorted (then the positions are the indexes) or
//      dense (then no sort and no join: the key is its own row position, and
//      one pass keeps the tuples whose key lies in [0, M), writing their
//      positions, their row and the next key, steps 3 and 4 included; on the
//      first hop into a large table a radix pass over the keys' top digit
//      goes first, so that the next-key reads of a tile share a slice of
//      the table in L2 instead of each missing it);
//   3. the sort-based join gives (tuple index, row of table t) pairs;
//   4. one gather kernel reads the earlier position columns through the tuple
//      index (late materialisation) and the next hop's key through the new
//      row of table t.
// The hop into table 2 carries the tuples' two earlier positions through its
// sort instead (an 8-byte payload: both positions ride the radix passes, and
// the join writes them with the new row), so its output needs no gather of
// them: after the key sort the tuple order is a random permutation, and two
// random 4-byte reads per tuple cost more than 8 more bytes per element in
// each radix pass.  Later hops keep the tuple index (more positions than one
// payload holds).
// Every hop's size stays on the device and bounds the next hop's kernels
// (their grids come from the caller's capacities), so the whole chain is one
// launch sequence with no host synchronisation.
#include "fragment.hpp"

namespace tqp {
namespace {

using JCfgChain = JoinCfg<256, 8, 4096>;
constexpr int CH_FILTER_BLOCK = 256;
// The first dense hop reads the next key at random rows of its table; from
// this many table rows (4 MB of keys, an XCD's L2) and as many tuples, the
// tuples are first partitioned by the key's high bits, so that the reads of
// a tile fall in one slice of the table.
constexpr int64_t CH_PART_MIN_ROWS = int64_t(1) << 20;
constexpr int CH_GATHER_BLOCK = 256, CH_GATHER_ITEMS = 4;

// Sort source of the hop into table 2: the tuples' keys with both earlier
// positions as the payload (table 1's in the high word).
struct SrcKeysPos2 {
    const uint32_t* keys;
    const int32_t* pos0;
    const int32_t* pos1;
    int64_t n_upper;
    const int64_t* d_n;
    __device__ int64_t size() const {
        if (!d_n) return n_upper;
        const int64_t n = *d_n;
        return n < n_upper ? n : n_upper;
    }
    __device__ bool load_key(int64_t i, uint32_t& k) const {
        k = keys[i];
        return true;
    }
    __device__ bool load(int64_t i, uint32_t& k, uint64_t& v) const {
        k = keys[i];
        v = ((uint64_t)(uint32_t)pos1[i] << 32) | (uint32_t)pos0[i];
        return true;
    }
};

// Sort source of the first hop's partition pass (dense rule): the tuples
// whose key lies in [0, M), with their tuple index; the rest take no part.
struct SrcDenseKeys {
    const int32_t* keys;
    int64_t M;
    int64_t n_upper;
    const int64_t* d_n;
    __device__ int64_t size() const {
        if (!d_n) return n_upper;
        const int64_t n = *d_n;
        return n < n_upper ? n : n_upper;
    }
    __device__ bool load_key(int64_t i, uint32_t& k) const {
        const int32_t x = keys[i];
        k = (uint32_t)x;
        return x >= 0 && (int64_t)x < M;
    }
    __device__ bool load(int64_t i, uint32_t& k, uint32_t& v) const {
        v = (uint32_t)i;
        return load_key(i, k);
    }
};

// Join output of that hop: both carried positions and the new row.
struct EmitPos3 {
    static constexpr bool ORDERED = true;
    int32_t* out0;
    int32_t* out1;
    int32_t* out_r;
    int64_t cap;
    struct Smem {};
    __device__ void init(Smem&) {}
    __device__ void operator()(int64_t o, uint32_t, uint64_t lp, uint32_t rp, Smem&) {
        if (o < cap) {
            out0[o] = (int32_t)(uint32_t)lp;
            out1[o] = (int32_t)(uint32_t)(lp >> 32);
            out_r[o] = (int32_t)rp;
        }
    }
    __device__ void finish(Smem&) {}
};

struct ChainGather {
    const int32_t* src[TQP_CHAIN_MAX_TABLES];   // earlier position columns, read through li
    int32_t* dst[TQP_CHAIN_MAX_TABLES];
    int32_t ncols;
    const int32_t* key_src;                     // the next hop's key column, read through rr (nullable)
    int32_t* key_dst;
};

// dst[c][i] = src[c][li[i]] and key_dst[i] = key_src[rr[i]] for i below the
// hop's tuple count (at most n_upper).  Positions come from the hop's own
// join or filter, so they are in range.
__global__ void __launch_bounds__(CH_GATHER_BLOCK)
k_chain_gather(ChainGather g, const int32_t* li, const int32_t* rr, int64_t n_upper, const int64_t* d_n) {
    int64_t n = *d_n;
    n = n < n_upper ? n : n_upper;
    const int64_t step = (int64_t)gridDim.x * CH_GATHER_BLOCK * CH_GATHER_ITEMS;
    for (int64_t base = (int64_t)blockIdx.x * CH_GATHER_BLOCK * CH_GATHER_ITEMS; base < n; base += step) {
        int32_t l[CH_GATHER_ITEMS], r[CH_GATHER_ITEMS];
        bool in[CH_GATHER_ITEMS];
#pragma unroll
        for (int j = 0; j < CH_GATHER_ITEMS; ++j) {
            const int64_t i = base + (int64_t)j * CH_GATHER_BLOCK + threadIdx.x;
            in[j] = i < n;
            const int64_t ic = in[j] ? i : base;
            l[j] = li[ic];
            r[j] = rr[ic];
        }
        for (int c = 0; c < g.ncols; ++c) {
            int32_t v[CH_GATHER_ITEMS];
#pragma unroll
            for (int j = 0; j < CH_GATHER_ITEMS; ++j) v[j] = g.src[c][l[j]];
#pragma unroll
            for (int j = 0; j < CH_GATHER_ITEMS; ++j)
                if (in[j]) g.dst[c][base + (int64_t)j * CH_GATHER_BLOCK + threadIdx.x] = v[j];
        }
        if (g.key_src) {
            int32_t v[CH_GATHER_ITEMS];
#pragma unroll
            for (int j = 0; j < CH_GATHER_ITEMS; ++j) v[j] = g.key_src[r[j]];
#pragma unroll
            for (int j = 0; j < CH_GATHER_ITEMS; ++j)
                if (in[j]) g.key_dst[base + (int64_t)j * CH_GATHER_BLOCK + threadIdx.x] = v[j];
        }
    }
}

// A hop by the dense rule in one pass: the tuples whose key k lies in
// [0, M) are kept in order (ballot per 64 tuples, block scan, decoupled
// look-back, as the filter), each written as its earlier positions (carried
// columns, or the tuple index itself on the first hop), its row k of the
// table, and the next hop's key read at row k.
struct ChainDense {
    const int32_t* key;
    int64_t M;
    const int32_t* src[TQP_CHAIN_MAX_TABLES];   // earlier position columns, in tuple order
    int32_t* dst[TQP_CHAIN_MAX_TABLES];
    int32_t ncols;
    int32_t* index_dst;                         // the tuple index (first hop), nullable
    int32_t* row_dst;
    const int32_t* key_src;                     // the next hop's key column (nullable)
    int32_t* key_dst;
};

// Rows per thread of a dense hop carrying nc position columns: every column
// of a tile is held in registers from its load to its store, so the tile
// shrinks as the columns grow.
constexpr int dense_items(int nc) { return nc <= 3 ? 16 : nc <= 5 ? 8 : 4; }
constexpr int dense_cols(int h) { return h == 1 ? 0 : h; }

template <int BLOCK, int NC>
__global__ void __launch_bounds__(BLOCK)
k_chain_dense(ChainDense d, int64_t n, const int64_t* d_n, int64_t cap, int64_t* d_count, uint64_t* status,
              uint32_t* tile_counter, uint32_t* flags) {
    constexpr int ITEMS = dense_items(NC), TILE = BLOCK * ITEMS, W = BLOCK / WAVE;
    __shared__ int64_t s_wave[W];
    __shared__ int64_t s_base;
    __shared__ uint32_t s_tile;
    const int tid = threadIdx.x, w = tid / WAVE, l = lane_id();
    if (d_n) {                                 // tuples counted on the device, at most n
        const int64_t t = *d_n;
        n = t < n ? t : n;
    }
    if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t ntiles = (n + TILE - 1) / TILE;
    if (tile >= ntiles) {
        if (ntiles == 0 && tile == 0 && tid == 0) *d_count = 0;
        return;
    }
    const int64_t chunk = tile * TILE + (int64_t)w * ITEMS * WAVE;
    // the keys and the carried positions of the whole tile are loaded before
    // any of it is written, so all of the tile's reads are in flight at once.
    // The streamed columns are read and written with the non-temporal hint:
    // they pass through once, and the L2 keeps the table slice the next-key
    // reads fall in.
    int32_t k[ITEMS];
    int32_t v[NC > 0 ? NC : 1][ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = chunk + j * WAVE + l;
        k[j] = __builtin_nontemporal_load(&d.key[i < n ? i : n - 1]);   // n >= 1: the tile exists
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int64_t i = chunk + j * WAVE + l;
            v[c][j] = __builtin_nontemporal_load(&d.src[c][i < n ? i : n - 1]);
        }
    bool ok[ITEMS];
    uint64_t m[ITEMS];
    int64_t wc = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        ok[j] = chunk + j * WAVE + l < n && k[j] >= 0 && (int64_t)k[j] < d.M;
        m[j] = ballot(ok[j]);
        wc += popc64(m[j]);
    }
    // the next keys of the kept tuples, in flight while the tile looks back
    int32_t nk[ITEMS];
    if (d.key_src && d.M > 0) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) nk[j] = d.key_src[ok[j] ? k[j] : 0];
    }
    if (l == 0) s_wave[w] = wc;
    __syncthreads();
    if (w == 0) {
        int64_t tot = 0;
        for (int ww = 0; ww < W; ++ww) tot += s_wave[ww];
        const int64_t base = lookback64(status, tile, tot, flags);
        if (tid == 0) {
            int64_t run = 0;
            for (int ww = 0; ww < W; ++ww) { const int64_t x = s_wave[ww]; s_wave[ww] = run; run += x; }
            s_base = base;
            if (tile == ntiles - 1) {
                *d_count = base + tot;
                if (base + tot > cap) set_flag(flags, FLAG_CAPACITY);
            }
        }
    }
    __syncthreads();
    int64_t pos = s_base + s_wave[w];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t o = ok[j] ? pos + popc64(m[j] & lanemask_lt()) : -1;
        pos += popc64(m[j]);
        if (o >= 0 && o < cap) {
            __builtin_nontemporal_store(k[j], &d.row_dst[o]);
            if (d.index_dst) __builtin_nontemporal_store((int32_t)(chunk + j * WAVE + l), &d.index_dst[o]);
            if (d.key_src) __builtin_nontemporal_store(nk[j], &d.key_dst[o]);
#pragma unroll
            for (int c = 0; c < NC; ++c) __builtin_nontemporal_store(v[c][j], &d.dst[c][o]);
        }
    }
}

template <int NC>
tqp_status dense_launch(tqp_ctx* ctx, hipStream_t s, const ChainDense& d, int64_t n, const int64_t* d_n, int64_t cap,
                        int64_t* d_count, uint64_t* status, uint32_t* counter) {
    if (d.ncols != NC) {
        if constexpr (NC + 1 < TQP_CHAIN_MAX_TABLES)
            return dense_launch<NC + 1>(ctx, s, d, n, d_n, cap, d_count, status, counter);
        else
            return fail(TQP_ERR_INVALID, "tqp_join_chain: %d position columns in a dense hop", d.ncols);
    }
    constexpr int64_t TILE = (int64_t)CH_FILTER_BLOCK * dense_items(NC);
    TQP_LAUNCH(ctx, s, "chain_dense",
               (k_chain_dense<CH_FILTER_BLOCK, NC><<<grid_for(n, TILE, 0), CH_FILTER_BLOCK, 0, s>>>(
                   d, n, d_n, cap, d_count, status, counter, ctx->d_err)));
    return TQP_OK;
}

template <class Cfg>
struct HopBufs {
    bool dense = false, sorted = false;
    bool carry = false;                      // the hop into table 2: earlier positions ride the sort
    int64_t n_left = 0;                      // host bound on the tuples entering the hop
    RadixBufs<Cfg, uint32_t> lsort, rsort;
    RadixBufs<Cfg, uint64_t> lsort2;         // carry: the key sort with both positions
    int lowb = 0;                            // key bits the left sort leaves to the join tiles
    int64_t nbkt = 0;                        // 2^lowb-key buckets of the right keys
    int64_t* rbstart = nullptr;              // the start of every bucket in the sorted right keys
    uint64_t* lsv2 = nullptr;
    JoinBufs join;
    uint64_t* fstatus = nullptr;             // dense rule: the filter's look-back words
    uint32_t* fcounter = nullptr;
    bool part = false;                       // dense first hop: partition pass before the gather
    int part_bits = 0;
    RadixBufs<Cfg, uint32_t> psort;
    uint32_t* pk = nullptr;                  // partitioned keys and tuple indexes
    uint32_t* pv = nullptr;
    uint32_t *lsk = nullptr, *lsv = nullptr, *rsk = nullptr, *rsv = nullptr;
    int32_t* li = nullptr;                   // tuple index of every output tuple
    int64_t* d_cnt = nullptr;                // tuples after the hop
};

template <class Cfg>
struct ChainBufs {
    int hops = 0;
    HopBufs<Cfg> hop[TQP_CHAIN_MAX_TABLES];
    int32_t* cols[2][TQP_CHAIN_MAX_TABLES] = {};   // ping-pong position columns of the inner hops
    int32_t* key[2] = {};                          // ping-pong next-hop keys
};

template <class Cfg>
void chain_reserve(Arena& a, const tqp_chain_table* t, int nt, int64_t* d_count, ChainBufs<Cfg>& b) {
    const int H = nt - 1;
    b.hops = H;
    int64_t inner_cap = 0;
    for (int h = 1; h <= H; ++h) {
        HopBufs<Cfg>& hb = b.hop[h];
        const int kb = norm_key_bits(t[h].key_bits);
        hb.dense = t[h].rule == TQP_CHAIN_PK_DENSE;
        hb.sorted = t[h].rule == TQP_CHAIN_PK_SORTED;
        hb.n_left = h == 1 ? t[0].n_rows : t[h - 1].cap;
        if (hb.dense) {
            hb.part = h == 1 && h < H && t[h].n_rows >= CH_PART_MIN_ROWS && hb.n_left >= CH_PART_MIN_ROWS;
            if (hb.part) {
                // one radix pass over the top digit of the keys below M
                int pb = 1;
                while (pb < 31 && (int64_t(1) << pb) < t[h].n_rows) ++pb;
                hb.part_bits = pb;
                hb.psort = radix_reserve<Cfg, uint32_t>(a, hb.n_left, pb, pb > Cfg::RADIX_BITS ? pb - Cfg::RADIX_BITS : 0);
                hb.pk = a.scratch<uint32_t>(hb.n_left);
                hb.pv = a.scratch<uint32_t>(hb.n_left);
            }
            const int64_t tile = (int64_t)CH_FILTER_BLOCK * dense_items(hb.part ? 1 : dense_cols(h));
            const int64_t tiles = (hb.n_left + tile - 1) / tile;
            hb.fstatus = a.zero<uint64_t>(tiles);
            hb.fcounter = a.zero<uint32_t>(1);
        } else {
            hb.carry = h == 2;
            // as in the fused fragments: the left sort covers the key bits
            // above lowb and each join tile resolves the rest in LDS, its
            // window found from the right keys' bucket starts
            hb.lowb = join_low_bits(hb.n_left, kb, Cfg::RADIX_BITS, JCfgChain::TILE, JCfgChain::RWIN);
            if (hb.lowb > 0) {
                hb.nbkt = int64_t(1) << (kb - hb.lowb);
                hb.rbstart = a.scratch<int64_t>(hb.nbkt + 1);
            }
            if (hb.carry) {
                hb.lsort2 = radix_reserve<Cfg, uint64_t>(a, hb.n_left, kb, hb.lowb);
                hb.lsv2 = a.scratch<uint64_t>(hb.n_left);
            } else {
                hb.lsort = radix_reserve<Cfg, uint32_t>(a, hb.n_left, kb, hb.lowb);
                hb.lsv = a.scratch<uint32_t>(hb.n_left);
            }
            hb.lsk = a.scratch<uint32_t>(hb.n_left);
            if (!hb.sorted) {
                hb.rsort = radix_reserve<Cfg, uint32_t>(a, t[h].n_rows, kb);
                hb.rsk = a.scratch<uint32_t>(t[h].n_rows);
                hb.rsv = a.scratch<uint32_t>(t[h].n_rows);
            }
            hb.join = join_reserve<JCfgChain>(a, hb.n_left);
        }
        hb.li = a.scratch<int32_t>(t[h].cap);
        hb.d_cnt = h == H ? d_count : a.zero<int64_t>(1);
        if (h < H && t[h].cap > inner_cap) inner_cap = t[h].cap;
    }
    for (int s = 0; s < 2; ++s) {
        for (int u = 0; u < H; ++u) b.cols[s][u] = a.scratch<int32_t>(inner_cap);
        b.key[s] = a.scratch<int32_t>(inner_cap);
    }
}

template <class Cfg>
tqp_status chain_launch(tqp_ctx* ctx, const tqp_chain_table* t, int nt, int32_t* const* out_rows,
                        const ChainBufs<Cfg>& b, hipStream_t s) {
    const int H = nt - 1;
    tqp_status st;
    const int32_t* cur = t[0].key_out;              // the tuples' keys into the next table
    const int64_t* d_prev = nullptr;                // tuples entering the hop (device), null: all of table 0
    int32_t* const* prev_cols = nullptr;
    for (int h = 1; h <= H; ++h) {
        const HopBufs<Cfg>& hb = b.hop[h];
        const int kb = norm_key_bits(t[h].key_bits);
        const uint32_t mask = key_mask_for(kb);
        int32_t* const* dst = h == H ? out_rows : b.cols[h & 1];
        // hop 1: the tuple index is table 0's row position, so it goes to its column directly
        int32_t* li = h == 1 ? dst[0] : hb.li;
        int32_t* rr = dst[h];
        int32_t* next_key = b.key[h & 1];
        if (hb.dense) {
            ChainDense d{};
            d.key = cur;
            d.M = t[h].n_rows;
            if (h == 1) {
                d.index_dst = dst[0];
            } else {
                d.ncols = dense_cols(h);
                for (int u = 0; u < h; ++u) {
                    d.src[u] = prev_cols[u];
                    d.dst[u] = dst[u];
                }
            }
            d.row_dst = rr;
            if (h < H) {
                d.key_src = t[h].key_out;
                d.key_dst = next_key;
            }
            const int64_t* dn = d_prev;
            if (hb.part) {
                // the kept tuples partitioned by their key's top digit (the
                // tuple index as the payload), then the pass below reads them
                // in that order: its index becomes the carried position
                SrcDenseKeys psrc{cur, t[h].n_rows, hb.n_left, d_prev};
                if ((st = radix_launch<Cfg, uint32_t>(hb.psort, psrc, hb.n_left, true, nullptr,
                                                      key_mask_for(hb.part_bits), hb.pk, hb.pv, ctx, s,
                                                      "chain_dense_part", "chain_dense_part")) != TQP_OK)
                    return st;
                d.key = reinterpret_cast<const int32_t*>(hb.pk);
                d.index_dst = nullptr;
                d.ncols = 1;
                d.src[0] = reinterpret_cast<const int32_t*>(hb.pv);
                d.dst[0] = dst[0];
                dn = hb.psort.d_cnt;
            }
            if ((st = dense_launch<0>(ctx, s, d, hb.n_left, dn, t[h].cap, hb.d_cnt, hb.fstatus, hb.fcounter)) != TQP_OK)
                return st;
            cur = next_key;
            d_prev = hb.d_cnt;
            prev_cols = dst;
            continue;
        } else {
            if (hb.carry) {
                SrcKeysPos2 lsrc{reinterpret_cast<const uint32_t*>(cur), prev_cols[0], prev_cols[1], hb.n_left, d_prev};
                if ((st = radix_launch<Cfg, uint64_t>(hb.lsort2, lsrc, hb.n_left, true, nullptr, mask, hb.lsk, hb.lsv2,
                                                      ctx, s, "chain_sort_left", "chain_sort_left")) != TQP_OK)
                    return st;
            } else {
                SrcKeysIndex lsrc{reinterpret_cast<const uint32_t*>(cur), hb.n_left, d_prev};
                if ((st = radix_launch<Cfg, uint32_t>(hb.lsort, lsrc, hb.n_left, true, nullptr, mask, hb.lsk, hb.lsv,
                                                      ctx, s, "chain_sort_left", "chain_sort_left")) != TQP_OK)
                    return st;
            }
            const uint32_t* rk = reinterpret_cast<const uint32_t*>(t[h].key_pk);
            const uint32_t* rp = nullptr;           // sorted by the caller: the positions are the indexes
            if (!hb.sorted) {
                SrcKeysIndex rsrc{reinterpret_cast<const uint32_t*>(t[h].key_pk), t[h].n_rows, nullptr};
                if ((st = radix_launch<Cfg, uint32_t>(hb.rsort, rsrc, t[h].n_rows, true, nullptr, mask, hb.rsk,
                                                      hb.rsv, ctx, s, "chain_sort_right", "chain_sort_right")) !=
                    TQP_OK)
                    return st;
                rk = hb.rsk;
                rp = hb.rsv;
            }
            // the start of every 2^lowb-key bucket of the sorted right keys
            // (an empty right side gives empty windows by search)
            const int64_t* rbstart = hb.lowb > 0 && t[h].n_rows > 0 ? hb.rbstart : nullptr;
            if (rbstart)
                TQP_LAUNCH(ctx, s, "chain_bucket_bounds",
                           k_bucket_bounds<<<grid_for(hb.nbkt + 1, 256, 0), 256, 0, s>>>(rk, t[h].n_rows, nullptr,
                                                                                          hb.lowb, hb.nbkt,
                                                                                          hb.rbstart));
            // left elements that took part in the sort: the histogram's count
            if (hb.carry) {
                EmitPos3 e{dst[0], dst[1], rr, t[h].cap};
                if ((st = join_launch<JCfgChain, uint64_t, uint32_t, EmitPos3>(
                         ctx, s, "chain_join", hb.join, hb.lsk, hb.lsv2, hb.n_left, hb.lsort2.d_cnt, rk, rp,
                         t[h].n_rows, nullptr, hb.d_cnt, t[h].cap, e, hb.lowb, nullptr, rbstart, hb.nbkt)) != TQP_OK)
                    return st;
            } else {
                EmitPairs e{li, rr, t[h].cap};
                if ((st = join_launch<JCfgChain, uint32_t, uint32_t, EmitPairs>(
                         ctx, s, "chain_join", hb.join, hb.lsk, hb.lsv, hb.n_left, hb.lsort.d_cnt, rk, rp,
                         t[h].n_rows, nullptr, hb.d_cnt, t[h].cap, e, hb.lowb, nullptr, rbstart, hb.nbkt)) != TQP_OK)
                    return st;
            }
        }
        // earlier position columns through the tuple index, the next key through the new row
        ChainGather g{};
        g.ncols = h == 1 || hb.carry ? 0 : h;      // hop 1: the tuple index is the row; carry: written by the join
        for (int u = 0; u < g.ncols; ++u) {
            g.src[u] = prev_cols[u];
            g.dst[u] = dst[u];
        }
        if (h < H) {
            g.key_src = t[h].key_out;
            g.key_dst = next_key;
        }
        if (g.ncols > 0 || g.key_src) {
            const int grid = grid_for(t[h].cap, (int64_t)CH_GATHER_BLOCK * CH_GATHER_ITEMS, (int64_t)ctx->num_cus * 16);
            TQP_LAUNCH(ctx, s, "chain_gather",
                       k_chain_gather<<<grid, CH_GATHER_BLOCK, 0, s>>>(g, li, rr, t[h].cap, hb.d_cnt));
        }
        cur = next_key;
        d_prev = hb.d_cnt;
        prev_cols = dst;
    }
    return TQP_OK;
}

tqp_status check_chain(const tqp_chain_table* t, int nt, int32_t* const* out_rows, const int64_t* d_count) {
    if (!t || !out_rows || !d_count) return fail(TQP_ERR_INVALID, "tqp_join_chain: null argument");
    if (nt < 2 || nt > TQP_CHAIN_MAX_TABLES)
        return fail(TQP_ERR_UNSUPPORTED, "tqp_join_chain: %d tables (2..%d)", nt, TQP_CHAIN_MAX_TABLES);
    for (int u = 0; u < nt; ++u) {
        if (t[u].n_rows < 0 || (u > 0 && t[u].cap < 0))
            return fail(TQP_ERR_INVALID, "tqp_join_chain: table %d: negative size", u);
        if (t[u].n_rows > MAX_ELEMS || (u > 0 && t[u].cap > MAX_ELEMS))
            return fail(TQP_ERR_UNSUPPORTED, "tqp_join_chain: table %d: too large", u);
        if (u + 1 < nt && t[u].n_rows > 0 && !t[u].key_out)
            return fail(TQP_ERR_INVALID, "tqp_join_chain: table %d has no outgoing key column", u);
        if (u > 0 && t[u].n_rows > 0 && !t[u].key_pk && t[u].rule != TQP_CHAIN_PK_DENSE)
            return fail(TQP_ERR_INVALID, "tqp_join_chain: table %d has no key column", u);
        if (u > 0 && t[u].rule != 0 && t[u].rule != TQP_CHAIN_PK_SORTED && t[u].rule != TQP_CHAIN_PK_DENSE)
            return fail(TQP_ERR_INVALID, "tqp_join_chain: table %d: rule %d", u, t[u].rule);
        if (t[nt - 1].cap > 0 && !out_rows[u])
            return fail(TQP_ERR_INVALID, "tqp_join_chain: no output column for table %d", u);
    }
    return TQP_OK;
}

}  // namespace
}  // namespace tqp

using namespace tqp;

extern "C" tqp_status tqp_join_chain(tqp_ctx* ctx, const tqp_chain_table* tables, int ntables,
                                     int32_t* const* out_rows, int64_t* d_count, void* ws, size_t* ws_bytes,
                                     hipStream_t stream) {
    clear_error();
    if (!ctx) return fail(TQP_ERR_INVALID, "tqp_join_chain: null context");
    tqp_status st = check_chain(tables, ntables, out_rows, d_count);
    if (st != TQP_OK) return st;
    return with_radix_cfg(ctx->digit_bits, [&](auto cfg) -> tqp_status {
        using Cfg = decltype(cfg);
        ChainBufs<Cfg> b;
        Arena a;
        auto plan = [&](Arena& ar) { chain_reserve<Cfg>(ar, tables, ntables, d_count, b); };
        tqp_status s2 = with_workspace(ctx, ws, ws_bytes, stream, plan, a);
        if (s2 != TQP_OK || !ws) return s2;
        if ((s2 = fill_zero(a.base, a.zsize, stream, ctx)) != TQP_OK) return s2;
        return chain_launch<Cfg>(ctx, tables, ntables, out_rows, b, stream);
    });
}
