// General fragments (tqp_fragment_run): the operators of Section 5 composed
// by a descriptor instead of the two fixed fragment shapes.
//
//   1. predicates  Section 5.1's expressions: each side's predicate program is
//                  evaluated once into a keep byte per row (tqp_eval's kernel);
//   2. join        Algorithm 1: both key columns radix-sorted with their row
//                  ids, the keep column fused into the sort's first pass so
//                  dropped rows are never written; the sort-based join gives
//                  (fact row, dim row) pairs (late materialisation).  As in
//                  the fused fragments, the sorts leave the low key bits a
//                  join tile resolves in LDS unsorted on the fact side, and
//                  the dim side gets the same high-bit passes plus one
//                  finishing pass per 4096-key span.  Without a join the kept
//                  fact rows are compacted instead;
//      Two plan rules of the hand-optimised plans (Section 6.6) carry what
//      the join's output needs through the key sorts instead of row ids: when
//      the only use of the fact rows after the join is one aggregate's value
//      program over fact columns, the program runs over the fact rows in
//      order before the sort and its value rides the sort (8-byte payload);
//      when the only use of the dim rows is one int32 group column, that
//      column rides the dim sort.  The join then emits those values directly
//      and nothing is read through row ids (the fused fragments' layout);
//   3. group key   the group columns read through the pairs and packed into
//                  one key (Algorithm 2's concatenated group columns);
//   4. values      every aggregate's program evaluated over the joined rows,
//                  its columns read through the pairs;
//   5. group sort  Algorithm 2: the packed keys radix-sorted with the
//                  joined-row index; for COUNT(DISTINCT v) the rows are first
//                  sorted by v (two 32-bit passes) so the final stable sort
//                  orders them by (key, v).  When one aggregate alone has a
//                  value (the others COUNT) and none is COUNT(DISTINCT), the
//                  value itself rides the sort as an 8-byte payload instead,
//                  so the reduction reads it in order;
//   6. runs        the first row of every run of equal keys compacted into the
//                  group starts (a ballot per 64 rows and a decoupled
//                  look-back), then every run reduced: sum, count, min, max,
//                  average and the number of value changes (distinct values).
//                  A wave takes 64 consecutive groups: each lane reduces its
//                  own group when every one of them is short, and the whole
//                  wave reduces each long one;
//   7. top-k       ORDER BY the first aggregate DESC, key ASC LIMIT k, as
//                  tqp_topk.
// Every size after step 1 (kept rows, joined rows, groups) stays on the
// device: the grids come from the caller's bounds and the kernels read the
// counts.
#include "filter.hpp"
#include "fragment.hpp"

namespace tqp {
namespace {

using JCfgGen = JoinCfg<256, 8, 4096>;
constexpr int GF_FILTER_BLOCK = 256, GF_FILTER_ITEMS = 16;
constexpr int GF_HEAD_BLOCK = 256, GF_HEAD_ITEMS = 8;
constexpr int GF_AGG_BLOCK = 256;
constexpr int GF_MAX_COLS = 64;
// Group keys of at least this many bits take the bucket group-by (when it
// applies): a bucket then holds 2^8 or more keys, enough slots that a block's
// LDS updates rarely meet on one.
constexpr int GF_BUCKET_MIN_BITS = 16;
// Group keys of at most this many bits (no COUNT(DISTINCT)) take the direct
// group-by: every block reduces its rows into an LDS slot per (aggregate,
// key), with no group sort (Algorithm 2's runs are then whole key values).
constexpr int GF_DIRECT_MAX_BITS = 9;
constexpr int GF_DIRECT_BLOCK = 256;
constexpr int GF_DIRECT_PARTS = 256;    // its blocks (each writes one part of the slots)
constexpr int64_t GF_LORDER_MIN_BYTES = int64_t(256) << 20;   // MI355X's infinity cache

// Sort source: the int32 key column with the row id as payload, rows whose
// keep byte is zero left out (keep null: every row).
struct SrcKeepRow {
    const int32_t* key;
    const uint8_t* keep;
    int64_t n;
    __device__ int64_t size() const { return n; }
    __device__ bool load_key(int64_t i, uint32_t& k) const {
        k = (uint32_t)key[i];
        return keep ? keep[i] != 0 : true;
    }
    __device__ bool load(int64_t i, uint32_t& k, uint32_t& v) const {
        k = (uint32_t)key[i];
        v = (uint32_t)i;
        return keep ? keep[i] != 0 : true;
    }
};

// Sort sources that carry a value instead of the row id: a precomputed int64
// per row (the fact value program), or an int32 column (the dim group column).
struct SrcKeepVal64 {
    const int32_t* key;
    const uint8_t* keep;
    const int64_t* val;
    int64_t n;
    __device__ int64_t size() const { return n; }
    __device__ bool load_key(int64_t i, uint32_t& k) const {
        k = (uint32_t)key[i];
        return keep ? keep[i] != 0 : true;
    }
    __device__ bool load(int64_t i, uint32_t& k, uint64_t& v) const {
        k = (uint32_t)key[i];
        v = (uint64_t)val[i];
        return keep ? keep[i] != 0 : true;
    }
};
struct SrcKeepCol {
    const int32_t* key;
    const uint8_t* keep;
    const int32_t* col;
    int64_t n;
    __device__ int64_t size() const { return n; }
    __device__ bool load_key(int64_t i, uint32_t& k) const {
        k = (uint32_t)key[i];
        return keep ? keep[i] != 0 : true;
    }
    __device__ bool load(int64_t i, uint32_t& k, uint32_t& v) const {
        k = (uint32_t)key[i];
        v = (uint32_t)col[i];
        return keep ? keep[i] != 0 : true;
    }
};

// Join output with a carried fact value: (value, dim row or carried dim value).
struct EmitValRow {
    static constexpr bool ORDERED = true;
    int64_t* out_v;
    int32_t* out_r;
    int64_t cap;
    struct Smem {};
    __device__ void init(Smem&) {}
    __device__ void operator()(int64_t o, uint32_t, uint64_t lp, uint32_t rp, Smem&) {
        if (o < cap) {
            out_v[o] = (int64_t)lp;
            out_r[o] = (int32_t)rp;
        }
    }
    __device__ void finish(Smem&) {}
};

// Sort source over the joined rows: row j = perm[i] (or i), key from an
// int32 array (MODE 0), the low word of an int64 array (MODE 1) or its high
// word with the sign bit flipped (MODE 2, so unsigned order is signed order);
// the payload is j.
template <int MODE>
struct SrcPermKey {
    const void* base;
    const uint32_t* perm;
    int64_t n_upper;
    const int64_t* d_n;
    __device__ int64_t size() const {
        const int64_t n = *d_n;
        return n < n_upper ? n : n_upper;
    }
    __device__ uint32_t key_of(int64_t j) const {
        if constexpr (MODE == 0) return static_cast<const uint32_t*>(base)[j];
        else if constexpr (MODE == 1) return (uint32_t)static_cast<const uint64_t*>(base)[j];
        else return (uint32_t)(static_cast<const uint64_t*>(base)[j] >> 32) ^ 0x80000000u;
    }
    __device__ bool load_key(int64_t i, uint32_t& k) const {
        k = key_of(perm ? (int64_t)perm[i] : i);
        return true;
    }
    __device__ bool load(int64_t i, uint32_t& k, uint32_t& v) const {
        const uint32_t j = perm ? perm[i] : (uint32_t)i;
        k = key_of(j);
        v = j;
        return true;
    }
};

// Sort source over the joined rows: the packed key with the one valued
// aggregate's value as the payload.
struct SrcKeyVal64 {
    const uint32_t* key;
    const int64_t* val;
    int64_t n_upper;
    const int64_t* d_n;
    __device__ int64_t size() const {
        const int64_t n = *d_n;
        return n < n_upper ? n : n_upper;
    }
    __device__ bool load_key(int64_t i, uint32_t& k) const {
        k = key[i];
        return true;
    }
    __device__ bool load(int64_t i, uint32_t& k, uint64_t& v) const {
        k = key[i];
        v = (uint64_t)val[i];
        return true;
    }
};

// The group sort's source when the one group column rode the dim sort: the
// key is that column's value (the join wrote it where the dim row would be),
// given whole to the histogram, which raises the key-range flag for a value
// outside the key width, and masked to the width for the passes.
struct SrcColKeyVal64 {
    const int32_t* key;
    const int64_t* val;
    int64_t n_upper;
    const int64_t* d_n;
    uint32_t mask;
    __device__ int64_t size() const {
        const int64_t n = *d_n;
        return n < n_upper ? n : n_upper;
    }
    __device__ bool load_key(int64_t i, uint32_t& k) const {
        k = (uint32_t)key[i];
        return true;
    }
    __device__ bool load(int64_t i, uint32_t& k, uint64_t& v) const {
        k = (uint32_t)key[i] & mask;
        v = (uint64_t)val[i];
        return true;
    }
};

struct GroupCols {
    const void* col[TQP_FRAGMENT_MAX_GROUP_COLS];
    int32_t type[TQP_FRAGMENT_MAX_GROUP_COLS];
    int32_t side[TQP_FRAGMENT_MAX_GROUP_COLS];      // 0: read through the fact row, 1: the dim row, 2: at the joined row
    int32_t bits[TQP_FRAGMENT_MAX_GROUP_COLS];
    int32_t n;
};

__device__ __forceinline__ int64_t gf_load(const void* col, int type, int64_t r) {
    switch (type) {
        case TQP_I8: return static_cast<const int8_t*>(col)[r];
        case TQP_I32: return static_cast<const int32_t*>(col)[r];
        default: return static_cast<const int64_t*>(col)[r];
    }
}

// gkey[i] = the group columns of joined row i packed, first most significant.
__global__ void __launch_bounds__(256)
k_gf_pack(GroupCols g, const int32_t* li, const int32_t* ri, int64_t n_upper, const int64_t* d_n, uint32_t* gkey,
          uint32_t* flags) {
    int64_t n = *d_n;
    n = n < n_upper ? n : n_upper;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t v = 0;
        for (int c = 0; c < g.n; ++c) {
            const int64_t r = g.side[c] == 2 ? i : g.side[c] ? (int64_t)ri[i] : (int64_t)li[i];
            const int64_t x = gf_load(g.col[c], g.type[c], r);
            const int64_t lim = int64_t(1) << g.bits[c];
            bad |= x < 0 || x >= lim;
            v = (v << g.bits[c]) | (uint32_t)(x & (lim - 1));
        }
        gkey[i] = v;
    }
    if (__any(bad) && lane_id() == 0) set_flag(flags, FLAG_KEY_RANGE);
}

// Group starts: the positions i < n (n = *d_n, at most n_upper) of the
// sorted keys where a run of equal keys begins, compacted in order into
// start[]; *d_groups = their number.  Ballot per 64 rows, block scan,
// decoupled look-back (as the filter).
__global__ void __launch_bounds__(GF_HEAD_BLOCK)
k_gf_heads(const uint32_t* skey, int64_t n_upper, const int64_t* d_n, int64_t* start, int64_t* d_groups,
           uint64_t* status, uint32_t* tile_counter, uint32_t* flags) {
    constexpr int TILE = GF_HEAD_BLOCK * GF_HEAD_ITEMS, W = GF_HEAD_BLOCK / WAVE;
    __shared__ int64_t s_wave[W];
    __shared__ int64_t s_base;
    __shared__ uint32_t s_tile;
    const int tid = threadIdx.x, w = tid / WAVE, l = lane_id();
    int64_t n = *d_n;
    n = n < n_upper ? n : n_upper;
    if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t ntiles = (n + TILE - 1) / TILE;
    if (tile >= ntiles) {
        if (ntiles == 0 && tile == 0 && tid == 0) *d_groups = 0;
        return;
    }
    const int64_t chunk = tile * TILE + (int64_t)w * GF_HEAD_ITEMS * WAVE;
    uint64_t m[GF_HEAD_ITEMS];
    int64_t wc = 0;
#pragma unroll
    for (int j = 0; j < GF_HEAD_ITEMS; ++j) {
        const int64_t i = chunk + j * WAVE + l;
        const bool in = i < n;
        const int64_t ic = in ? i : n - 1;
        const bool head = in && (ic == 0 || skey[ic] != skey[ic - 1]);
        m[j] = ballot(head);
        wc += popc64(m[j]);
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
            if (tile == ntiles - 1) *d_groups = base + tot;
        }
    }
    __syncthreads();
    int64_t pos = s_base + s_wave[w];
#pragma unroll
    for (int j = 0; j < GF_HEAD_ITEMS; ++j) {
        const int64_t i = chunk + j * WAVE + l;
        if ((m[j] >> l) & 1) start[pos + popc64(m[j] & lanemask_lt())] = i;
        pos += popc64(m[j]);
    }
}

struct AggSet {
    const int64_t* val[TQP_FRAGMENT_MAX_AGGS];   // values per joined row, read through perm (null for COUNT)
    const int64_t* sval;                         // or the values of aggregate sk in sorted order
    int32_t sk;
    void* out[TQP_FRAGMENT_MAX_AGGS];
    int32_t op[TQP_FRAGMENT_MAX_AGGS];
    int32_t n;
};

__device__ __forceinline__ uint64_t gf_ord(int64_t x) { return (uint64_t)x ^ (uint64_t(1) << 63); }
__device__ __forceinline__ int64_t gf_unord(uint64_t u) { return (int64_t)(u ^ (uint64_t(1) << 63)); }

constexpr int GF_LANE_GROUP = 64;    // runs at most this long are reduced by one lane

// Partial reduction of rows [b, e) of one run, taking every `step`-th row
// from b (one lane: step 1; a wave: its lane offset and step 64).
struct GfPart {
    int64_t cnt = 0, dist = 0;
    int64_t sum[TQP_FRAGMENT_MAX_AGGS];
    uint64_t mn[TQP_FRAGMENT_MAX_AGGS], mx[TQP_FRAGMENT_MAX_AGGS];
    __device__ void clear() {
#pragma unroll
        for (int k = 0; k < TQP_FRAGMENT_MAX_AGGS; ++k) { sum[k] = 0; mn[k] = ~uint64_t(0); mx[k] = 0; }
        cnt = 0;
        dist = 0;
    }
    __device__ void add(const AggSet& a, const uint32_t* perm, const int64_t* dval, int64_t s, int64_t i) {
        const uint32_t j = perm ? perm[i] : 0u;
        ++cnt;
#pragma unroll
        for (int k = 0; k < TQP_FRAGMENT_MAX_AGGS; ++k) {
            if (k >= a.n) continue;
            const int64_t* vk = a.val[k];
            if (!vk && !(a.sval && k == a.sk)) continue;
            const int64_t v = vk ? vk[j] : a.sval[i];
            sum[k] = (int64_t)((uint64_t)sum[k] + (uint64_t)v);
            const uint64_t o = gf_ord(v);
            mn[k] = o < mn[k] ? o : mn[k];
            mx[k] = o > mx[k] ? o : mx[k];
        }
        // rows are in (key, distinct value) order: a value starts where it differs from the row before
        if (dval) dist += (i == s || dval[j] != dval[perm[i - 1]]) ? 1 : 0;
    }
};

__device__ __forceinline__ void gf_write(const AggSet& a, const GfPart& p, int64_t g, int64_t cnt) {
#pragma unroll
    for (int k = 0; k < TQP_FRAGMENT_MAX_AGGS; ++k) {
        if (k >= a.n) continue;
        int64_t* o64 = static_cast<int64_t*>(a.out[k]);
        switch (a.op[k]) {
            case TQP_AGG_COUNT: o64[g] = cnt; break;
            case TQP_AGG_SUM: o64[g] = p.sum[k]; break;
            case TQP_AGG_MIN: o64[g] = gf_unord(p.mn[k]); break;
            case TQP_AGG_MAX: o64[g] = gf_unord(p.mx[k]); break;
            case TQP_AGG_AVG: static_cast<double*>(a.out[k])[g] = (double)p.sum[k] / (double)cnt; break;
            default: o64[g] = p.dist; break;
        }
    }
}

// The bucket group-by's outputs that are not written by its kernel: the
// COUNTs other than the one it writes (cnt), and AVG (one IEEE division of
// the exact int64 sum).
__global__ void k_gf_bucket_out(AggSet a, const int64_t* v, const int64_t* cnt, const int64_t* d_groups,
                                int64_t gcap) {
    int64_t G = *d_groups;
    G = G < gcap ? G : gcap;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G; g += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < TQP_FRAGMENT_MAX_AGGS; ++k) {
            if (k >= a.n) continue;
            if (a.op[k] == TQP_AGG_COUNT && a.out[k] != cnt) static_cast<int64_t*>(a.out[k])[g] = cnt[g];
            if (a.op[k] == TQP_AGG_AVG) static_cast<double*>(a.out[k])[g] = (double)v[g] / (double)cnt[g];
        }
    }
}

// The direct group-by.  Slot (k, g) of aggregate k and key g holds the sum
// (SUM, AVG), the largest ord(v) (MAX) or the largest ~ord(v) (MIN), where
// ord flips the sign bit so that unsigned order is signed order: every slot
// starts at 0 and only adds or takes maxima.  Slot (n, g) counts the rows.
// Each block reduces a grid-stride share of the joined rows in LDS and writes
// its slots to part[block].
__global__ void __launch_bounds__(GF_DIRECT_BLOCK)
k_gf_direct(const uint32_t* gkey, AggSet a, int64_t n_upper, const int64_t* d_n, int gbits, uint64_t* part) {
    extern __shared__ unsigned long long dslot[];
    const int G2 = 1 << gbits, nslot = (a.n + 1) << gbits;
    for (int i = threadIdx.x; i < nslot; i += GF_DIRECT_BLOCK) dslot[i] = 0;
    __syncthreads();
    int64_t n = *d_n;
    n = n < n_upper ? n : n_upper;
    const uint32_t gmask = (uint32_t)G2 - 1;
    for (int64_t i = (int64_t)blockIdx.x * GF_DIRECT_BLOCK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * GF_DIRECT_BLOCK) {
        const uint32_t g = gkey[i] & gmask;
        atomicAdd(&dslot[(a.n << gbits) + g], 1ull);
#pragma unroll
        for (int k = 0; k < TQP_FRAGMENT_MAX_AGGS; ++k) {
            if (k >= a.n || !a.val[k]) continue;
            const int64_t v = a.val[k][i];
            unsigned long long* sl = &dslot[(k << gbits) + g];
            if (a.op[k] == TQP_AGG_MIN) atomicMax(sl, (unsigned long long)~gf_ord(v));
            else if (a.op[k] == TQP_AGG_MAX) atomicMax(sl, (unsigned long long)gf_ord(v));
            else atomicAdd(sl, (unsigned long long)v);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nslot; i += GF_DIRECT_BLOCK) part[(int64_t)blockIdx.x * nslot + i] = dslot[i];
}

// Slot s of every block's part reduced by one wave: red[s].
__global__ void __launch_bounds__(WAVE)
k_gf_direct_reduce(const uint64_t* part, int nparts, AggSet a, int gbits, uint64_t* red) {
    const int nslot = (a.n + 1) << gbits, sl = blockIdx.x, k = sl >> gbits;
    const bool takes_max = k < a.n && (a.op[k] == TQP_AGG_MIN || a.op[k] == TQP_AGG_MAX);
    uint64_t acc = 0;
    for (int b = lane_id(); b < nparts; b += WAVE) {
        const uint64_t x = part[(int64_t)b * nslot + sl];
        acc = takes_max ? (x > acc ? x : acc) : acc + x;
    }
    acc = takes_max ? wave_max(acc) : wave_sum(acc);
    if (lane_id() == 0) red[sl] = acc;
}

// The non-empty keys in ascending order with their aggregates (one block of
// 2^GF_DIRECT_MAX_BITS threads, one key each).
__global__ void __launch_bounds__(1 << GF_DIRECT_MAX_BITS)
k_gf_direct_out(const uint64_t* red, AggSet a, int gbits, int32_t* out_key, int64_t gcap, int64_t* d_ngroups,
                int64_t* d_written, uint32_t* flags) {
    __shared__ int64_t scratch[(1 << GF_DIRECT_MAX_BITS) / WAVE];
    const int g = threadIdx.x, G2 = 1 << gbits;
    const int64_t cnt = g < G2 ? (int64_t)red[((int64_t)a.n << gbits) + g] : 0;
    int64_t total;
    const int64_t pos = block_excl_sum<1 << GF_DIRECT_MAX_BITS>((int64_t)(cnt > 0), scratch, &total);
    if (cnt > 0 && pos < gcap) {
        out_key[pos] = g;
#pragma unroll
        for (int k = 0; k < TQP_FRAGMENT_MAX_AGGS; ++k) {
            if (k >= a.n) continue;
            const uint64_t x = red[((int64_t)k << gbits) + g];
            int64_t* o64 = static_cast<int64_t*>(a.out[k]);
            switch (a.op[k]) {
                case TQP_AGG_COUNT: o64[pos] = cnt; break;
                case TQP_AGG_SUM: o64[pos] = (int64_t)x; break;
                case TQP_AGG_MIN: o64[pos] = gf_unord(~x); break;
                case TQP_AGG_MAX: o64[pos] = gf_unord(x); break;
                default: static_cast<double*>(a.out[k])[pos] = (double)(int64_t)x / (double)cnt; break;
            }
        }
    }
    if (g == 0) {
        *d_ngroups = total;
        *d_written = total < gcap ? total : gcap;
        if (total > gcap) set_flag(flags, FLAG_CAPACITY);
    }
}

// Every group's aggregates: each wave takes 64 consecutive groups (grid-stride);
// a lane reduces its own group when all 64 are at most GF_LANE_GROUP rows,
// else the wave reduces the long ones one at a time and the lanes the rest.
// The run of group g is [start[g], start[g + 1]) of the sorted keys; values
// come through perm, or in sorted order (a.sval).
__global__ void __launch_bounds__(GF_AGG_BLOCK)
k_gf_agg(const uint32_t* skey, const uint32_t* perm, const int64_t* start, const int64_t* d_groups,
         const int64_t* d_rows, int64_t rows_upper, AggSet a, const int64_t* dval, int32_t* out_key, int64_t gcap,
         int64_t* d_ngroups, int64_t* d_written, uint32_t* flags) {
    const int64_t G = *d_groups;
    int64_t J = *d_rows;
    J = J < rows_upper ? J : rows_upper;
    const int64_t Gw = G < gcap ? G : gcap;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *d_ngroups = G;
        *d_written = Gw;
        if (G > gcap) set_flag(flags, FLAG_CAPACITY);
    }
    const int l = lane_id();
    const int64_t wid = ((int64_t)blockIdx.x * GF_AGG_BLOCK + threadIdx.x) / WAVE;
    const int64_t nw = (int64_t)gridDim.x * GF_AGG_BLOCK / WAVE;
    for (int64_t g0 = wid * WAVE; g0 < Gw; g0 += nw * WAVE) {
        const int64_t g = g0 + l;
        const bool has = g < Gw;
        const int64_t s = has ? start[g] : 0, e = has ? (g + 1 < G ? start[g + 1] : J) : 0;
        const bool lng = e - s > GF_LANE_GROUP;
        if (has && !lng) {
            GfPart p;
            p.clear();
            for (int64_t i = s; i < e; ++i) p.add(a, perm, dval, s, i);
            out_key[g] = (int32_t)skey[s];
            gf_write(a, p, g, p.cnt);
        }
        uint64_t big = ballot(has && lng);
        while (big) {
            const int src = __ffsll((unsigned long long)big) - 1;
            big &= big - 1;
            const int64_t gs = wave_read(s, src), ge = wave_read(e, src), gg = g0 + src;
            GfPart p;
            p.clear();
            for (int64_t i = gs + l; i < ge; i += WAVE) p.add(a, perm, dval, gs, i);
            const int64_t cnt = wave_sum(p.cnt);
            p.dist = wave_sum(p.dist);
#pragma unroll
            for (int k = 0; k < TQP_FRAGMENT_MAX_AGGS; ++k) {
                if (k >= a.n) continue;
                p.sum[k] = wave_sum(p.sum[k]);
                p.mn[k] = wave_min(p.mn[k]);
                p.mx[k] = wave_max(p.mx[k]);
            }
            if (l == 0) {
                out_key[gg] = (int32_t)skey[gs];
                gf_write(a, p, gg, cnt);
            }
        }
    }
}

// The keyed form of the bucket group-by: the fact value rides the fact sort
// (VT: int64 bits, or int32 bits under a declared 32-bit width), the join
// emits (group key, value) with the group sort's digit counts, and the group
// sort is its passes alone.
template <class Cfg, class VT>
struct GenKv {
    RadixBufs<Cfg, VT> fsort, gsort;
    VT* fsv = nullptr;
    uint32_t* gk_in = nullptr;
    VT* gv_in = nullptr;
    uint32_t* gk = nullptr;
    VT* gv = nullptr;
};

template <class Cfg>
struct GenBufs {
    bool join = false;
    int distinct = -1;                       // the COUNT(DISTINCT) aggregate, if any
    int gbits = 1;
    uint8_t* fkeep = nullptr;                // predicate keep bytes (1: the row takes part)
    uint8_t* dkeep = nullptr;
    RadixBufs<Cfg, uint32_t> fsort, dsort, sa, sb, sc;
    int flowb = 0;                           // fact key bits left to the join tiles
    int64_t nspans = 0, nmbkt = 0;
    uint32_t *dsk_full = nullptr, *dsv_full = nullptr;   // dim keys after the finishing pass
    int64_t* mbstart = nullptr;              // start of every 2^flowb-key bucket in them
    int vsort = -1;                          // the one valued aggregate whose value rides the group sort
    bool fpush = false;                      // that value rides the fact sort (fact-only program)
    int dpush = -1;                          // the dim column that rides the dim sort, or -1
    int64_t* fval = nullptr;                 // fpush: the program over every fact row
    RadixBufs<Cfg, uint64_t> fsort64;
    uint64_t* fsv64 = nullptr;
    int64_t* jval = nullptr;                 // fpush: the value of every joined row
    RadixBufs<Cfg, uint64_t> sv;
    uint64_t* vc = nullptr;
    // the bucket group-by: the group sort covers the key bits above lowb, and
    // one block per bucket of 2^lowb keys reduces it in LDS
    bool bucket = false;
    int lowb = 0;
    int64_t nbuckets = 0;
    int64_t* bstarts = nullptr;
    uint64_t* bstatus = nullptr;
    uint32_t* bcounter = nullptr;
    int64_t *bval = nullptr, *bcnt = nullptr;   // per group: the value's reduction, the row count
    bool reads_fact = false;                 // group columns or value programs read fact columns after the join
    int fact_row_bytes = 0;                  // their bytes per fact row
    bool lorder = false;                     // the joined rows put in fact-row order before the gathers
    RadixBufs<Cfg, uint32_t> lsort;
    int32_t *li2 = nullptr, *ri2 = nullptr;
    bool direct = false;                     // the direct group-by (few keys)
    int64_t dparts = 0;                      // its blocks, one part each
    uint64_t *dpart = nullptr, *dred = nullptr;
    bool kv = false;                         // the keyed form (one group column carried by the dim sort)
    bool v32 = false;                        // its value carried in 32 bits
    int32_t* fval32 = nullptr;
    GenKv<Cfg, uint64_t> kv64;
    GenKv<Cfg, uint32_t> kv32;
    JoinBufs jb;
    uint32_t *fsk = nullptr, *fsv = nullptr, *dsk = nullptr, *dsv = nullptr;
    uint64_t* fstatus = nullptr;             // no join: the compaction of the kept fact rows
    uint32_t* fcounter = nullptr;
    int32_t *li = nullptr, *ri = nullptr;
    int64_t* d_join = nullptr;
    uint32_t* gkey = nullptr;
    int64_t* vals[TQP_FRAGMENT_MAX_AGGS] = {};
    uint32_t *ka = nullptr, *pa = nullptr, *kb = nullptr, *pb = nullptr, *kc = nullptr, *pc = nullptr;
    int64_t* gstart = nullptr;
    uint64_t* hstatus = nullptr;
    uint32_t* hcounter = nullptr;
    int64_t* d_groups = nullptr;
    int64_t* d_written = nullptr;
    TopkBufs topk;
    int64_t* tcnt = nullptr;                 // the top rows' third column (not returned)
};

int gf_group_bits(const tqp_fragment& f) {
    int b = 0;
    for (int i = 0; i < f.n_group; ++i) b += f.group[i].bits;
    return b > 0 ? b : 1;
}

template <class Cfg>
void gen_reserve(Arena& a, const tqp_fragment& f, const tqp_fragment_out& o, GenBufs<Cfg>& b) {
    const int kb = norm_key_bits(f.key_bits);
    const int64_t N = f.n_fact, J = f.join_cap;
    b.join = f.fact_key >= 0;
    b.gbits = gf_group_bits(f);
    for (int k = 0; k < f.n_agg; ++k)
        if (f.aggs[k].op == TQP_AGG_COUNT_DISTINCT) b.distinct = k;
    int valued = 0;
    for (int k = 0; k < f.n_agg; ++k)
        if (f.aggs[k].op != TQP_AGG_COUNT) {
            ++valued;
            b.vsort = k;
        }
    if (valued != 1 || b.distinct >= 0) b.vsort = -1;
    b.bucket = b.vsort >= 0 && b.gbits >= GF_BUCKET_MIN_BITS;
    b.direct = b.distinct < 0 && b.gbits <= GF_DIRECT_MAX_BITS;
    if (b.bucket) {
        b.lowb = bucket_low_bits(b.gbits, Cfg::RADIX_BITS);
        b.nbuckets = int64_t(1) << (b.gbits - b.lowb);
    }
    if (b.join) {
        // what the join's output is used for: columns of each side read after it
        auto prog_sides = [&](const tqp_xinstr* pr, int np, bool& uses_f, bool& uses_d) {
            for (int i = 0; i < np; ++i)
                if (pr[i].op == TQP_X_COL) (pr[i].arg < f.n_fact_cols ? uses_f : uses_d) = true;
        };
        bool group_f = false, group_d = false;
        int gd = -1;
        bool gd_one = true;
        for (int i = 0; i < f.n_group; ++i) {
            const int c = f.group[i].col;
            if (c < f.n_fact_cols) {
                group_f = true;
            } else {
                group_d = true;
                if (gd >= 0 && gd != c) gd_one = false;
                gd = c;
            }
        }
        bool prog_f = false, prog_d = false;
        for (int k = 0; k < f.n_agg; ++k)
            if (f.aggs[k].op != TQP_AGG_COUNT) prog_sides(f.aggs[k].prog, f.aggs[k].nprog, prog_f, prog_d);
        // the fact rows serve only the one valued aggregate, whose program reads
        // only fact columns; evaluated over every fact row, it must not divide
        // (a zero divisor on a row the join drops would raise the value flag)
        bool divides = false;
        if (b.vsort >= 0)
            for (int i = 0; i < f.aggs[b.vsort].nprog; ++i)
                divides |= f.aggs[b.vsort].prog[i].op == TQP_X_DIV || f.aggs[b.vsort].prog[i].op == TQP_X_MOD;
        b.fpush = b.vsort >= 0 && prog_f && !prog_d && !group_f && !divides;
        // the dim rows serve only one int32 group column
        if (group_d && gd_one && !prog_d && f.dim_cols[gd - f.n_fact_cols].type == TQP_I32) b.dpush = gd - f.n_fact_cols;
        // bytes of the fact columns read through the pairs (per fact row)
        {
            uint64_t seen = 0;
            auto mark = [&](int c) {
                if (c < f.n_fact_cols && !((seen >> c) & 1)) {
                    seen |= uint64_t(1) << c;
                    const int t = f.fact_cols[c].type;
                    b.fact_row_bytes += t == TQP_I64 ? 8 : t == TQP_I32 ? 4 : 1;
                }
            };
            for (int i = 0; i < f.n_group; ++i) mark(f.group[i].col);
            for (int k = 0; k < f.n_agg; ++k)
                if (f.aggs[k].op != TQP_AGG_COUNT)
                    for (int i = 0; i < f.aggs[k].nprog; ++i)
                        if (f.aggs[k].prog[i].op == TQP_X_COL) mark((int)f.aggs[k].prog[i].arg);
        }
        b.reads_fact = group_f || prog_f;
        b.kv = b.bucket && b.fpush && b.dpush >= 0 && f.n_group == 1;
        b.v32 = b.kv && f.value_bits == 32;
    }
    if (f.n_fact_pred > 0) b.fkeep = a.scratch<uint8_t>(N);
    if (b.join) {
        if (f.n_dim_pred > 0) b.dkeep = a.scratch<uint8_t>(f.n_dim);
        b.flowb = join_low_bits(N, kb, Cfg::RADIX_BITS, JCfgGen::TILE, JCfgGen::RWIN);
        if (b.flowb > FINISH_LOG2) b.flowb = FINISH_LOG2;
        // the fact sorts' first pass looks back instead of reading per-tile
        // counts, as the custkey fragment's fact sort: over tens of millions
        // of rows the plain histogram costs less than the counting one
        auto kv_reserve = [&](auto& k) {
            using VT = typename std::remove_pointer<decltype(k.fsv)>::type;
            k.fsort = radix_reserve<Cfg, VT>(a, N, kb, b.flowb, false);
            k.fsv = a.scratch<VT>(N);
            k.gsort = radix_reserve<Cfg, VT>(a, J, b.gbits, b.lowb, false);     // digit counts from the join
            k.gk_in = a.scratch<uint32_t>(J);
            k.gv_in = a.scratch<VT>(J);
            k.gk = a.scratch<uint32_t>(J);
            k.gv = a.scratch<VT>(J);
        };
        if (b.kv) {
            if (b.v32) {
                b.fval32 = a.scratch<int32_t>(N);
                kv_reserve(b.kv32);
            } else {
                b.fval = a.scratch<int64_t>(N);
                kv_reserve(b.kv64);
            }
        } else if (b.fpush) {
            b.fval = a.scratch<int64_t>(N);
            b.fsort64 = radix_reserve<Cfg, uint64_t>(a, N, kb, b.flowb, false);
            b.fsv64 = a.scratch<uint64_t>(N);
            b.jval = a.scratch<int64_t>(J);
        } else {
            b.fsort = radix_reserve<Cfg, uint32_t>(a, N, kb, b.flowb, false);
            b.fsv = a.scratch<uint32_t>(N);
        }
        b.dsort = radix_reserve<Cfg, uint32_t>(a, f.n_dim, kb, b.flowb);
        if (b.flowb > 0) {
            b.dsk_full = a.scratch<uint32_t>(f.n_dim);
            b.dsv_full = a.scratch<uint32_t>(f.n_dim);
            b.nspans = ((int64_t(1) << kb) + FINISH_SPAN - 1) >> FINISH_LOG2;
            b.nmbkt = b.nspans << (FINISH_LOG2 - b.flowb);
            b.mbstart = a.scratch<int64_t>(b.nmbkt + 1);
        }
        b.fsk = a.scratch<uint32_t>(N);
        b.dsk = a.scratch<uint32_t>(f.n_dim);
        b.dsv = a.scratch<uint32_t>(f.n_dim);
        b.jb = join_reserve<JCfgGen>(a, N);
        if (!b.kv) b.ri = a.scratch<int32_t>(J);
    } else {
        const int64_t tiles = (N + GF_FILTER_BLOCK * GF_FILTER_ITEMS - 1) / (GF_FILTER_BLOCK * GF_FILTER_ITEMS);
        b.fstatus = a.zero<uint64_t>(tiles);
        b.fcounter = a.zero<uint32_t>(1);
    }
    if (!b.fpush) b.li = a.scratch<int32_t>(J);
    b.d_join = a.zero<int64_t>(1);
    // No result depends on the joined rows' order (groups come in key order,
    // every aggregate is order-free).  With fact columns read through the
    // pairs, sorting the pairs by fact row turns those reads from random into
    // one forward sweep; the top 16 bits of the row suffice (two passes):
    // rows then come in runs of nearby rows, which the caches serve.  Worth
    // it when those columns outgrow the chip's last-level cache (random
    // reads of a table that fits it are served there).
    if (b.join && !b.fpush && b.reads_fact && N * b.fact_row_bytes > GF_LORDER_MIN_BYTES) {
        int rb = 1;
        while (rb < 31 && (int64_t(1) << rb) < N) ++rb;
        b.lorder = true;
        b.lsort = radix_reserve<Cfg, uint32_t>(a, J, rb, rb > 16 ? rb - 16 : 0);
        b.li2 = a.scratch<int32_t>(J);
        b.ri2 = a.scratch<int32_t>(J);
    }
    if (!b.kv) b.gkey = a.scratch<uint32_t>(J);
    for (int k = 0; k < f.n_agg; ++k)
        if (f.aggs[k].op != TQP_AGG_COUNT) b.vals[k] = b.fpush && k == b.vsort ? b.jval : a.scratch<int64_t>(J);
    if (b.distinct >= 0) {
        b.sa = radix_reserve<Cfg, uint32_t>(a, J, 32);
        b.sb = radix_reserve<Cfg, uint32_t>(a, J, 32);
        b.ka = a.scratch<uint32_t>(J);
        b.pa = a.scratch<uint32_t>(J);
        b.kb = a.scratch<uint32_t>(J);
        b.pb = a.scratch<uint32_t>(J);
    }
    if (b.direct) {
        const int64_t nslot = (int64_t)(f.n_agg + 1) << b.gbits;
        b.dparts = GF_DIRECT_PARTS;
        b.dpart = a.scratch<uint64_t>(b.dparts * nslot);
        b.dred = a.scratch<uint64_t>(nslot);
        b.d_written = a.zero<int64_t>(1);
        if (f.topk > 0) {
            b.topk = topk_reserve(a, o.gcap, f.topk);
            b.tcnt = a.scratch<int64_t>(f.topk);
        }
        return;
    }
    if (b.bucket) {
        if (!b.kv) {
            b.sv = radix_reserve<Cfg, uint64_t>(a, J, b.gbits, b.lowb);
            b.kc = a.scratch<uint32_t>(J);
            b.vc = a.scratch<uint64_t>(J);
        }
        b.bstarts = a.scratch<int64_t>(b.nbuckets + 1);
        b.bstatus = a.zero<uint64_t>(b.nbuckets);
        b.bcounter = a.zero<uint32_t>(1);
        b.bval = a.scratch<int64_t>(o.gcap);
        b.bcnt = a.scratch<int64_t>(o.gcap);
        if (f.topk > 0) {
            // candidates: the first k groups of every bucket
            b.topk = topk_reserve(a, std::min<int64_t>(o.gcap, b.nbuckets * f.topk), f.topk);
            b.tcnt = a.scratch<int64_t>(f.topk);
        }
        return;
    }
    b.kc = a.scratch<uint32_t>(J);
    if (b.vsort >= 0) {
        b.sv = radix_reserve<Cfg, uint64_t>(a, J, b.gbits);
        b.vc = a.scratch<uint64_t>(J);
    } else {
        b.sc = radix_reserve<Cfg, uint32_t>(a, J, b.gbits);
        b.pc = a.scratch<uint32_t>(J);
    }
    b.gstart = a.scratch<int64_t>(J + 1);
    const int64_t htiles = (J + GF_HEAD_BLOCK * GF_HEAD_ITEMS - 1) / (GF_HEAD_BLOCK * GF_HEAD_ITEMS);
    b.hstatus = a.zero<uint64_t>(htiles);
    b.hcounter = a.zero<uint32_t>(1);
    b.d_groups = a.zero<int64_t>(1);
    b.d_written = a.zero<int64_t>(1);
    if (f.topk > 0) {
        b.topk = topk_reserve(a, o.gcap, f.topk);
        b.tcnt = a.scratch<int64_t>(f.topk);
    }
}

// The joined row's columns (fact, then dim) and the row arrays they are read through.
struct JoinedCols {
    tqp_column col[GF_MAX_COLS];
    const int32_t* idx[GF_MAX_COLS];
    int n = 0;
};

// The group-by by buckets, over the keys sorted on their bits above lowb
// with the one valued aggregate's value (Algorithm 2 with the last digit
// resolved in LDS, as in the custkey fragment): every bucket's block reduces
// the value (sum, min or max) and counts the rows per key in LDS and writes
// its groups in key order, with its first k groups as top-k candidates when
// the fragment has a top-k.  Groups come out in ascending key order, as from
// the full sort.  bhist: the digit counts of a one-pass group sort (the
// buckets), else the bucket starts are searched for.
template <class Cfg, class AV>
tqp_status bucket_groupby(tqp_ctx* ctx, const tqp_fragment& f, const tqp_fragment_out& o, const GenBufs<Cfg>& b,
                          const uint32_t* keys, const AV* vals, const uint32_t* bhist, hipStream_t s) {
    const int64_t J = f.join_cap;
    const int vop = f.aggs[b.vsort].op;
    int64_t* vout = vop == TQP_AGG_AVG ? b.bval : static_cast<int64_t*>(f.aggs[b.vsort].out);
    int64_t* cout = b.bcnt;
    bool finish = false;
    for (int k = 0; k < f.n_agg; ++k) {
        if (f.aggs[k].op == TQP_AGG_COUNT) {
            if (cout == b.bcnt) cout = static_cast<int64_t*>(f.aggs[k].out);
            else finish = true;
        }
        finish |= f.aggs[k].op == TQP_AGG_AVG;
    }
    SegOut so{o.key, vout, cout, nullptr, o.gcap, o.d_ngroups};
    if (!bhist) {
        TQP_LAUNCH(ctx, s, "fragment_bucket_bounds",
                   k_bucket_bounds<<<grid_for(b.nbuckets + 1, 256, 0), 256, 0, s>>>(keys, J, b.d_join, b.lowb,
                                                                                      b.nbuckets, b.bstarts));
    }
    TopCand* cand = f.topk > 0 ? b.topk.filtered : nullptr;
    int64_t* d_cand = f.topk > 0 ? b.topk.d_nf : nullptr;
    const bool bycnt = f.topk > 0 && f.aggs[0].op == TQP_AGG_COUNT;
    constexpr int SLOTS = 1 << BUCKET_LOWB_MAX;
    auto go = [&](auto kern) -> tqp_status {
        TQP_LAUNCH(ctx, s, "fragment_bucket_agg",
                   kern<<<(unsigned)b.nbuckets, 1024, 0, s>>>(keys, vals, b.bstarts, bhist, b.lowb, b.nbuckets,
                                                              b.bstatus, b.bcounter, so, ctx->d_err, cand, d_cand,
                                                              f.topk));
        return TQP_OK;
    };
    tqp_status st;
    if (vop == TQP_AGG_MIN)
        st = bycnt ? go(k_bucket_agg<1024, SLOTS, AV, BUCKET_MIN, true>)
                   : go(k_bucket_agg<1024, SLOTS, AV, BUCKET_MIN, false>);
    else if (vop == TQP_AGG_MAX)
        st = bycnt ? go(k_bucket_agg<1024, SLOTS, AV, BUCKET_MAX, true>)
                   : go(k_bucket_agg<1024, SLOTS, AV, BUCKET_MAX, false>);
    else
        st = bycnt ? go(k_bucket_agg<1024, SLOTS, AV, BUCKET_SUM, true>)
                   : go(k_bucket_agg<1024, SLOTS, AV, BUCKET_SUM, false>);
    if (st != TQP_OK) return st;
    if (finish && o.gcap > 0) {
        AggSet as{};
        as.n = f.n_agg;
        for (int k = 0; k < f.n_agg; ++k) {
            as.out[k] = f.aggs[k].out;
            as.op[k] = f.aggs[k].op;
        }
        TQP_LAUNCH(ctx, s, "fragment_bucket_out",
                   k_gf_bucket_out<<<grid_for(o.gcap, 256, (int64_t)ctx->num_cus * 8), 256, 0, s>>>(
                       as, vout, cout, o.d_ngroups, o.gcap));
    }
    // ORDER BY the first aggregate DESC, key ASC LIMIT k, over the candidates
    if (f.topk > 0)
        return topk_launch_candidates(b.topk, cout, f.topk, o.top_key, o.top_val, b.tcnt, o.d_topk, s, ctx);
    return TQP_OK;
}

// The one valued aggregate's program over every fact row, in row order (it
// then rides the fact sort).
template <class Cfg>
tqp_status fact_value(tqp_ctx* ctx, const tqp_fragment& f, const GenBufs<Cfg>& b, void* out, int mode,
                      hipStream_t s) {
    const tqp_agg& ag = f.aggs[b.vsort];
    return eval_program(ctx, f.fact_cols, nullptr, f.n_fact_cols, f.n_fact, nullptr, ag.prog, ag.nprog, out, s,
                        "tqp_fragment_run", "fragment_fact_value", mode);
}

// The keyed bucket group-by from the fact value on (the dim side and the
// fact predicate already launched): the value program over every fact row,
// the fact sort carrying it, the join emitting (group key, value) with the
// group sort's digit counts, the group sort's passes, the buckets.
template <class Cfg, class VT>
tqp_status kv_launch(tqp_ctx* ctx, const tqp_fragment& f, const tqp_fragment_out& o, const GenBufs<Cfg>& b,
                     const GenKv<Cfg, VT>& k, const uint32_t* rk, const uint32_t* rv, hipStream_t s) {
    constexpr bool V32 = sizeof(VT) == 4;
    const int kb = norm_key_bits(f.key_bits);
    const int64_t N = f.n_fact, J = f.join_cap;
    const int32_t* fkey = static_cast<const int32_t*>(f.fact_cols[f.fact_key].data);
    tqp_status st;
    void* fv = V32 ? static_cast<void*>(b.fval32) : static_cast<void*>(b.fval);
    if (N > 0 && (st = fact_value(ctx, f, b, fv, V32 ? XOUT_I32 : XOUT_I64, s)) != TQP_OK) return st;
    if constexpr (V32) {
        SrcKeepCol fs{fkey, b.fkeep, b.fval32, N};
        st = radix_launch<Cfg, uint32_t>(k.fsort, fs, N, true, nullptr, key_mask_for(kb), b.fsk, k.fsv, ctx, s,
                                         "fragment_sort_fact", "fragment_sort_fact");
    } else {
        SrcKeepVal64 fs{fkey, b.fkeep, b.fval, N};
        st = radix_launch<Cfg, uint64_t>(k.fsort, fs, N, true, nullptr, key_mask_for(kb), b.fsk, k.fsv, ctx, s,
                                         "fragment_sort_fact", "fragment_sort_fact");
    }
    if (st != TQP_OK) return st;
    if ((st = side_join(ctx, s)) != TQP_OK) return st;
    using Emit = EmitKeyVal<JCfgGen::BLOCK, Cfg::RADIX_BITS, VT>;
    Emit e{};
    e.out_key = k.gk_in;
    e.out_val = k.gv_in;
    e.cap = J;
    e.key_mask = key_mask_for(b.gbits);
    e.flags = ctx->d_err;
    e.hist = k.gsort.hist;
    e.npass = k.gsort.pd.npass;
    for (int p = 0; p < k.gsort.pd.npass && p < Emit::NP; ++p) {
        e.shift[p] = k.gsort.pd.shift[p];
        e.bits[p] = k.gsort.pd.bits[p];
    }
    const int64_t* rbstart = b.flowb > 0 && f.n_dim > 0 ? b.mbstart : nullptr;
    if ((st = join_launch<JCfgGen, VT, uint32_t, Emit>(ctx, s, "fragment_join", b.jb, b.fsk, k.fsv, N, k.fsort.d_cnt,
                                                       rk, rv, f.n_dim, b.dsort.d_cnt, b.d_join, J, e, b.flowb,
                                                       nullptr, rbstart, b.nmbkt)) != TQP_OK)
        return st;
    if (o.d_join) TQP_TRY_HIP(hipMemcpyAsync(o.d_join, b.d_join, 8, hipMemcpyDeviceToDevice, s));
    SrcPairs<VT> gsrc{k.gk_in, k.gv_in, J, b.d_join};
    if ((st = radix_launch<Cfg, VT>(k.gsort, gsrc, J, false, b.d_join, key_mask_for(b.gbits), k.gk, k.gv, ctx, s,
                                    "fragment_sort_group", "fragment_sort_group")) != TQP_OK)
        return st;
    using AV = typename std::conditional<V32, int32_t, int64_t>::type;
    return bucket_groupby<Cfg, AV>(ctx, f, o, b, k.gk, reinterpret_cast<const AV*>(k.gv),
                                   k.gsort.pd.npass == 1 ? k.gsort.hist : nullptr, s);
}

// The direct group-by over the packed keys and the aggregates' values of the
// joined rows: per-block LDS slots, the blocks' parts reduced per slot, the
// non-empty keys written in ascending order; then the top-k as for sorted
// groups.
template <class Cfg>
tqp_status direct_groupby(tqp_ctx* ctx, const tqp_fragment& f, const tqp_fragment_out& o, const GenBufs<Cfg>& b,
                          hipStream_t s) {
    const int64_t J = f.join_cap;
    AggSet as{};
    as.n = f.n_agg;
    as.sk = -1;
    for (int k = 0; k < f.n_agg; ++k) {
        as.val[k] = f.aggs[k].op == TQP_AGG_COUNT ? nullptr : b.vals[k];
        as.out[k] = f.aggs[k].out;
        as.op[k] = f.aggs[k].op;
    }
    // an empty side joins nothing and no value column was evaluated: the
    // blocks see no rows (the join count is 0), so no value is read
    const int nslot = (f.n_agg + 1) << b.gbits;
    const size_t lds = (size_t)nslot * sizeof(uint64_t);
    TQP_LAUNCH(ctx, s, "fragment_direct",
               k_gf_direct<<<(unsigned)b.dparts, GF_DIRECT_BLOCK, lds, s>>>(b.gkey, as, J, b.d_join, b.gbits,
                                                                          b.dpart));
    TQP_LAUNCH(ctx, s, "fragment_direct_reduce",
               k_gf_direct_reduce<<<(unsigned)nslot, WAVE, 0, s>>>(b.dpart, (int)b.dparts, as, b.gbits, b.dred));
    TQP_LAUNCH(ctx, s, "fragment_direct_out",
               k_gf_direct_out<<<1, 1 << GF_DIRECT_MAX_BITS, 0, s>>>(b.dred, as, b.gbits, o.key, o.gcap,
                                                                    o.d_ngroups, b.d_written, ctx->d_err));
    if (f.topk > 0) {
        const int64_t* v0 = static_cast<const int64_t*>(f.aggs[0].out);
        return topk_launch(b.topk, o.key, v0, v0, b.d_written, f.topk, o.top_key, o.top_val, b.tcnt, o.d_topk, s,
                           ctx);
    }
    return TQP_OK;
}

template <class Cfg>
tqp_status gen_launch(tqp_ctx* ctx, const tqp_fragment& f, const tqp_fragment_out& o, const GenBufs<Cfg>& b,
                      hipStream_t s) {
    const int kb = norm_key_bits(f.key_bits);
    const int64_t N = f.n_fact, J = f.join_cap;
    tqp_status st;
    // 1. predicates and 2. the join's sorts.  With a join the dim side (its
    // predicate, its sort and the finishing pass) runs on the side stream
    // beside the fact side, and the join waits for both.
    const hipStream_t sd = b.join ? ctx->side : s;
    if (b.join && (st = side_fork(ctx, s)) != TQP_OK) return st;
    if (b.dkeep && f.n_dim > 0 &&
        (st = eval_program(ctx, f.dim_cols, nullptr, f.n_dim_cols, f.n_dim, nullptr, f.dim_pred, f.n_dim_pred, b.dkeep,
                           sd, "tqp_fragment_run", "fragment_dim_pred", XOUT_FLAG)) != TQP_OK)
        return st;
    const uint32_t* rk = b.dsk;
    const uint32_t* rv = b.dsv;
    if (b.join) {
        const int32_t* dkey = static_cast<const int32_t*>(f.dim_cols[f.dim_key].data);
        if (b.dpush >= 0) {
            SrcKeepCol ds{dkey, b.dkeep, static_cast<const int32_t*>(f.dim_cols[b.dpush].data), f.n_dim};
            if ((st = radix_launch<Cfg, uint32_t>(b.dsort, ds, f.n_dim, true, nullptr, key_mask_for(kb), b.dsk,
                                                  b.dsv, ctx, sd, "fragment_sort_dim", "fragment_sort_dim")) != TQP_OK)
                return st;
        } else {
            SrcKeepRow ds{dkey, b.dkeep, f.n_dim};
            if ((st = radix_launch<Cfg, uint32_t>(b.dsort, ds, f.n_dim, true, nullptr, key_mask_for(kb), b.dsk,
                                                  b.dsv, ctx, sd, "fragment_sort_dim", "fragment_sort_dim")) != TQP_OK)
                return st;
        }
        if (b.flowb > 0 && f.n_dim > 0) {
            // the low bits of the dim keys, span by span, and every bucket's start
            TQP_LAUNCH(ctx, sd, "fragment_finish_dim",
                       k_finish_sort<<<(unsigned)b.nspans, FINISH_BLOCK, 0, sd>>>(b.dsk, b.dsv, f.n_dim, b.dsk_full,
                                                                               b.dsv_full, b.flowb, b.mbstart,
                                                                               b.dsort.d_cnt));
            rk = b.dsk_full;
            rv = b.dsv_full;
        }
    }
    if (b.fkeep && N > 0 &&
        (st = eval_program(ctx, f.fact_cols, nullptr, f.n_fact_cols, N, nullptr, f.fact_pred, f.n_fact_pred, b.fkeep,
                           s, "tqp_fragment_run", "fragment_fact_pred", XOUT_FLAG)) != TQP_OK)
        return st;
    // 2. join, or the kept fact rows
    if (b.kv)
        return b.v32 ? kv_launch<Cfg, uint32_t>(ctx, f, o, b, b.kv32, rk, rv, s)
                     : kv_launch<Cfg, uint64_t>(ctx, f, o, b, b.kv64, rk, rv, s);
    if (b.join) {
        const int32_t* fkey = static_cast<const int32_t*>(f.fact_cols[f.fact_key].data);
        const int64_t* fsort_cnt;
        if (b.fpush) {
            // the one value program over every fact row, in row order, before the sort
            if (N > 0 && (st = fact_value(ctx, f, b, b.fval, XOUT_I64, s)) != TQP_OK) return st;
            SrcKeepVal64 fs{fkey, b.fkeep, b.fval, N};
            if ((st = radix_launch<Cfg, uint64_t>(b.fsort64, fs, N, true, nullptr, key_mask_for(kb), b.fsk, b.fsv64,
                                                  ctx, s, "fragment_sort_fact", "fragment_sort_fact")) != TQP_OK)
                return st;
            fsort_cnt = b.fsort64.d_cnt;
        } else {
            SrcKeepRow fs{fkey, b.fkeep, N};
            if ((st = radix_launch<Cfg, uint32_t>(b.fsort, fs, N, true, nullptr, key_mask_for(kb), b.fsk, b.fsv, ctx,
                                                  s, "fragment_sort_fact", "fragment_sort_fact")) != TQP_OK)
                return st;
            fsort_cnt = b.fsort.d_cnt;
        }
        if ((st = side_join(ctx, s)) != TQP_OK) return st;
        const int64_t* rbstart = b.flowb > 0 && f.n_dim > 0 ? b.mbstart : nullptr;
        if (b.fpush) {
            EmitValRow e{b.jval, b.ri, J};
            if ((st = join_launch<JCfgGen, uint64_t, uint32_t, EmitValRow>(
                     ctx, s, "fragment_join", b.jb, b.fsk, b.fsv64, N, fsort_cnt, rk, rv, f.n_dim, b.dsort.d_cnt,
                     b.d_join, J, e, b.flowb, nullptr, rbstart, b.nmbkt)) != TQP_OK)
                return st;
        } else {
            EmitPairs e{b.li, b.ri, J};
            if ((st = join_launch<JCfgGen, uint32_t, uint32_t, EmitPairs>(
                     ctx, s, "fragment_join", b.jb, b.fsk, b.fsv, N, fsort_cnt, rk, rv, f.n_dim, b.dsort.d_cnt,
                     b.d_join, J, e, b.flowb, nullptr, rbstart, b.nmbkt)) != TQP_OK)
                return st;
        }
    } else {
        FilterPreds fp{};
        if (b.fkeep) {
            fp.np = 1;
            fp.col[0] = b.fkeep;
            fp.type[0] = TQP_I8;
            fp.op[0] = CMP_NE;
            fp.k[0] = 0;
        }
        constexpr int64_t TILE = GF_FILTER_BLOCK * GF_FILTER_ITEMS;
        TQP_LAUNCH(ctx, s, "fragment_rows",
                   (k_filter<GF_FILTER_BLOCK, GF_FILTER_ITEMS><<<grid_for(N, TILE, 0), GF_FILTER_BLOCK, 0, s>>>(
                       fp, N, nullptr, b.li, nullptr, J, b.d_join, b.fstatus, b.fcounter, ctx->d_err)));
    }
    if (o.d_join) TQP_TRY_HIP(hipMemcpyAsync(o.d_join, b.d_join, 8, hipMemcpyDeviceToDevice, s));
    int32_t* li = b.li;
    int32_t* ri = b.ri;
    if (b.lorder) {
        SrcPairs<uint32_t> lp{reinterpret_cast<const uint32_t*>(b.li), reinterpret_cast<const uint32_t*>(b.ri), J,
                              b.d_join};
        if ((st = radix_launch<Cfg, uint32_t>(b.lsort, lp, J, true, nullptr, 0xFFFFFFFFu,
                                              reinterpret_cast<uint32_t*>(b.li2), reinterpret_cast<uint32_t*>(b.ri2),
                                              ctx, s, "fragment_sort_rows", "fragment_sort_rows")) != TQP_OK)
            return st;
        li = b.li2;
        ri = b.ri2;
    }
    // the joined rows' columns: fact columns through li, dim columns through ri
    JoinedCols jc;
    for (int c = 0; c < f.n_fact_cols; ++c) {
        jc.col[jc.n] = f.fact_cols[c];
        jc.idx[jc.n++] = li;
    }
    if (b.join)
        for (int c = 0; c < f.n_dim_cols; ++c) {
            jc.col[jc.n] = f.dim_cols[c];
            jc.idx[jc.n++] = ri;
        }
    // 3. group key
    GroupCols g{};
    g.n = f.n_group;
    for (int i = 0; i < f.n_group; ++i) {
        const int c = f.group[i].col;
        g.col[i] = jc.col[c].data;
        g.type[i] = jc.col[c].type;
        g.side[i] = c >= f.n_fact_cols ? 1 : 0;
        if (b.dpush >= 0 && c >= f.n_fact_cols) {
            // the dim sort carried this column: the join wrote its values where the rows would be
            g.col[i] = ri;
            g.type[i] = TQP_I32;
            g.side[i] = 2;
        }
        g.bits[i] = f.group[i].bits;
    }
    // the one group column carried by the dim sort, with the bucket group-by
    // (which masks the key as the pack would): the group sort reads it directly
    const bool direct_key = b.bucket && f.n_group == 1 && g.side[0] == 2;
    if (!direct_key) {
        TQP_LAUNCH(ctx, s, "fragment_pack",
                   k_gf_pack<<<grid_for(J, 256 * 4, (int64_t)ctx->num_cus * 8), 256, 0, s>>>(
                       g, li, ri, J, b.d_join, b.gkey, ctx->d_err));
    }
    // 4. aggregate values (an empty side joins nothing: no row is read, and
    // its columns may be null)
    const bool no_rows = N == 0 || (b.join && f.n_dim == 0);
    for (int k = 0; k < f.n_agg; ++k) {
        if (!b.vals[k] || no_rows || (b.fpush && k == b.vsort)) continue;     // fpush: the join wrote it
        if ((st = eval_program(ctx, jc.col, jc.idx, jc.n, J, b.d_join, f.aggs[k].prog, f.aggs[k].nprog, b.vals[k], s,
                               "tqp_fragment_run", "fragment_value")) != TQP_OK)
            return st;
    }
    if (b.direct) return direct_groupby(ctx, f, o, b, s);
    // 5. group sort (distinct values first, low word then high word)
    const uint32_t* perm_in = nullptr;
    if (b.distinct >= 0) {
        SrcPermKey<1> a1{b.vals[b.distinct], nullptr, J, b.d_join};
        if ((st = radix_launch<Cfg, uint32_t>(b.sa, a1, J, true, nullptr, ~0u, b.ka, b.pa, ctx, s, "fragment_sort_value",
                                              "fragment_sort_value")) != TQP_OK)
            return st;
        SrcPermKey<2> a2{b.vals[b.distinct], b.pa, J, b.d_join};
        if ((st = radix_launch<Cfg, uint32_t>(b.sb, a2, J, true, nullptr, ~0u, b.kb, b.pb, ctx, s, "fragment_sort_value",
                                              "fragment_sort_value")) != TQP_OK)
            return st;
        perm_in = b.pb;
    }
    if (direct_key) {
        SrcColKeyVal64 a3{b.ri, b.vals[b.vsort], J, b.d_join, key_mask_for(b.gbits)};
        if ((st = radix_launch<Cfg, uint64_t>(b.sv, a3, J, true, nullptr, key_mask_for(b.gbits), b.kc, b.vc, ctx, s,
                                              "fragment_sort_group", "fragment_sort_group")) != TQP_OK)
            return st;
        return bucket_groupby<Cfg, int64_t>(ctx, f, o, b, b.kc, reinterpret_cast<const int64_t*>(b.vc),
                                            b.sv.pd.npass == 1 ? b.sv.hist : nullptr, s);
    }
    if (b.vsort >= 0) {
        SrcKeyVal64 a3{b.gkey, b.vals[b.vsort], J, b.d_join};
        if ((st = radix_launch<Cfg, uint64_t>(b.sv, a3, J, true, nullptr, key_mask_for(b.gbits), b.kc, b.vc, ctx, s,
                                              "fragment_sort_group", "fragment_sort_group")) != TQP_OK)
            return st;
        if (b.bucket)
            return bucket_groupby<Cfg, int64_t>(ctx, f, o, b, b.kc, reinterpret_cast<const int64_t*>(b.vc),
                                                b.sv.pd.npass == 1 ? b.sv.hist : nullptr, s);
    } else {
        SrcPermKey<0> a3{b.gkey, perm_in, J, b.d_join};
        if ((st = radix_launch<Cfg, uint32_t>(b.sc, a3, J, true, nullptr, key_mask_for(b.gbits), b.kc, b.pc, ctx, s,
                                              "fragment_sort_group", "fragment_sort_group")) != TQP_OK)
            return st;
    }
    // 6. runs: group starts, then one wave per group
    TQP_LAUNCH(ctx, s, "fragment_heads",
               k_gf_heads<<<grid_for(J, GF_HEAD_BLOCK * GF_HEAD_ITEMS, 0), GF_HEAD_BLOCK, 0, s>>>(
                   b.kc, J, b.d_join, b.gstart, b.d_groups, b.hstatus, b.hcounter, ctx->d_err));
    AggSet as{};
    as.n = f.n_agg;
    as.sk = b.vsort;
    as.sval = b.vsort >= 0 ? reinterpret_cast<const int64_t*>(b.vc) : nullptr;
    for (int k = 0; k < f.n_agg; ++k) {
        as.val[k] = k == b.vsort ? nullptr : b.vals[k];
        as.out[k] = f.aggs[k].out;
        as.op[k] = f.aggs[k].op;
    }
    const int64_t* dval = b.distinct >= 0 ? b.vals[b.distinct] : nullptr;
    const int64_t gw = (o.gcap + WAVE - 1) / WAVE;   // waves of 64 groups
    const int64_t waves = gw < (int64_t)ctx->num_cus * 32 ? gw : (int64_t)ctx->num_cus * 32;
    TQP_LAUNCH(ctx, s, "fragment_agg",
               k_gf_agg<<<grid_for(waves, GF_AGG_BLOCK / WAVE, 0), GF_AGG_BLOCK, 0, s>>>(
                   b.kc, b.pc, b.gstart, b.d_groups, b.d_join, J, as, dval, o.key, o.gcap, o.d_ngroups, b.d_written,
                   ctx->d_err));
    // 7. top-k over the first aggregate
    if (f.topk > 0) {
        const int64_t* v0 = static_cast<const int64_t*>(f.aggs[0].out);
        if ((st = topk_launch(b.topk, o.key, v0, v0, b.d_written, f.topk, o.top_key, o.top_val, b.tcnt, o.d_topk, s,
                              ctx)) != TQP_OK)
            return st;
    }
    return TQP_OK;
}

tqp_status check_general(tqp_ctx* ctx, const tqp_fragment* f, const tqp_fragment_out* o) {
    const char* who = "tqp_fragment_run";
    if (!f || !o) return fail(TQP_ERR_INVALID, "%s: null fragment or output", who);
    if (f->n_fact < 0 || f->n_dim < 0 || f->join_cap < 0 || o->gcap < 0) return fail(TQP_ERR_INVALID, "%s: negative size", who);
    if (f->n_fact > MAX_ELEMS || f->n_dim > MAX_ELEMS || f->join_cap > MAX_ELEMS || o->gcap > MAX_ELEMS)
        return fail(TQP_ERR_UNSUPPORTED, "%s: too large", who);
    const bool join = f->fact_key >= 0;
    const int nd = join ? f->n_dim_cols : 0;
    if (f->n_fact_cols < 1 || f->n_fact_cols + nd > GF_MAX_COLS || (join && f->n_dim_cols < 1) ||
        !f->fact_cols || (join && !f->dim_cols))
        return fail(TQP_ERR_INVALID, "%s: columns", who);
    auto col_ok = [&](const tqp_column& c, int64_t rows) {
        return (c.type == TQP_I8 || c.type == TQP_I32 || c.type == TQP_I64) && (rows == 0 || c.data);
    };
    for (int c = 0; c < f->n_fact_cols; ++c)
        if (!col_ok(f->fact_cols[c], f->n_fact)) return fail(TQP_ERR_INVALID, "%s: fact column %d", who, c);
    for (int c = 0; c < nd; ++c)
        if (!col_ok(f->dim_cols[c], f->n_dim)) return fail(TQP_ERR_INVALID, "%s: dim column %d", who, c);
    if (join) {
        if (f->fact_key >= f->n_fact_cols || f->fact_cols[f->fact_key].type != TQP_I32 || f->dim_key < 0 ||
            f->dim_key >= f->n_dim_cols || f->dim_cols[f->dim_key].type != TQP_I32)
            return fail(TQP_ERR_INVALID, "%s: join keys must be int32 columns", who);
    }
    if (f->n_group < 0 || f->n_group > TQP_FRAGMENT_MAX_GROUP_COLS || (f->n_group > 0 && !f->group))
        return fail(TQP_ERR_UNSUPPORTED, "%s: %d group columns", who, f->n_group);
    int bits = 0;
    for (int i = 0; i < f->n_group; ++i) {
        if (f->group[i].col < 0 || f->group[i].col >= f->n_fact_cols + nd || f->group[i].bits < 1)
            return fail(TQP_ERR_INVALID, "%s: group column %d", who, i);
        bits += f->group[i].bits;
    }
    if (bits > 31) return fail(TQP_ERR_UNSUPPORTED, "%s: group key of %d bits", who, bits);
    if (f->n_agg < 0 || f->n_agg > TQP_FRAGMENT_MAX_AGGS || (f->n_agg > 0 && !f->aggs))
        return fail(TQP_ERR_UNSUPPORTED, "%s: %d aggregates", who, f->n_agg);
    int ndist = 0;
    for (int k = 0; k < f->n_agg; ++k) {
        const tqp_agg& a = f->aggs[k];
        if (a.op < TQP_AGG_COUNT || a.op > TQP_AGG_COUNT_DISTINCT)
            return fail(TQP_ERR_INVALID, "%s: aggregate %d: op %d", who, k, a.op);
        if (o->gcap > 0 && !a.out) return fail(TQP_ERR_INVALID, "%s: aggregate %d has no output", who, k);
        ndist += a.op == TQP_AGG_COUNT_DISTINCT;
    }
    if (ndist > 1) return fail(TQP_ERR_UNSUPPORTED, "%s: at most one COUNT(DISTINCT)", who);
    if (f->value_bits != 0 && f->value_bits != 32 && f->value_bits != 64)
        return fail(TQP_ERR_UNSUPPORTED, "%s: value_bits = %d (0, 32 or 64)", who, f->value_bits);
    if (f->topk < 0 || f->topk > 1024 || (f->topk > 0 && (f->n_agg < 1 || f->aggs[0].op == TQP_AGG_AVG)))
        return fail(TQP_ERR_UNSUPPORTED, "%s: topk %d (1..1024 over an integer first aggregate)", who, f->topk);
    if (f->topk > 0 && (!o->top_key || !o->top_val || !o->d_topk)) return fail(TQP_ERR_INVALID, "%s: top outputs", who);
    if (!o->key || !o->d_ngroups) return fail(TQP_ERR_INVALID, "%s: null output", who);
    // every program checked before anything is launched
    tqp_status st;
    if (f->n_fact_pred > 0 &&
        (st = eval_program(ctx, f->fact_cols, nullptr, f->n_fact_cols, 0, nullptr, f->fact_pred, f->n_fact_pred,
                           nullptr, nullptr, "tqp_fragment_run: fact predicate", "")) != TQP_OK)
        return st;
    if (join && f->n_dim_pred > 0 &&
        (st = eval_program(ctx, f->dim_cols, nullptr, f->n_dim_cols, 0, nullptr, f->dim_pred, f->n_dim_pred, nullptr,
                           nullptr, "tqp_fragment_run: dim predicate", "")) != TQP_OK)
        return st;
    JoinedCols jc;
    for (int c = 0; c < f->n_fact_cols; ++c) jc.col[jc.n++] = f->fact_cols[c];
    for (int c = 0; c < nd; ++c) jc.col[jc.n++] = f->dim_cols[c];
    for (int k = 0; k < f->n_agg; ++k) {
        const tqp_agg& a = f->aggs[k];
        if (a.op == TQP_AGG_COUNT) continue;
        if (!a.prog) return fail(TQP_ERR_INVALID, "%s: aggregate %d has no program", who, k);
        if ((st = eval_program(ctx, jc.col, nullptr, jc.n, 0, nullptr, a.prog, a.nprog, nullptr, nullptr,
                               "tqp_fragment_run: aggregate", "")) != TQP_OK)
            return st;
    }
    return TQP_OK;
}

}  // namespace
}  // namespace tqp

using namespace tqp;

extern "C" tqp_status tqp_fragment_run(tqp_ctx* ctx, const tqp_fragment* f, const tqp_fragment_out* o, void* ws,
                                       size_t* ws_bytes, hipStream_t stream) {
    clear_error();
    if (!ctx) return fail(TQP_ERR_INVALID, "tqp_fragment_run: null context");
    tqp_status st = check_general(ctx, f, o);
    if (st != TQP_OK) return st;
    tqp_fragment fd = *f;
    if (fd.fact_key < 0) {
        fd.n_dim_cols = 0;
        fd.n_dim = 0;
        fd.n_dim_pred = 0;
    }
    return with_radix_cfg(ctx->digit_bits, [&](auto cfg) -> tqp_status {
        using Cfg = decltype(cfg);
        GenBufs<Cfg> b;
        Arena a;
        auto plan = [&](Arena& ar) { gen_reserve<Cfg>(ar, fd, *o, b); };
        tqp_status s2 = with_workspace(ctx, ws, ws_bytes, stream, plan, a);
        if (s2 != TQP_OK || !ws) return s2;
        if ((s2 = fill_zero(a.base, a.zsize, stream, ctx)) != TQP_OK) return s2;
        return gen_launch<Cfg>(ctx, fd, *o, b, stream);
    });
}
