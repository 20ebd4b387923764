// Hash-based equi-join (Section 5.3, Algorithm 3), the variant of the join
// the paper measures against the sort-based one, in the partitioned form the
// section names as the next step.
//
// The paper builds a table of m slots indexed by a hash of the key from one
// side, probes it with the other, and repeats build and probe as many times
// as the most crowded slot holds rows, because a PyTorch scatter keeps one
// row per slot.  Here both sides are first split into 2^P partitions by the
// top bits of h = key * odd constant mod 2^32 (a bijection of the key, so
// equal keys and only equal keys share h), and each partition is joined in
// LDS, where a table build and its probes cost no HBM traffic:
//
//   partition  radix passes per side over the top P bits of h (the sort's
//              histogram, a pre-counted 8-bit pass and, for P > 8, a second
//              pass), rows carried as (h, row); P leaves up to about 2000
//              right rows per partition (one build of a 4096-slot table);
//   plan       the partition starts (one search per partition) and a list of
//              work items: (partition, chunk of left rows);
//   join       persistent blocks take items.  For every chunk of at most
//              PJ_RCAP right rows of the item's partition the block builds
//              an LDS table keyed by key + 1: one slot per distinct key
//              (linear probing, one compare-and-swap per row), the rows of a
//              key counted, an exclusive scan of the counts over the slots,
//              then every right row placed in its key's run (the slot's
//              count-then-scan layout: inserts are O(1) per row whatever the
//              number of duplicates, and the matches of a key are one
//              contiguous run).  Each left row then finds its key's run with
//              one probe; a round of left rows reserves its output range
//              with one atomic add and writes (lrow, rrow) pairs, short runs
//              by the row's own lane, long runs by the whole wave.
//
// Output rows come in no fixed order (partition order, then the order in
// which rounds reserve their ranges); the set of pairs is exact.
#include "dev.hpp"
#include "host.hpp"

namespace tqp {
namespace {

constexpr uint32_t PJ_MUL = 0x9E3779B1u;        // odd: key -> h is a bijection mod 2^32
constexpr int PJ_BLOCK = 512;
constexpr int PJ_ITEMS = 2;                      // left rows per thread per round
constexpr int PJ_ROUND = PJ_BLOCK * PJ_ITEMS;
constexpr int PJ_RCAP = 2048;                    // right rows per table build
constexpr int PJ_LOG2S = 12;                     // table slots: 4096 (load factor <= 0.5)
constexpr int PJ_S = 1 << PJ_LOG2S;
constexpr int PJ_LCHUNK = 16384;                 // left rows per work item
constexpr int PJ_MAXP = 16;                      // partition bits: at most two 8-bit radix passes
constexpr int PJ_LANE_MAX = 4;                   // an item with a longer run is written by the whole wave
constexpr int PJ_WAVE_RUN = 32;                  // runs this long: one at a time, 64 consecutive pairs per step
constexpr int PJ_PLAN_BLOCK = 1024;

static_assert(PJ_RCAP % PJ_BLOCK == 0, "right rows split evenly over the block");
static_assert(PJ_S % PJ_BLOCK == 0, "slots split evenly over the block");
static_assert(32 - PJ_MAXP - PJ_LOG2S >= 0, "slot bits lie below the partition bits");

// Rows as (h, row): row = the caller's row id, or the element index.  A
// negative key is reported and its row left out.
struct SrcHashRows {
    const int32_t* key;
    const int32_t* row;
    int64_t n_upper;
    const int64_t* d_n;
    uint32_t* flags;
    __device__ int64_t size() const {
        if (!d_n) return n_upper;
        const int64_t n = *d_n;
        return n < n_upper ? n : n_upper;
    }
    __device__ bool load_key(int64_t i, uint32_t& k) const {
        const int32_t x = key[i];
        if (x < 0) set_flag(flags, FLAG_KEY_RANGE);
        k = (uint32_t)x * PJ_MUL;
        return x >= 0;
    }
    __device__ bool load(int64_t i, uint32_t& k, uint32_t& v) const {
        const int32_t x = key[i];
        k = (uint32_t)x * PJ_MUL;
        v = row ? (uint32_t)row[i] : (uint32_t)i;
        return x >= 0;
    }
};

constexpr uint32_t pj_inv(uint32_t a) {
    uint32_t x = a;                                  // Newton's iteration for the inverse mod 2^32
    for (int i = 0; i < 5; ++i) x *= 2u - a * x;
    return x;
}
constexpr uint32_t PJ_INV = pj_inv(PJ_MUL);
static_assert(PJ_MUL * PJ_INV == 1u, "PJ_INV inverts PJ_MUL");

// Start of every partition in the partitioned hashes of one side: start[p]
// = first row whose top P bits of h are >= p, start[2^P] = the row count (one
// binary search per partition).
__global__ void __launch_bounds__(256)
k_pj_bounds(const uint32_t* h, const int64_t* d_cnt, int P, int64_t* start) {
    const int64_t np = int64_t(1) << P;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > np) return;
    const int64_t n = *d_cnt;
    if (p == np) {
        start[p] = n;
        return;
    }
    const int sh = 32 - P;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)(h[mid] >> sh) < p) lo = mid + 1;
        else hi = mid;
    }
    start[p] = lo;
}

// The work items: a partition with rows on both sides gives ceil(left rows /
// LCHUNK) items; item_pre[p] = the items of the partitions before p (np + 1
// entries).  One block.
__global__ void __launch_bounds__(PJ_PLAN_BLOCK)
k_pj_plan(const int64_t* lstart, const int64_t* rstart, int np, int64_t* item_pre) {
    __shared__ int64_t s_w[PJ_PLAN_BLOCK / WAVE];
    __shared__ int64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int p0 = 0; p0 < np; p0 += PJ_PLAN_BLOCK) {
        const int p = p0 + threadIdx.x;
        const int64_t nl = p < np ? lstart[p + 1] - lstart[p] : 0, nr = p < np ? rstart[p + 1] - rstart[p] : 0;
        const int64_t it = (nl > 0 && nr > 0) ? (nl + PJ_LCHUNK - 1) / PJ_LCHUNK : 0;
        int64_t ti;
        const int64_t ei = block_excl_sum<PJ_PLAN_BLOCK>(it, s_w, &ti);
        if (p < np) item_pre[p] = s_carry + ei;
        __syncthreads();
        if (threadIdx.x == 0) s_carry += ti;
        __syncthreads();
    }
    if (threadIdx.x == 0) item_pre[np] = s_carry;
}

struct PjSmem {
    uint32_t key[PJ_S];          // key + 1, 0 = free
    uint32_t cur[PJ_S];          // count, then (after the scan and placement) the end of the key's run
    uint32_t rows[PJ_RCAP];      // right rows grouped by key
    int64_t w64[PJ_BLOCK / WAVE];
    uint32_t w32[PJ_BLOCK / WAVE];
    int64_t base;
    int64_t item;
    int32_t part;
};

__device__ __forceinline__ uint32_t pj_slot(uint32_t h, int P) {
    return (h >> (32 - P - PJ_LOG2S)) & (PJ_S - 1);
}

// Builds the table of right rows [r0, r1) of a partition (hashes rh, rows rv).
__device__ void pj_build(PjSmem& sm, const uint32_t* rh, const uint32_t* rv, int64_t r0, int64_t r1, int P) {
    constexpr int RPT = PJ_RCAP / PJ_BLOCK;
    for (int i = threadIdx.x; i < PJ_S; i += PJ_BLOCK) {
        sm.key[i] = 0;
        sm.cur[i] = 0;
    }
    __syncthreads();
    uint32_t slot[RPT], val[RPT];
    bool in[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int64_t i = r0 + threadIdx.x + (int64_t)j * PJ_BLOCK;
        in[j] = i < r1;
        const int64_t ic = in[j] ? i : r0;         // r1 > r0: the chunk is not empty
        const uint32_t h = rh[ic];
        val[j] = rv[ic];
        slot[j] = pj_slot(h, P);
        const uint32_t k1 = h * PJ_INV + 1u;      // key + 1, never 0 for keys in [0, 2^31)
        if (in[j]) {
            // at most PJ_RCAP keys in PJ_S slots: a free or matching slot is always reached
            for (;;) {
                const uint32_t old = atomicCAS(&sm.key[slot[j]], 0u, k1);
                if (old == 0u || old == k1) break;
                slot[j] = (slot[j] + 1) & (PJ_S - 1);
            }
            atomicAdd(&sm.cur[slot[j]], 1u);
        }
    }
    __syncthreads();
    // count -> start of the key's run: wave w scans its contiguous slice of
    // slots 64 at a time (consecutive lanes, consecutive words: no bank
    // conflicts), then adds the totals of the slices before it
    {
        constexpr int W = PJ_BLOCK / WAVE, SLICE = PJ_S / W;
        const int w = threadIdx.x / WAVE, l = lane_id();
        uint32_t carry = 0;
        for (int c = w * SLICE; c < (w + 1) * SLICE; c += WAVE) {
            const uint32_t x = sm.cur[c + l];
            const uint32_t inc = wave_incl_sum(x);
            sm.cur[c + l] = carry + inc - x;
            carry += wave_read(inc, WAVE - 1);
        }
        if (l == 0) sm.w32[w] = carry;
        __syncthreads();
        uint32_t off = 0;
        for (int ww = 0; ww < w; ++ww) off += sm.w32[ww];
        if (off)
            for (int c = w * SLICE; c < (w + 1) * SLICE; c += WAVE) sm.cur[c + l] += off;
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < RPT; ++j)
        if (in[j]) sm.rows[atomicAdd(&sm.cur[slot[j]], 1u)] = val[j];   // cur ends at the run's end
    __syncthreads();
}

// Joins left rows [l0, l1) of a partition against the table in sm.
__device__ void pj_probe(PjSmem& sm, const uint32_t* lh, const uint32_t* lv, int64_t l0, int64_t l1, int P,
                         int32_t* out_l, int32_t* out_r, int64_t cap, int64_t* total) {
    const int w = threadIdx.x / WAVE, l = lane_id();
    for (int64_t b = l0; b < l1; b += PJ_ROUND) {
        uint32_t start[PJ_ITEMS], cnt[PJ_ITEMS], lrow[PJ_ITEMS];
        // item j of lane l of wave w: row b + (w * ITEMS + j) * 64 + l (coalesced)
#pragma unroll
        for (int j = 0; j < PJ_ITEMS; ++j) {
            const int64_t i = b + (int64_t)(w * PJ_ITEMS + j) * WAVE + l;
            const bool in = i < l1;
            const int64_t ic = in ? i : l0;
            const uint32_t h = lh[ic];
            lrow[j] = lv[ic];
            uint32_t s = pj_slot(h, P);
            const uint32_t k1 = h * PJ_INV + 1u;
            start[j] = 0;
            cnt[j] = 0;
            if (in) {
                for (;;) {
                    const uint32_t kk = sm.key[s];
                    if (kk == k1) {
                        const uint32_t e = sm.cur[s];
                        const uint32_t st = s ? sm.cur[s - 1] : 0u;       // the run before ends where this begins
                        start[j] = st;
                        cnt[j] = e - st;
                        break;
                    }
                    if (kk == 0u) break;
                    s = (s + 1) & (PJ_S - 1);
                }
            }
        }
        // output offsets: wave scans in item order, then the waves before, then one atomic per round
        int64_t off[PJ_ITEMS];
        int64_t run = 0;
#pragma unroll
        for (int j = 0; j < PJ_ITEMS; ++j) {
            const int64_t inc = wave_incl_sum((int64_t)cnt[j]);
            off[j] = run + inc - cnt[j];
            run += wave_read(inc, WAVE - 1);
        }
        if (l == 0) sm.w64[w] = run;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t t = 0;
            for (int ww = 0; ww < PJ_BLOCK / WAVE; ++ww) t += sm.w64[ww];
            sm.base = t ? atomic_add(total, t) : 0;
        }
        __syncthreads();
        int64_t wbase = sm.base;
        for (int ww = 0; ww < w; ++ww) wbase += sm.w64[ww];
#pragma unroll
        for (int j = 0; j < PJ_ITEMS; ++j) {
            if (!__any(cnt[j] > (uint32_t)PJ_LANE_MAX)) {
                // every run of the item is short: each lane writes its own
                const int64_t o = wbase + off[j];
                for (uint32_t q = 0; q < cnt[j]; ++q) {
                    if (o + q < cap) {
                        out_l[o + q] = (int32_t)lrow[j];
                        out_r[o + q] = (int32_t)sm.rows[start[j] + q];
                    }
                }
            } else {
                // some run is long.  Runs of at least PJ_WAVE_RUN pairs: the
                // whole wave writes each; the shorter ones: the wave writes
                // their pairs 64 at a time, each lane finding the left row its
                // pair belongs to
                const bool lng = cnt[j] >= (uint32_t)PJ_WAVE_RUN;
                const int64_t oc2 = lng ? 0 : (int64_t)cnt[j];
                const int64_t incl2 = wave_incl_sum(oc2);
                const int64_t excl2 = incl2 - oc2, tot2 = wave_read(incl2, WAVE - 1);
                const int64_t o = wbase + off[j];
                for (int64_t q0 = 0; q0 < tot2; q0 += WAVE) {
                    const int64_t q = q0 + l;
                    const int src = wave_run_owner(excl2, q);
                    const int64_t t = q - wave_shfl(excl2, src);
                    const uint32_t st = wave_shfl(start[j], src);
                    const int32_t lr = (int32_t)wave_shfl(lrow[j], src);
                    const int64_t oo = wave_shfl(o, src) + t;
                    if (q < tot2 && oo < cap) {
                        out_l[oo] = lr;
                        out_r[oo] = (int32_t)sm.rows[st + t];
                    }
                }
                uint64_t m = ballot(lng);
                while (m) {
                    const int src = __ffsll((unsigned long long)m) - 1;
                    m &= m - 1;
                    const int64_t oo = wave_read(o, src);
                    const uint32_t c = wave_read(cnt[j], src);
                    const uint32_t st = wave_read(start[j], src);
                    const int32_t lr = (int32_t)wave_read(lrow[j], src);
                    for (uint32_t q = l; q < c; q += WAVE) {
                        if (oo + q < cap) {
                            out_l[oo + q] = lr;
                            out_r[oo + q] = (int32_t)sm.rows[st + q];
                        }
                    }
                }
            }
        }
        __syncthreads();         // sm.base and sm.w64 are rewritten by the next round
    }
}

// Three blocks per CU: 40 KB of LDS each, and at most 84 VGPRs (6 waves per
// SIMD; two left rows per thread and round keep the spills to a few).
__global__ void __launch_bounds__(PJ_BLOCK, 6)
k_pj_join(const uint32_t* lh, const uint32_t* lv, const uint32_t* rh, const uint32_t* rv, const int64_t* lstart,
          const int64_t* rstart, const int64_t* item_pre, int P, uint32_t* counter, int32_t* out_l, int32_t* out_r,
          int64_t cap, int64_t* total) {
    __shared__ PjSmem sm;
    const int np = 1 << P;
    const int64_t nitems = item_pre[np];
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t g = atomicAdd(counter, 1u);
            sm.item = g;
            if (g < nitems) {
                int lo = 0, hi = np - 1;                  // the last partition p with item_pre[p] <= g
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (item_pre[mid] <= g) lo = mid;
                    else hi = mid - 1;
                }
                sm.part = lo;
            }
        }
        __syncthreads();
        const int64_t g = sm.item;
        const int p = sm.part;
        __syncthreads();
        if (g >= nitems) break;
        const int64_t lc = g - item_pre[p];
        const int64_t l0 = lstart[p] + lc * PJ_LCHUNK;
        const int64_t l1 = l0 + PJ_LCHUNK < lstart[p + 1] ? l0 + PJ_LCHUNK : lstart[p + 1];
        for (int64_t r0 = rstart[p]; r0 < rstart[p + 1]; r0 += PJ_RCAP) {
            const int64_t r1 = r0 + PJ_RCAP < rstart[p + 1] ? r0 + PJ_RCAP : rstart[p + 1];
            pj_build(sm, rh, rv, r0, r1, P);
            pj_probe(sm, lh, lv, l0, l1, P, out_l, out_r, cap, total);
        }
    }
}

__global__ void k_pj_finish(const int64_t* total, int64_t cap, int64_t* d_count, uint32_t* flags) {
    const int64_t t = *total;
    *d_count = t;
    if (t > cap) set_flag(flags, FLAG_CAPACITY);
}

// Partition bits for nr right rows: the fewest that leave at most about
// 31/32 of PJ_RCAP right rows per partition on average (so that most
// partitions take one table build; larger ones take several), at most
// PJ_MAXP, at least one.
int pj_bits(int64_t nr) {
    int P = 1;
    while (P < PJ_MAXP && (nr >> P) > PJ_RCAP - PJ_RCAP / 32) ++P;
    return P;
}

}  // namespace
}  // namespace tqp

using namespace tqp;

extern "C" {

tqp_status tqp_hash_join(tqp_ctx* ctx, const int32_t* lkey, const int32_t* lrow, int64_t nl, const int64_t* d_nl,
                         const int32_t* rkey, const int32_t* rrow, int64_t nr, const int64_t* d_nr, int32_t* out_l,
                         int32_t* out_r, int64_t cap, int64_t* d_count, void* ws, size_t* ws_bytes,
                         hipStream_t stream) {
    clear_error();
    if (!ctx || !d_count || nl < 0 || nr < 0 || cap < 0 || (nl > 0 && !lkey) || (nr > 0 && !rkey) ||
        (cap > 0 && (!out_l || !out_r)))
        return fail(TQP_ERR_INVALID, "tqp_hash_join: null pointer or negative size");
    if (nl > MAX_ELEMS || nr > MAX_ELEMS) return fail(TQP_ERR_UNSUPPORTED, "tqp_hash_join: input too large");
    const int P = pj_bits(nr);
    const int np = 1 << P;
    using Cfg = R8;            // P > 8 bits take two 8-bit passes (longer digit runs per write than wider digits)
    RadixBufs<Cfg, uint32_t> lb, rb;
    uint32_t *lh = nullptr, *lv = nullptr, *rh = nullptr, *rv = nullptr, *counter = nullptr;
    int64_t *lstart = nullptr, *rstart = nullptr, *item_pre = nullptr, *total = nullptr;
    Arena a;
    auto plan = [&](Arena& ar) {
        lb = radix_reserve<Cfg, uint32_t>(ar, nl, 32, 32 - P);
        rb = radix_reserve<Cfg, uint32_t>(ar, nr, 32, 32 - P);
        counter = ar.zero<uint32_t>(1);
        total = ar.zero<int64_t>(1);
        lh = ar.scratch<uint32_t>(nl);
        lv = ar.scratch<uint32_t>(nl);
        rh = ar.scratch<uint32_t>(nr);
        rv = ar.scratch<uint32_t>(nr);
        lstart = ar.scratch<int64_t>(np + 1);
        rstart = ar.scratch<int64_t>(np + 1);
        item_pre = ar.scratch<int64_t>(np + 1);
    };
    tqp_status st = with_workspace(ctx, ws, ws_bytes, stream, plan, a);
    if (st != TQP_OK || !ws) return st;
    if ((st = fill_zero(a.base, a.zsize, stream, ctx)) != TQP_OK) return st;
    // both sides into 2^P partitions by the top bits of h (one or two passes each; an
    // empty side launches nothing and leaves its histogram zero)
    SrcHashRows ls{lkey, lrow, nl, d_nl, ctx->d_err};
    SrcHashRows rs{rkey, rrow, nr, d_nr, ctx->d_err};
    if ((st = radix_launch<Cfg, uint32_t>(lb, ls, nl, true, nullptr, ~0u, lh, lv, ctx, stream, "hashjoin_part_l",
                                          "hashjoin_part_l")) != TQP_OK)
        return st;
    if ((st = radix_launch<Cfg, uint32_t>(rb, rs, nr, true, nullptr, ~0u, rh, rv, ctx, stream, "hashjoin_part_r",
                                          "hashjoin_part_r")) != TQP_OK)
        return st;
    TQP_LAUNCH(ctx, stream, "hashjoin_bounds",
               k_pj_bounds<<<grid_for(np + 1, 256, 0), 256, 0, stream>>>(lh, lb.d_cnt, P, lstart));
    TQP_LAUNCH(ctx, stream, "hashjoin_bounds",
               k_pj_bounds<<<grid_for(np + 1, 256, 0), 256, 0, stream>>>(rh, rb.d_cnt, P, rstart));
    TQP_LAUNCH(ctx, stream, "hashjoin_plan",
               k_pj_plan<<<1, PJ_PLAN_BLOCK, 0, stream>>>(lstart, rstart, np, item_pre));
    static const int per_cu = [] {
        int b = 2;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_pj_join, PJ_BLOCK, 0) != hipSuccess) b = 2;
        return b < 1 ? 1 : b;
    }();
    // items: at most one per partition plus one per LCHUNK left rows
    const int64_t items_upper = (nl + PJ_LCHUNK - 1) / PJ_LCHUNK + np;
    if (nl > 0 && nr > 0) {
        const int grid = grid_for(items_upper, 1, (int64_t)ctx->num_cus * per_cu);
        TQP_LAUNCH(ctx, stream, "hashjoin_join",
                   k_pj_join<<<grid, PJ_BLOCK, 0, stream>>>(lh, lv, rh, rv, lstart, rstart, item_pre, P, counter,
                                                            out_l, out_r, cap, total));
    }
    TQP_LAUNCH(ctx, stream, "hashjoin_finish", k_pj_finish<<<1, 1, 0, stream>>>(total, cap, d_count, ctx->d_err));
    return TQP_OK;
}

}  // extern "C"
