// Hash-based group-by aggregation: the alternative to the sort-based
// aggregation of Section 5.4 / Algorithm 2.  Section 6 traces the paper's
// loss on aggregation-heavy queries to its sorting, against systems that
// aggregate in hash tables; this is that hash aggregation, so the two can be
// compared on the same inputs.  It also evaluates the aggregates Section 4
// lists besides sum and count: min, max and count with DISTINCT.
//
// Table: open addressing over m = 2^log2m slots of 32 bytes (the power of two
// at or above 2 * gcap), home slot a multiplicative hash of the key, linear
// probing.  A slot holds key + 1 (0 = free), count, sum, and min / max in an
// order-preserving unsigned encoding, so that a zero-filled table is a valid
// empty one and min and max are both unsigned atomic maxima:
//   ord(v) = v ^ 2^63           max  = max ord(v)
//   nmin   = max ~ord(v)        min  = ~nmin ^ 2^63
// A row finds its group's slot (claiming the first free one with a
// compare-and-swap when the key is new) and adds itself with atomics.  New
// groups stop being admitted once gcap exist (TQP_DEVERR_CAPACITY), and a
// probe gives up after HA_PROBE_LIMIT slots, so every probe ends even on
// a full table.  Probes read slots with plain loads, which another CU's
// claim may not have reached yet (a free slot read from a stale line): a
// free slot is always confirmed by the compare-and-swap or an agent-scope
// load.
//
// Few groups (gcap <= HA_LDS_GROUPS): each block first aggregates its rows
// in a table in LDS and merges its groups into the global table at the end,
// so the global atomics per block are one per group, not one per row.
//
// COUNT(DISTINCT d): a second table of 64-bit entries (key + 1, d) as a set;
// the row that inserts a pair adds one to its group's distinct count.
//
// Output: one row per group in no fixed order (slot order, compacted by wave
// ballots), the group count in *d_ngroups.
#include "dev.hpp"
#include "host.hpp"

namespace tqp {
namespace {

constexpr int HA_BLOCK = 256;
constexpr int HA_ITEMS = 4;                 // rows per thread per step, probed in lockstep
constexpr int HA_LDS = 1024;                // slots of the per-block table
constexpr int64_t HA_LDS_GROUPS = HA_LDS / 2;
constexpr uint32_t HA_PROBE_LIMIT = 4096;
constexpr unsigned long long ORD_BIAS = 1ull << 63;

struct alignas(32) HaSlot {
    uint32_t key1;                  // key + 1, 0 = free
    uint32_t cnt;
    unsigned long long sum;         // two's-complement int64 sum
    unsigned long long nmin;        // max of ~ord(v)
    unsigned long long max;         // max of ord(v)
};
static_assert(sizeof(HaSlot) == 32, "one slot per 32-byte sector");

__device__ __forceinline__ uint32_t ha_home(uint64_t key, int log2m) {
    return log2m ? (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - log2m)) : 0u;
}

template <class T>
__device__ __forceinline__ void add_nr(T* p, T v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void max_nr(unsigned long long* p, unsigned long long v) {
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct HaArgs {
    const int32_t* gkey;
    const int64_t* val;
    const int32_t* dval;
    int64_t n_upper;
    const int64_t* d_n;
    HaSlot* table;
    int log2m;
    uint32_t* ndist;                // per slot, COUNT(DISTINCT)
    unsigned long long* set;        // (key + 1) << 32 | d, 0 = free
    int log2s;
    uint32_t* d_groups;             // groups admitted so far
    uint32_t gcap;
    uint32_t* flags;
};

__device__ __forceinline__ int64_t ha_rows(const HaArgs& a) {
    int64_t n = a.n_upper;
    if (a.d_n) { const int64_t t = *a.d_n; n = t < n ? t : n; }
    return n;
}

// Finds (or creates) the global slots of ITEMS keys in lockstep: one round of
// slot loads for all live items per step.  slot[j] = -1 when the item is not
// live or its group could not be admitted.
template <int IT>
__device__ __forceinline__ void ha_find(const HaArgs& a, const uint32_t (&k1)[IT], const bool (&in)[IT],
                                        int32_t (&slot)[IT]) {
    const uint32_t mask = (uint32_t)((uint64_t(1) << a.log2m) - 1);
    const uint32_t limit = mask + 1 < HA_PROBE_LIMIT ? mask + 1 : HA_PROBE_LIMIT;
    uint32_t s[IT];
    bool live[IT];
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        s[j] = ha_home(k1[j], a.log2m);
        live[j] = in[j];
        slot[j] = -1;
    }
    for (uint32_t p = 0; p < limit; ++p) {
        bool any = false;
#pragma unroll
        for (int j = 0; j < IT; ++j) any |= live[j];
        if (!any) break;
        uint32_t cur[IT];
#pragma unroll
        for (int j = 0; j < IT; ++j) cur[j] = live[j] ? a.table[s[j]].key1 : 0u;
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            if (!live[j]) continue;
            bool done = cur[j] == k1[j];
            if (!done && cur[j] == 0u) {
                // The plain load may come from a stale cache line, so a 0 is
                // confirmed by the compare-and-swap, or, once gcap groups
                // exist, by an agent-scope load before the row is refused.
                uint32_t old;
                if (ld_relaxed(a.d_groups) >= a.gcap) {
                    old = ld_relaxed(&a.table[s[j]].key1);
                    if (old == 0u) {
                        set_flag(a.flags, FLAG_CAPACITY);     // a new group beyond gcap
                        live[j] = false;
                        continue;
                    }
                } else {
                    old = atomicCAS(&a.table[s[j]].key1, 0u, k1[j]);
                    if (old == 0u) add_nr(a.d_groups, 1u);
                }
                done = old == 0u || old == k1[j];
            }
            if (done) {
                slot[j] = (int32_t)s[j];
                live[j] = false;
            } else {
                s[j] = (s[j] + 1) & mask;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < IT; ++j)
        if (live[j]) set_flag(a.flags, FLAG_CAPACITY);      // probe limit reached
}

// Inserts the pairs (key + 1, d) into the set; ins[j] is true for the item
// that inserted its pair (the first row of that pair to arrive).
template <int IT>
__device__ __forceinline__ void ha_distinct(const HaArgs& a, const uint32_t (&k1)[IT], const int32_t (&d)[IT],
                                            const bool (&in)[IT], bool (&ins)[IT]) {
    const uint32_t mask = (uint32_t)((uint64_t(1) << a.log2s) - 1);
    const uint32_t limit = mask + 1 < HA_PROBE_LIMIT ? mask + 1 : HA_PROBE_LIMIT;
    unsigned long long e[IT];
    uint32_t s[IT];
    bool live[IT];
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        e[j] = ((unsigned long long)k1[j] << 32) | (uint32_t)d[j];
        s[j] = ha_home(e[j], a.log2s);
        live[j] = in[j];
        ins[j] = false;
    }
    for (uint32_t p = 0; p < limit; ++p) {
        bool any = false;
#pragma unroll
        for (int j = 0; j < IT; ++j) any |= live[j];
        if (!any) break;
        unsigned long long cur[IT];
#pragma unroll
        for (int j = 0; j < IT; ++j) cur[j] = live[j] ? a.set[s[j]] : 0ull;
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            if (!live[j]) continue;
            bool done = cur[j] == e[j];
            if (!done && cur[j] == 0ull) {
                const unsigned long long old = atomicCAS(&a.set[s[j]], 0ull, e[j]);
                ins[j] = old == 0ull;
                done = old == 0ull || old == e[j];
            }
            if (done) live[j] = false;
            else s[j] = (s[j] + 1) & mask;
        }
    }
#pragma unroll
    for (int j = 0; j < IT; ++j)
        if (live[j]) set_flag(a.flags, FLAG_CAPACITY);
}

// Loads ITEMS rows: row r of step `base` is base + j * HA_BLOCK + tid, so each
// item's loads are coalesced across the block.
template <bool VAL, bool DIST>
__device__ __forceinline__ void ha_load(const HaArgs& a, int64_t n, int64_t base, uint32_t (&k1)[HA_ITEMS],
                                        bool (&in)[HA_ITEMS], int64_t (&v)[HA_ITEMS], int32_t (&d)[HA_ITEMS]) {
#pragma unroll
    for (int j = 0; j < HA_ITEMS; ++j) {
        const int64_t i = base + (int64_t)j * HA_BLOCK + threadIdx.x;
        const bool ok = i < n;
        const int32_t k = ok ? a.gkey[i] : 0;
        if (ok && k < 0) set_flag(a.flags, FLAG_KEY_RANGE);
        in[j] = ok && k >= 0;
        k1[j] = (uint32_t)k + 1u;
        v[j] = VAL && ok ? a.val[i] : 0;
        d[j] = DIST && ok ? a.dval[i] : 0;
    }
}

template <bool VAL, bool MINMAX>
__device__ __forceinline__ void ha_update(HaSlot* t, int32_t s, int64_t v) {
    add_nr(&t[s].cnt, 1u);
    if (VAL) add_nr(&t[s].sum, (unsigned long long)v);
    if (MINMAX) {
        const unsigned long long o = (unsigned long long)v ^ ORD_BIAS;
        max_nr(&t[s].max, o);
        max_nr(&t[s].nmin, ~o);
    }
}

// Every row straight into the global table (many groups).
template <bool VAL, bool MINMAX, bool DIST>
__global__ void __launch_bounds__(HA_BLOCK) k_ha_global(HaArgs a) {
    const int64_t n = ha_rows(a);
    const int64_t step = (int64_t)gridDim.x * HA_BLOCK * HA_ITEMS;
    for (int64_t base = (int64_t)blockIdx.x * HA_BLOCK * HA_ITEMS; base < n; base += step) {
        uint32_t k1[HA_ITEMS];
        bool in[HA_ITEMS];
        int64_t v[HA_ITEMS];
        int32_t d[HA_ITEMS];
        ha_load<VAL, DIST>(a, n, base, k1, in, v, d);
        int32_t slot[HA_ITEMS];
        ha_find(a, k1, in, slot);
#pragma unroll
        for (int j = 0; j < HA_ITEMS; ++j)
            if (slot[j] >= 0) ha_update<VAL, MINMAX>(a.table, slot[j], v[j]);
        if (DIST) {
            bool ok[HA_ITEMS], ins[HA_ITEMS];
#pragma unroll
            for (int j = 0; j < HA_ITEMS; ++j) ok[j] = slot[j] >= 0;
            ha_distinct(a, k1, d, ok, ins);
#pragma unroll
            for (int j = 0; j < HA_ITEMS; ++j)
                if (ins[j]) add_nr(&a.ndist[slot[j]], 1u);
        }
    }
}

// Few groups: a per-block LDS table first, merged into the global table at
// the end.  A row whose LDS probe fails (more groups than the LDS table
// holds, which only an input with more than gcap groups reaches) goes to the
// global table directly.
template <bool VAL, bool MINMAX, bool DIST>
__global__ void __launch_bounds__(HA_BLOCK) k_ha_local(HaArgs a) {
    constexpr int SV = VAL ? HA_LDS : 1, SM = MINMAX ? HA_LDS : 1, SD = DIST ? HA_LDS : 1;
    __shared__ uint32_t s_key[HA_LDS];
    __shared__ uint32_t s_cnt[HA_LDS];
    __shared__ unsigned long long s_sum[SV];
    __shared__ unsigned long long s_max[SM];
    __shared__ unsigned long long s_nmin[SM];
    __shared__ uint32_t s_nd[SD];
    for (int i = threadIdx.x; i < HA_LDS; i += HA_BLOCK) {
        s_key[i] = 0u;
        s_cnt[i] = 0u;
        if (VAL) s_sum[i] = 0ull;
        if (MINMAX) s_max[i] = 0ull, s_nmin[i] = 0ull;
        if (DIST) s_nd[i] = 0u;
    }
    __syncthreads();
    const int lg = 31 - __clz(HA_LDS);
    const int64_t n = ha_rows(a);
    const int64_t step = (int64_t)gridDim.x * HA_BLOCK * HA_ITEMS;
    for (int64_t base = (int64_t)blockIdx.x * HA_BLOCK * HA_ITEMS; base < n; base += step) {
        uint32_t k1[HA_ITEMS];
        bool in[HA_ITEMS];
        int64_t v[HA_ITEMS];
        int32_t d[HA_ITEMS];
        ha_load<VAL, DIST>(a, n, base, k1, in, v, d);
        int32_t ls[HA_ITEMS];
        bool spill[HA_ITEMS];
#pragma unroll
        for (int j = 0; j < HA_ITEMS; ++j) {
            ls[j] = -1;
            spill[j] = false;
            if (!in[j]) continue;
            uint32_t s = ha_home(k1[j], lg);
            for (int p = 0; p < HA_LDS; ++p) {
                uint32_t cur = s_key[s];
                if (cur == 0u) cur = atomicCAS(&s_key[s], 0u, k1[j]);
                if (cur == 0u || cur == k1[j]) { ls[j] = (int32_t)s; break; }
                s = (s + 1) & (HA_LDS - 1);
            }
            spill[j] = ls[j] < 0;
            if (ls[j] >= 0) {
                atomicAdd(&s_cnt[ls[j]], 1u);
                if (VAL) atomicAdd(&s_sum[ls[j]], (unsigned long long)v[j]);
                if (MINMAX) {
                    const unsigned long long o = (unsigned long long)v[j] ^ ORD_BIAS;
                    atomicMax(&s_max[ls[j]], o);
                    atomicMax(&s_nmin[ls[j]], ~o);
                }
            }
        }
        // rows the LDS table could not take
        int32_t gs[HA_ITEMS];
        bool any_spill = false;
#pragma unroll
        for (int j = 0; j < HA_ITEMS; ++j) any_spill |= spill[j];
        if (__any(any_spill)) {
            ha_find(a, k1, spill, gs);
#pragma unroll
            for (int j = 0; j < HA_ITEMS; ++j)
                if (gs[j] >= 0) ha_update<VAL, MINMAX>(a.table, gs[j], v[j]);
        } else {
#pragma unroll
            for (int j = 0; j < HA_ITEMS; ++j) gs[j] = -1;
        }
        if (DIST) {
            bool ok[HA_ITEMS], ins[HA_ITEMS];
#pragma unroll
            for (int j = 0; j < HA_ITEMS; ++j) ok[j] = ls[j] >= 0 || gs[j] >= 0;
            ha_distinct(a, k1, d, ok, ins);
#pragma unroll
            for (int j = 0; j < HA_ITEMS; ++j) {
                if (!ins[j]) continue;
                if (ls[j] >= 0) atomicAdd(&s_nd[ls[j]], 1u);
                else add_nr(&a.ndist[gs[j]], 1u);
            }
        }
    }
    __syncthreads();
    // merge this block's groups
    for (int i0 = 0; i0 < HA_LDS; i0 += HA_BLOCK) {
        const int i = i0 + threadIdx.x;
        uint32_t k1[1] = {s_key[i]};
        bool in[1] = {k1[0] != 0u};
        int32_t gs[1];
        ha_find(a, k1, in, gs);
        if (gs[0] >= 0) {
            HaSlot* t = a.table;
            add_nr(&t[gs[0]].cnt, s_cnt[i]);
            if (VAL) add_nr(&t[gs[0]].sum, s_sum[i]);
            if (MINMAX) {
                max_nr(&t[gs[0]].max, s_max[i]);
                max_nr(&t[gs[0]].nmin, s_nmin[i]);
            }
            if (DIST && s_nd[i]) add_nr(&a.ndist[gs[0]], s_nd[i]);
        }
    }
}

struct HaOut {
    int32_t* key;
    int64_t* cnt;
    int64_t* sum;
    int64_t* min;
    int64_t* max;
    int64_t* ndist;
    int64_t gcap;
};

// Compaction of the occupied slots: one atomic per wave reserves the wave's
// output rows.
__global__ void __launch_bounds__(256)
k_ha_emit(const HaSlot* t, int64_t m, const uint32_t* ndist, HaOut o, unsigned long long* d_out) {
    const int l = lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x - l); b < m; b += stride) {
        const int64_t i = b + l;
        const bool occ = i < m && t[i].key1 != 0u;
        const uint64_t mk = ballot(occ);
        if (!mk) continue;
        unsigned long long base = 0;
        if (l == 0) base = atomicAdd(d_out, (unsigned long long)popc64(mk));
        base = __shfl(base, 0);
        const int64_t r = (int64_t)base + popc64(mk & lanemask_lt());
        if (occ && r < o.gcap) {
            const HaSlot s = t[i];
            o.key[r] = (int32_t)(s.key1 - 1u);
            o.cnt[r] = s.cnt;
            if (o.sum) o.sum[r] = (int64_t)s.sum;
            if (o.max) o.max[r] = (int64_t)(s.max ^ ORD_BIAS);
            if (o.min) o.min[r] = (int64_t)(~s.nmin ^ ORD_BIAS);
            if (o.ndist) o.ndist[r] = ndist[i];
        }
    }
}

__global__ void k_ha_finish(const unsigned long long* d_out, int64_t gcap, int64_t* d_ngroups, uint32_t* flags) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t g = (int64_t)*d_out;
        *d_ngroups = g;
        if (g > gcap) set_flag(flags, FLAG_CAPACITY);
    }
}

template <bool VAL, bool MINMAX, bool DIST>
tqp_status ha_run(tqp_ctx* ctx, const HaArgs& a, bool local, int64_t n, hipStream_t stream) {
    static const int per_cu[2] = {
        [] {
            int b = 4;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_ha_global<VAL, MINMAX, DIST>, HA_BLOCK, 0) !=
                hipSuccess)
                b = 4;
            return b < 1 ? 1 : b;
        }(),
        [] {
            int b = 2;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_ha_local<VAL, MINMAX, DIST>, HA_BLOCK, 0) !=
                hipSuccess)
                b = 2;
            return b < 1 ? 1 : b;
        }()};
    const int grid = grid_for(n, (int64_t)HA_BLOCK * HA_ITEMS, (int64_t)ctx->num_cus * per_cu[local ? 1 : 0]);
    if (local) {
        TQP_LAUNCH(ctx, stream, "hashagg_local", k_ha_local<VAL, MINMAX, DIST><<<grid, HA_BLOCK, 0, stream>>>(a));
    } else {
        TQP_LAUNCH(ctx, stream, "hashagg_global", k_ha_global<VAL, MINMAX, DIST><<<grid, HA_BLOCK, 0, stream>>>(a));
    }
    return TQP_OK;
}

}  // namespace
}  // namespace tqp

using namespace tqp;

extern "C" {

tqp_status tqp_hash_groupby(tqp_ctx* ctx, const int32_t* gkey, int64_t n, const int64_t* d_n, const int64_t* val,
                            const int32_t* dval, int32_t* out_key, int64_t* out_cnt, int64_t* out_sum,
                            int64_t* out_min, int64_t* out_max, int64_t* out_ndist, int64_t gcap,
                            int64_t* d_ngroups, void* ws, size_t* ws_bytes, hipStream_t stream) {
    clear_error();
    if (!ctx || !d_ngroups || n < 0 || gcap < 0 || (n > 0 && !gkey) || (gcap > 0 && (!out_key || !out_cnt)))
        return fail(TQP_ERR_INVALID, "tqp_hash_groupby: null pointer or negative size");
    if ((out_sum || out_min || out_max) && n > 0 && !val)
        return fail(TQP_ERR_INVALID, "tqp_hash_groupby: sum, min or max asked for without a value column");
    if (out_ndist && n > 0 && !dval)
        return fail(TQP_ERR_INVALID, "tqp_hash_groupby: count distinct asked for without its column");
    if (n > MAX_ELEMS || gcap > MAX_ELEMS)
        return fail(TQP_ERR_UNSUPPORTED, "tqp_hash_groupby: n = %lld, gcap = %lld", (long long)n, (long long)gcap);
    const bool want_val = out_sum || out_min || out_max;
    const bool want_mm = out_min || out_max;
    const bool want_dist = out_ndist != nullptr;
    int log2m = 0;
    while ((int64_t(1) << log2m) < 2 * gcap) ++log2m;
    const int64_t m = int64_t(1) << log2m;
    int log2s = 0;
    if (want_dist)
        while ((int64_t(1) << log2s) < 2 * n) ++log2s;
    const int64_t sm = want_dist ? int64_t(1) << log2s : 0;
    HaSlot* table = nullptr;
    uint32_t *ndist = nullptr, *d_groups = nullptr;
    unsigned long long *set = nullptr, *d_out = nullptr;
    Arena ar;
    auto plan = [&](Arena& p) {
        table = p.zero<HaSlot>(m);
        ndist = want_dist ? p.zero<uint32_t>(m) : nullptr;
        set = want_dist ? p.zero<unsigned long long>(sm) : nullptr;
        d_groups = p.zero<uint32_t>(1);
        d_out = p.zero<unsigned long long>(1);
    };
    tqp_status st = with_workspace(ctx, ws, ws_bytes, stream, plan, ar);
    if (st != TQP_OK || !ws) return st;
    if ((st = fill_zero(ar.base, ar.zsize, stream, ctx)) != TQP_OK) return st;
    HaArgs a{gkey, val, dval, n, d_n, table, log2m, ndist, set, log2s, d_groups, (uint32_t)gcap, ctx->d_err};
    const bool local = gcap <= HA_LDS_GROUPS;
    if (n > 0) {
        if (want_dist) {
            if (want_mm) st = ha_run<true, true, true>(ctx, a, local, n, stream);
            else if (want_val) st = ha_run<true, false, true>(ctx, a, local, n, stream);
            else st = ha_run<false, false, true>(ctx, a, local, n, stream);
        } else {
            if (want_mm) st = ha_run<true, true, false>(ctx, a, local, n, stream);
            else if (want_val) st = ha_run<true, false, false>(ctx, a, local, n, stream);
            else st = ha_run<false, false, false>(ctx, a, local, n, stream);
        }
        if (st != TQP_OK) return st;
    }
    HaOut o{out_key, out_cnt, out_sum, out_min, out_max, out_ndist, gcap};
    TQP_LAUNCH(ctx, stream, "hashagg_emit",
               k_ha_emit<<<grid_for(m, 256 * 4, (int64_t)ctx->num_cus * 8), 256, 0, stream>>>(table, m, ndist, o,
                                                                                              d_out));
    TQP_LAUNCH(ctx, stream, "hashagg_finish", k_ha_finish<<<1, 64, 0, stream>>>(d_out, gcap, d_ngroups, ctx->d_err));
    return TQP_OK;
}

}  // extern "C"
