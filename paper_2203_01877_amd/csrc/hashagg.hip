// Hash-based group-by aggregation: the alternative to the sort-based
// aggregation of Section 5.4 / Algorithm 2.  Section 6 traces the paper's
// loss on aggregation-heavy queries to its sorting, against systems that
// aggregate in hash tables; this is that hash aggregation, so the two can be
// compared on the same inputs.  It also evaluates the aggregates that the
// introduction of Section 5 lists besides sum and count: min, max and count
// with DISTINCT.
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
// Few groups (a table of 2 * gcap slots fits in 64 KB of LDS, 128 KB with
// distinct counts: gcap <= 2048 for sum and count, 1024 with everything):
// each block first aggregates its rows in a table in LDS and merges its
// groups into the global table at the end, so the global atomics per block
// are one per group, not one per row.
//
// Many groups with sum / min / max (a partitioned hash aggregation): the
// global table would take every row's update as device-scope atomics, which
// on a chip of eight L2 caches are performed beyond them, far below the HBM
// rate.  Instead one radix pass (two above 2^16 partitions) moves the rows,
// values alongside, into 2^P partitions by the top P bits of h = key * HP_MUL
// mod 2^32 (odd, so h is a bijection of the key and the key is h * HP_INV);
// then one block per partition aggregates it in an LDS table keyed by the
// next bits of h and writes its groups straight out.  P is chosen so that a
// partition holds about a quarter of its table's slots; a partition that
// still overflows its table sets TQP_DEVERR_CAPACITY.
//
// COUNT(DISTINCT d): a second table of 64-bit entries (key + 1, d) as a set;
// the row that inserts a pair adds one to its group's distinct count.  With
// many groups the rows are partitioned as above but carry d (and, with a
// value column, their row index), partitions are sized by rows too (about
// 1024), and each block keeps its partition's pairs in an LDS set, falling
// back to the global set only when that fills (k_hpd_agg).  A plain COUNT(*) with more groups than an LDS
// table holds takes the global table directly.
//
// Output: one row per group in no fixed order (slot order, compacted by wave
// ballots), the group count in *d_ngroups.
#include "dev.hpp"
#include "host.hpp"
#include "radix.hpp"

namespace tqp {
namespace {

constexpr int HA_BLOCK = 256;
constexpr int HA_ITEMS = 4;                 // rows per thread per step, probed in lockstep
constexpr int HA_LDS_MIN = 256;             // slots of the per-block table: 2 * gcap (or 4 * gcap), at least this
constexpr int HA_LDS_BYTES = 65536;         // LDS of a partition's table
// LDS of the per-block table: 64 KB, or 128 KB (of the 160 KB of a CU) with
// distinct counts, which have no partitioned path to fall back on
constexpr int ha_local_bytes(bool dist) { return dist ? 131072 : 65536; }
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
constexpr int ha_lds_slot_bytes() {
    return 8 + (VAL ? 8 : 0) + (MINMAX ? 16 : 0) + (DIST ? 4 : 0);
}

// The table has S = 2^lg slots in dynamic LDS (S * ha_lds_slot_bytes bytes):
// the 8-byte columns first, then the 4-byte ones.
// With distinct counts the block also keeps the (key + 1, d) pairs it has
// seen in an LDS set of HA_LSET slots: only a pair new to the block is tried
// in the global set, and one found there is not counted again.  A probe of
// the LDS set stops after HA_LSET_PROBE slots (the pair then goes to the
// global set, as does every later copy of it: slots are never freed, so they
// meet the same full run).  The set is used only when gcap <= HA_LSET_GROUPS:
// with more groups the pairs seen by a block outgrow it and the probes only
// add work.
constexpr int HA_LSET = 2048;
constexpr int HA_LSET_PROBE = 16;
constexpr int64_t HA_LSET_GROUPS = 64;

template <bool VAL, bool MINMAX, bool DIST>
__global__ void __launch_bounds__(HA_BLOCK) k_ha_local(HaArgs a, int lg, int pset) {
    extern __shared__ __align__(16) unsigned long long ha_smem[];
    const int S = 1 << lg;
    unsigned long long* s_pset = ha_smem;
    unsigned long long* s_sum = s_pset + (DIST && pset ? HA_LSET : 0);
    unsigned long long* s_max = s_sum + (VAL ? S : 0);
    unsigned long long* s_nmin = s_max + (MINMAX ? S : 0);
    uint32_t* s_key = reinterpret_cast<uint32_t*>(s_nmin + (MINMAX ? S : 0));
    uint32_t* s_cnt = s_key + S;
    uint32_t* s_nd = s_cnt + S;
    for (int i = threadIdx.x; i < S; i += HA_BLOCK) {
        s_key[i] = 0u;
        s_cnt[i] = 0u;
        if (VAL) s_sum[i] = 0ull;
        if (MINMAX) s_max[i] = 0ull, s_nmin[i] = 0ull;
        if (DIST) s_nd[i] = 0u;
    }
    if (DIST && pset)
        for (int i = threadIdx.x; i < HA_LSET; i += HA_BLOCK) s_pset[i] = 0ull;
    __syncthreads();
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
            for (int p = 0; p < S; ++p) {
                uint32_t cur = s_key[s];
                if (cur == 0u) cur = atomicCAS(&s_key[s], 0u, k1[j]);
                if (cur == 0u || cur == k1[j]) { ls[j] = (int32_t)s; break; }
                s = (s + 1) & (S - 1);
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
            for (int j = 0; j < HA_ITEMS; ++j) {
                ok[j] = ls[j] >= 0 || gs[j] >= 0;
                if (!ok[j] || !pset) continue;
                // seen before in this block: already tried globally, nothing to count
                const unsigned long long pe = ((unsigned long long)k1[j] << 32) | (uint32_t)d[j];
                uint32_t ps = ha_home(pe, 31 - __clz(HA_LSET));
                for (int q = 0; q < HA_LSET_PROBE; ++q) {
                    unsigned long long cur = s_pset[ps];
                    if (cur == 0ull) cur = atomicCAS(&s_pset[ps], 0ull, pe);
                    if (cur == 0ull) break;                        // new to the block
                    if (cur == pe) { ok[j] = false; break; }
                    ps = (ps + 1) & (HA_LSET - 1);
                }                                                  // a full run: try globally
            }
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
    for (int i0 = 0; i0 < S; i0 += HA_BLOCK) {
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

// Compaction of the occupied slots.  A block takes chunks of HE_PER * 256
// slots; one atomic per chunk reserves the chunk's output rows (a counter
// shared by every wave would serialise the waves on one address).
constexpr int HE_PER = 16;

__global__ void __launch_bounds__(256)
k_ha_emit(const HaSlot* t, int64_t m, const uint32_t* ndist, HaOut o, unsigned long long* d_out) {
    __shared__ int64_t s_w[256 / WAVE];
    __shared__ unsigned long long s_base;
    const int tid = threadIdx.x, w = tid / WAVE, l = lane_id();
    constexpr int64_t CH = (int64_t)256 * HE_PER;
    for (int64_t c0 = (int64_t)blockIdx.x * CH; c0 < m; c0 += (int64_t)gridDim.x * CH) {
        uint32_t occ = 0;
#pragma unroll
        for (int q = 0; q < HE_PER; ++q) {
            const int64_t i = c0 + (int64_t)q * 256 + tid;
            if (i < m && t[i].key1 != 0u) occ |= 1u << q;
        }
        const int64_t cnt = __popc(occ);
        const int64_t incl = wave_incl_sum(cnt);
        if (l == WAVE - 1) s_w[w] = incl;
        __syncthreads();
        int64_t before = 0, tot = 0;
#pragma unroll
        for (int ww = 0; ww < 256 / WAVE; ++ww) {
            if (ww < w) before += s_w[ww];
            tot += s_w[ww];
        }
        if (tid == 0) s_base = tot ? atomicAdd(d_out, (unsigned long long)tot) : 0ull;
        __syncthreads();
        int64_t r = (int64_t)s_base + before + incl - cnt;
#pragma unroll
        for (int q = 0; q < HE_PER; ++q) {
            if (!((occ >> q) & 1u)) continue;
            const int64_t i = c0 + (int64_t)q * 256 + tid;
            if (r < o.gcap) {
                const HaSlot s = t[i];
                o.key[r] = (int32_t)(s.key1 - 1u);
                o.cnt[r] = s.cnt;
                if (o.sum) o.sum[r] = (int64_t)s.sum;
                if (o.max) o.max[r] = (int64_t)(s.max ^ ORD_BIAS);
                if (o.min) o.min[r] = (int64_t)(~s.nmin ^ ORD_BIAS);
                if (o.ndist) o.ndist[r] = ndist[i];
            }
            ++r;
        }
        __syncthreads();
    }
}

__global__ void k_ha_finish(const unsigned long long* d_out, int64_t gcap, int64_t* d_ngroups, uint32_t* flags) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t g = (int64_t)*d_out;
        *d_ngroups = g;
        if (g > gcap) set_flag(flags, FLAG_CAPACITY);
    }
}

// ---------------------------------------------------------------- partitioned
constexpr uint32_t HP_MUL = 0x9E3779B1u;
constexpr uint32_t inv_odd(uint32_t a) {
    uint32_t x = a;                                   // Newton's iteration for the inverse mod 2^32
    for (int i = 0; i < 5; ++i) x *= 2u - a * x;
    return x;
}
constexpr uint32_t HP_INV = inv_odd(HP_MUL);
static_assert(HP_MUL * HP_INV == 1u, "HP_INV inverts HP_MUL");
constexpr int HP_BLOCK = 1024;
constexpr int HP_MIN_BITS = 8;                  // at least 256 partitions: one block per CU or more

// Rows as (h, value); a negative key is reported and its row left out.
struct SrcHashPart {
    const int32_t* key;
    const int64_t* val;
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
        k = (uint32_t)x * HP_MUL;
        return x >= 0;
    }
    __device__ bool load(int64_t i, uint32_t& k, uint64_t& v) const {
        const int32_t x = key[i];
        k = (uint32_t)x * HP_MUL;
        v = (uint64_t)val[i];
        return x >= 0;
    }
};

// start[p] = first row of partition p (rows sorted by their top P bits of h),
// start[2^P] = the row count.
__global__ void __launch_bounds__(256)
k_hp_bounds(const uint32_t* h, const int64_t* d_cnt, int P, int64_t* start) {
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

// One block per partition: LDS table of 2^lg slots, keyed by key + 1, home
// slot from the bits of h below the partition bits; then the block's groups
// are written at an offset reserved with one atomic.
template <bool MINMAX>
__global__ void __launch_bounds__(HP_BLOCK)
k_hp_agg(const uint32_t* h, const uint64_t* v, const int64_t* start, int P, int lg, HaOut o,
         unsigned long long* d_out, uint32_t* flags) {
    extern __shared__ __align__(16) unsigned long long ha_smem[];
    __shared__ int64_t s_w[HP_BLOCK / WAVE];
    __shared__ unsigned long long s_base;
    const int S = 1 << lg;
    unsigned long long* s_sum = ha_smem;
    unsigned long long* s_max = s_sum + S;
    unsigned long long* s_nmin = s_max + (MINMAX ? S : 0);
    uint32_t* s_key = reinterpret_cast<uint32_t*>(s_nmin + (MINMAX ? S : 0));
    uint32_t* s_cnt = s_key + S;
    const int tid = threadIdx.x;
    for (int i = tid; i < S; i += HP_BLOCK) {
        s_key[i] = 0u;
        s_cnt[i] = 0u;
        s_sum[i] = 0ull;
        if (MINMAX) s_max[i] = 0ull, s_nmin[i] = 0ull;
    }
    __syncthreads();
    const int64_t b = start[blockIdx.x], e = start[blockIdx.x + 1];
    const int hs = P + lg <= 32 ? 32 - lg : P;     // h << P >> hs: lg bits below the partition bits
    for (int64_t i0 = b; i0 < e; i0 += (int64_t)HP_BLOCK * HA_ITEMS) {
        uint32_t hh[HA_ITEMS];
        uint64_t vv[HA_ITEMS];
#pragma unroll
        for (int j = 0; j < HA_ITEMS; ++j) {
            const int64_t i = i0 + (int64_t)j * HP_BLOCK + tid;
            hh[j] = i < e ? h[i] : 0u;
            vv[j] = i < e ? v[i] : 0ull;
        }
#pragma unroll
        for (int j = 0; j < HA_ITEMS; ++j) {
            const int64_t i = i0 + (int64_t)j * HP_BLOCK + tid;
            if (i >= e) continue;
            const uint32_t k1 = hh[j] * HP_INV + 1u;
            uint32_t sl = P < 32 ? ((hh[j] << P) >> hs) & (uint32_t)(S - 1) : 0u;
            int found = -1;
            for (int q = 0; q < S; ++q) {
                uint32_t cur = s_key[sl];
                if (cur == 0u) cur = atomicCAS(&s_key[sl], 0u, k1);
                if (cur == 0u || cur == k1) { found = (int)sl; break; }
                sl = (sl + 1) & (uint32_t)(S - 1);
            }
            if (found < 0) {
                set_flag(flags, FLAG_CAPACITY);       // more groups in this partition than slots
                continue;
            }
            atomicAdd(&s_cnt[found], 1u);
            atomicAdd(&s_sum[found], (unsigned long long)vv[j]);
            if (MINMAX) {
                const unsigned long long ov = vv[j] ^ ORD_BIAS;
                atomicMax(&s_max[found], ov);
                atomicMax(&s_nmin[found], ~ov);
            }
        }
    }
    __syncthreads();
    // compaction of the occupied slots: slot q * HP_BLOCK + tid is bit q of occ
    const int per = S > HP_BLOCK ? S / HP_BLOCK : 1;
    uint32_t occ = 0;
    for (int q = 0; q < per; ++q) {
        const int i = q * HP_BLOCK + tid;
        if (i < S && s_key[i] != 0u) occ |= 1u << q;
    }
    const int64_t cnt = __popc(occ);
    const int64_t incl = wave_incl_sum(cnt);
    const int w = tid / WAVE;
    if (lane_id() == WAVE - 1) s_w[w] = incl;
    __syncthreads();
    int64_t before = 0, tot = 0;
    for (int ww = 0; ww < HP_BLOCK / WAVE; ++ww) {
        if (ww < w) before += s_w[ww];
        tot += s_w[ww];
    }
    if (tid == 0) s_base = tot ? atomicAdd(d_out, (unsigned long long)tot) : 0ull;
    __syncthreads();
    int64_t r = (int64_t)s_base + before + incl - cnt;
    for (int q = 0; q < per; ++q) {
        if (!((occ >> q) & 1u)) continue;
        const int i = q * HP_BLOCK + tid;
        if (r < o.gcap) {
            o.key[r] = (int32_t)(s_key[i] - 1u);
            o.cnt[r] = s_cnt[i];
            if (o.sum) o.sum[r] = (int64_t)s_sum[i];
            if (MINMAX) {
                if (o.max) o.max[r] = (int64_t)(s_max[i] ^ ORD_BIAS);
                if (o.min) o.min[r] = (int64_t)(~s_nmin[i] ^ ORD_BIAS);
            }
        }
        ++r;
    }
}

// ---------------------------------------------------------------- partitioned, with distinct counts
// Rows as (h, payload).  With a value column the payload (PL = uint64_t) is
// the distinct value in the high half and the row index in the low half, and
// the value is read through the index by the aggregating block; without one
// (COUNT and COUNT(DISTINCT) only, PL = uint32_t) it is the distinct value.
template <class PL>
struct SrcHashPartIdx {
    const int32_t* key;
    const int32_t* dval;
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
        k = (uint32_t)x * HP_MUL;
        return x >= 0;
    }
    __device__ bool load(int64_t i, uint32_t& k, PL& v) const {
        const int32_t x = key[i];
        k = (uint32_t)x * HP_MUL;
        if constexpr (sizeof(PL) == 8) v = ((uint64_t)(uint32_t)dval[i] << 32) | (uint32_t)i;
        else v = (uint32_t)dval[i];
        return x >= 0;
    }
};

constexpr int HPD_BLOCK = 256;
constexpr int HPD_SET = 2048;                   // LDS pair-set slots of a partition (about 1024 rows each)

// One block per partition, with COUNT(DISTINCT d): the group table as in
// k_hp_agg plus a set of the partition's (key + 1, d) pairs in LDS.  The row
// that inserts a pair adds one to its group's distinct count.  A pair the
// full LDS set cannot take goes to the global set (a partition with far more
// rows than expected, e.g. one very frequent key); the LDS set never loses an
// entry, so a pair is never counted in both.
template <bool VAL, bool MINMAX>
__global__ void __launch_bounds__(HPD_BLOCK)
k_hpd_agg(const uint32_t* h, const typename std::conditional<VAL, uint64_t, uint32_t>::type* pay, const int64_t* start, int P, int lg, const int64_t* val,
          const int32_t* dval, unsigned long long* gset, int log2s, HaOut o, unsigned long long* d_out,
          uint32_t* flags) {
    extern __shared__ __align__(16) unsigned long long ha_smem[];
    __shared__ int64_t s_w[HPD_BLOCK / WAVE];
    __shared__ unsigned long long s_base;
    const int S = 1 << lg;
    unsigned long long* s_set = ha_smem;
    unsigned long long* s_sum = s_set + HPD_SET;
    unsigned long long* s_max = s_sum + (VAL ? S : 0);
    unsigned long long* s_nmin = s_max + (MINMAX ? S : 0);
    uint32_t* s_key = reinterpret_cast<uint32_t*>(s_nmin + (MINMAX ? S : 0));
    uint32_t* s_cnt = s_key + S;
    uint32_t* s_nd = s_cnt + S;
    const int tid = threadIdx.x;
    for (int i = tid; i < HPD_SET; i += HPD_BLOCK) s_set[i] = 0ull;
    for (int i = tid; i < S; i += HPD_BLOCK) {
        s_key[i] = 0u;
        s_cnt[i] = 0u;
        s_nd[i] = 0u;
        if (VAL) s_sum[i] = 0ull;
        if (MINMAX) s_max[i] = 0ull, s_nmin[i] = 0ull;
    }
    __syncthreads();
    const int64_t b = start[blockIdx.x], e = start[blockIdx.x + 1];
    const int hs = P + lg <= 32 ? 32 - lg : P;
    const uint32_t smask = (uint32_t)((uint64_t(1) << log2s) - 1);
    const uint32_t slimit = smask + 1 < HA_PROBE_LIMIT ? smask + 1 : HA_PROBE_LIMIT;
    for (int64_t i0 = b; i0 < e; i0 += (int64_t)HPD_BLOCK * HA_ITEMS) {
        uint32_t hh[HA_ITEMS];
        uint64_t pl[HA_ITEMS];
#pragma unroll
        for (int j = 0; j < HA_ITEMS; ++j) {
            const int64_t i = i0 + (int64_t)j * HPD_BLOCK + tid;
            hh[j] = i < e ? h[i] : 0u;
            pl[j] = i < e ? (uint64_t)pay[i] : 0ull;
        }
        int64_t vv[HA_ITEMS];
        int32_t dd[HA_ITEMS];
#pragma unroll
        for (int j = 0; j < HA_ITEMS; ++j) {
            const int64_t i = i0 + (int64_t)j * HPD_BLOCK + tid;
            vv[j] = VAL && i < e ? val[(uint32_t)pl[j]] : 0;                // the row index, low half
            dd[j] = VAL ? (int32_t)(pl[j] >> 32) : (int32_t)(uint32_t)pl[j];
        }
#pragma unroll
        for (int j = 0; j < HA_ITEMS; ++j) {
            const int64_t i = i0 + (int64_t)j * HPD_BLOCK + tid;
            if (i >= e) continue;
            const uint32_t k1 = hh[j] * HP_INV + 1u;
            uint32_t sl = P < 32 ? ((hh[j] << P) >> hs) & (uint32_t)(S - 1) : 0u;
            int found = -1;
            for (int q = 0; q < S; ++q) {
                uint32_t cur = s_key[sl];
                if (cur == 0u) cur = atomicCAS(&s_key[sl], 0u, k1);
                if (cur == 0u || cur == k1) { found = (int)sl; break; }
                sl = (sl + 1) & (uint32_t)(S - 1);
            }
            if (found < 0) {
                set_flag(flags, FLAG_CAPACITY);
                continue;
            }
            atomicAdd(&s_cnt[found], 1u);
            if (VAL) atomicAdd(&s_sum[found], (unsigned long long)vv[j]);
            if (MINMAX) {
                const unsigned long long ov = (unsigned long long)vv[j] ^ ORD_BIAS;
                atomicMax(&s_max[found], ov);
                atomicMax(&s_nmin[found], ~ov);
            }
            // the pair, first in the LDS set, then (when that is full) in the global one
            const unsigned long long pe = ((unsigned long long)k1 << 32) | (uint32_t)dd[j];
            uint32_t ps = ha_home(pe, 31 - __clz(HPD_SET));
            int inserted = -1;                          // 1 new, 0 already there, -1 no room
            for (int q = 0; q < HPD_SET; ++q) {
                unsigned long long cur = s_set[ps];
                if (cur == 0ull) cur = atomicCAS(&s_set[ps], 0ull, pe);
                if (cur == 0ull) { inserted = 1; break; }
                if (cur == pe) { inserted = 0; break; }
                ps = (ps + 1) & (HPD_SET - 1);
            }
            if (inserted < 0) {
                uint32_t gs = ha_home(pe, log2s);
                for (uint32_t q = 0; q < slimit; ++q) {
                    unsigned long long cur = gset[gs];
                    if (cur == 0ull) cur = atomicCAS(&gset[gs], 0ull, pe);
                    if (cur == 0ull) { inserted = 1; break; }
                    if (cur == pe) { inserted = 0; break; }
                    gs = (gs + 1) & smask;
                }
                if (inserted < 0) set_flag(flags, FLAG_CAPACITY);
            }
            if (inserted == 1) atomicAdd(&s_nd[found], 1u);
        }
    }
    __syncthreads();
    const int per = S > HPD_BLOCK ? S / HPD_BLOCK : 1;
    uint32_t occ = 0;
    for (int q = 0; q < per; ++q) {
        const int i = q * HPD_BLOCK + tid;
        if (i < S && s_key[i] != 0u) occ |= 1u << q;
    }
    const int64_t cnt = __popc(occ);
    const int64_t incl = wave_incl_sum(cnt);
    const int w = tid / WAVE;
    if (lane_id() == WAVE - 1) s_w[w] = incl;
    __syncthreads();
    int64_t before = 0, tot = 0;
    for (int ww = 0; ww < HPD_BLOCK / WAVE; ++ww) {
        if (ww < w) before += s_w[ww];
        tot += s_w[ww];
    }
    if (tid == 0) s_base = tot ? atomicAdd(d_out, (unsigned long long)tot) : 0ull;
    __syncthreads();
    int64_t r = (int64_t)s_base + before + incl - cnt;
    for (int q = 0; q < per; ++q) {
        if (!((occ >> q) & 1u)) continue;
        const int i = q * HPD_BLOCK + tid;
        if (r < o.gcap) {
            o.key[r] = (int32_t)(s_key[i] - 1u);
            o.cnt[r] = s_cnt[i];
            o.ndist[r] = s_nd[i];
            if (VAL && o.sum) o.sum[r] = (int64_t)s_sum[i];
            if (MINMAX) {
                if (o.max) o.max[r] = (int64_t)(s_max[i] ^ ORD_BIAS);
                if (o.min) o.min[r] = (int64_t)(~s_nmin[i] ^ ORD_BIAS);
            }
        }
        ++r;
    }
}

template <bool VAL, bool MINMAX>
constexpr int hpd_slot_bytes() {
    return 12 + (VAL ? 8 : 0) + (MINMAX ? 16 : 0);
}

template <bool VAL, bool MINMAX>
tqp_status hpd_run(tqp_ctx* ctx, const int32_t* gkey, const int64_t* val, const int32_t* dval, int64_t n,
                   const int64_t* d_n, HaOut o, int64_t gcap, int64_t* d_ngroups, void* ws, size_t* ws_bytes,
                   hipStream_t stream) {
    // partitions of about 1024 rows and about 256 groups
    int P = HP_MIN_BITS;
    while (((n >> P) > 1024 || (gcap >> P) > 256) && P < 24) ++P;
    const int64_t per = (gcap + (int64_t(1) << P) - 1) >> P;
    int lg = 8;
    while ((int64_t(1) << lg) < 4 * per && lg < 10) ++lg;
    int log2s = 0;
    while ((int64_t(1) << log2s) < 2 * n) ++log2s;
    using PL = typename std::conditional<VAL, uint64_t, uint32_t>::type;
    RadixBufs<R8, PL> rb;
    uint32_t* hk = nullptr;
    PL* hi = nullptr;
    int64_t* start = nullptr;
    unsigned long long *gset = nullptr, *d_out = nullptr;
    Arena ar;
    auto plan = [&](Arena& p) {
        rb = radix_reserve<R8, PL>(p, n, 32, 32 - P);
        d_out = p.zero<unsigned long long>(1);
        gset = p.zero<unsigned long long>(int64_t(1) << log2s);
        hk = p.scratch<uint32_t>(n);
        hi = p.scratch<PL>(n);
        start = p.scratch<int64_t>((int64_t(1) << P) + 1);
    };
    tqp_status st = with_workspace(ctx, ws, ws_bytes, stream, plan, ar);
    if (st != TQP_OK || !ws) return st;
    if ((st = fill_zero(ar.base, ar.zsize, stream, ctx)) != TQP_OK) return st;
    SrcHashPartIdx<PL> src{gkey, dval, n, d_n, ctx->d_err};
    st = radix_launch<R8, PL>(rb, src, n, true, nullptr, ~0u, hk, hi, ctx, stream, "hashpart_pass",
                                    "hashpart_pass");
    if (st != TQP_OK) return st;
    const int64_t np = int64_t(1) << P;
    TQP_LAUNCH(ctx, stream, "hashpart_bounds",
               k_hp_bounds<<<grid_for(np + 1, 256, 0), 256, 0, stream>>>(hk, rb.d_cnt, P, start));
    const size_t lds = (size_t)HPD_SET * 8 + ((size_t)1 << lg) * hpd_slot_bytes<VAL, MINMAX>();
    TQP_LAUNCH(ctx, stream, "hashpart_distinct",
               k_hpd_agg<VAL, MINMAX><<<(unsigned)np, HPD_BLOCK, lds, stream>>>(hk, hi, start, P, lg, val, dval, gset,
                                                                                log2s, o, d_out, ctx->d_err));
    TQP_LAUNCH(ctx, stream, "hashagg_finish", k_ha_finish<<<1, 64, 0, stream>>>(d_out, gcap, d_ngroups, ctx->d_err));
    return TQP_OK;
}

template <bool MINMAX>
constexpr int hp_slot_bytes() {
    return 16 + (MINMAX ? 16 : 0);
}

// Partition bits and LDS table size for gcap groups: about S / 4 groups per
// partition, S at most 64 KB of LDS and at most 32 slots per thread.
template <bool MINMAX>
void hp_plan(int64_t gcap, int& P, int& lg) {
    int lmax = 0;
    while ((int64_t(2) << lmax) * hp_slot_bytes<MINMAX>() <= HA_LDS_BYTES) ++lmax;
    P = HP_MIN_BITS;
    while ((gcap >> P) > ((int64_t(1) << lmax) >> 2) && P < 24) ++P;
    const int64_t per = (gcap + (int64_t(1) << P) - 1) >> P;
    lg = 8;
    while ((int64_t(1) << lg) < 4 * per && lg < lmax) ++lg;
}

// log2 of the LDS table's slots for gcap groups, or -1 when it would not fit
// (the global table then takes every row).
template <bool VAL, bool MINMAX, bool DIST>
int ha_lds_log2(int64_t gcap) {
    int lg = 0;
    while ((int64_t(1) << lg) < 2 * gcap || (1 << lg) < HA_LDS_MIN) ++lg;
    const int64_t set = DIST && gcap <= HA_LSET_GROUPS ? HA_LSET * 8 : 0;
    // A table sized by the group bound (not by its minimum) gets twice the
    // slots when they fit: at a quarter full its linear probes stay short,
    // and a wave waits for its longest (SUM and COUNT over 1000 groups:
    // 0.63 -> 0.54 ms for 60M rows).  A minimum-size table keeps its size:
    // doubling it only adds clearing and merging.
    const int64_t bytes = ha_lds_slot_bytes<VAL, MINMAX, DIST>();
    if ((int64_t(1) << lg) > HA_LDS_MIN && (int64_t(1) << (lg + 1)) * bytes + set <= ha_local_bytes(DIST)) return lg + 1;
    return ((int64_t(1) << lg) * bytes + set <= ha_local_bytes(DIST)) ? lg : -1;
}

template <bool VAL, bool MINMAX, bool DIST>
tqp_status ha_run(tqp_ctx* ctx, const HaArgs& a, int64_t gcap, int64_t n, hipStream_t stream) {
    static const int per_cu_global = [] {
        int b = 4;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_ha_global<VAL, MINMAX, DIST>, HA_BLOCK, 0) !=
            hipSuccess)
            b = 4;
        return b < 1 ? 1 : b;
    }();
    static int per_cu_local[2][32] = {};            // by the pair set's use and log2 of the LDS slots
    const int lg = ha_lds_log2<VAL, MINMAX, DIST>(gcap);
    if (lg >= 0) {
        const int pset = DIST && gcap <= HA_LSET_GROUPS;
        const size_t lds = ((size_t)1 << lg) * ha_lds_slot_bytes<VAL, MINMAX, DIST>() + (pset ? HA_LSET * 8 : 0);
        int& per_cu = per_cu_local[pset][lg];
        if (!per_cu) {
            if (lds > 65536 &&
                hipFuncSetAttribute(reinterpret_cast<const void*>(k_ha_local<VAL, MINMAX, DIST>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
                return fail(TQP_ERR_HIP, "tqp_hash_groupby: %zu bytes of LDS refused", lds);
            int b = 1;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_ha_local<VAL, MINMAX, DIST>, HA_BLOCK, lds) !=
                hipSuccess)
                b = 1;
            per_cu = b < 1 ? 1 : b;
        }
        const int grid = grid_for(n, (int64_t)HA_BLOCK * HA_ITEMS, (int64_t)ctx->num_cus * per_cu);
        TQP_LAUNCH(ctx, stream, "hashagg_local",
                   k_ha_local<VAL, MINMAX, DIST><<<grid, HA_BLOCK, lds, stream>>>(a, lg, pset));
    } else {
        const int grid = grid_for(n, (int64_t)HA_BLOCK * HA_ITEMS, (int64_t)ctx->num_cus * per_cu_global);
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
    // many groups with sum / min / max: partitioned (no global table)
    const bool part = want_val && !want_dist && n > 0 &&
                      (want_mm ? ha_lds_log2<true, true, false>(gcap) : ha_lds_log2<true, false, false>(gcap)) < 0;
    if (part) {
        int P = 0, lg = 0;
        if (want_mm) hp_plan<true>(gcap, P, lg);
        else hp_plan<false>(gcap, P, lg);
        RadixBufs<R8, uint64_t> rb;
        uint32_t* hk = nullptr;
        uint64_t* hv = nullptr;
        int64_t* start = nullptr;
        unsigned long long* d_out = nullptr;
        Arena ar;
        auto plan = [&](Arena& p) {
            rb = radix_reserve<R8, uint64_t>(p, n, 32, 32 - P);
            d_out = p.zero<unsigned long long>(1);
            hk = p.scratch<uint32_t>(n);
            hv = p.scratch<uint64_t>(n);
            start = p.scratch<int64_t>((int64_t(1) << P) + 1);
        };
        tqp_status st = with_workspace(ctx, ws, ws_bytes, stream, plan, ar);
        if (st != TQP_OK || !ws) return st;
        if ((st = fill_zero(ar.base, ar.zsize, stream, ctx)) != TQP_OK) return st;
        SrcHashPart src{gkey, val, n, d_n, ctx->d_err};
        st = radix_launch<R8, uint64_t>(rb, src, n, true, nullptr, ~0u, hk, hv, ctx, stream, "hashpart_pass",
                                        "hashpart_pass");
        if (st != TQP_OK) return st;
        const int64_t np = int64_t(1) << P;
        TQP_LAUNCH(ctx, stream, "hashpart_bounds",
                   k_hp_bounds<<<grid_for(np + 1, 256, 0), 256, 0, stream>>>(hk, rb.d_cnt, P, start));
        HaOut o{out_key, out_cnt, out_sum, out_min, out_max, nullptr, gcap};
        if (want_mm) {
            const size_t lds = ((size_t)1 << lg) * hp_slot_bytes<true>();
            TQP_LAUNCH(ctx, stream, "hashpart_agg",
                       k_hp_agg<true><<<(unsigned)np, HP_BLOCK, lds, stream>>>(hk, hv, start, P, lg, o, d_out,
                                                                                 ctx->d_err));
        } else {
            const size_t lds = ((size_t)1 << lg) * hp_slot_bytes<false>();
            TQP_LAUNCH(ctx, stream, "hashpart_agg",
                       k_hp_agg<false><<<(unsigned)np, HP_BLOCK, lds, stream>>>(hk, hv, start, P, lg, o, d_out,
                                                                                  ctx->d_err));
        }
        TQP_LAUNCH(ctx, stream, "hashagg_finish",
                   k_ha_finish<<<1, 64, 0, stream>>>(d_out, gcap, d_ngroups, ctx->d_err));
        return TQP_OK;
    }
    // distinct counts with many groups: partitioned too
    if (want_dist && n > 0) {
        const int lg_local = want_mm ? ha_lds_log2<true, true, true>(gcap)
                             : want_val ? ha_lds_log2<true, false, true>(gcap)
                                        : ha_lds_log2<false, false, true>(gcap);
        if (lg_local < 0) {
            HaOut o{out_key, out_cnt, out_sum, out_min, out_max, out_ndist, gcap};
            if (want_mm) return hpd_run<true, true>(ctx, gkey, val, dval, n, d_n, o, gcap, d_ngroups, ws, ws_bytes, stream);
            if (want_val)
                return hpd_run<true, false>(ctx, gkey, val, dval, n, d_n, o, gcap, d_ngroups, ws, ws_bytes, stream);
            return hpd_run<false, false>(ctx, gkey, val, dval, n, d_n, o, gcap, d_ngroups, ws, ws_bytes, stream);
        }
    }
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
    if (n > 0) {
        if (want_dist) {
            if (want_mm) st = ha_run<true, true, true>(ctx, a, gcap, n, stream);
            else if (want_val) st = ha_run<true, false, true>(ctx, a, gcap, n, stream);
            else st = ha_run<false, false, true>(ctx, a, gcap, n, stream);
        } else {
            if (want_mm) st = ha_run<true, true, false>(ctx, a, gcap, n, stream);
            else if (want_val) st = ha_run<true, false, false>(ctx, a, gcap, n, stream);
            else st = ha_run<false, false, false>(ctx, a, gcap, n, stream);
        }
        if (st != TQP_OK) return st;
    }
    HaOut o{out_key, out_cnt, out_sum, out_min, out_max, out_ndist, gcap};
    TQP_LAUNCH(ctx, stream, "hashagg_emit",
               k_ha_emit<<<grid_for(m, 256 * HE_PER, (int64_t)ctx->num_cus * 4), 256, 0, stream>>>(table, m, ndist, o,
                                                                                              d_out));
    TQP_LAUNCH(ctx, stream, "hashagg_finish", k_ha_finish<<<1, 64, 0, stream>>>(d_out, gcap, d_ngroups, ctx->d_err));
    return TQP_OK;
}

}  // extern "C"
