// LSD radix sort of (key, payload) pairs: one histogram read for all digit
// passes, then one "onesweep" kernel per pass that ranks a tile in LDS with
// 64-lane ballots, finds its global digit offsets by decoupled look-back and
// writes the tile out digit by digit.  Stable, ascending, key-width trimmed.
//
// The sort is the first step of the sort-based join (Algorithm 1: both key
// columns are sorted with their row ids) and of the sort-based aggregation
// (Algorithm 2: the packed group key is sorted, Section 5.4 names radix sort).
#pragma once
#include <type_traits>

#include "dev.hpp"

namespace tqp {

struct NoVal {};

// ------------------------------------------------------------------ sources
// A source yields, for index i of its domain, whether the element takes part,
// its key and its payload.  size() may depend on a device-side count.

// Loads are branch-free and unconditional (callers clamp the index), so the
// compiler keeps every item's loads of a thread in flight together.

// Plain (key, value) arrays, optionally bounded by a device count.
template <class V>
struct SrcPairs {
    const uint32_t* keys;
    const V* vals;             // not null (SrcKeysIndex pairs keys with their index)
    int64_t n_upper;
    const int64_t* d_n;
    __device__ int64_t size() const {
        if (!d_n) return n_upper;
        int64_t n = *d_n;
        return n < n_upper ? n : n_upper;
    }
    __device__ bool load_key(int64_t i, uint32_t& k) const {
        k = keys[i];
        return true;
    }
    __device__ bool load(int64_t i, uint32_t& k, V& v) const {
        k = keys[i];
        v = vals[i];
        return true;
    }
};

// Keys with their element index as the payload.
struct SrcKeysIndex {
    const uint32_t* keys;
    int64_t n_upper;
    const int64_t* d_n;
    __device__ int64_t size() const {
        if (!d_n) return n_upper;
        int64_t n = *d_n;
        return n < n_upper ? n : n_upper;
    }
    __device__ bool load_key(int64_t i, uint32_t& k) const {
        k = keys[i];
        return true;
    }
    __device__ bool load(int64_t i, uint32_t& k, uint32_t& v) const {
        k = keys[i];
        v = (uint32_t)i;
        return true;
    }
};

template <>
struct SrcPairs<NoVal> {
    const uint32_t* keys;
    const NoVal* vals;
    int64_t n_upper;
    const int64_t* d_n;
    __device__ int64_t size() const {
        if (!d_n) return n_upper;
        int64_t n = *d_n;
        return n < n_upper ? n : n_upper;
    }
    __device__ bool load_key(int64_t i, uint32_t& k) const {
        k = keys[i];
        return true;
    }
    __device__ bool load(int64_t i, uint32_t& k, NoVal&) const {
        k = keys[i];
        return true;
    }
};

// Predicate constants of a pushed-down comparison.
enum CmpOp : int32_t { CMP_LT = 0, CMP_LE = 1, CMP_GT = 2, CMP_GE = 3, CMP_EQ = 4, CMP_NE = 5 };

// Branch-free on purpose: with a switch, the compiler waits for each item's
// loads before the next item's (it will not move loads across the branches),
// so a thread kept one item in flight instead of all of them.  Operators
// outside CMP_LT..CMP_EQ compare for inequality.
__device__ __forceinline__ bool cmp_eval(int64_t x, int32_t op, int64_t k) {
    const bool lt = x < k, eq = x == k;
    bool r = (op == CMP_LT) & lt;
    r |= (op == CMP_LE) & (lt | eq);
    r |= (op == CMP_GT) & !(lt | eq);
    r |= (op == CMP_GE) & !lt;
    r |= (op == CMP_EQ) & eq;
    r |= (op < CMP_LT || op > CMP_EQ) & !eq;
    return r;
}

// key column + one filter column (date < D, seg == c ...), payload = row id.
// This fuses the filter (Section 3.1: predicate -> selection) into the first
// sort pass: rows that fail the predicate are never written.
template <class FT>
struct SrcFilterRowid {
    const int32_t* key;
    const FT* fcol;
    int32_t op;
    int64_t k;
    int64_t n;
    int64_t row0;              // row id offset (a fragment over a row range of a larger table)
    __device__ int64_t size() const { return n; }
    __device__ bool load_key(int64_t i, uint32_t& kk) const {
        kk = (uint32_t)key[i];
        return cmp_eval((int64_t)fcol[i], op, k);
    }
    __device__ bool load(int64_t i, uint32_t& kk, uint32_t& v) const {
        kk = (uint32_t)key[i];
        v = (uint32_t)(row0 + i);
        return cmp_eval((int64_t)fcol[i], op, k);
    }
};

// fact key + date filter, payload = price * (100 - disc) computed on the fly
// (the revenue expression evaluated before the join instead of after it),
// carried as VT: uint64_t (the int64 value), or uint32_t when the caller
// declares that every kept row's revenue lies in [0, 2^32) (a kept row
// outside is reported through the pass's value-range flag).
// MASK: the histogram kernel, which evaluates the predicate anyway, stores it
// as one bit per row (mask, one 64-bit word per 64 rows); the pass then reads
// that bit instead of the 4-byte date.
template <class VT, bool MASK = false>
struct SrcFilterRevenue {
    static constexpr bool CHECKS = sizeof(VT) < 8;
    static constexpr bool WRITES_MASK = MASK;
    const int32_t* key;
    const int32_t* date;
    const int64_t* price;
    const int64_t* disc;
    int32_t op;
    int64_t k;
    int64_t n;
    uint64_t* mask;            // MASK: ceil(n / 64) words
    __device__ int64_t size() const { return n; }
    __device__ bool load_key(int64_t i, uint32_t& kk) const {
        kk = (uint32_t)key[i];
        return cmp_eval((int64_t)date[i], op, k);
    }
    // price and disc are read with the key and the predicate, whatever the
    // predicate says, so a row costs one memory round trip instead of two
    // (the rows the filter drops cost their 16 bytes).  bad collects kept
    // rows whose value does not fit VT.
    __device__ bool load(int64_t i, uint32_t& kk, VT& v, uint32_t& bad) const {
        kk = (uint32_t)key[i];
        const int64_t p = price[i], d = disc[i];
        const int64_t rev = p * (100 - d);
        v = (VT)rev;
        bool ok;
        if constexpr (MASK) ok = (mask[i >> 6] >> (i & 63)) & 1;
        else ok = cmp_eval((int64_t)date[i], op, k);
        if constexpr (CHECKS) bad |= (uint32_t)ok & (uint32_t)((uint64_t)rev >> 32 != 0);
        return ok;
    }
    __device__ bool load(int64_t i, uint32_t& kk, VT& v) const {
        uint32_t unused = 0;
        return load(i, kk, v, unused);
    }
};

// Sources with WRITES_MASK = true get their predicate bits from the histogram
// kernel.
template <class S, class = void>
struct SrcWritesMask : std::false_type {};
template <class S>
struct SrcWritesMask<S, std::void_t<decltype(S::WRITES_MASK)>> : std::integral_constant<bool, S::WRITES_MASK> {};

// Sources with CHECKS = true take a fourth load argument that collects values
// outside their declared width.
template <class S, class = void>
struct SrcChecks : std::false_type {};
template <class S>
struct SrcChecks<S, std::void_t<decltype(S::CHECKS)>> : std::integral_constant<bool, S::CHECKS> {};

// key column + int32 payload column, no filter (the mid table side).
struct SrcKeyCol {
    const int32_t* key;
    const int32_t* val;
    int64_t n;
    __device__ int64_t size() const { return n; }
    __device__ bool load_key(int64_t i, uint32_t& kk) const {
        kk = (uint32_t)key[i];
        return true;
    }
    __device__ bool load(int64_t i, uint32_t& kk, uint32_t& v) const {
        kk = (uint32_t)key[i];
        v = (uint32_t)val[i];
        return true;
    }
};

// ------------------------------------------------------------------ sinks
template <class V>
struct DstPairs {
    uint32_t* keys;
    V* vals;
    __device__ void store(int64_t i, uint32_t k, const V& v) const {
        keys[i] = k;
        vals[i] = v;
    }
};
template <>
struct DstPairs<NoVal> {
    uint32_t* keys;
    NoVal* vals;
    __device__ void store(int64_t i, uint32_t k, const NoVal&) const { keys[i] = k; }
};

template <class V> struct ValBytes { static constexpr int value = sizeof(V); };
template <> struct ValBytes<NoVal> { static constexpr int value = 0; };

// ------------------------------------------------------------------ config
// ITEMS_NARROW_: items per thread when the payload has at most 4 bytes (the
// staged tile then takes less LDS, so the tile can be longer: longer digit
// runs per tile, fewer look-backs per element).
template <int RB, int BLOCK_, int ITEMS_, int LB_ = 16, int ITEMS_NARROW_ = ITEMS_>
struct RadixCfg {
    template <class V>
    using ForVal = RadixCfg<RB, BLOCK_, (ValBytes<V>::value <= 4 ? ITEMS_NARROW_ : ITEMS_), LB_, ITEMS_NARROW_>;
    static constexpr int LOOKBACK = LB_;     // predecessors read per look-back round
    static constexpr int RADIX_BITS = RB;
    static constexpr int RADIX = 1 << RB;
    static constexpr int BLOCK = BLOCK_;
    static constexpr int ITEMS = ITEMS_;
    static constexpr int TILE = BLOCK_ * ITEMS_;
    static constexpr int WAVES = BLOCK_ / WAVE;
    static constexpr int MAX_PASSES = (32 + RB - 1) / RB;
};

constexpr uint32_t ST_AGG = 1u << 30;       // tile aggregate published
constexpr uint32_t ST_INC = 2u << 30;       // inclusive prefix published
constexpr uint32_t ST_VAL = (1u << 30) - 1;

struct PassDesc {
    int32_t shift[8];
    int32_t bits[8];
    int32_t npass;
};

// ------------------------------------------------------------------ histogram
constexpr int HIST_ITEMS = 8;

// One read of the input: digit histograms of every pass (LDS-privatised, then
// merged with one global atomic per bin and block), the number of elements
// that take part, and the key-width check.
template <class Cfg, class Src>
__global__ void __launch_bounds__(Cfg::BLOCK)
k_radix_hist(Src src, PassDesc pd, uint32_t key_mask, uint32_t* hist, int64_t* d_count,
             uint32_t* flags) {
    constexpr int R = Cfg::RADIX;
    __shared__ uint32_t h[Cfg::MAX_PASSES * R];
    __shared__ uint32_t s_cnt;
    __shared__ uint32_t s_bad;
    for (int i = threadIdx.x; i < pd.npass * R; i += Cfg::BLOCK) h[i] = 0;
    if (threadIdx.x == 0) { s_cnt = 0; s_bad = 0; }
    __syncthreads();
    const int64_t n = src.size();
    uint32_t cnt = 0, bad = 0;
    // HIST_ITEMS loads per thread are issued before any counter update, so
    // each wave keeps that many requests in flight.
    constexpr int U = HIST_ITEMS;
    const int64_t step = (int64_t)gridDim.x * Cfg::BLOCK * U;
    for (int64_t base = (int64_t)blockIdx.x * Cfg::BLOCK * U + threadIdx.x; base < n; base += step) {
        uint32_t kk[U];
        bool ok[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int64_t i = base + (int64_t)j * Cfg::BLOCK;
            const bool in = i < n;
            ok[j] = src.load_key(in ? i : n - 1, kk[j]) && in;     // base < n, so n >= 1
        }
        if constexpr (SrcWritesMask<Src>::value) {
            // the 64 rows of item j of a wave are consecutive and 64-aligned
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const uint64_t m = ballot(ok[j]);
                const int64_t i0 = base - lane_id() + (int64_t)j * Cfg::BLOCK;
                if (lane_id() == 0 && i0 < n) src.mask[i0 >> 6] = m;
            }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (!ok[j]) continue;
            const uint32_t k = kk[j];
            ++cnt;
            bad |= k & ~key_mask;
            for (int p = 0; p < pd.npass; ++p) {
                uint32_t d = (k >> pd.shift[p]) & ((1u << pd.bits[p]) - 1);
                atomicAdd(&h[p * R + d], 1u);
            }
        }
    }
    cnt = wave_sum(cnt);
    if (lane_id() == 0 && cnt) atomicAdd(&s_cnt, cnt);
    if (bad) atomicOr(&s_bad, 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < pd.npass * R; i += Cfg::BLOCK)
        if (h[i]) atomic_add(&hist[i], h[i]);
    if (threadIdx.x == 0) {
        if (d_count && s_cnt) atomic_add(d_count, (int64_t)s_cnt);
        if (s_bad) set_flag(flags, FLAG_KEY_RANGE);
    }
}

// Pre-counted first pass.  The histogram kernel below walks the tiles of the
// first pass itself (block c owns the contiguous tiles [c*tpc, (c+1)*tpc)),
// so besides the global histograms it records, per tile and digit, the count
// of earlier tiles of the same chunk (pre), and per chunk and digit the chunk
// total (ctot).  A one-block-per-digit scan turns the chunk totals into chunk
// bases (cbase: the digit's global start plus the counts of earlier chunks).
// The first pass then knows every tile's global offsets up front and needs no
// look-back: its tiles run in any order.
constexpr int COUNT_CHUNKS = 512;        // chunks (blocks) of the counting kernel, at most 1024
constexpr int CHUNK_SCAN_BLOCK = 1024;

template <class Cfg, class Src>
__global__ void __launch_bounds__(Cfg::BLOCK)
k_radix_hist_tiles(Src src, PassDesc pd, uint32_t key_mask, uint32_t* hist, int64_t* d_count,
                   uint32_t* flags, uint32_t* pre, uint32_t* ctot, int tpc, int64_t ntiles_cap) {
    constexpr int R = Cfg::RADIX, ITEMS = Cfg::ITEMS, TILE = Cfg::TILE;
    // h[0, R): the chunk's first-pass counts so far; h[R, npass*R): later
    // passes' counts over the chunk.  The counters only grow: a tile's
    // counts are the difference of two readings.  (Clearing them between
    // tiles raced with the next tile's increments: the back edge of the tile
    // loop reached its barrier with the clearing stores still in flight, and
    // another wave's increments could land first and be erased.)
    __shared__ uint32_t h[Cfg::MAX_PASSES * R];
    __shared__ uint32_t s_cnt;
    __shared__ uint32_t s_bad;
    constexpr int PER = (R + Cfg::BLOCK - 1) / Cfg::BLOCK;   // digits per thread
    uint32_t run[PER];                    // digit tid + q * BLOCK: the chunk's count before the tile
#pragma unroll
    for (int q = 0; q < PER; ++q) run[q] = 0;
    for (int i = threadIdx.x; i < pd.npass * R; i += Cfg::BLOCK) h[i] = 0;
    if (threadIdx.x == 0) { s_cnt = 0; s_bad = 0; }
    __syncthreads();
    const int64_t n = src.size();
    int64_t ntiles = (n + TILE - 1) / TILE;
    if (ntiles > ntiles_cap) ntiles = ntiles_cap;          // the tiles pre holds
    const int64_t t0 = (int64_t)blockIdx.x * tpc;
    const int64_t t1 = t0 + tpc < ntiles ? t0 + tpc : ntiles;
    const int sh0 = pd.shift[0];
    const uint32_t m0 = (1u << pd.bits[0]) - 1;
    uint32_t cnt = 0, bad = 0;
    // the next tile's loads are issued before the current tile is counted
    uint32_t kc[ITEMS], kn[ITEMS];
    bool oc[ITEMS], on[ITEMS];
    auto load = [&](int64_t t, uint32_t* kk, bool* ok) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int64_t i = t * TILE + (int64_t)j * Cfg::BLOCK + threadIdx.x;
            const bool in = i < n;
            ok[j] = src.load_key(in ? i : n - 1, kk[j]) && in;     // t < ntiles, so n >= 1
        }
    };
    if (t0 < t1) load(t0, kc, oc);
    for (int64_t t = t0; t < t1; ++t) {
        if (t + 1 < t1) load(t + 1, kn, on);
        __syncthreads();                      // the previous tile's readings are taken
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            if (!oc[j]) continue;
            const uint32_t k = kc[j];
            ++cnt;
            bad |= k & ~key_mask;
            atomicAdd(&h[(k >> sh0) & m0], 1u);
            for (int p = 1; p < pd.npass; ++p)
                atomicAdd(&h[p * R + ((k >> pd.shift[p]) & ((1u << pd.bits[p]) - 1))], 1u);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int d = threadIdx.x + q * Cfg::BLOCK;
            if (d < R) {
                const uint32_t c = h[d];      // through this tile
                // taken before this thread reaches the next barrier (the
                // compiler does not wait for LDS on the loop's back edge),
                // so that no increment of the next tile can reach it
                asm volatile("" : : "v"(c));
                pre[t * R + d] = run[q];
                run[q] = c;
            }
        }
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) { kc[j] = kn[j]; oc[j] = on[j]; }
    }
    cnt = wave_sum(cnt);
    if (lane_id() == 0 && cnt) atomicAdd(&s_cnt, cnt);
    if (bad) atomicOr(&s_bad, 1u);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int d = threadIdx.x + q * Cfg::BLOCK;
        if (d < R) {
            ctot[(int64_t)blockIdx.x * R + d] = run[q];
            if (run[q]) atomic_add(&hist[d], run[q]);
        }
    }
    for (int i = R + threadIdx.x; i < pd.npass * R; i += Cfg::BLOCK)
        if (h[i]) atomic_add(&hist[i], h[i]);
    if (threadIdx.x == 0) {
        if (d_count && s_cnt) atomic_add(d_count, (int64_t)s_cnt);
        if (s_bad) set_flag(flags, FLAG_KEY_RANGE);
    }
}

// cbase[c][d] = (count of digits below d) + (count of d in chunks before c);
// one block per digit, one thread per chunk.
__global__ void k_radix_chunk_scan(const uint32_t* ctot, int nchunks, const uint32_t* hist0, int R,
                                   uint32_t* cbase);

// ------------------------------------------------------------------ one pass
// LDS of one pass: the per-wave digit counters are only live while ranking and
// the staged tile only while scattering, so the two share storage.
template <class Cfg, class V>
struct PassSmem {
    static constexpr int R = Cfg::RADIX;
    struct Stage {
        uint32_t keys[Cfg::TILE];
        typename std::conditional<ValBytes<V>::value == 0, char, V>::type
            vals[ValBytes<V>::value == 0 ? 1 : Cfg::TILE];
    };
    union {
        uint32_t wave_hist[Cfg::WAVES][R];
        Stage stage;
    } u;
    uint32_t local_start[R];
    int32_t delta[R];
    uint32_t scratch[Cfg::WAVES];
    uint32_t tile;
};

// Exclusive prefix of digit d over the tiles before `tile` (one thread per
// digit).  Walks back from tile - 1 reading LOOKBACK_WINDOW status words per
// round (the loads are issued together, so a round costs one memory round
// trip however many tiles it covers), adding aggregates until it meets an
// inclusive prefix.
template <int LOOKBACK_WINDOW>
__device__ __forceinline__ uint32_t radix_lookback(const uint32_t* status, int64_t tile, int R, int d,
                                                   uint32_t* flags) {
    uint32_t excl = 0;
    int64_t j = tile - 1;
    uint32_t spins = 0;
    while (j >= 0) {
        uint32_t s[LOOKBACK_WINDOW];
#pragma unroll
        for (int i = 0; i < LOOKBACK_WINDOW; ++i)
            s[i] = (j - i >= 0) ? ld_relaxed(status + (j - i) * R + d) : ST_INC;
        uint32_t acc = 0;
        int used = 0;
        bool done = false, stall = false;
#pragma unroll
        for (int i = 0; i < LOOKBACK_WINDOW; ++i) {
            if (done || stall) continue;
            const uint32_t f = s[i] & ~ST_VAL;
            if (f == 0) { stall = true; continue; }
            acc += s[i] & ST_VAL;
            used = i + 1;
            if (f == ST_INC) done = true;
        }
        excl += acc;
        j -= used;
        if (done) break;
        if (stall) {
            if (++spins > SPIN_LIMIT) { set_flag(flags, FLAG_SPIN_LIMIT); break; }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return excl;
}

// One tile of one pass (shared by the single-input kernel and the batched
// kernel).  The caller has obtained the tile id in increasing order from a
// counter, so every predecessor of the tile is held by a running block.
// Global offsets of a pre-counted first pass (see k_radix_hist_tiles).
struct PassCounts {
    const uint32_t* pre;
    const uint32_t* cbase;
    int tpc;
};

template <class Cfg, class Src, class V, bool COUNTED = false>
__device__ __forceinline__ void radix_pass_tile(const Src& src, const DstPairs<V>& dst, int shift, int bits,
                                                const uint32_t* hist, uint32_t* status, uint32_t tile,
                                                int64_t n, uint32_t* flags, PassSmem<Cfg, V>& sm,
                                                PassCounts pc = {}) {
    constexpr int R = Cfg::RADIX, ITEMS = Cfg::ITEMS, TILE = Cfg::TILE, W = Cfg::WAVES;
    const int tid = threadIdx.x, w = tid / WAVE, l = lane_id();
    for (int i = tid; i < W * R; i += Cfg::BLOCK) (&sm.u.wave_hist[0][0])[i] = 0;
    __syncthreads();
    const uint32_t dmask = (1u << bits) - 1;
    const int nd = (int)dmask + 1;            // digits of this pass (<= R)
    // Load: wave w owns the contiguous chunk [w*ITEMS*64, (w+1)*ITEMS*64) of the
    // tile, item j of lane l is element chunk + j*64 + l (coalesced loads).
    const int64_t base = (int64_t)tile * TILE + (int64_t)w * ITEMS * WAVE;
    uint32_t key[ITEMS];
    V val[ITEMS];
    uint32_t pos[ITEMS];
    bool valid[ITEMS];
    uint32_t bad = 0;
    // pre-counted: the tile's global digit offsets, read with the items
    constexpr int PER = (R + Cfg::BLOCK - 1) / Cfg::BLOCK;
    uint32_t goff[PER];
    if constexpr (COUNTED) {
        const int64_t c = tile / pc.tpc;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int d = tid + q * Cfg::BLOCK;
            goff[q] = d < nd ? pc.cbase[c * R + d] + pc.pre[(int64_t)tile * R + d] : 0;
        }
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = base + j * WAVE + l;
        const bool in = i < n;
        if constexpr (SrcChecks<Src>::value)
            valid[j] = src.load(in ? i : n - 1, key[j], val[j], bad) && in;   // n >= 1: the tile exists
        else
            valid[j] = src.load(in ? i : n - 1, key[j], val[j]) && in;
    }
    if constexpr (SrcChecks<Src>::value) {
        if (bad) set_flag(flags, FLAG_VALUE_RANGE);
    }

    // Rank: peers with the same digit found by one ballot per digit bit (a
    // lane differs from this one where the ballot of a bit disagrees with this
    // lane's bit); the per-wave counter of the digit gives the rank of earlier
    // items.  Full-width digits (the common case) unroll without bounds.
    auto rank = [&](auto full) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t d = valid[j] ? (key[j] >> shift) & dmask : 0;
            uint32_t dlo = 0, dhi = 0;
#pragma unroll
            for (int b = 0; b < Cfg::RADIX_BITS; ++b) {
                if (decltype(full)::value || b < bits) {
                    const uint32_t bit = (d >> b) & 1u;
                    const uint64_t t = ballot(bit != 0);
                    const uint32_t m = 0u - bit;
                    dlo |= (uint32_t)t ^ m;
                    dhi |= (uint32_t)(t >> 32) ^ m;
                }
            }
            const uint64_t peers = ballot(valid[j]) & ~(((uint64_t)dhi << 32) | dlo);
            if (valid[j]) {
                const uint32_t before = sm.u.wave_hist[w][d];
                const uint64_t lower = peers & lanemask_lt();
                pos[j] = before + popc64(lower);
                if ((peers >> l) == 1) sm.u.wave_hist[w][d] = before + popc64(peers);   // last peer
            }
        }
    };
    if (bits == Cfg::RADIX_BITS) rank(std::true_type{});
    else rank(std::false_type{});
    __syncthreads();

    // Per digit: exclusive prefix over waves (in place), tile count, publish
    // the tile aggregate as early as possible.
    for (int d = tid; d < R; d += Cfg::BLOCK) {
        uint32_t run = 0;
#pragma unroll
        for (int ww = 0; ww < W; ++ww) {
            const uint32_t c = sm.u.wave_hist[ww][d];
            sm.u.wave_hist[ww][d] = run;
            run += c;
        }
        sm.local_start[d] = run;   // tile count for now; scanned below
        if constexpr (!COUNTED) {
            if (d < nd) st_relaxed(status + (int64_t)tile * R + d, (tile == 0 ? ST_INC : ST_AGG) | run);
        }
    }
    __syncthreads();
    // Tile-local digit starts (exclusive scan of the tile counts, in place).
    const uint32_t tile_total = block_excl_scan_array<Cfg::BLOCK>(sm.local_start, R, sm.scratch);
    if constexpr (COUNTED) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int d = tid + q * Cfg::BLOCK;
            if (d < nd) sm.delta[d] = (int32_t)goff[q] - (int32_t)sm.local_start[d];
        }
    } else {
        // Global digit base: exclusive scan of this pass's histogram.
        const int per = (R + Cfg::BLOCK - 1) / Cfg::BLOCK;
        const int b0 = tid * per;
        uint32_t loc = 0;
        for (int i = 0; i < per; ++i)
            if (b0 + i < nd) loc += hist[b0 + i];
        uint32_t tot;
        uint32_t off = block_excl_sum<Cfg::BLOCK>(loc, sm.scratch, &tot);
        for (int i = 0; i < per; ++i) {
            const int d = b0 + i;
            if (d < nd) {
                sm.delta[d] = (int32_t)off - (int32_t)sm.local_start[d];
                off += hist[d];
            }
        }
    }
    // Positions inside the tile, while the per-wave offsets are still in LDS.
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if (valid[j]) {
            const uint32_t d = (key[j] >> shift) & dmask;
            pos[j] += sm.local_start[d] + sm.u.wave_hist[w][d];
        }
    }
    __syncthreads();
    // Stage the tile in digit order (overwrites the counters) ...
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if (valid[j]) {
            sm.u.stage.keys[pos[j]] = key[j];
            if constexpr (ValBytes<V>::value != 0) sm.u.stage.vals[pos[j]] = val[j];
        }
    }
    // ... while one thread per digit looks back for the tile's global offset.
    for (int d = tid; d < nd && !COUNTED; d += Cfg::BLOCK) {
        if (tile != 0) {
            const uint32_t excl = radix_lookback<Cfg::LOOKBACK>(status, tile, R, d, flags);
            st_relaxed(status + (int64_t)tile * R + d,
                       ST_INC | (excl + (d + 1 < R ? sm.local_start[d + 1] : tile_total) - sm.local_start[d]));
            sm.delta[d] += (int32_t)excl;
        }
    }
    __syncthreads();
    // Coalesced write-out: consecutive LDS slots of one digit go to
    // consecutive global positions.
    for (uint32_t p = tid; p < tile_total; p += Cfg::BLOCK) {
        const uint32_t k = sm.u.stage.keys[p];
        const uint32_t d = (k >> shift) & dmask;
        const int64_t g = (int64_t)p + sm.delta[d];
        if constexpr (ValBytes<V>::value != 0) dst.store(g, k, sm.u.stage.vals[p]);
        else dst.store(g, k, NoVal{});
    }
}

// Tag only separates the launches of different sorts in a profile (the
// kernel symbol carries it); it changes nothing in the code.
template <class Cfg, class Src, class V, int Tag = 0>
__global__ void __launch_bounds__(Cfg::BLOCK)
k_radix_pass(Src src, DstPairs<V> dst, int shift, int bits, const uint32_t* hist,
             uint32_t* status, uint32_t* tile_counter, uint32_t* flags) {
    __shared__ PassSmem<Cfg, V> sm;
    if (threadIdx.x == 0) sm.tile = atomicAdd(tile_counter, 1u);
    __syncthreads();
    const uint32_t tile = sm.tile;
    const int64_t n = src.size();
    if ((int64_t)tile >= (n + Cfg::TILE - 1) / Cfg::TILE) return;
    radix_pass_tile<Cfg, Src, V>(src, dst, shift, bits, hist, status, tile, n, flags, sm);
}

// First pass with pre-counted offsets: tile = block, no waits.
template <class Cfg, class Src, class V, int Tag = 0>
__global__ void __launch_bounds__(Cfg::BLOCK)
k_radix_pass_counted(Src src, DstPairs<V> dst, int shift, int bits, PassCounts pc, uint32_t* flags) {
    __shared__ PassSmem<Cfg, V> sm;
    const uint32_t tile = blockIdx.x;
    const int64_t n = src.size();
    if ((int64_t)tile >= (n + Cfg::TILE - 1) / Cfg::TILE) return;
    radix_pass_tile<Cfg, Src, V, true>(src, dst, shift, bits, nullptr, nullptr, tile, n, flags, sm, pc);
}

// ---------------------------------------------------------- finishing pass
// Completes the sort of keys already sorted on their bits above lowb
// (lowb <= FINISH_LOG2): the rows whose key lies in one span [s << FINISH_LOG2,
// (s + 1) << FINISH_LOG2) are contiguous (two 64-way wave searches find
// them), so one block per span counting-sorts them in LDS (count per key,
// scan, scatter).  Equal keys end up in arbitrary order.  With bstart (and
// 0 < lowb <= FINISH_LOG2), each block also records where every bucket of
// 2^lowb key values in its span starts in the output, and the last block the
// end of the last bucket: bstart[b] = lower_bound(kout, b << lowb) for b in
// [0, nspans << (FINISH_LOG2 - lowb)].  With d_n, the keys are the first
// min(n, *d_n).
constexpr int FINISH_LOG2 = 12;
constexpr int FINISH_SPAN = 1 << FINISH_LOG2;
constexpr int FINISH_BLOCK = 256;
__global__ void k_finish_sort(const uint32_t* kin, const uint32_t* vin, int64_t n, uint32_t* kout, uint32_t* vout,
                              int lowb, int64_t* bstart, const int64_t* d_n = nullptr);

}  // namespace tqp
