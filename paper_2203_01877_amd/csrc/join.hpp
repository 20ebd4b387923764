// Sort-based equi-join over two key-sorted inputs (Section 5.2, Algorithm 1).
//
// The paper computes, per distinct key, the histogram product
// leftHist[k] * rightHist[k] (the bucket size), its prefix sum (the output
// offsets) and then finds each output slot's bucket by binary search
// (bucketize), splitting the in-bucket offset into a left part (quotient) and
// a right part (remainder).  Here the same quantities are computed per left
// element instead of per key, which needs no key-domain-sized arrays:
//
//   count(i)  = upper_bound(R, L[i]) - lower_bound(R, L[i])   (= rightHist[L[i]])
//   offset(i) = sum of count over left elements before i      (prefix sum, int64)
//
// Output slot o belongs to the left element i with offset(i) <= o <
// offset(i+1) (the bucket search) and pairs it with right element
// lower_bound(R, L[i]) + (o - offset(i)) (the remainder).  Over one bucket of
// equal keys this is exactly the left-major quotient / remainder order of
// Algorithm 1.
//
// One kernel does all of it per tile of left elements: the tile's window of
// R is found with two wave-wide searches and staged in LDS, counts come from
// LDS binary searches, the tile's output base from a block scan plus a
// decoupled look-back, and the tile's outputs are expanded in place.  The
// kernel is persistent: each block pulls tiles from a counter until none is
// left, so emitters can accumulate across tiles and flush once.
#pragma once
#include "dev.hpp"

namespace tqp {

template <int BLOCK_, int ITEMS_, int RWIN_>
struct JoinCfg {
    static constexpr int BLOCK = BLOCK_;
    static constexpr int ITEMS = ITEMS_;
    static constexpr int TILE = BLOCK_ * ITEMS_;
    static constexpr int RWIN = RWIN_;
    static constexpr int WAVES = BLOCK_ / WAVE;
};

// Window rows each thread loads per round while building a tile's LDS table
// (the expanding kernel has fewer registers to spare than the counting one).
constexpr int TABLE_ITEMS = 4;
constexpr int COUNT_TABLE_ITEMS = 8;

// Join kinds: the inner join, and the left semi, left anti and left outer
// joins of the operator list at the start of Section 5, which Section 5.2
// reaches by small changes to the sort-based join.  Only the number of output
// rows per left element changes: semi keeps an element with at least one
// match once, anti keeps one with none, outer emits an unmatched element once
// with no right row.  A missing right row is written as -1 (JOIN_NONE).
constexpr int JOIN_INNER = 0, JOIN_SEMI = 1, JOIN_ANTI = 2, JOIN_OUTER = 3;
constexpr uint32_t JOIN_NONE = 0xFFFFFFFFu;
template <int KIND>
__device__ __forceinline__ int64_t join_out_rows(int64_t matches) {
    if constexpr (KIND == JOIN_SEMI) return matches > 0;
    else if constexpr (KIND == JOIN_ANTI) return matches == 0;
    else if constexpr (KIND == JOIN_OUTER) return matches > 0 ? matches : 1;
    else return matches;
}

// When every element of a wave's round has at most JOIN_LANE_MAX output
// rows, each lane emits its own.  Otherwise runs of JOIN_WAVE_RUN rows or
// more are emitted by the whole wave one run at a time (64 consecutive rows
// per step), and the rest of the round's rows 64 at a time, each lane finding
// the element its row belongs to (load-balanced expansion: full lanes
// whatever the mix of short run lengths).  Aggregating emitters keep the
// simpler form: short runs by their lane, each longer run by the whole wave.
constexpr int JOIN_LANE_MAX = 4;
constexpr int JOIN_WAVE_RUN = 32;      // runs this long are written by the whole wave, one at a time

// ------------------------------------------------------------------ emitters
// Index pairs (late materialisation: the join returns row-index pairs).
struct EmitPairs {
    static constexpr bool ORDERED = true;      // writes at the output positions
    int32_t* out_l;
    int32_t* out_r;
    int64_t cap;
    struct Smem {};
    __device__ void init(Smem&) {}
    __device__ void operator()(int64_t o, uint32_t, uint32_t lp, uint32_t rp, Smem&) {
        if (o < cap) {
            out_l[o] = (int32_t)lp;
            if (out_r) out_r[o] = (int32_t)rp;
        }
    }
    __device__ void finish(Smem&) {}
};

// (group key from the right side, value V from the left side), with the
// digit histograms of the following group-key sort accumulated on the way.
template <int BLOCK, int RB, class V = uint64_t>
struct EmitKeyVal {
    static constexpr bool ORDERED = true;
    static constexpr int R = 1 << RB;
    static constexpr int NP = (32 + RB - 1) / RB;
    uint32_t* out_key;
    V* out_val;
    int64_t cap;
    uint32_t key_mask;         // group keys must fit the declared width
    uint32_t* flags;
    uint32_t* hist;            // NP * R global digit counts of out_key (null: none)
    int32_t npass;
    int32_t shift[NP];
    int32_t bits[NP];
    struct Smem {
        uint32_t h[NP * R];
    };
    __device__ void init(Smem& s) {
        if (hist)
            for (int i = threadIdx.x; i < npass * R; i += BLOCK) s.h[i] = 0;
    }
    __device__ void operator()(int64_t o, uint32_t, uint64_t lp, uint32_t rp, Smem& s) {
        if (o < cap) {
            const uint32_t key = rp & key_mask;        // a key outside the width enters masked
            out_key[o] = key;
            out_val[o] = lp;
            if (rp & ~key_mask) set_flag(flags, FLAG_KEY_RANGE);
            if (hist)
                for (int p = 0; p < npass; ++p)
                    atomicAdd(&s.h[p * R + ((key >> shift[p]) & ((1u << bits[p]) - 1))], 1u);
        }
    }
    __device__ void finish(Smem& s) {
        if (!hist) return;
        __syncthreads();
        for (int i = threadIdx.x; i < npass * R; i += BLOCK)
            if (s.h[i]) atomic_add(&hist[i], s.h[i]);
    }
};

// Flags-fragment aggregation fused into the join output (the small-G direct
// path): gather price / disc / flags of the left row, evaluate the revenue
// expression and accumulate sum, count and sum(price) per packed group
// flagA * 2 + flagB in registers; flush once per block.  flagA in 0..2 and
// flagB in 0..1 give the six groups 0..5; a row with a flag outside its
// domain is left out and sets FLAG_VALUE_RANGE.
template <int BLOCK>
struct EmitFlagsAgg {
    static constexpr bool ORDERED = false;     // aggregates only: positions unused
    static constexpr int G = 6;
    const int64_t* price;
    const int64_t* disc;
    const int8_t* flagA;
    const int8_t* flagB;
    int64_t* acc;              // [G][3] global: sum, count, sum(price)
    uint32_t* flags;
    int64_t s[G], c[G], p[G];
    struct Smem {
        int64_t a[BLOCK / WAVE][G * 3];
    };
    __device__ void init(Smem&) {
#pragma unroll
        for (int g = 0; g < G; ++g) { s[g] = 0; c[g] = 0; p[g] = 0; }
    }
    __device__ void operator()(int64_t, uint32_t, uint32_t lp, uint32_t, Smem&) {
        const int64_t pr = price[lp];
        const int64_t v = pr * (100 - disc[lp]);
        const int fa = flagA[lp], fb = flagB[lp];
        const bool ok = (unsigned)fa <= 2u && (unsigned)fb <= 1u;
        const int g = ok ? fa * 2 + fb : -1;
        if (!ok) set_flag(flags, FLAG_VALUE_RANGE);
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const bool on = (g == k);
            s[k] += on ? v : 0;
            c[k] += on ? 1 : 0;
            p[k] += on ? pr : 0;
        }
    }
    // Block-wide sums of the register accumulators added to dst[G][3], which
    // are then cleared (the batched join flushes after every tile).
    __device__ void flush(Smem& sm, int64_t* dst) {
        const int w = threadIdx.x / WAVE;
#pragma unroll
        for (int k = 0; k < G; ++k) {
            int64_t a = wave_sum(s[k]), b = wave_sum(c[k]), d = wave_sum(p[k]);
            if (lane_id() == 0) { sm.a[w][k * 3] = a; sm.a[w][k * 3 + 1] = b; sm.a[w][k * 3 + 2] = d; }
            s[k] = 0; c[k] = 0; p[k] = 0;
        }
        __syncthreads();
        if (threadIdx.x < G * 3) {
            int64_t t = 0;
            for (int ww = 0; ww < BLOCK / WAVE; ++ww) t += sm.a[ww][threadIdx.x];
            if (t) atomic_add(&dst[threadIdx.x], t);
        }
        __syncthreads();
    }
    __device__ void finish(Smem& sm) { flush(sm, acc); }
};

// ------------------------------------------------------------------ kernels
// R window of every left tile: [lower_bound(R, first key), upper_bound(R, last
// key)).  One thread per tile; all tiles search at once, or, given the start
// of every bucket of 2^lowb key values in R (rbstart[0..nbkt]), read it there.
__global__ void k_join_windows(const uint32_t* lkey, int64_t nl_upper, const int64_t* d_nl,
                               const uint32_t* rkey, int64_t nr_upper, const int64_t* d_nr, int tile_size,
                               int64_t* win, int lowb, const int64_t* rbstart, int64_t nbkt);

template <class Cfg, class RP>
struct JoinSmem {
    // Direct table of the tile's key range: for key value v in [kmin, kmin + KRANGE),
    // first[v - kmin] = first right position (relative to the window) with
    // that key, cnt[...] = number of right rows with it (rightHist of v).
    int32_t first[Cfg::RWIN];
    int32_t cnt[Cfg::RWIN];
    RP rpay[Cfg::RWIN];
    int64_t wave[Cfg::WAVES];
    int64_t base;
    uint32_t tile;
    int32_t seg;
};

// One left tile (shared by the single-input kernel and the batched kernel):
// match counts, output base by look-back, expansion into the emitter.  When
// the tile's key range and its R window both fit RWIN, counts and first
// matches come from a direct LDS table built from the window (two LDS reads
// per left element) and the right payloads are staged in LDS; otherwise from
// binary searches over the window in global memory.  ntiles is the number of
// tiles of this left input; the last one stores the join size.
//
// The right keys must be fully sorted.  The left keys need only be sorted on
// their bits above lowb: every key of the tile then lies in its bucket-aligned
// range, and each left element is looked up on its own, so the pairs of a
// tile come out in the tile's element order instead of key order (the same
// pairs; lowb = 0 keeps the canonical order).
// What a left tile needs before its rows are read: its R window and its
// first and last left keys.  The persistent kernels load it one tile ahead,
// so that a tile's row loads and window loads go out together.
struct TileGeo {
    int64_t wlo, whi;
    uint32_t kfirst, klast;
};
__device__ __forceinline__ TileGeo tile_geo(const uint32_t* lkey, int64_t nl, const int64_t* win, int64_t tile,
                                            int tile_size) {
    const int64_t t0 = tile * tile_size;
    const int64_t tl = (t0 + tile_size < nl ? t0 + tile_size : nl) - 1;
    return TileGeo{win[2 * tile], win[2 * tile + 1], lkey[t0], lkey[tl]};
}

// Key range of a left tile whose keys are sorted on their bits above lowb
// (lowb = 0: fully sorted): from the bucket of its first key to the end of
// the bucket of its last key.
__device__ __forceinline__ void tile_key_range(const TileGeo& g, int lowb, uint32_t& kmin, uint32_t& kmax) {
    kmin = (g.kfirst >> lowb) << lowb;
    kmax = ((g.klast >> lowb) << lowb) | ((1u << lowb) - 1);
}

// Output rows of one left tile, for the counting kernel of the two-kernel
// join: the same direct table (counts only) or global searches as join_tile,
// with no payload traffic.  The value is returned to every thread.
template <class Cfg, class RP, int KIND = JOIN_INNER>
__device__ __forceinline__ int64_t join_tile_count(const uint32_t* lkey, int64_t nl, const uint32_t* rkey,
                                                   const TileGeo& g, int64_t tile, JoinSmem<Cfg, RP>& sm,
                                                   int lowb) {
    constexpr int TILE = Cfg::TILE, ITEMS = Cfg::ITEMS, RWIN = Cfg::RWIN, W = Cfg::WAVES;
    const int tid = threadIdx.x, w = tid / WAVE, l = lane_id();
    const int64_t t0 = tile * TILE;
    uint32_t kmin, kmax;
    tile_key_range(g, lowb, kmin, kmax);
    const int64_t wlo = g.wlo, whi = g.whi;
    const int64_t wn = whi - wlo;
    const bool direct = wn <= RWIN && (int64_t)kmax - (int64_t)kmin < RWIN;
    // The tile's keys and the first round of window keys are loaded together
    // (clamped indexes: no branch between the loads); the table is cleared
    // while they are in flight.
    const int64_t chunk = t0 + (int64_t)w * ITEMS * WAVE;
    uint32_t key[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = chunk + j * WAVE + l;
        key[j] = lkey[i < nl ? i : nl - 1];                 // the tile exists, so nl >= 1
    }
    uint32_t kk0[COUNT_TABLE_ITEMS];
    if (direct && wn > 0) {
#pragma unroll
        for (int u = 0; u < COUNT_TABLE_ITEMS; ++u) {
            const int i = tid + u * Cfg::BLOCK;
            kk0[u] = rkey[wlo + (i < wn ? i : wn - 1)];
        }
    }
    if (direct) {
        const int range = (int)(kmax - kmin) + 1;
        for (int i = tid; i < range; i += Cfg::BLOCK) sm.cnt[i] = 0;
    }
    __syncthreads();
    if (direct) {
        // keys outside [kmin, kmax] occur only in inputs that break the
        // declared key width (already flagged): they are skipped, never
        // indexed
        const uint32_t range = kmax - kmin + 1;
        if (wn > 0) {
#pragma unroll
            for (int u = 0; u < COUNT_TABLE_ITEMS; ++u) {
                const uint32_t v = kk0[u] - kmin;
                if (tid + u * Cfg::BLOCK < wn && v < range) atomicAdd(&sm.cnt[v], 1);
            }
        }
        for (int i0 = tid + Cfg::BLOCK * COUNT_TABLE_ITEMS; i0 < wn; i0 += Cfg::BLOCK * COUNT_TABLE_ITEMS) {
            uint32_t kk[COUNT_TABLE_ITEMS];
#pragma unroll
            for (int u = 0; u < COUNT_TABLE_ITEMS; ++u) {
                const int i = i0 + u * Cfg::BLOCK;
                kk[u] = rkey[wlo + (i < wn ? i : wn - 1)];
            }
#pragma unroll
            for (int u = 0; u < COUNT_TABLE_ITEMS; ++u) {
                const uint32_t v = kk[u] - kmin;
                if (i0 + u * Cfg::BLOCK < wn && v < range) atomicAdd(&sm.cnt[v], 1);
            }
        }
        __syncthreads();
    }
    int64_t c = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = chunk + j * WAVE + l;
        if (i < nl) {
            if (direct) {
                const uint32_t v = key[j] - kmin;
                c += join_out_rows<KIND>(v <= kmax - kmin ? sm.cnt[v] : 0);
            } else {
                const int64_t lb = lower_bound_glb(rkey, wlo, whi, key[j]);
                c += join_out_rows<KIND>(upper_bound_glb(rkey, lb, whi, key[j]) - lb);
            }
        }
    }
    c = wave_sum(c);
    if (l == 0) sm.wave[w] = c;
    __syncthreads();
    int64_t tot = 0;
    for (int ww = 0; ww < W; ++ww) tot += sm.wave[ww];
    __syncthreads();
    return tot;
}

// base: the tile's output base (emitters that write at output positions;
// the counting kernel's totals give it).  Emitters that only aggregate add
// the tile's total to *d_count instead.
template <class Cfg, class LP, class RP, class Emit, int KIND = JOIN_INNER>
__device__ __forceinline__ void join_tile(const uint32_t* lkey, const LP* lpay, int64_t nl, const uint32_t* rkey,
                                          const RP* rpay, const TileGeo& g, int64_t tile, int64_t base,
                                          int64_t* d_count, Emit& e, typename Emit::Smem& esm,
                                          JoinSmem<Cfg, RP>& sm, int lowb = 0) {
    constexpr int TILE = Cfg::TILE, ITEMS = Cfg::ITEMS, RWIN = Cfg::RWIN, W = Cfg::WAVES;
    const int tid = threadIdx.x, w = tid / WAVE, l = lane_id();
    const int64_t t0 = tile * TILE;
    uint32_t kmin, kmax;
    tile_key_range(g, lowb, kmin, kmax);
    const int64_t wlo = g.wlo, whi = g.whi;
    const int64_t wn = whi - wlo;
    const bool direct = wn <= RWIN && (int64_t)kmax - (int64_t)kmin < RWIN;
    if (direct) {
        const int range = (int)(kmax - kmin) + 1;
        for (int i = tid; i < range; i += Cfg::BLOCK) {
            sm.cnt[i] = 0;
            sm.first[i] = RWIN;
        }
    }
    // The wave's contiguous chunk of the tile, 64 elements per round.
    const int64_t chunk = t0 + (int64_t)w * ITEMS * WAVE;
    uint32_t key[ITEMS];
    LP pay[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = chunk + j * WAVE + l;
        key[j] = 0;
        if (i < nl) {
            key[j] = lkey[i];
            pay[j] = lpay ? lpay[i] : (LP)i;
        }
    }
    __syncthreads();
    if (direct) {
        // TABLE_ITEMS window rows per thread and round, loaded before any is
        // used (clamped index: no branch between the loads)
        auto build = [&](auto load_pay) {
            for (int i0 = tid; i0 < wn; i0 += Cfg::BLOCK * TABLE_ITEMS) {
                uint32_t kk[TABLE_ITEMS];
                RP pp[TABLE_ITEMS];
#pragma unroll
                for (int u = 0; u < TABLE_ITEMS; ++u) {
                    const int i = i0 + u * Cfg::BLOCK;
                    const int ic = i < wn ? i : (int)wn - 1;
                    kk[u] = rkey[wlo + ic];
                    pp[u] = load_pay(wlo + ic);
                }
#pragma unroll
                for (int u = 0; u < TABLE_ITEMS; ++u) {
                    const int i = i0 + u * Cfg::BLOCK;
                    if (i < wn) {
                        const uint32_t v = kk[u] - kmin;     // window keys lie in [kmin, kmax] (others skipped)
                        if (v <= kmax - kmin) {
                            atomicMin(&sm.first[v], i);
                            atomicAdd(&sm.cnt[v], 1);
                        }
                        sm.rpay[i] = pp[u];
                    }
                }
            }
        };
        if (rpay) build([&](int64_t r) { return rpay[r]; });
        else build([&](int64_t r) { return (RP)r; });
        __syncthreads();
    }
    // Match count and first match of each element: rightHist of its key.
    // first is relative to the window (windows hold fewer than 2^31 rows).
    // The per-element output offsets are not kept: the emit phase redoes the
    // wave scans, which costs less than holding them across the look-back.
    int32_t cnt[ITEMS], first[ITEMS];
    int64_t wave_total = 0;
    // output rows of item j (its matches for the inner join)
    auto out_rows = [&](int j) -> int64_t {
        if constexpr (KIND == JOIN_INNER) return cnt[j];
        else return chunk + j * WAVE + l < nl ? join_out_rows<KIND>(cnt[j]) : 0;
    };
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = chunk + j * WAVE + l;
        cnt[j] = 0;
        first[j] = 0;
        if (i < nl) {
            if (direct) {
                const uint32_t v = key[j] - kmin;
                if (v <= kmax - kmin) {
                    cnt[j] = sm.cnt[v];
                    first[j] = sm.first[v];
                }
            } else {
                const int64_t lb = lower_bound_glb(rkey, wlo, whi, key[j]);
                const int64_t ub = upper_bound_glb(rkey, lb, whi, key[j]);
                first[j] = (int32_t)(lb - wlo);
                cnt[j] = (int32_t)(ub - lb);
            }
        }
        wave_total += wave_sum(out_rows(j));
    }
    if (l == 0) sm.wave[w] = wave_total;
    __syncthreads();
    // Wave bases: the tile's base plus the totals of the waves before.
    if (!Emit::ORDERED && tid == 0) {
        int64_t tot = 0;
        for (int ww = 0; ww < W; ++ww) tot += sm.wave[ww];
        if (tot) atomic_add(d_count, tot);
    }
    int64_t wbase = base;
    for (int ww = 0; ww < w; ++ww) wbase += sm.wave[ww];
    // Expansion: output o of element i pairs it with right element first + (o - offset(i)).
    auto right = [&](int64_t r) -> RP {        // r relative to the window
        if (direct) return sm.rpay[r];
        return rpay ? rpay[wlo + r] : (RP)(wlo + r);
    };
    // Writing emitters read the first match of every element ahead of the
    // stores (independent reads: their latencies overlap); the aggregating
    // ones keep their registers for the gathers.
    constexpr bool AHEAD = Emit::ORDERED && (KIND == JOIN_INNER || KIND == JOIN_OUTER);
    RP r0[AHEAD ? ITEMS : 1];
    if constexpr (AHEAD) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) r0[j] = cnt[j] > 0 ? right(first[j]) : RP{};
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t oc = out_rows(j);
        const int64_t incl = wave_incl_sum(oc);
        const int64_t o = wbase + incl - oc;
        wbase += wave_read(incl, WAVE - 1);
        if constexpr (KIND == JOIN_SEMI || KIND == JOIN_ANTI) {
            if (oc) e(o, key[j], pay[j], (RP)JOIN_NONE, esm);
            continue;
        }
        if constexpr (!Emit::ORDERED) {
            // aggregating emitters (fewer registers to spare): short runs by
            // their own lane, each long one by the whole wave
            if constexpr (KIND == JOIN_OUTER) {
                if (oc && cnt[j] == 0) e(o, key[j], pay[j], (RP)JOIN_NONE, esm);
            }
            const bool small = cnt[j] <= JOIN_LANE_MAX;
            if (small)
                for (int t = 0; t < cnt[j]; ++t) e(o + t, key[j], pay[j], right(first[j] + t), esm);
            uint64_t heavy = ballot(!small);
            while (heavy) {
                const int src = __ffsll((unsigned long long)heavy) - 1;
                heavy &= heavy - 1;
                const int c = wave_read(cnt[j], src);
                const int64_t f = wave_read(first[j], src);
                const int64_t oo = wave_read(o, src);
                const uint32_t kk = wave_read(key[j], src);
                const LP pp = wave_read(pay[j], src);
                for (int q = l; q < c; q += WAVE) e(oo + q, kk, pp, right(f + q), esm);
            }
        } else if (!__any(cnt[j] > JOIN_LANE_MAX)) {
            // every element of the round has a short run: each lane writes its own
            if constexpr (KIND == JOIN_OUTER) {
                if (oc && cnt[j] == 0) e(o, key[j], pay[j], (RP)JOIN_NONE, esm);
            }
            if constexpr (AHEAD) {
                if (cnt[j] > 0) {
                    e(o, key[j], pay[j], r0[j], esm);
                    for (int t = 1; t < cnt[j]; ++t) e(o + t, key[j], pay[j], right(first[j] + t), esm);
                }
            } else {
                for (int t = 0; t < cnt[j]; ++t) e(o + t, key[j], pay[j], right(first[j] + t), esm);
            }
        } else {
            // some run is long.  Runs of at least JOIN_WAVE_RUN rows: the
            // whole wave writes each, 64 consecutive rows per step; the
            // shorter ones: the wave writes their rows 64 at a time, each
            // lane finding the element its row belongs to
            const bool lng = cnt[j] >= JOIN_WAVE_RUN;
            const int64_t oc2 = lng ? 0 : oc;
            const int64_t incl2 = wave_incl_sum(oc2);
            const int64_t excl2 = incl2 - oc2, tot2 = wave_read(incl2, WAVE - 1);
            for (int64_t q0 = 0; q0 < tot2; q0 += WAVE) {
                const int64_t q = q0 + l;
                const int src = wave_run_owner(excl2, q);
                const int64_t t = q - wave_shfl(excl2, src);
                const uint32_t kk = wave_shfl(key[j], src);
                const LP pp = wave_shfl(pay[j], src);
                const int32_t f = wave_shfl(first[j], src);
                const int32_t c = wave_shfl(cnt[j], src);
                const int64_t oo = wave_shfl(o, src);
                if (q < tot2) {
                    if (KIND == JOIN_OUTER && c == 0) e(oo, kk, pp, (RP)JOIN_NONE, esm);
                    else e(oo + t, kk, pp, right(f + t), esm);
                }
            }
            uint64_t heavy = ballot(lng);
            while (heavy) {
                const int src = __ffsll((unsigned long long)heavy) - 1;
                heavy &= heavy - 1;
                const int c = wave_read(cnt[j], src);
                const int64_t f = wave_read(first[j], src);
                const int64_t oo = wave_read(o, src);
                const uint32_t kk = wave_read(key[j], src);
                const LP pp = wave_read(pay[j], src);
                for (int q = l; q < c; q += WAVE) e(oo + q, kk, pp, right(f + q), esm);
            }
        }
    }
    __syncthreads();
}

// Tiles [t0, t1) of block b when ntiles tiles are split into contiguous
// ranges over the grid (the counting and expanding kernels split alike).
__device__ __forceinline__ void join_block_range(int64_t ntiles, int64_t& t0, int64_t& t1) {
    const int64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    t0 = (int64_t)blockIdx.x * per;
    t1 = t0 + per < ntiles ? t0 + per : ntiles;
    if (t0 > t1) t0 = t1;
}

// Per-tile output counts (first kernel of the two-kernel join): tile_cnt of
// every tile and blk_total of every block's contiguous range of tiles.
template <class Cfg, int KIND = JOIN_INNER>
__global__ void __launch_bounds__(Cfg::BLOCK)
k_join_count(const uint32_t* lkey, int64_t nl_upper, const int64_t* d_nl, const uint32_t* rkey,
             const int64_t* win, int64_t* tile_cnt, int64_t* blk_total, int lowb) {
    __shared__ JoinSmem<Cfg, uint8_t> sm;
    int64_t nl = nl_upper;
    if (d_nl) { const int64_t t = *d_nl; nl = t < nl ? t : nl; }
    const int64_t ntiles = (nl + Cfg::TILE - 1) / Cfg::TILE;
    int64_t t0, t1, sum = 0;
    join_block_range(ntiles, t0, t1);
    TileGeo g{};
    if (t0 < t1) g = tile_geo(lkey, nl, win, t0, Cfg::TILE);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const TileGeo cur = g;
        if (tile + 1 < t1) g = tile_geo(lkey, nl, win, tile + 1, Cfg::TILE);     // one tile ahead
        const int64_t t = join_tile_count<Cfg, uint8_t, KIND>(lkey, nl, rkey, cur, tile, sm, lowb);
        if (threadIdx.x == 0) tile_cnt[tile] = t;
        sum += t;
    }
    if (threadIdx.x == 0) blk_total[blockIdx.x] = sum;
}

// The join.  Emitters that write at output positions: each block expands its
// contiguous range of tiles, the first at the sum of the earlier blocks'
// totals and each next one after the previous tile's count; the last block
// stores the join size (also to d_count_out, if not null).  Aggregating
// emitters: tiles are pulled from a
// counter.  The kernel is persistent, so emitters can accumulate across tiles
// and flush once.
template <class Cfg, class LP, class RP, class Emit, int KIND = JOIN_INNER>
__global__ void __launch_bounds__(Cfg::BLOCK)
k_join(const uint32_t* lkey, const LP* lpay, int64_t nl_upper, const int64_t* d_nl,
       const uint32_t* rkey, const RP* rpay, const int64_t* win, uint32_t* tile_counter, const int64_t* tile_cnt,
       const int64_t* blk_total, int64_t* d_count, int64_t* d_count_out, int64_t cap, Emit emit, uint32_t* flags,
       int lowb) {
    __shared__ JoinSmem<Cfg, RP> sm;
    __shared__ typename Emit::Smem esm;
    int64_t nl = nl_upper;
    if (d_nl) { int64_t t = *d_nl; nl = t < nl ? t : nl; }
    const int64_t ntiles = (nl + Cfg::TILE - 1) / Cfg::TILE;
    Emit e = emit;
    e.init(esm);
    if constexpr (Emit::ORDERED) {
        if (threadIdx.x < WAVE) {
            int64_t acc = 0;
            for (int64_t b = threadIdx.x; b < blockIdx.x; b += WAVE) acc += blk_total[b];
            acc = wave_sum(acc);
            if (threadIdx.x == 0) sm.base = acc;
        }
        __syncthreads();
        int64_t run = sm.base;
        int64_t t0, t1;
        join_block_range(ntiles, t0, t1);
        for (int64_t tile = t0; tile < t1; ++tile) {
            const int64_t base = run;
            run += tile_cnt[tile];
            join_tile<Cfg, LP, RP, Emit, KIND>(lkey, lpay, nl, rkey, rpay, tile_geo(lkey, nl, win, tile, Cfg::TILE),
                                               tile, base, d_count, e, esm, sm, lowb);
        }
        if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
            *d_count = run;
            if (d_count_out) *d_count_out = run;
            if (run > cap) set_flag(flags, FLAG_CAPACITY);
        }
    } else {
        for (;;) {
            if (threadIdx.x == 0) sm.tile = atomicAdd(tile_counter, 1u);
            __syncthreads();
            const int64_t tile = sm.tile;
            if (tile >= ntiles) break;
            join_tile<Cfg, LP, RP, Emit, KIND>(lkey, lpay, nl, rkey, rpay, tile_geo(lkey, nl, win, tile, Cfg::TILE),
                                               tile, 0, d_count, e, esm, sm, lowb);
        }
    }
    e.finish(esm);
}

}  // namespace tqp
