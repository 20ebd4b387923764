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

template <class Cfg, class LP>
struct JoinSmem {
    static_assert(Cfg::WAVES >= 2, "the two window searches run on waves 0 and 1");
    uint32_t lkey[Cfg::TILE];
    LP lpay[Cfg::TILE];
    int64_t off[Cfg::TILE + 1];
    int32_t lb[Cfg::TILE];
    uint32_t rkey[Cfg::RWIN];
    int64_t scratch[Cfg::WAVES];
    int64_t win_lo, win_hi, tile_base;
    uint32_t tile;
};

// ------------------------------------------------------------------ emitters
// Index pairs (late materialisation: the join returns row-index pairs).
struct EmitPairs {
    int32_t* out_l;
    int32_t* out_r;
    int64_t cap;
    struct Smem {};
    __device__ void init(Smem&) {}
    __device__ void operator()(int64_t o, uint32_t, uint32_t lp, uint32_t rp, Smem&) {
        if (o < cap) {
            out_l[o] = (int32_t)lp;
            out_r[o] = (int32_t)rp;
        }
    }
    __device__ void finish(Smem&) {}
};

// (group key from the right side, 64-bit value from the left side), with the
// digit histograms of the following group-key sort accumulated on the way.
template <int BLOCK, int RB>
struct EmitKeyVal {
    static constexpr int R = 1 << RB;
    static constexpr int NP = (32 + RB - 1) / RB;
    uint32_t* out_key;
    uint64_t* out_val;
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
            out_key[o] = rp;
            out_val[o] = lp;
            if (rp & ~key_mask) set_flag(flags, FLAG_KEY_RANGE);
            if (hist)
                for (int p = 0; p < npass; ++p)
                    atomicAdd(&s.h[p * R + ((rp >> shift[p]) & ((1u << bits[p]) - 1))], 1u);
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
// flagA * 2 + flagB in registers; flush once per block.
template <int BLOCK>
struct EmitFlagsAgg {
    static constexpr int G = 8;
    const int64_t* price;
    const int64_t* disc;
    const int8_t* flagA;
    const int8_t* flagB;
    int64_t* acc;              // [G][3] global: sum, count, sum(price)
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
        const int g = flagA[lp] * 2 + flagB[lp];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const bool on = (g == k);
            s[k] += on ? v : 0;
            c[k] += on ? 1 : 0;
            p[k] += on ? pr : 0;
        }
    }
    __device__ void finish(Smem& sm) {
        const int w = threadIdx.x / WAVE;
#pragma unroll
        for (int k = 0; k < G; ++k) {
            int64_t a = wave_sum(s[k]), b = wave_sum(c[k]), d = wave_sum(p[k]);
            if (lane_id() == 0) { sm.a[w][k * 3] = a; sm.a[w][k * 3 + 1] = b; sm.a[w][k * 3 + 2] = d; }
        }
        __syncthreads();
        if (threadIdx.x < G * 3) {
            int64_t t = 0;
            for (int ww = 0; ww < BLOCK / WAVE; ++ww) t += sm.a[ww][threadIdx.x];
            if (t) atomic_add(&acc[threadIdx.x], t);
        }
    }
};

// ------------------------------------------------------------------ kernel
template <class Cfg, class LP, class RP, class Emit>
__global__ void __launch_bounds__(Cfg::BLOCK)
k_join(const uint32_t* lkey, const LP* lpay, int64_t nl_upper, const int64_t* d_nl,
       const uint32_t* rkey, const RP* rpay, int64_t nr_upper, const int64_t* d_nr,
       uint64_t* status, uint32_t* tile_counter, int64_t* d_count, int64_t cap, Emit emit,
       uint32_t* flags) {
    constexpr int TILE = Cfg::TILE, ITEMS = Cfg::ITEMS, BLOCK = Cfg::BLOCK, RWIN = Cfg::RWIN;
    __shared__ JoinSmem<Cfg, LP> sm;
    __shared__ typename Emit::Smem esm;
    const int tid = threadIdx.x, w = tid / WAVE;

    int64_t nl = nl_upper, nr = nr_upper;
    if (d_nl) { int64_t t = *d_nl; nl = t < nl ? t : nl; }
    if (d_nr) { int64_t t = *d_nr; nr = t < nr ? t : nr; }
    const int64_t ntiles = (nl + TILE - 1) / TILE;
    Emit e = emit;
    e.init(esm);
    if (ntiles == 0 && blockIdx.x == 0 && tid == 0) *d_count = 0;

    for (;;) {
        if (tid == 0) sm.tile = atomicAdd(tile_counter, 1u);
        __syncthreads();
        const int64_t tile = sm.tile;
        if (tile >= ntiles) break;
        const int64_t t0 = tile * TILE;
        const int tn = (int)((nl - t0) < TILE ? (nl - t0) : TILE);

        for (int i = tid; i < tn; i += BLOCK) {
            sm.lkey[i] = lkey[t0 + i];
            sm.lpay[i] = lpay ? lpay[t0 + i] : (LP)(t0 + i);
        }
        __syncthreads();
        // R window of the tile's key range.
        if (w == 0) {
            int64_t lo = wave_bound(rkey, nr, sm.lkey[0], false);
            if (lane_id() == 0) sm.win_lo = lo;
        } else if (w == 1) {
            int64_t hi = wave_bound(rkey, nr, sm.lkey[tn - 1], true);
            if (lane_id() == 0) sm.win_hi = hi;
        }
        __syncthreads();
        const int64_t wlo = sm.win_lo, whi = sm.win_hi;
        const int64_t wn = whi - wlo;
        const bool in_lds = wn <= RWIN;
        if (in_lds)
            for (int i = tid; i < wn; i += BLOCK) sm.rkey[i] = rkey[wlo + i];
        __syncthreads();

        // Per left element: first match and match count (blocked layout).
        int64_t tsum = 0;
        int64_t cnt[ITEMS];
        int32_t first[ITEMS];
        uint32_t prev_key = 0;
        int64_t prev_lb = -1, prev_cnt = 0;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int i = tid * ITEMS + j;
            cnt[j] = 0;
            first[j] = 0;
            if (i < tn) {
                const uint32_t k = sm.lkey[i];
                if (prev_lb >= 0 && k == prev_key) {
                    first[j] = (int32_t)prev_lb;
                    cnt[j] = prev_cnt;
                } else {
                    int64_t lb, ub;
                    if (in_lds) {
                        lb = wlo + lower_bound_lds(sm.rkey, (int)wn, k);
                        ub = wlo + upper_bound_lds(sm.rkey, (int)wn, k);
                    } else {
                        lb = lower_bound_glb(rkey, wlo, whi, k);
                        ub = upper_bound_glb(rkey, lb, whi, k);
                    }
                    first[j] = (int32_t)lb;
                    cnt[j] = ub - lb;
                    prev_key = k;
                    prev_lb = lb;
                    prev_cnt = cnt[j];
                }
                tsum += cnt[j];
            }
        }
        int64_t ttot;
        int64_t toff = block_excl_sum<BLOCK>(tsum, sm.scratch, &ttot);
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int i = tid * ITEMS + j;
            if (i < tn) {
                sm.off[i] = toff;
                sm.lb[i] = first[j];
                toff += cnt[j];
            }
        }
        if (tid == 0) {
            const int64_t base = lookback64(status, tile, ttot, flags);
            sm.tile_base = base;
            if (tile == ntiles - 1) {
                *d_count = base + ttot;
                if (base + ttot > cap) set_flag(flags, FLAG_CAPACITY);
            }
        }
        __syncthreads();
        const int64_t base = sm.tile_base;
        // Expansion: output slot q of the tile -> (left element, right element).
        for (int64_t q = tid; q < ttot; q += BLOCK) {
            int lo = 0, hi = tn;      // last i with off[i] <= q
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (sm.off[mid] <= q) lo = mid; else hi = mid;
            }
            const int64_t r = (int64_t)sm.lb[lo] + (q - sm.off[lo]);
            e(base + q, sm.lkey[lo], sm.lpay[lo], rpay ? rpay[r] : (RP)r, esm);
        }
        __syncthreads();
    }
    e.finish(esm);
}

}  // namespace tqp
