// Band join: the non-equi join that Section 5.2 reaches with a small change
// to the sort-based join.  On key-sorted inputs the right rows matching left
// element i, |lkey[i] - rkey[j]| <= w, are one contiguous range
// [lower_bound(R, lkey[i] - w), upper_bound(R, lkey[i] + w)) of the right
// side, so the histogram product of Algorithm 1 becomes the length of that
// range and the expansion pairs output slot o with lo(i) + (o - offset(i)).
//
// Two kernels over the same contiguous tile ranges, as in the equi-join:
// count (per-tile and per-block totals of the range lengths), then expand.
// A tile stages the right keys its elements can reach in LDS when they fit
// and searches there; otherwise it searches the right keys in HBM.
#include "dev.hpp"
#include "host.hpp"

namespace tqp {
namespace {

constexpr int BJ_BLOCK = 256;
constexpr int BJ_ITEMS = 8;
constexpr int BJ_TILE = BJ_BLOCK * BJ_ITEMS;
constexpr int BJ_RWIN = 4096;          // right keys a tile may stage in LDS
constexpr int BJ_LANE_MAX = 4;         // longer ranges in an item: the wave writes the item's rows together
constexpr int BJ_WAVE_RUN = 32;        // ranges this long: one at a time, 64 consecutive rows per step

struct BandSmem {
    uint32_t rk[BJ_RWIN];
    int64_t wave[BJ_BLOCK / WAVE];
    int64_t base;
    int64_t wlo, whi;
};

__device__ __forceinline__ void bj_block_range(int64_t ntiles, int64_t& t0, int64_t& t1) {
    const int64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    t0 = (int64_t)blockIdx.x * per;
    t1 = t0 + per < ntiles ? t0 + per : ntiles;
    if (t0 > t1) t0 = t1;
}

// Bounds of key k's band, clamped to the key type: [k - w, k + w].
__device__ __forceinline__ uint32_t band_lo(uint32_t k, int64_t w) {
    const int64_t v = (int64_t)k - w;
    return v < 0 ? 0u : (uint32_t)v;
}
__device__ __forceinline__ uint32_t band_hi(uint32_t k, int64_t w) {
    const int64_t v = (int64_t)k + w;
    return v > 0x7FFFFFFF ? 0x7FFFFFFFu : (uint32_t)v;
}

// First position in keys[lo, hi) (LDS or HBM) whose key is >= v (or > v when upper).
template <class P>
__device__ __forceinline__ int64_t band_search(P keys, int64_t lo, int64_t hi, uint32_t v, bool upper) {
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        const uint32_t x = keys[mid];
        if (upper ? x <= v : x < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One tile: loads its keys, finds the right window of the whole tile, stages
// it in LDS when it fits, and returns each element's range [lo, lo + cnt)
// (absolute right positions).
__device__ __forceinline__ void band_tile(const uint32_t* lkey, int64_t nl, const uint32_t* rkey, int64_t nr,
                                          int64_t w, int64_t tile, uint32_t (&key)[BJ_ITEMS],
                                          bool (&in)[BJ_ITEMS], int64_t (&lo)[BJ_ITEMS],
                                          int32_t (&cnt)[BJ_ITEMS], BandSmem& sm) {
    const int tid = threadIdx.x, wv = tid / WAVE, l = lane_id();
    const int64_t t0 = tile * BJ_TILE;
    const int64_t tl = (t0 + BJ_TILE < nl ? t0 + BJ_TILE : nl) - 1;
    const int64_t chunk = t0 + (int64_t)wv * BJ_ITEMS * WAVE;
#pragma unroll
    for (int j = 0; j < BJ_ITEMS; ++j) {
        const int64_t i = chunk + j * WAVE + l;
        in[j] = i < nl;
        key[j] = lkey[in[j] ? i : nl - 1];                  // the tile exists, so nl >= 1
    }
    if (tid == 0) {
        sm.wlo = band_search(rkey, 0, nr, band_lo(lkey[t0], w), false);
        sm.whi = band_search(rkey, sm.wlo, nr, band_hi(lkey[tl], w), true);
    }
    __syncthreads();
    const int64_t wlo = sm.wlo, whi = sm.whi;
    const bool staged = whi - wlo <= BJ_RWIN;
    if (staged)
        for (int64_t r = tid; r < whi - wlo; r += BJ_BLOCK) sm.rk[r] = rkey[wlo + r];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < BJ_ITEMS; ++j) {
        int64_t a = 0, b = 0;
        if (in[j]) {
            // keys above the declared type or out of order only shrink the window; the searches stay in it
            if (staged) {
                a = wlo + band_search(sm.rk, 0, whi - wlo, band_lo(key[j], w), false);
                b = wlo + band_search(sm.rk, a - wlo, whi - wlo, band_hi(key[j], w), true);
            } else {
                a = band_search(rkey, wlo, whi, band_lo(key[j], w), false);
                b = band_search(rkey, a, whi, band_hi(key[j], w), true);
            }
        }
        lo[j] = a;
        cnt[j] = (int32_t)(b - a);
    }
    __syncthreads();                                        // the staged keys are read before the next tile
}

__global__ void __launch_bounds__(BJ_BLOCK)
k_band_count(const uint32_t* lkey, int64_t nl_upper, const int64_t* d_nl, const uint32_t* rkey, int64_t nr_upper,
             const int64_t* d_nr, int64_t w, int64_t* tile_cnt, int64_t* blk_total) {
    __shared__ BandSmem sm;
    int64_t nl = nl_upper, nr = nr_upper;
    if (d_nl) { const int64_t t = *d_nl; nl = t < nl ? t : nl; }
    if (d_nr) { const int64_t t = *d_nr; nr = t < nr ? t : nr; }
    const int64_t ntiles = (nl + BJ_TILE - 1) / BJ_TILE;
    int64_t t0, t1, sum = 0;
    bj_block_range(ntiles, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        uint32_t key[BJ_ITEMS];
        bool in[BJ_ITEMS];
        int64_t lo[BJ_ITEMS];
        int32_t cnt[BJ_ITEMS];
        band_tile(lkey, nl, rkey, nr, w, tile, key, in, lo, cnt, sm);
        int64_t c = 0;
#pragma unroll
        for (int j = 0; j < BJ_ITEMS; ++j) c += cnt[j];
        c = wave_sum(c);
        if (lane_id() == 0) sm.wave[threadIdx.x / WAVE] = c;
        __syncthreads();
        int64_t t = 0;
        for (int ww = 0; ww < BJ_BLOCK / WAVE; ++ww) t += sm.wave[ww];
        __syncthreads();
        if (threadIdx.x == 0) tile_cnt[tile] = t;
        sum += t;
    }
    if (threadIdx.x == 0) blk_total[blockIdx.x] = sum;
}

__global__ void __launch_bounds__(BJ_BLOCK)
k_band_expand(const uint32_t* lkey, const int32_t* lrow, int64_t nl_upper, const int64_t* d_nl, const uint32_t* rkey,
              const int32_t* rrow, int64_t nr_upper, const int64_t* d_nr, int64_t w, const int64_t* tile_cnt,
              const int64_t* blk_total, int32_t* out_l, int32_t* out_r, int64_t cap, int64_t* d_count,
              uint32_t* flags) {
    __shared__ BandSmem sm;
    const int tid = threadIdx.x, wv = tid / WAVE, l = lane_id();
    int64_t nl = nl_upper, nr = nr_upper;
    if (d_nl) { const int64_t t = *d_nl; nl = t < nl ? t : nl; }
    if (d_nr) { const int64_t t = *d_nr; nr = t < nr ? t : nr; }
    const int64_t ntiles = (nl + BJ_TILE - 1) / BJ_TILE;
    if (tid < WAVE) {
        int64_t acc = 0;
        for (int64_t b = tid; b < blockIdx.x; b += WAVE) acc += blk_total[b];
        acc = wave_sum(acc);
        if (tid == 0) sm.base = acc;
    }
    __syncthreads();
    int64_t run = sm.base;
    int64_t t0, t1;
    bj_block_range(ntiles, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        uint32_t key[BJ_ITEMS];
        bool in[BJ_ITEMS];
        int64_t lo[BJ_ITEMS];
        int32_t cnt[BJ_ITEMS];
        band_tile(lkey, nl, rkey, nr, w, tile, key, in, lo, cnt, sm);
        int64_t wt = 0;
#pragma unroll
        for (int j = 0; j < BJ_ITEMS; ++j) wt += wave_sum((int64_t)cnt[j]);
        if (l == 0) sm.wave[wv] = wt;
        __syncthreads();
        int64_t wbase = run;
        for (int ww = 0; ww < wv; ++ww) wbase += sm.wave[ww];
        run += tile_cnt[tile];
        __syncthreads();
        const int64_t chunk = tile * BJ_TILE + (int64_t)wv * BJ_ITEMS * WAVE;
#pragma unroll
        for (int j = 0; j < BJ_ITEMS; ++j) {
            const int64_t incl = wave_incl_sum((int64_t)cnt[j]);
            const int64_t o = wbase + incl - cnt[j];
            wbase += wave_read(incl, WAVE - 1);
            const int64_t i = chunk + j * WAVE + l;
            const int32_t lp = lrow ? lrow[in[j] ? i : 0] : (int32_t)i;
            if (!__any(cnt[j] > BJ_LANE_MAX)) {
                for (int t = 0; t < cnt[j]; ++t)
                    if (o + t < cap) {
                        out_l[o + t] = lp;
                        out_r[o + t] = rrow ? rrow[lo[j] + t] : (int32_t)(lo[j] + t);
                    }
            } else {
                // some range is wide.  Ranges of at least BJ_WAVE_RUN rows: the
                // whole wave writes each; the shorter ones: the wave writes
                // their rows 64 at a time, each lane finding the left element
                // its row belongs to
                const bool lng = cnt[j] >= BJ_WAVE_RUN;
                const int64_t oc2 = lng ? 0 : (int64_t)cnt[j];
                const int64_t incl2 = wave_incl_sum(oc2);
                const int64_t excl2 = incl2 - oc2, tot2 = wave_read(incl2, WAVE - 1);
                for (int64_t q0 = 0; q0 < tot2; q0 += WAVE) {
                    const int64_t q = q0 + l;
                    const int src = wave_run_owner(excl2, q);
                    const int64_t t = q - wave_shfl(excl2, src);
                    const int64_t f = wave_shfl(lo[j], src);
                    const int32_t pp = wave_shfl(lp, src);
                    const int64_t oo = wave_shfl(o, src) + t;
                    if (q < tot2 && oo < cap) {
                        out_l[oo] = pp;
                        out_r[oo] = rrow ? rrow[f + t] : (int32_t)(f + t);
                    }
                }
                uint64_t heavy = ballot(lng);
                while (heavy) {
                    const int src = __ffsll((unsigned long long)heavy) - 1;
                    heavy &= heavy - 1;
                    const int c = wave_read(cnt[j], src);
                    const int64_t f = wave_read(lo[j], src);
                    const int64_t oo = wave_read(o, src);
                    const int32_t pp = wave_read(lp, src);
                    for (int q = l; q < c; q += WAVE)
                        if (oo + q < cap) {
                            out_l[oo + q] = pp;
                            out_r[oo + q] = rrow ? rrow[f + q] : (int32_t)(f + q);
                        }
                }
            }
        }
    }
    if (blockIdx.x == gridDim.x - 1 && tid == 0) {
        *d_count = run;
        if (run > cap) set_flag(flags, FLAG_CAPACITY);
    }
}

}  // namespace
}  // namespace tqp

using namespace tqp;

extern "C" {

tqp_status tqp_join_band(tqp_ctx* ctx, const int32_t* lkey, const int32_t* lrow, int64_t nl, const int64_t* d_nl,
                         const int32_t* rkey, const int32_t* rrow, int64_t nr, const int64_t* d_nr, int64_t w,
                         int32_t* out_l, int32_t* out_r, int64_t cap, int64_t* d_count, void* ws, size_t* ws_bytes,
                         hipStream_t stream) {
    clear_error();
    if (!ctx || !d_count || nl < 0 || nr < 0 || cap < 0 || w < 0 || (nl > 0 && !lkey) || (nr > 0 && !rkey) ||
        (cap > 0 && (!out_l || !out_r)))
        return fail(TQP_ERR_INVALID, "tqp_join_band: null pointer or negative size or band");
    if (nl > MAX_ELEMS || nr > MAX_ELEMS) return fail(TQP_ERR_UNSUPPORTED, "tqp_join_band: input too large");
    const int64_t tiles = (nl + BJ_TILE - 1) / BJ_TILE;
    static const int per_cu = [] {
        int a = 4, b = 4;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_band_count, BJ_BLOCK, 0) != hipSuccess) a = 4;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_band_expand, BJ_BLOCK, 0) != hipSuccess) b = 4;
        const int c = a < b ? a : b;
        return c < 1 ? 1 : c;
    }();
    const int grid = grid_for(tiles, 1, (int64_t)ctx->num_cus * per_cu);
    int64_t *tile_cnt = nullptr, *blk_total = nullptr;
    Arena a;
    auto plan = [&](Arena& ar) {
        tile_cnt = ar.scratch<int64_t>(tiles > 0 ? tiles : 1);
        blk_total = ar.scratch<int64_t>(tiles > 0 ? tiles : 1);
    };
    tqp_status st = with_workspace(ctx, ws, ws_bytes, stream, plan, a);
    if (st != TQP_OK || !ws) return st;
    const uint32_t* lk = reinterpret_cast<const uint32_t*>(lkey);
    const uint32_t* rk = reinterpret_cast<const uint32_t*>(rkey);
    if (tiles == 0) {
        // no left rows: the join is empty
        TQP_LAUNCH(ctx, stream, "band_empty",
                   k_fill_u32<<<1, 64, 0, stream>>>(reinterpret_cast<uint32_t*>(d_count), 2, 0u));
        return TQP_OK;
    }
    TQP_LAUNCH(ctx, stream, "band_count",
               k_band_count<<<grid, BJ_BLOCK, 0, stream>>>(lk, nl, d_nl, rk, nr, d_nr, w, tile_cnt, blk_total));
    TQP_LAUNCH(ctx, stream, "band_expand",
               k_band_expand<<<grid, BJ_BLOCK, 0, stream>>>(lk, lrow, nl, d_nl, rk, rrow, nr, d_nr, w, tile_cnt,
                                                            blk_total, out_l, out_r, cap, d_count, ctx->d_err));
    return TQP_OK;
}

}  // extern "C"
