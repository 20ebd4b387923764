// Filter (Section 3.1): a conjunction of column-versus-constant comparisons
// evaluated per row, then stream compaction into a selection vector of row ids
// (the index form of the bitmap filter), with an optional carried column.
//
// Per tile: one ballot per 64 rows gives the wave's survivors and each lane's
// rank among them; a block scan and a decoupled look-back give the tile's
// output base.  The row count stays on the device (and the input's may come
// from the device: d_n).
#pragma once
#include "dev.hpp"
#include "radix.hpp"

namespace tqp {

constexpr int FILTER_MAX_PREDS = 4;

struct FilterPreds {
    const void* col[FILTER_MAX_PREDS];
    int32_t type[FILTER_MAX_PREDS];    // 1 = int8, 2 = int32, 3 = int64
    int32_t op[FILTER_MAX_PREDS];
    int64_t k[FILTER_MAX_PREDS];
    int32_t np;
    // ok[j] for rows idx[j] (already clamped into range): per predicate, the
    // column type is decided once and all the rows' values are loaded before
    // any is compared, so they are in flight together.
    template <int ITEMS>
    __device__ void eval(const int64_t (&idx)[ITEMS], bool (&ok)[ITEMS]) const {
        for (int p = 0; p < np; ++p) {
            int64_t x[ITEMS];
            if (type[p] == 1) {
                const int8_t* c = (const int8_t*)col[p];
#pragma unroll
                for (int j = 0; j < ITEMS; ++j) x[j] = c[idx[j]];
            } else if (type[p] == 2) {
                const int32_t* c = (const int32_t*)col[p];
#pragma unroll
                for (int j = 0; j < ITEMS; ++j) x[j] = c[idx[j]];
            } else {
                const int64_t* c = (const int64_t*)col[p];
#pragma unroll
                for (int j = 0; j < ITEMS; ++j) x[j] = c[idx[j]];
            }
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) ok[j] = ok[j] & cmp_eval(x[j], op[p], k[p]);
        }
    }
};

template <int BLOCK, int ITEMS>
__global__ void __launch_bounds__(BLOCK)
k_filter(FilterPreds fp, int64_t n, const int32_t* carry, int32_t* out_row, int32_t* out_carry,
         int64_t cap, int64_t* d_count, uint64_t* status, uint32_t* tile_counter, uint32_t* flags,
         const int64_t* d_n = nullptr) {
    constexpr int TILE = BLOCK * ITEMS, W = BLOCK / WAVE;
    __shared__ int64_t s_wave[W];
    __shared__ int64_t s_base;
    __shared__ uint32_t s_tile;
    const int tid = threadIdx.x, w = tid / WAVE, l = lane_id();
    if (d_n) {                                 // rows counted on the device, at most n
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
    uint64_t m[ITEMS];
    int64_t wc = 0;
    int64_t idx[ITEMS];
    bool ok[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = chunk + j * WAVE + l;
        ok[j] = i < n;
        idx[j] = ok[j] ? i : n - 1;       // n >= 1: the tile exists
    }
    fp.eval<ITEMS>(idx, ok);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        m[j] = ballot(ok[j]);
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
        const int64_t i = chunk + j * WAVE + l;
        if ((m[j] >> l) & 1) {
            const int64_t o = pos + popc64(m[j] & lanemask_lt());
            if (o < cap) {
                out_row[o] = (int32_t)i;
                if (out_carry) out_carry[o] = carry[i];
            }
        }
        pos += popc64(m[j]);
    }
}

}  // namespace tqp
