// Hash-based equi-join (Section 5.3, Algorithm 3), the variant of the join
// the paper measures against the sort-based one.
//
// The paper builds a table of m slots indexed by a hash of the key from one
// side, probes it with the other, and repeats build and probe as many times
// as the most crowded slot holds rows, because a PyTorch scatter keeps one
// row per slot.  On the GPU a slot conflict can be resolved in the table
// itself (open addressing, linear probing), so one build and one probe
// suffice:
//
//   build   every right row claims the first free slot at or after the home
//           slot of its key with a 64-bit compare-and-swap of (row + 1, key);
//   count   every left element scans from its key's home slot to the first
//           free slot and counts the entries with an equal key (the per-tile
//           and per-block totals give the output offsets, as in the
//           sort-based join);
//   expand  the same scan again, writing (lrow, rrow) at the element's offset.
//
// m is the power of two at or above 2 * nr (at most half full, so every scan
// ends), the home slot a multiplicative (Fibonacci) hash of the key: the
// paper's key mod m would pile the duplicates of consecutive keys into one
// run of slots.  Inputs need not be sorted.  Output rows follow the left
// input order; the rows of one left element follow the table, i.e. no fixed
// right order.
#include "dev.hpp"
#include "host.hpp"

namespace tqp {
namespace {

constexpr int HJ_BLOCK = 256;
constexpr int HJ_ITEMS = 8;
constexpr int HJ_TILE = HJ_BLOCK * HJ_ITEMS;
constexpr int HJ_REG = 2;          // matches per element kept in registers between count and write

__device__ __forceinline__ uint32_t hj_home(uint32_t key, int log2m) {
    return log2m ? (uint32_t)(((uint64_t)key * 0x9E3779B97F4A7C15ull) >> (64 - log2m)) : 0u;
}

__global__ void __launch_bounds__(256)
k_hash_build(const uint32_t* rkey, int64_t nr_upper, const int64_t* d_nr, unsigned long long* table,
             int log2m) {
    int64_t nr = nr_upper;
    if (d_nr) { const int64_t t = *d_nr; nr = t < nr ? t : nr; }
    const uint32_t mask = (uint32_t)((uint64_t(1) << log2m) - 1);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nr; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = rkey[i];
        const unsigned long long e = ((unsigned long long)(i + 1) << 32) | k;
        uint32_t s = hj_home(k, log2m);
        // the table is at most half full: a free slot is always reached
        while (atomicCAS(&table[s], 0ull, e) != 0ull) s = (s + 1) & mask;
    }
}

// Scans the runs of a thread's ITEMS elements in lockstep (one round of slot
// loads per step, issued together); visit(j, row) sees every entry whose key
// equals the element's.
template <class Visit>
__device__ __forceinline__ void hash_walk(const uint32_t (&key)[HJ_ITEMS], const bool (&in)[HJ_ITEMS],
                                          const unsigned long long* table, int log2m, Visit visit) {
    const uint32_t mask = (uint32_t)((uint64_t(1) << log2m) - 1);
    uint32_t s[HJ_ITEMS];
    bool live[HJ_ITEMS];
#pragma unroll
    for (int j = 0; j < HJ_ITEMS; ++j) {
        s[j] = hj_home(key[j], log2m);
        live[j] = in[j];
    }
    for (;;) {
        bool any = false;
#pragma unroll
        for (int j = 0; j < HJ_ITEMS; ++j) any |= live[j];
        if (!any) break;
        unsigned long long e[HJ_ITEMS];
#pragma unroll
        for (int j = 0; j < HJ_ITEMS; ++j) e[j] = table[s[j]];
#pragma unroll
        for (int j = 0; j < HJ_ITEMS; ++j) {
            if (live[j]) {
                if (e[j] == 0ull) {
                    live[j] = false;
                } else {
                    if ((uint32_t)e[j] == key[j]) visit(j, (uint32_t)(e[j] >> 32) - 1u);
                    s[j] = (s[j] + 1) & mask;
                }
            }
        }
    }
}

__device__ __forceinline__ void hj_block_range(int64_t ntiles, int64_t& t0, int64_t& t1) {
    const int64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    t0 = (int64_t)blockIdx.x * per;
    t1 = t0 + per < ntiles ? t0 + per : ntiles;
    if (t0 > t1) t0 = t1;
}

__device__ __forceinline__ void hj_load(const uint32_t* lkey, int64_t nl, int64_t tile, uint32_t (&key)[HJ_ITEMS],
                                        bool (&in)[HJ_ITEMS]) {
    const int w = threadIdx.x / WAVE, l = lane_id();
    const int64_t chunk = tile * HJ_TILE + (int64_t)w * HJ_ITEMS * WAVE;
#pragma unroll
    for (int j = 0; j < HJ_ITEMS; ++j) {
        const int64_t i = chunk + j * WAVE + l;
        in[j] = i < nl;
        key[j] = lkey[in[j] ? i : nl - 1];                  // the tile exists, so nl >= 1
    }
}

__global__ void __launch_bounds__(HJ_BLOCK)
k_hash_count(const uint32_t* lkey, int64_t nl_upper, const int64_t* d_nl, const unsigned long long* table, int log2m,
             int64_t* tile_cnt, int64_t* blk_total) {
    __shared__ int64_t s_wave[HJ_BLOCK / WAVE];
    int64_t nl = nl_upper;
    if (d_nl) { const int64_t t = *d_nl; nl = t < nl ? t : nl; }
    const int64_t ntiles = (nl + HJ_TILE - 1) / HJ_TILE;
    int64_t t0, t1, sum = 0;
    hj_block_range(ntiles, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        uint32_t key[HJ_ITEMS];
        bool in[HJ_ITEMS];
        hj_load(lkey, nl, tile, key, in);
        int64_t c = 0;
        hash_walk(key, in, table, log2m, [&](int, uint32_t) { ++c; });
        c = wave_sum(c);
        if (lane_id() == 0) s_wave[threadIdx.x / WAVE] = c;
        __syncthreads();
        int64_t t = 0;
        for (int w = 0; w < HJ_BLOCK / WAVE; ++w) t += s_wave[w];
        __syncthreads();
        if (threadIdx.x == 0) tile_cnt[tile] = t;
        sum += t;
    }
    if (threadIdx.x == 0) blk_total[blockIdx.x] = sum;
}

__global__ void __launch_bounds__(HJ_BLOCK)
k_hash_expand(const uint32_t* lkey, const int32_t* lrow, int64_t nl_upper, const int64_t* d_nl,
              const int32_t* rrow, const unsigned long long* table, int log2m, const int64_t* tile_cnt,
              const int64_t* blk_total, int32_t* out_l, int32_t* out_r, int64_t cap, int64_t* d_count,
              uint32_t* flags) {
    __shared__ int64_t s_wave[HJ_BLOCK / WAVE];
    __shared__ int64_t s_base;
    const int tid = threadIdx.x, w = tid / WAVE, l = lane_id();
    int64_t nl = nl_upper;
    if (d_nl) { const int64_t t = *d_nl; nl = t < nl ? t : nl; }
    const int64_t ntiles = (nl + HJ_TILE - 1) / HJ_TILE;
    if (tid < WAVE) {
        int64_t acc = 0;
        for (int64_t b = tid; b < blockIdx.x; b += WAVE) acc += blk_total[b];
        acc = wave_sum(acc);
        if (tid == 0) s_base = acc;
    }
    __syncthreads();
    int64_t run = s_base;
    int64_t t0, t1;
    hj_block_range(ntiles, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        uint32_t key[HJ_ITEMS];
        bool in[HJ_ITEMS];
        hj_load(lkey, nl, tile, key, in);
        // first walk: counts, and the first HJ_REG matches of each element
        int32_t cnt[HJ_ITEMS];
        uint32_t m[HJ_ITEMS][HJ_REG];
#pragma unroll
        for (int j = 0; j < HJ_ITEMS; ++j) cnt[j] = 0;
        hash_walk(key, in, table, log2m, [&](int j, uint32_t node) {
#pragma unroll
            for (int q = 0; q < HJ_REG; ++q)
                if (cnt[j] == q) m[j][q] = node;
            ++cnt[j];
        });
        // offsets: wave scans over the elements in order, then the waves before
        int64_t wt = 0;
#pragma unroll
        for (int j = 0; j < HJ_ITEMS; ++j) wt += wave_sum((int64_t)cnt[j]);
        if (l == 0) s_wave[w] = wt;
        __syncthreads();
        int64_t wbase = run;
        for (int ww = 0; ww < w; ++ww) wbase += s_wave[ww];
        run += tile_cnt[tile];
        __syncthreads();
        const int64_t chunk = tile * HJ_TILE + (int64_t)w * HJ_ITEMS * WAVE;
        bool more = false;
        int64_t o0[HJ_ITEMS];
#pragma unroll
        for (int j = 0; j < HJ_ITEMS; ++j) {
            const int64_t incl = wave_incl_sum((int64_t)cnt[j]);
            const int64_t o = wbase + incl - cnt[j];
            wbase += wave_read(incl, WAVE - 1);
            o0[j] = o;
            const int64_t i = chunk + j * WAVE + l;
            const int32_t lp = lrow ? lrow[in[j] ? i : 0] : (int32_t)i;
#pragma unroll
            for (int q = 0; q < HJ_REG; ++q) {
                if (q < cnt[j] && o + q < cap) {
                    out_l[o + q] = lp;
                    out_r[o + q] = rrow ? rrow[m[j][q]] : (int32_t)m[j][q];
                }
            }
            more |= cnt[j] > HJ_REG;
        }
        // elements with more matches: a second walk writes the rest
        if (__any(more)) {
            int32_t seen[HJ_ITEMS];
#pragma unroll
            for (int j = 0; j < HJ_ITEMS; ++j) seen[j] = 0;
            hash_walk(key, in, table, log2m, [&](int j, uint32_t node) {
                const int32_t q = seen[j]++;
                if (q >= HJ_REG && o0[j] + q < cap) {
                    const int64_t i = chunk + j * WAVE + l;
                    out_l[o0[j] + q] = lrow ? lrow[i] : (int32_t)i;
                    out_r[o0[j] + q] = rrow ? rrow[node] : (int32_t)node;
                }
            });
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

tqp_status tqp_hash_join(tqp_ctx* ctx, const int32_t* lkey, const int32_t* lrow, int64_t nl, const int64_t* d_nl,
                         const int32_t* rkey, const int32_t* rrow, int64_t nr, const int64_t* d_nr, int32_t* out_l,
                         int32_t* out_r, int64_t cap, int64_t* d_count, void* ws, size_t* ws_bytes,
                         hipStream_t stream) {
    clear_error();
    if (!ctx || !d_count || nl < 0 || nr < 0 || cap < 0 || (nl > 0 && !lkey) || (nr > 0 && !rkey) ||
        (cap > 0 && (!out_l || !out_r)))
        return fail(TQP_ERR_INVALID, "tqp_hash_join: null pointer or negative size");
    if (nl > MAX_ELEMS || nr > MAX_ELEMS) return fail(TQP_ERR_UNSUPPORTED, "tqp_hash_join: input too large");
    int log2m = 0;
    while ((int64_t(1) << log2m) < 2 * nr) ++log2m;
    const int64_t m = int64_t(1) << log2m;
    const int64_t tiles = (nl + HJ_TILE - 1) / HJ_TILE;
    static const int per_cu = [] {
        int a = 4, b = 4;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_hash_count, HJ_BLOCK, 0) != hipSuccess) a = 4;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_hash_expand, HJ_BLOCK, 0) != hipSuccess) b = 4;
        const int c = a < b ? a : b;
        return c < 1 ? 1 : c;
    }();
    const int grid = grid_for(tiles, 1, (int64_t)ctx->num_cus * per_cu);
    unsigned long long* table = nullptr;
    int64_t *tile_cnt = nullptr, *blk_total = nullptr;
    Arena a;
    auto plan = [&](Arena& ar) {
        table = ar.zero<unsigned long long>(m);
        tile_cnt = ar.scratch<int64_t>(tiles > 0 ? tiles : 1);
        blk_total = ar.scratch<int64_t>(tiles > 0 ? tiles : 1);
    };
    tqp_status st = with_workspace(ctx, ws, ws_bytes, stream, plan, a);
    if (st != TQP_OK || !ws) return st;
    if ((st = fill_zero(a.base, a.zsize, stream, ctx)) != TQP_OK) return st;
    const uint32_t* rk = reinterpret_cast<const uint32_t*>(rkey);
    const uint32_t* lk = reinterpret_cast<const uint32_t*>(lkey);
    if (nr > 0) {
        TQP_LAUNCH(ctx, stream, "hash_build",
                   k_hash_build<<<grid_for(nr, 256 * 4, (int64_t)ctx->num_cus * 8), 256, 0, stream>>>(
                       rk, nr, d_nr, table, log2m));
    }
    if (tiles == 0) {
        // no left rows: the join is empty
        TQP_LAUNCH(ctx, stream, "hash_empty", k_fill_u32<<<1, 64, 0, stream>>>(
                                                  reinterpret_cast<uint32_t*>(d_count), 2, 0u));
        return TQP_OK;
    }
    TQP_LAUNCH(ctx, stream, "hash_count",
               k_hash_count<<<grid, HJ_BLOCK, 0, stream>>>(lk, nl, d_nl, table, log2m, tile_cnt, blk_total));
    TQP_LAUNCH(ctx, stream, "hash_expand",
               k_hash_expand<<<grid, HJ_BLOCK, 0, stream>>>(lk, lrow, nl, d_nl, rrow, table, log2m, tile_cnt,
                                                            blk_total, out_l, out_r, cap, d_count, ctx->d_err));
    return TQP_OK;
}

}  // extern "C"
