// ORDER BY sum DESC, key ASC, first k rows (the sort operator of Section 5
// applied to the aggregated groups).
//
// Each level sorts chunks of CH candidates in LDS with a bitonic network and
// keeps the first k of each chunk, so a level shrinks the candidate set by
// CH / k; the last level has one chunk.  The order is total because group
// keys are unique, so every level's survivors are exactly the chunk's true
// first k.
#pragma once
#include "dev.hpp"

namespace tqp {

struct TopCand {
    int64_t sum;
    int32_t key;
    int32_t idx;               // group index, -1 for padding
};

__device__ __forceinline__ bool top_before(const TopCand& a, const TopCand& b) {
    if (a.idx < 0) return false;
    if (b.idx < 0) return true;
    if (a.sum != b.sum) return a.sum > b.sum;
    return a.key < b.key;
}

template <int BLOCK, int CH>
__global__ void __launch_bounds__(BLOCK)
k_topk_level(const int32_t* gkey, const int64_t* gsum, int64_t n_upper, const int64_t* d_n,
             const TopCand* cin, TopCand* cout, int k) {
    __shared__ TopCand c[CH];
    int64_t n = n_upper;
    if (d_n) { int64_t t = *d_n; n = t < n ? t : n; }
    const int64_t c0 = (int64_t)blockIdx.x * CH;
    for (int i = threadIdx.x; i < CH; i += BLOCK) {
        const int64_t g = c0 + i;
        TopCand x;
        x.sum = 0; x.key = 0; x.idx = -1;
        if (g < n) {
            if (cin) x = cin[g];
            else { x.sum = gsum[g]; x.key = gkey[g]; x.idx = (int32_t)g; }
        }
        c[i] = x;
    }
    __syncthreads();
    // bitonic sort into "before" order
    for (int size = 2; size <= CH; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < CH / 2; t += BLOCK) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool asc = ((lo & size) == 0);
                TopCand a = c[lo], b = c[hi];
                const bool swap = asc ? top_before(b, a) : top_before(a, b);
                if (swap) { c[lo] = b; c[hi] = a; }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < k; i += BLOCK) cout[(int64_t)blockIdx.x * k + i] = c[i];
}

// Final rows: key, sum, count of the first min(k, G) candidates.
__global__ void k_topk_emit(const TopCand* c, int k, const int64_t* gcnt, int32_t* out_key,
                            int64_t* out_sum, int64_t* out_cnt, int32_t* d_k);

}  // namespace tqp
