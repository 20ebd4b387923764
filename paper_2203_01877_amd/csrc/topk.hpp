// ORDER BY sum DESC, key ASC, first k rows (the sort operator of Section 5
// applied to the aggregated groups).
//
// Each level sorts chunks of CH candidates in LDS with a bitonic network and
// keeps the first k of each chunk, so a level shrinks the candidate set by
// CH / k; the last level has one chunk.  The order is total because group
// keys are unique, so every level's survivors are exactly the chunk's true
// first k.
//
// Before the levels, the first k rows of a sample of the groups give a
// threshold T (the sample's k-th row): a group ordered after T cannot be in
// the overall first k, since the sample already holds k rows ordered before
// it.  One streaming pass keeps the other groups, so the levels sort a few
// thousand candidates instead of every group.
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

// Number of candidates entering level `level` when level 0 gets n0: each level
// leaves k per chunk of CH, and at least one (possibly padded) chunk.
__device__ __forceinline__ int64_t topk_level_n(int64_t n0, int level, int CH, int k) {
    int64_t n = n0;
    for (int l = 0; l < level; ++l) {
        int64_t b = (n + CH - 1) / CH;
        n = (b < 1 ? 1 : b) * k;
    }
    return n;
}

// One level.  Level 0 reads the groups themselves (cin == null: gkey / gsum)
// or the filtered candidates; level l > 0 reads the previous level's output.
// The level-0 count is min(*d_n0, n_upper) (n_upper when d_n0 is null) and
// later counts follow from it.  Block 0 always writes its k rows (padding
// included), so every level leaves at least one valid chunk.
template <int BLOCK, int CH>
__global__ void __launch_bounds__(BLOCK)
k_topk_level(const int32_t* gkey, const int64_t* gsum, int64_t n_upper, const int64_t* d_n0,
             const TopCand* cin, TopCand* cout, int k, int level) {
    __shared__ TopCand c[CH];
    int64_t n0 = n_upper;
    if (d_n0) { const int64_t t = *d_n0; n0 = t < n0 ? t : n0; }
    const int64_t n = topk_level_n(n0, level, CH, k);
    // A level after the first single-chunk level receives that chunk's k
    // sorted rows: nothing left to do but pass them on.
    if (level > 0 && topk_level_n(n0, level - 1, CH, k) <= CH) {
        if (blockIdx.x == 0)
            for (int i = threadIdx.x; i < k; i += BLOCK) cout[i] = cin[i];
        return;
    }
    const int64_t c0 = (int64_t)blockIdx.x * CH;
    if (c0 >= n && blockIdx.x != 0) return;
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
    // Bitonic sort into "before" order, one compare-exchange per thread and
    // stage.  Pairs at a stride below 128 lie in the 128 slots of one wave, so
    // only the wider strides need a block barrier.
    static_assert(BLOCK * 2 == CH, "one compare-exchange per thread");
    const int t = threadIdx.x;
    for (int size = 2; size <= CH; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int lo = 2 * t - (t & (stride - 1));
            const int hi = lo + stride;
            const bool asc = ((lo & size) == 0);
            const TopCand a = c[lo], b = c[hi];
            if (asc ? top_before(b, a) : top_before(a, b)) { c[lo] = b; c[hi] = a; }
            if (stride >= 2 * WAVE || stride == 1) __syncthreads();
            else __builtin_amdgcn_wave_barrier();
        }
    }
    for (int i = threadIdx.x; i < k; i += BLOCK) cout[(int64_t)blockIdx.x * k + i] = c[i];
}

// Keeps the groups not ordered after the threshold thr[k-1] (all groups when
// the sample had fewer than k).  Order of the kept candidates is irrelevant.
__global__ void k_topk_filter(const int32_t* gkey, const int64_t* gsum, int64_t n_upper, const int64_t* d_n,
                              const TopCand* thr, int k, TopCand* out, int64_t* d_out);

// Final rows: key, sum, count of the first min(k, G) candidates.
__global__ void k_topk_emit(const TopCand* c, int k, const int64_t* gcnt, int32_t* out_key,
                            int64_t* out_sum, int64_t* out_cnt, int32_t* d_k);

}  // namespace tqp
