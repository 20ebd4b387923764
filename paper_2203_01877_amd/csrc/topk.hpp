// ORDER BY sum DESC, key ASC, first k rows (the sort operator of Section 5
// applied to the aggregated groups).
//
// 1. Threshold.  One block finds, by radix select, the exact k-th largest sum
//    T of a sample of the groups (runs spread evenly over them).  The sample
//    holds k groups whose sum is at least T, so no group with a smaller sum
//    can be among the overall first k.
// 2. Filter.  One streaming pass keeps the groups with sum >= T.
//    (Steps 1-2 alternative, in the custkey fragment: each group-by bucket
//    block appends its own first k groups, a superset of the overall first
//    k, as it writes them; see k_bucket_agg.)
// 3. Chunk levels (only when many groups survive).  Each level keeps the
//    first k of each chunk of CH candidates (radix select in one block); a
//    level runs only while its input exceeds TOPK_DIRECT.
// 4. Final.  One block selects the exact k-th remaining candidate by radix
//    select on (sum, key), gathers the k candidates not after it and sorts
//    them.
//
// The order is total because group keys are unique, so each step keeps
// exactly the true first k of what it sees.
#pragma once
#include "dev.hpp"

namespace tqp {

struct TopCand {
    int64_t sum;
    int32_t key;
    int32_t idx;               // group index, -1 for padding
};

constexpr int TOPK_CH = 2048;          // candidates per LDS chunk
constexpr int TOPK_BLOCK = 1024;       // one compare-exchange per thread and stage
constexpr int TOPK_SAMPLE_PER = 32;    // sample rows per thread of the threshold block
constexpr int64_t TOPK_DIRECT = 16384; // largest candidate count the final block takes directly
constexpr int TOPK_MAX_LEVELS = 32;
constexpr int TOPK_K_MAX = 1024;       // largest k
constexpr int TOPK_FINAL_PER = 16;     // candidates per thread of the final block

// Outputs of the chunk levels (kernel argument by value).
struct TopkLevels {
    TopCand* out[TOPK_MAX_LEVELS];
};

__device__ __forceinline__ bool top_before(const TopCand& a, const TopCand& b) {
    if (a.idx < 0) return false;
    if (b.idx < 0) return true;
    if (a.sum != b.sum) return a.sum > b.sum;
    return a.key < b.key;
}

// Candidates entering level `level` when the filter kept n0: each level
// leaves k per chunk of CH.
__device__ __forceinline__ int64_t topk_level_n(int64_t n0, int level, int k) {
    int64_t n = n0;
    for (int l = 0; l < level; ++l) n = (n + TOPK_CH - 1) / TOPK_CH * k;
    return n;
}

// Radix select in one block over up to BLOCK * PER candidates held in
// registers.  A candidate's order key is the unsigned image of its sum
// (sign bit flipped, so unsigned order = signed order), followed, when LO,
// by the complement of its group key (a smaller key sorts first on equal
// sums).  Returns in (t_hi, t_lo) the need-th largest order key.  Digits are
// bytes, from the top; bytes shared by the largest and smallest hi are fixed
// up front, and a wave whose matching lanes all hold the same byte counts
// them with one LDS atomic.
template <int BLOCK, int PER, bool LO>
struct BlockSelect {
    uint32_t h[256];
    uint64_t wmax[BLOCK / WAVE], wmin[BLOCK / WAVE];
    uint32_t wlo[BLOCK / WAVE];
    uint64_t prefix_hi;
    uint32_t prefix_lo;
    uint32_t need;
    uint32_t whole;            // the chosen byte's candidates are all selected
};

template <int BLOCK, int PER, bool LO>
__device__ __forceinline__ void block_select(BlockSelect<BLOCK, PER, LO>& sm, const uint64_t (&hi)[PER],
                                             const uint32_t (&lo)[PER], const bool (&valid)[PER], int need,
                                             uint64_t& t_hi, uint32_t& t_lo) {
    const int tid = threadIdx.x, w = tid / WAVE, l = lane_id();
    uint64_t mx = 0, mn = ~uint64_t(0);
#pragma unroll
    for (int j = 0; j < PER; ++j)
        if (valid[j]) { mx = hi[j] > mx ? hi[j] : mx; mn = hi[j] < mn ? hi[j] : mn; }
    mx = wave_max(mx);
    mn = wave_min(mn);
    if (l == 0) { sm.wmax[w] = mx; sm.wmin[w] = mn; }
    __syncthreads();
    if (tid == 0) {
        uint64_t M = 0, m = ~uint64_t(0);
        for (int ww = 0; ww < BLOCK / WAVE; ++ww) {
            M = sm.wmax[ww] > M ? sm.wmax[ww] : M;
            m = sm.wmin[ww] < m ? sm.wmin[ww] : m;
        }
        // bytes above the highest differing bit of max and min are common
        const int same = M == m ? 8 : __clzll((long long)(M ^ m)) / 8;
        sm.prefix_hi = same == 8 ? M : (same == 0 ? 0 : M & (~uint64_t(0) << (64 - 8 * same)));
        sm.prefix_lo = 0;
        sm.need = (uint32_t)need;
        sm.whole = 0;
        sm.wmax[0] = (uint64_t)same;
    }
    __syncthreads();
    const int same = (int)sm.wmax[0];
    const int top = (LO ? 11 : 7) - same;          // first byte to resolve, counted from the bottom
    for (int p = top; p >= 0; --p) {
        for (int i = tid; i < 256; i += BLOCK) sm.h[i] = 0;
        __syncthreads();
        // bytes 7..4 of the order key's hi... : byte p >= 4 (with LO) lives in hi
        const bool in_hi = LO ? p >= 4 : true;
        const int sh = LO ? (in_hi ? 8 * (p - 4) : 8 * p) : 8 * p;
        const uint64_t mhi = in_hi ? (sh + 8 >= 64 ? 0 : ~uint64_t(0) << (sh + 8)) : ~uint64_t(0);
        const uint32_t mlo = in_hi ? 0u : (sh + 8 >= 32 ? 0u : ~0u << (sh + 8));
        const uint64_t phi = sm.prefix_hi & mhi;
        const uint32_t plo = sm.prefix_lo & mlo;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const bool match = valid[j] && (hi[j] & mhi) == phi && (lo[j] & mlo) == plo;
            const uint32_t d = in_hi ? (uint32_t)(hi[j] >> sh) & 255u : (lo[j] >> sh) & 255u;
            const uint64_t mm = ballot(match);
            if (!mm) continue;
            const int lead = __ffsll((unsigned long long)mm) - 1;
            const uint32_t d0 = wave_read(d, lead);
            if (!ballot(match && d != d0)) {
                if (l == lead) atomicAdd(&sm.h[d0], (uint32_t)popc64(mm));
            } else if (match) {
                atomicAdd(&sm.h[d], 1u);
            }
        }
        __syncthreads();
        if (tid < WAVE) {
            // lane l owns bytes 255-4l .. 252-4l, scanned from the top
            uint32_t c[4];
            uint32_t own = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) { c[q] = sm.h[255 - 4 * tid - q]; own += c[q]; }
            const uint32_t incl = wave_incl_sum(own);
            const uint32_t above = incl - own;
            const uint32_t nd = sm.need;
            if (above < nd && nd <= incl) {
                uint32_t acc = above;
                int q = 0;
                while (acc + c[q] < nd) { acc += c[q]; ++q; }
                const uint32_t byte = (uint32_t)(255 - 4 * tid - q);
                if (in_hi) sm.prefix_hi |= (uint64_t)byte << sh;
                else sm.prefix_lo |= byte << sh;
                sm.need = nd - acc;
                sm.whole = c[q] == nd - acc;
            }
        }
        __syncthreads();
        if (sm.whole) {
            // every candidate under the chosen prefix is selected: the
            // need-th largest is the smallest of them
            const int shn = sh;
            const uint64_t mhi2 = in_hi ? (shn >= 64 ? 0 : ~uint64_t(0) << shn) : ~uint64_t(0);
            const uint32_t mlo2 = in_hi ? 0u : (shn >= 32 ? 0u : ~0u << shn);
            const uint64_t phi2 = sm.prefix_hi & mhi2;
            const uint32_t plo2 = sm.prefix_lo & mlo2;
            uint64_t bh = ~uint64_t(0);
#pragma unroll
            for (int j = 0; j < PER; ++j)
                if (valid[j] && (hi[j] & mhi2) == phi2 && (lo[j] & mlo2) == plo2 && hi[j] < bh) bh = hi[j];
            bh = wave_min(bh);
            if (l == 0) sm.wmin[w] = bh;
            __syncthreads();
            uint64_t mh = ~uint64_t(0);
            for (int ww = 0; ww < BLOCK / WAVE; ++ww) mh = sm.wmin[ww] < mh ? sm.wmin[ww] : mh;
            uint32_t bl = ~0u;
            if (LO) {
#pragma unroll
                for (int j = 0; j < PER; ++j)
                    if (valid[j] && hi[j] == mh && (lo[j] & mlo2) == plo2 && lo[j] < bl) bl = lo[j];
                bl = wave_min(bl);
                if (l == 0) sm.wlo[w] = bl;
                __syncthreads();
                for (int ww = 0; ww < BLOCK / WAVE; ++ww) bl = sm.wlo[ww] < bl ? sm.wlo[ww] : bl;
            }
            t_hi = mh;
            t_lo = LO ? bl : 0;
            __syncthreads();
            return;
        }
    }
    t_hi = sm.prefix_hi;
    t_lo = sm.prefix_lo;
}

__device__ __forceinline__ uint64_t order_hi(int64_t sum) { return (uint64_t)sum ^ (uint64_t(1) << 63); }
__device__ __forceinline__ uint32_t order_lo(int32_t key) { return ~(uint32_t)key; }

// Step 1: thr[0] = k-th largest sum of the sample (INT64_MIN when the sample,
// hence the whole input, has fewer than k groups).
template <int BLOCK, int PER>
__global__ void __launch_bounds__(BLOCK)
k_topk_thresh(const int64_t* gsum, int64_t n_upper, const int64_t* d_n, int k, int64_t* thr) {
    __shared__ BlockSelect<BLOCK, PER, false> sm;
    int64_t n = n_upper;
    if (d_n) { const int64_t t = *d_n; n = t < n ? t : n; }
    const int64_t m = n < (int64_t)BLOCK * PER ? n : (int64_t)BLOCK * PER;
    if (m < k) {
        if (threadIdx.x == 0) thr[0] = INT64_MIN;
        return;
    }
    // PER runs of BLOCK consecutive groups, spread evenly over the groups
    // (one run per load round, so every load of the block is contiguous)
    const int64_t run = n > m ? n / PER : BLOCK;   // >= BLOCK when n > m
    uint64_t hi[PER];
    uint32_t lo[PER];
    bool valid[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int64_t i = (int64_t)j * BLOCK + threadIdx.x;
        valid[j] = i < m;
        // clamped index (the sample has at least k >= 1 rows): no branch between the loads
        hi[j] = order_hi(gsum[valid[j] ? (int64_t)j * run + threadIdx.x : 0]);
        lo[j] = 0;
    }
    uint64_t t_hi;
    uint32_t t_lo;
    block_select<BLOCK, PER, false>(sm, hi, lo, valid, k, t_hi, t_lo);
    if (threadIdx.x == 0) thr[0] = (int64_t)(t_hi ^ (uint64_t(1) << 63));
}

// Step 2: keeps the groups with sum >= thr[0]; the order of the kept
// candidates is irrelevant.
__global__ void k_topk_filter(const int32_t* gkey, const int64_t* gsum, int64_t n_upper, const int64_t* d_n,
                              const int64_t* thr, TopCand* out, int64_t* d_out);

// Step 3, level `level`: runs only while its input count exceeds TOPK_DIRECT.
// Each block keeps the first k of its chunk of CH candidates (radix select,
// then a gather, in no particular order; padding when the chunk holds fewer).
// Block 0 always writes its k rows.
template <int BLOCK, int CH>
__global__ void __launch_bounds__(BLOCK)
k_topk_level(const int64_t* d_n0, const TopCand* cin, TopCand* cout, int k, int level) {
    constexpr int PER = CH / BLOCK;
    static_assert(PER * BLOCK == CH, "whole chunks per block");
    __shared__ BlockSelect<BLOCK, PER, true> sm;
    __shared__ int s_n;
    const int64_t n = topk_level_n(*d_n0, level, k);
    if (n <= TOPK_DIRECT) return;
    const int64_t c0 = (int64_t)blockIdx.x * CH;
    if (c0 >= n && blockIdx.x != 0) return;
    const int tid = threadIdx.x;
    uint64_t hi[PER];
    uint32_t lo[PER];
    int32_t idx[PER];
    bool valid[PER];
    int nv = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int64_t g = c0 + (int64_t)j * BLOCK + tid;
        TopCand x;
        x.sum = 0; x.key = 0; x.idx = -1;
        if (g < n) x = cin[g];
        valid[j] = x.idx >= 0;
        hi[j] = order_hi(x.sum);
        lo[j] = order_lo(x.key);
        idx[j] = x.idx;
        nv += valid[j];
    }
    nv = wave_sum(nv);
    if (tid == 0) s_n = 0;
    __syncthreads();
    if (lane_id() == 0 && nv) atomicAdd(&s_n, nv);
    __syncthreads();
    const int need = s_n < k ? s_n : k;
    __syncthreads();
    if (tid == 0) s_n = 0;
    uint64_t t_hi = 0;
    uint32_t t_lo = 0;
    if (need > 0) block_select<BLOCK, PER, true>(sm, hi, lo, valid, need, t_hi, t_lo);
    __syncthreads();
    TopCand* dst = cout + (int64_t)blockIdx.x * k;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        if (need > 0 && valid[j] && (hi[j] > t_hi || (hi[j] == t_hi && lo[j] >= t_lo))) {
            const int slot = atomicAdd(&s_n, 1);
            if (slot < need) {
                TopCand x;
                x.sum = (int64_t)(hi[j] ^ (uint64_t(1) << 63));
                x.key = (int32_t)~lo[j];
                x.idx = idx[j];
                dst[slot] = x;
            }
        }
    }
    for (int i = need + tid; i < k; i += BLOCK) {
        TopCand x;
        x.sum = 0; x.key = 0; x.idx = -1;
        dst[i] = x;
    }
}

// Step 4: one block.  The input is the first level whose count is at most
// TOPK_DIRECT (the filtered candidates, or level l's output).  A radix select
// on (sum, key) gives the exact k-th candidate; the k candidates not after it
// are gathered in LDS, sorted by a bitonic network over the next power of two
// and written out with their counts.
template <int BLOCK, int PER>
__global__ void __launch_bounds__(BLOCK)
k_topk_final(const int64_t* d_n0, const TopCand* filtered, TopkLevels lvl, int levels, int k,
             const int64_t* gcnt, int32_t* out_key, int64_t* out_sum, int64_t* out_cnt, int32_t* d_k) {
    static_assert(BLOCK * PER >= TOPK_DIRECT, "the final block holds every candidate");
    __shared__ BlockSelect<BLOCK, PER, true> sm;
    __shared__ TopCand c[TOPK_K_MAX];
    __shared__ int s_n;
    int64_t n = *d_n0;
    const TopCand* src = filtered;
    for (int l = 0; l < levels && n > TOPK_DIRECT; ++l) {
        src = lvl.out[l];
        n = (n + TOPK_CH - 1) / TOPK_CH * k;
    }
    const int tid = threadIdx.x;
    if (tid == 0) s_n = 0;
    __syncthreads();
    uint64_t hi[PER];
    uint32_t lo[PER];
    bool valid[PER];
    int32_t idx[PER];
    int nvalid = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int64_t i = (int64_t)j * BLOCK + tid;
        TopCand x;
        x.sum = 0; x.key = 0; x.idx = -1;
        if (i < n) x = src[i];
        valid[j] = x.idx >= 0;
        hi[j] = order_hi(x.sum);
        lo[j] = order_lo(x.key);
        idx[j] = x.idx;
        nvalid += valid[j];
    }
    nvalid = wave_sum(nvalid);
    if (lane_id() == 0) atomicAdd(&s_n, nvalid);
    __syncthreads();
    const int total = s_n;
    const int kk = total < k ? total : k;
    __syncthreads();
    if (tid == 0) s_n = 0;
    uint64_t t_hi = 0;
    uint32_t t_lo = 0;
    if (kk > 0) block_select<BLOCK, PER, true>(sm, hi, lo, valid, kk, t_hi, t_lo);
    __syncthreads();
    // the kk candidates whose order key is at least the kk-th one
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const bool take = kk > 0 && valid[j] && (hi[j] > t_hi || (hi[j] == t_hi && lo[j] >= t_lo));
        if (take) {
            const int slot = atomicAdd(&s_n, 1);
            TopCand x;
            x.sum = (int64_t)(hi[j] ^ (uint64_t(1) << 63));
            x.key = (int32_t)~lo[j];
            x.idx = idx[j];
            if (slot < kk) c[slot] = x;      // more only if keys repeat
        }
    }
    __syncthreads();
    int P = 1;
    while (P < kk) P <<= 1;
    for (int i = kk + tid; i < P; i += BLOCK) c[i].idx = -1;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = tid; t < P / 2; t += BLOCK) {
                const int a = 2 * t - (t & (stride - 1));
                const int b = a + stride;
                const bool asc = ((a & size) == 0);
                const TopCand x = c[a], y = c[b];
                if (asc ? top_before(y, x) : top_before(x, y)) { c[a] = y; c[b] = x; }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < kk; i += BLOCK) {
        const TopCand x = c[i];
        out_key[i] = x.key;
        out_sum[i] = x.sum;
        out_cnt[i] = gcnt[x.idx];
    }
    if (tid == 0) *d_k = kk;
}

}  // namespace tqp
