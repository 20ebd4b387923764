// Sort-based group-by, second half (Section 5.4, Algorithm 2): over keys that
// are already sorted, mark the first element of every run of equal keys
// (uniqueConsecutive), number the runs (the inverse index) and reduce each
// run's values: sum, count and the sum behind an average.
//
// Each wave walks a contiguous chunk of the tile 64 elements at a time: run
// heads come from one ballot, the run number from a popcount plus the tile's
// base (block scan + decoupled look-back over the head counts), the partial
// sums from a segmented wave scan with the open run carried from one round to
// the next.  A run that lies entirely inside one chunk is stored; the pieces of
// a run cut by a chunk boundary are added atomically into zeroed outputs
// (integer adds, so the result does not depend on their order).
#pragma once
#include "dev.hpp"
#include "topk.hpp"

namespace tqp {

template <int BLOCK_, int ITEMS_>
struct SegCfg {
    static constexpr int BLOCK = BLOCK_;
    static constexpr int ITEMS = ITEMS_;
    static constexpr int TILE = BLOCK_ * ITEMS_;
    static constexpr int WAVES = BLOCK_ / WAVE;
};

// Values stored next to the sorted keys.
struct ValsDirect {
    const int64_t* v;
    const int64_t* a;          // nullable
    __device__ void get(int64_t i, int64_t& x, int64_t& y) const {
        x = v[i];
        y = a ? a[i] : 0;
    }
};

// Values reached through the sort permutation (Algorithm 2 permutes every
// data column by the sorted order of the group keys).
struct ValsGather {
    const int32_t* perm;
    const int64_t* v;
    const int64_t* a;          // nullable
    __device__ void get(int64_t i, int64_t& x, int64_t& y) const {
        const int32_t r = perm[i];
        x = v[r];
        y = a ? a[r] : 0;
    }
};

struct SegOut {
    int32_t* key;
    int64_t* sum;
    int64_t* cnt;
    int64_t* sa;               // nullable: sum of the averaged column
    int64_t gcap;
    int64_t* d_ngroups;
};

__device__ __forceinline__ void seg_flush(const SegOut& o, int64_t seg, int64_t v, int64_t c, int64_t a,
                                          bool complete) {
    if (seg < 0 || seg >= o.gcap) return;
    if (complete) {
        o.sum[seg] = v;
        o.cnt[seg] = c;
        if (o.sa) o.sa[seg] = a;
    } else {
        atomic_add(&o.sum[seg], v);
        atomic_add(&o.cnt[seg], c);
        if (o.sa) atomic_add(&o.sa[seg], a);
    }
}

template <class Cfg, class VS, bool AVG>
__global__ void __launch_bounds__(Cfg::BLOCK)
k_segreduce(const uint32_t* keys, VS vs, int64_t n_upper, const int64_t* d_n, uint64_t* status,
            uint32_t* tile_counter, SegOut out, uint32_t* flags) {
    constexpr int ITEMS = Cfg::ITEMS, TILE = Cfg::TILE, W = Cfg::WAVES;
    __shared__ int64_t s_scan[W];
    __shared__ int64_t s_wave[W];
    __shared__ int64_t s_base;
    __shared__ uint32_t s_tile;
    __shared__ int64_t s_pseg[W], s_pv[W], s_pc[W], s_pa[W];   // each wave's unfinished last run
    const int tid = threadIdx.x, w = tid / WAVE, l = lane_id();

    int64_t n = n_upper;
    if (d_n) { int64_t t = *d_n; n = t < n ? t : n; }
    if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t ntiles = (n + TILE - 1) / TILE;
    if (tile >= ntiles) {
        if (ntiles == 0 && tile == 0 && tid == 0) *out.d_ngroups = 0;
        return;
    }

    // Keys and run heads of the wave's contiguous chunk, 64 per round.
    const int64_t chunk = tile * TILE + (int64_t)w * ITEMS * WAVE;
    uint32_t key[ITEMS];
    uint64_t hm[ITEMS];
    int64_t wave_heads = 0;
    uint32_t prev[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {          // clamped indices: no branch between the loads
        const int64_t i = chunk + j * WAVE + l;
        const int64_t ic = i < n ? i : n - 1;  // n >= 1: the tile exists
        key[j] = keys[ic];
        prev[j] = keys[ic > 0 ? ic - 1 : 0];
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = chunk + j * WAVE + l;
        const bool head = i < n && (i == 0 || prev[j] != key[j]);
        if (i >= n) key[j] = 0;
        hm[j] = ballot(head);
        wave_heads += popc64(hm[j]);
    }
    if (l == 0) s_wave[w] = wave_heads;
    __syncthreads();
    if (w == 0) {
        int64_t tot = 0;
        for (int ww = 0; ww < W; ++ww) tot += s_wave[ww];
        const int64_t base = lookback64(status, tile, tot, flags);
        if (tid == 0) {
            int64_t run = 0;
            for (int ww = 0; ww < W; ++ww) { s_scan[ww] = run; run += s_wave[ww]; }
            s_base = base;
            if (tile == ntiles - 1) {
                *out.d_ngroups = base + tot;
                if (base + tot > out.gcap) set_flag(flags, FLAG_CAPACITY);
            }
        }
    }
    __syncthreads();
    const int64_t seg_base = s_base + s_scan[w];

    int64_t open_v = 0, open_c = 0, open_a = 0, open_seg = -1;
    bool has_open = false, open_here = false;
    int64_t heads_so_far = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t i = chunk + j * WAVE + l;
        const bool valid = i < n;
        const uint64_t h = hm[j];
        if (has_open && (h & 1)) {              // the open run ended at the previous round
            if (l == 0) seg_flush(out, open_seg, open_v, open_c, open_a, open_here);
            has_open = false;
        }
        const uint64_t upto = h & lanemask_le();
        const int64_t seg = seg_base + heads_so_far + popc64(upto) - 1;
        const bool head = (h >> l) & 1;
        if (valid && head && seg < out.gcap) out.key[seg] = key[j];
        int64_t x = 0, y = 0;
        if (valid) vs.get(i, x, y);
        int64_t v = wave_seg_incl_sum(x, h);
        int64_t c = wave_seg_incl_sum((int32_t)(valid ? 1 : 0), h);
        int64_t a = AVG ? wave_seg_incl_sum(y, h) : 0;
        const bool cont = upto == 0;            // run began before this round
        if (cont && has_open) { v += open_v; c += open_c; a += open_a; }
        const bool here = cont ? (has_open && open_here) : true;
        const bool last_global = valid && (i == n - 1);
        const bool next_head = (l < WAVE - 1) && ((h >> (l + 1)) & 1);
        if (valid && (next_head || last_global)) seg_flush(out, seg, v, c, a, here);
        const int64_t i63 = chunk + j * WAVE + (WAVE - 1);
        if (i63 < n - 1) {                      // lane 63 valid and not the global end: run stays open
            open_v = wave_read(v, WAVE - 1);
            open_c = wave_read(c, WAVE - 1);
            if (AVG) open_a = wave_read(a, WAVE - 1);
            open_seg = wave_read(seg, WAVE - 1);
            open_here = wave_read((int)here, WAVE - 1) != 0;
            has_open = true;
        } else {
            has_open = false;
        }
        heads_so_far += popc64(h);
    }
    bool partial = false;
    if (has_open) {                             // the chunk's last run may continue past it
        const int64_t last = chunk + (int64_t)ITEMS * WAVE - 1;
        const uint32_t lk = wave_read(key[ITEMS - 1], WAVE - 1);
        const bool ends = keys[last + 1] != lk;
        if (open_here && ends) {
            if (l == 0) seg_flush(out, open_seg, open_v, open_c, open_a, true);
        } else {
            partial = true;
        }
    }
    // The waves' unfinished runs are merged in the block before they are added
    // to the output: adjacent waves of a long run share one set of atomics.
    if (l == 0) {
        s_pseg[w] = partial ? open_seg : -1;
        s_pv[w] = open_v;
        s_pc[w] = open_c;
        s_pa[w] = open_a;
    }
    __syncthreads();
    if (tid == 0) {
        int64_t cs = -1, cv = 0, cc = 0, ca = 0;
        for (int ww = 0; ww < W; ++ww) {
            const int64_t sg = s_pseg[ww];
            if (sg != cs) {
                if (cs >= 0) seg_flush(out, cs, cv, cc, ca, false);
                cs = sg;
                cv = cc = ca = 0;
            }
            if (sg >= 0) {
                cv += s_pv[ww];
                cc += s_pc[ww];
                ca += s_pa[ww];
            }
        }
        if (cs >= 0) seg_flush(out, cs, cv, cc, ca, false);
    }
}

// Group-by over keys sorted by their high bits only (Algorithm 2 with the
// last radix digit resolved in LDS): bucket b holds the keys whose bits above
// `lowb` equal b, contiguous in the sorted array.  One block per bucket (in
// bucket order, from a counter) accumulates sum and count per low-bit value in
// LDS, which is the counting sort of the last digit and the run reduction in
// one step, then writes the bucket's non-empty groups in ascending key order
// at the offset given by a look-back over the buckets' group counts.
constexpr int BUCKET_LOWB_MAX = 13;        // 8192 slots: 96 KB of LDS

// Start of every bucket in the high-bit-sorted keys (starts[nbuckets] = n),
// one binary search per bucket.
__global__ void k_bucket_bounds(const uint32_t* keys, int64_t n_upper, const int64_t* d_n, int lowb,
                                int64_t nbuckets, int64_t* starts);

// vals: int64 values (VT = int64_t), int32 values (VT = int32_t) or values in
// [0, 2^32) (VT = uint32_t).  OP: what the value column is reduced to (sum;
// min or max for signed values), written to out.sum.  With cand, each block also appends the first
// k of its groups in the order value DESC (the count with BYCNT), key ASC
// (step 1 of the top-k: the overall first k are among them) to cand,
// counting them in *d_cand.
enum : int { BUCKET_SUM = 0, BUCKET_MIN = 1, BUCKET_MAX = 2 };
template <int BLOCK, int SLOTS, class VT = int64_t, int OP = BUCKET_SUM, bool BYCNT = false>
__global__ void __launch_bounds__(BLOCK)
k_bucket_agg(const uint32_t* keys, const VT* vals, const int64_t* starts, const uint32_t* bhist, int lowb,
             int64_t nbuckets, uint64_t* status, uint32_t* counter, SegOut out, uint32_t* flags,
             TopCand* cand = nullptr, int64_t* d_cand = nullptr, int k = 0) {
    static_assert(SLOTS <= (1 << BUCKET_LOWB_MAX), "slot table larger than the LDS budget");
    static_assert(OP == BUCKET_SUM || std::is_same<VT, int64_t>::value || std::is_same<VT, int32_t>::value,
                  "min / max over signed values");
    constexpr int U = 8;                               // loads in flight per thread
    constexpr int PER = (SLOTS + BLOCK - 1) / BLOCK;   // most slots per thread
    __shared__ unsigned long long s_sum[SLOTS];
    __shared__ uint32_t s_cnt[SLOTS];
    __shared__ int64_t s_base;
    __shared__ int32_t s_wave[BLOCK / WAVE];
    __shared__ uint32_t s_b;
    __shared__ BlockSelect<BLOCK, PER, true> s_sel;
    __shared__ int32_t s_nc;
    const int tid = threadIdx.x, w = tid / WAVE, l = lane_id();
    if (tid == 0) s_b = atomicAdd(counter, 1u);
    const int slots = 1 << lowb;
    constexpr unsigned long long ident = OP == BUCKET_MIN ? 0x7FFFFFFFFFFFFFFFull
                                         : OP == BUCKET_MAX ? 0x8000000000000000ull : 0ull;
    for (int i = tid; i < slots; i += BLOCK) { s_sum[i] = ident; s_cnt[i] = 0; }
    __syncthreads();
    const int64_t b = s_b;
    if (b >= nbuckets) return;
    int64_t lo, hi;
    if (bhist) {
        // bucket b = digit b of the single sort pass: it starts after the
        // elements of the smaller digits
        if (w == 0) {
            int64_t acc = 0;
            for (int64_t d = l; d < b; d += WAVE) acc += bhist[d];
            acc = wave_sum(acc);
            if (l == 0) s_base = acc;
        }
        __syncthreads();
        lo = s_base;
        hi = lo + bhist[b];
        __syncthreads();
    } else {
        lo = starts[b];
        hi = starts[b + 1];
    }
    const uint32_t lmask = (uint32_t)slots - 1;
    for (int64_t i0 = lo + tid; i0 < hi; i0 += (int64_t)BLOCK * U) {
        uint32_t k[U];
        VT v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {          // clamped index: no branch between the loads
            const int64_t i = i0 + (int64_t)j * BLOCK;
            const int64_t ic = i < hi ? i : hi - 1;
            k[j] = keys[ic] & lmask;
            v[j] = vals[ic];
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (i0 + (int64_t)j * BLOCK < hi) {
                if constexpr (OP == BUCKET_MIN) {
                    atomicMin(reinterpret_cast<long long*>(&s_sum[k[j]]), (long long)v[j]);
                } else if constexpr (OP == BUCKET_MAX) {
                    atomicMax(reinterpret_cast<long long*>(&s_sum[k[j]]), (long long)v[j]);
                } else if constexpr (std::is_same<VT, uint32_t>::value) {
                    // 32-bit add on the low word; a wrap carries into the high word
                    uint32_t* w2 = reinterpret_cast<uint32_t*>(&s_sum[k[j]]);
                    const uint32_t old = atomicAdd(&w2[0], v[j]);
                    if (old + v[j] < old) atomicAdd(&w2[1], 1u);
                } else {
                    atomicAdd(&s_sum[k[j]], (unsigned long long)v[j]);
                }
                atomicAdd(&s_cnt[k[j]], 1u);
            }
        }
    }
    __syncthreads();
    // non-empty slots in ascending order -> local group index
    const int per = (slots + BLOCK - 1) / BLOCK;      // consecutive slots per thread
    int mine = 0;
    for (int q = 0; q < per; ++q) {
        const int sl = tid * per + q;
        if (sl < slots && s_cnt[sl]) ++mine;
    }
    const int incl = wave_incl_sum(mine);
    if (l == WAVE - 1) s_wave[w] = incl;
    __syncthreads();
    int total = 0, woff = 0;
    for (int ww = 0; ww < BLOCK / WAVE; ++ww) {
        if (ww < w) woff += s_wave[ww];
        total += s_wave[ww];
    }
    if (w == 0) {
        const int64_t base = lookback64(status, b, total, flags);
        if (tid == 0) {
            s_base = base;
            if (b == nbuckets - 1) {
                *out.d_ngroups = base + total;
                if (base + total > out.gcap) set_flag(flags, FLAG_CAPACITY);
            }
        }
    }
    __syncthreads();
    int64_t g = s_base + woff + incl - mine;
    // the block's groups as top-k candidates: order key (sum, ~key), group index
    uint64_t chi[PER];
    uint32_t clo[PER];
    int32_t cidx[PER];
    bool cval[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int sl = tid * per + q;
        cval[q] = false;
        chi[q] = 0;
        clo[q] = 0;
        cidx[q] = 0;
        if (q < per && sl < slots && s_cnt[sl]) {
            const int32_t key = (int32_t)((b << lowb) | sl);
            const int64_t sum = (int64_t)s_sum[sl];
            if (g < out.gcap) {
                out.key[g] = key;
                out.sum[g] = sum;
                out.cnt[g] = (int64_t)s_cnt[sl];
                chi[q] = order_hi(BYCNT ? (int64_t)s_cnt[sl] : sum);
                clo[q] = order_lo(key);
                cidx[q] = (int32_t)g;
                cval[q] = true;
            }
            ++g;
        }
    }
    if (!cand) return;
    // candidates stored (groups past the output capacity are not)
    int nv = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) nv += cval[q];
    nv = wave_sum(nv);
    if (tid == 0) s_nc = 0;
    __syncthreads();
    if (l == 0 && nv) atomicAdd(&s_nc, nv);
    __syncthreads();
    const int need = s_nc < k ? s_nc : k;
    if (need == 0) return;
    uint64_t t_hi;
    uint32_t t_lo;
    block_select<BLOCK, PER, true>(s_sel, chi, clo, cval, need, t_hi, t_lo);
    __syncthreads();
    if (tid == 0) {
        s_base = atomic_add(d_cand, (int64_t)need);
        s_nc = 0;
    }
    __syncthreads();
    // exactly need candidates are not after the need-th (group keys are unique)
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        if (cval[q] && (chi[q] > t_hi || (chi[q] == t_hi && clo[q] >= t_lo))) {
            const int slot = atomicAdd(&s_nc, 1);
            if (slot < need) {
                TopCand x;
                x.sum = (int64_t)(chi[q] ^ (uint64_t(1) << 63));
                x.key = (int32_t)~clo[q];
                x.idx = cidx[q];
                cand[s_base + slot] = x;
            }
        }
    }
}

// avg = (double)sum / (double)count, one IEEE division per group.
__global__ void k_avg(const int64_t* sa, const int64_t* cnt, double* avg, const int64_t* d_ngroups,
                      int64_t gcap);

}  // namespace tqp
