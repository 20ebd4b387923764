// Batched flags fragments: many fragments of uneven size run as one launch
// sequence of persistent kernels.  Every stage pulls (fragment side, tile)
// work items from one device counter per stage, so a block that waits in a
// look-back only ever waits on items handed out before its own.  The
// sequence can be captured into a hipGraph and replayed, and an autotuner
// picks the radix digit width and tile shape by timing the candidates.
#include <algorithm>
#include <vector>

#include "fragment.hpp"

namespace tqp {

// One sort input: the fact side or the dim side of one fragment.
struct BatchSeg {
    const int32_t* key;
    const void* fcol;          // filter column (int8 or int32)
    int32_t ftype;             // 1 = int8, 2 = int32
    int32_t op;
    int64_t k;
    int64_t row0;              // payload = row0 + row (global row id of the fact table)
    int64_t n;                 // rows
    int32_t npass;
    int32_t shift[8];
    int32_t bits[8];
    int64_t ntiles;            // tiles of n (upper bound for every pass)
    uint32_t* hist;            // npass * R
    uint32_t* status;          // npass * ntiles * R
    int64_t* d_cnt;            // rows that pass the filter
    uint32_t* bk[2];           // ping-pong keys: pass p writes bk[p & 1]
    uint32_t* bv[2];           // ping-pong row ids
};

struct BatchFrag {
    int32_t fseg, dseg;
    int32_t lowb;              // fact key bits the fact sort leaves to the join tiles
    const int64_t* price;
    const int64_t* disc;
    const int8_t* flagA;
    const int8_t* flagB;
    int64_t* acc;              // [8][3]
    int64_t* d_join;
    int64_t* win;
    tqp_flags_out out;
};

// Runtime-typed filter source of the first pass (int32 date or int8 seg).
struct SrcSeg {
    const BatchSeg* s;
    __device__ int64_t size() const { return s->n; }
    // Both typed reads are issued (the other at index 0, always in range) and
    // the value selected afterwards: no branch between the loads of a tile's
    // items.
    __device__ bool pass_row(int64_t i) const {
        const bool i8 = s->ftype == 1;
        const int64_t x8 = ((const int8_t*)s->fcol)[i8 ? i : 0];
        const int64_t x32 = ((const int32_t*)s->fcol)[i8 ? 0 : i];
        return cmp_eval(i8 ? x8 : x32, s->op, s->k);
    }
    __device__ bool load_key(int64_t i, uint32_t& kk) const {
        kk = (uint32_t)s->key[i];
        return pass_row(i);
    }
    __device__ bool load(int64_t i, uint32_t& kk, uint32_t& v) const {
        kk = (uint32_t)s->key[i];
        v = (uint32_t)(s->row0 + i);
        return pass_row(i);
    }
};

__device__ __forceinline__ int find_item(const int64_t* prefix, int count, int64_t g) {
    int lo = 0, hi = count;    // last i with prefix[i] <= g
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

constexpr int BATCH_HIST_CHUNK = 32768;

// Histograms of every pass of every segment.  Work item = (segment, chunk of
// BATCH_HIST_CHUNK rows); prefix holds the chunk offsets of the segments.
template <class Cfg>
__global__ void __launch_bounds__(Cfg::BLOCK)
k_batch_hist(const BatchSeg* segs, int nseg, const int64_t* prefix, uint32_t* counter, uint32_t key_mask_unused,
             uint32_t* flags) {
    constexpr int R = Cfg::RADIX;
    __shared__ uint32_t h[Cfg::MAX_PASSES * R];
    __shared__ uint32_t s_cnt, s_bad;
    __shared__ int64_t s_item;
    __shared__ int s_seg;
    (void)key_mask_unused;
    const int64_t total = prefix[nseg];
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t g = atomicAdd(counter, 1u);
            s_item = g;
            s_seg = g < total ? find_item(prefix, nseg, g) : -1;
            s_cnt = 0;
            s_bad = 0;
        }
        __syncthreads();
        const int64_t g = s_item;
        if (g >= total) break;
        const BatchSeg& sg = segs[s_seg];
        const int np = sg.npass;
        for (int i = threadIdx.x; i < np * R; i += Cfg::BLOCK) h[i] = 0;
        __syncthreads();
        const int64_t r0 = (g - prefix[s_seg]) * BATCH_HIST_CHUNK;
        const int64_t r1 = r0 + BATCH_HIST_CHUNK < sg.n ? r0 + BATCH_HIST_CHUNK : sg.n;
        SrcSeg src{&sg};
        const uint32_t kmask = sg.shift[np - 1] + sg.bits[np - 1] >= 32
                                   ? 0xFFFFFFFFu : ((1u << (sg.shift[np - 1] + sg.bits[np - 1])) - 1);
        uint32_t cnt = 0, bad = 0;
        constexpr int U = HIST_ITEMS;
        for (int64_t i0 = r0 + threadIdx.x; i0 < r1; i0 += (int64_t)Cfg::BLOCK * U) {
            uint32_t kk[U];
            bool ok[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {      // clamped index: no branch between the loads
                const int64_t i = i0 + (int64_t)j * Cfg::BLOCK;
                const bool in = i < r1;
                ok[j] = src.load_key(in ? i : r1 - 1, kk[j]) && in;
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                if (!ok[j]) continue;
                const uint32_t k = kk[j];
                ++cnt;
                bad |= k & ~kmask;
                for (int p = 0; p < np; ++p)
                    atomicAdd(&h[p * R + ((k >> sg.shift[p]) & ((1u << sg.bits[p]) - 1))], 1u);
            }
        }
        cnt = wave_sum(cnt);
        if (lane_id() == 0 && cnt) atomicAdd(&s_cnt, cnt);
        if (bad) atomicOr(&s_bad, 1u);
        __syncthreads();
        for (int i = threadIdx.x; i < np * R; i += Cfg::BLOCK)
            if (h[i]) atomic_add(&sg.hist[i], h[i]);
        if (threadIdx.x == 0) {
            if (s_cnt) atomic_add(sg.d_cnt, (int64_t)s_cnt);
            if (s_bad) set_flag(flags, FLAG_KEY_RANGE);
        }
        __syncthreads();
    }
}

// Pass p of every segment that has one; work item = (segment, tile).
template <class Cfg>
__global__ void __launch_bounds__(Cfg::BLOCK)
k_batch_pass(const BatchSeg* segs, int nseg, const int64_t* prefix, int p, uint32_t* counter, uint32_t* flags) {
    __shared__ PassSmem<Cfg, uint32_t> sm;
    __shared__ int s_seg;
    __shared__ int64_t s_item;
    const int64_t total = prefix[nseg];
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t g = atomicAdd(counter, 1u);
            s_item = g;
            s_seg = g < total ? find_item(prefix, nseg, g) : -1;
        }
        __syncthreads();
        const int64_t g = s_item;
        if (g >= total) break;
        const BatchSeg& sg = segs[s_seg];
        const int64_t tile = g - prefix[s_seg];
        DstPairs<uint32_t> dst{sg.bk[p & 1], sg.bv[p & 1]};
        uint32_t* st = sg.status + (int64_t)p * sg.ntiles * Cfg::RADIX;
        const uint32_t* hist = sg.hist + p * Cfg::RADIX;
        if (p == 0) {
            SrcSeg src{&sg};
            const int64_t n = sg.n;
            if (tile < (n + Cfg::TILE - 1) / Cfg::TILE)
                radix_pass_tile<Cfg, SrcSeg, uint32_t>(src, dst, sg.shift[0], sg.bits[0], hist, st, (uint32_t)tile, n,
                                                       flags, sm);
        } else {
            SrcPairs<uint32_t> src{sg.bk[(p - 1) & 1], sg.bv[(p - 1) & 1], sg.n, sg.d_cnt};
            const int64_t n = src.size();
            if (tile < (n + Cfg::TILE - 1) / Cfg::TILE)
                radix_pass_tile<Cfg, SrcPairs<uint32_t>, uint32_t>(src, dst, sg.shift[p], sg.bits[p], hist, st,
                                                                   (uint32_t)tile, n, flags, sm);
        }
        __syncthreads();
    }
}

// R windows of every join tile of every fragment (one thread per tile).
__global__ void k_batch_windows(const BatchSeg* segs, const BatchFrag* frags, int nfrag, const int64_t* prefix,
                                int tile_size) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= prefix[nfrag]) return;
    const int f = find_item(prefix, nfrag, g);
    const BatchFrag& fr = frags[f];
    const BatchSeg& L = segs[fr.fseg];
    const BatchSeg& R = segs[fr.dseg];
    const int64_t t = g - prefix[f];
    const int64_t nl = *L.d_cnt < L.n ? *L.d_cnt : L.n;
    const int64_t nr = *R.d_cnt < R.n ? *R.d_cnt : R.n;
    if (t * tile_size >= nl) return;
    const uint32_t* lk = L.bk[(L.npass - 1) & 1];
    const uint32_t* rk = R.bk[(R.npass - 1) & 1];
    const int64_t i1 = (t * tile_size + tile_size < nl ? t * tile_size + tile_size : nl) - 1;
    // the tile's keys are sorted on their bits above lowb: its key range runs
    // from its first key's bucket to the end of its last key's
    uint32_t kmin, kmax;
    tile_key_range(TileGeo{0, 0, lk[t * tile_size], lk[i1]}, fr.lowb, kmin, kmax);
    const int64_t lo = lower_bound_glb(rk, 0, nr, kmin);
    fr.win[2 * t] = lo;
    fr.win[2 * t + 1] = upper_bound_glb(rk, lo, nr, kmax);
}

// Join + gather + per-fragment aggregation; work item = (fragment, left tile).
template <class Cfg>
__global__ void __launch_bounds__(Cfg::BLOCK)
k_batch_join(const BatchSeg* segs, const BatchFrag* frags, int nfrag, const int64_t* prefix, uint32_t* counter,
             uint32_t* flags) {
    using Emit = EmitFlagsAgg<Cfg::BLOCK>;
    __shared__ JoinSmem<Cfg, uint32_t> sm;
    __shared__ typename Emit::Smem esm;
    __shared__ int64_t s_item;
    const int64_t total = prefix[nfrag];
    Emit e{};
    e.flags = flags;
    e.init(esm);
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t g = atomicAdd(counter, 1u);
            s_item = g;
            sm.seg = g < total ? find_item(prefix, nfrag, g) : -1;
        }
        __syncthreads();
        const int64_t g = s_item;
        if (g >= total) break;
        const BatchFrag& fr = frags[sm.seg];
        const BatchSeg& L = segs[fr.fseg];
        const BatchSeg& R = segs[fr.dseg];
        const int64_t tile = g - prefix[sm.seg];
        const int64_t nl = *L.d_cnt < L.n ? *L.d_cnt : L.n;
        const int64_t ntiles = (nl + Cfg::TILE - 1) / Cfg::TILE;
        if (tile < ntiles) {
            e.price = fr.price;
            e.disc = fr.disc;
            e.flagA = fr.flagA;
            e.flagB = fr.flagB;
            const uint32_t* lk = L.bk[(L.npass - 1) & 1];
            join_tile<Cfg, uint32_t, uint32_t, Emit>(lk, L.bv[(L.npass - 1) & 1], nl, R.bk[(R.npass - 1) & 1],
                                                     (const uint32_t*)nullptr,
                                                     tile_geo(lk, nl, fr.win, tile, Cfg::TILE), tile, 0, fr.d_join,
                                                     e, esm, sm, fr.lowb);
            e.flush(esm, fr.acc);
        }
        __syncthreads();
    }
}

// One thread per fragment: groups in ascending packed-key order.
__global__ void k_batch_finalize(const BatchFrag* frags, int nfrag) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nfrag) return;
    const BatchFrag& fr = frags[f];
    int64_t g = 0;
    for (int k = 0; k < 6; ++k) {
        const int64_t s = fr.acc[k * 3], c = fr.acc[k * 3 + 1], p = fr.acc[k * 3 + 2];
        if (c == 0) continue;
        fr.out.key[g] = k;
        fr.out.sum[g] = s;
        fr.out.cnt[g] = c;
        fr.out.avg[g] = (double)p / (double)c;
        ++g;
    }
    *fr.out.d_ngroups = g;
    if (fr.out.d_join) *fr.out.d_join = *fr.d_join;
}

}  // namespace tqp

using namespace tqp;

// ------------------------------------------------------------------ host side
namespace {

using BJCfg = JoinCfg<256, 8, 2048>;

// Candidate configurations the autotuner times.
enum { CAND_R4 = 0, CAND_R8S = 1, CAND_R8 = 2, CAND_R11 = 3, NCAND = 4 };
using CR4 = RadixCfg<4, 256, 8, 8>;
using CR8S = RadixCfg<8, 256, 8, 8>;
using CR8 = RadixCfg<8, 512, 8, 8>;
using CR11 = RadixCfg<11, 512, 8, 8>;
const char* const CAND_NAMES[NCAND] = {"digit4_tile2048", "digit8_tile2048", "digit8_tile4096", "digit11_tile4096"};
const int CAND_DIGITS[NCAND] = {4, 8, 8, 11};

struct CandPlan {
    int maxpass = 0;
    size_t zero_off = 0, zero_bytes = 0;
    BatchSeg* d_segs = nullptr;
    BatchFrag* d_frags = nullptr;
    int64_t* d_hist_prefix = nullptr;
    int64_t* d_pass_prefix = nullptr;    // [8][nseg + 1]
    int64_t* d_join_prefix = nullptr;
    uint32_t* counters = nullptr;        // 1 hist + 8 pass + 1 join
    int64_t hist_items = 0, join_tiles = 0;
    int64_t pass_items[8] = {0};
};

}  // namespace

// Host copies of one configuration's descriptor tables.
struct HostTables {
    std::vector<BatchSeg> segs;
    std::vector<BatchFrag> frags;
    std::vector<int64_t> hist_prefix, pass_prefix, join_prefix;
};

struct tqp_batch {
    tqp_ctx* ctx = nullptr;
    int nf = 0;
    int cand_mask = (1 << NCAND) - 1;    // configurations planned in the workspace
    std::vector<tqp_flags_fragment> frags;
    std::vector<tqp_flags_out> outs;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    CandPlan cand[NCAND];
    int chosen = CAND_R8;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<HostTables>* host = nullptr;   // host copies of the descriptor tables (kept for async uploads)
    float tuned_ms[NCAND] = {0, 0, 0, 0};
};

namespace {

template <class Cfg>
int cand_radix_bits() { return Cfg::RADIX_BITS; }

// Lays out (or sizes, when base is null) every candidate's workspace and
// builds its descriptor tables on the host.  Scratch buffers (the ping-pong
// keys and row ids) are shared; each candidate has its own zero region.

template <class Cfg>
void plan_candidate(tqp_batch* b, int c, char* base, size_t& off, size_t scratch_off, HostTables& ht) {
    const int F = b->nf, S = 2 * F;
    CandPlan& cp = b->cand[c];
    ht.segs.assign(S, BatchSeg{});
    ht.frags.assign(F, BatchFrag{});
    auto take = [&](size_t bytes) {
        size_t o = (off + 255) & ~size_t(255);
        off = o + bytes;
        return base ? base + o : nullptr;
    };
    const size_t z0 = (off + 255) & ~size_t(255);
    cp.maxpass = 0;
    size_t soff = scratch_off;
    auto stake = [&](size_t bytes) {
        size_t o = (soff + 255) & ~size_t(255);
        soff = o + bytes;
        return base ? base + o : nullptr;
    };
    for (int f = 0; f < F; ++f) {
        const tqp_flags_fragment& fr = b->frags[f];
        const int kb = norm_key_bits(fr.key_bits);
        // the fact sort covers the key bits above lowb (the join tiles resolve
        // the rest in LDS; at least one pass stays, which also compacts the
        // kept rows), the dim sort all of them
        int lowb = join_low_bits(fr.n_fact, kb, Cfg::RADIX_BITS, BJCfg::TILE, BJCfg::RWIN);
        lowb = lowb < kb - 1 ? lowb : kb - 1;
        PassDesc pds[2] = {make_passes(kb - lowb, Cfg::RADIX_BITS), make_passes(kb, Cfg::RADIX_BITS)};
        for (int q = 0; q < pds[0].npass; ++q) pds[0].shift[q] += lowb;
        for (int side = 0; side < 2; ++side) {
            const PassDesc& pd = pds[side];
            BatchSeg& sg = ht.segs[2 * f + side];
            sg.key = side == 0 ? fr.fk + fr.row0 : fr.pk;
            sg.fcol = side == 0 ? (const void*)(fr.date + fr.row0) : (const void*)fr.seg;
            sg.ftype = side == 0 ? 2 : 1;
            sg.op = side == 0 ? CMP_LT : CMP_EQ;
            sg.k = side == 0 ? fr.D : fr.c;
            sg.row0 = side == 0 ? fr.row0 : 0;
            sg.n = side == 0 ? fr.n_fact : fr.n_dim;
            sg.npass = pd.npass;
            for (int p = 0; p < 8; ++p) { sg.shift[p] = pd.shift[p]; sg.bits[p] = pd.bits[p]; }
            sg.ntiles = (sg.n + Cfg::TILE - 1) / Cfg::TILE;
            sg.hist = (uint32_t*)take((size_t)pd.npass * Cfg::RADIX * 4);
            sg.status = (uint32_t*)take((size_t)pd.npass * sg.ntiles * Cfg::RADIX * 4);
            sg.d_cnt = (int64_t*)take(8);
            for (int q = 0; q < 2; ++q) {
                sg.bk[q] = (uint32_t*)stake((size_t)sg.n * 4);
                sg.bv[q] = (uint32_t*)stake((size_t)sg.n * 4);
            }
            cp.maxpass = std::max(cp.maxpass, pd.npass);
        }
        BatchFrag& bf = ht.frags[f];
        bf.fseg = 2 * f;
        bf.dseg = 2 * f + 1;
        bf.lowb = lowb;
        bf.price = fr.price;
        bf.disc = fr.disc;
        bf.flagA = fr.flagA;
        bf.flagB = fr.flagB;
        bf.acc = (int64_t*)take(24 * 8);
        const int64_t jt = (fr.n_fact + BJCfg::TILE - 1) / BJCfg::TILE;
        bf.d_join = (int64_t*)take(8);
        bf.win = (int64_t*)stake((size_t)(2 * jt + 2) * 8);
        bf.out = b->outs[f];
    }
    cp.counters = (uint32_t*)take(16 * 4);
    cp.zero_off = z0;
    cp.zero_bytes = ((off + 255) & ~size_t(255)) - z0;
    // work-item prefixes
    ht.hist_prefix.assign(S + 1, 0);
    for (int s = 0; s < S; ++s)
        ht.hist_prefix[s + 1] = ht.hist_prefix[s] + (ht.segs[s].n + BATCH_HIST_CHUNK - 1) / BATCH_HIST_CHUNK;
    cp.hist_items = ht.hist_prefix[S];
    ht.pass_prefix.assign((size_t)8 * (S + 1), 0);
    for (int p = 0; p < 8; ++p) {
        int64_t* pp = &ht.pass_prefix[(size_t)p * (S + 1)];
        for (int s = 0; s < S; ++s) pp[s + 1] = pp[s] + (p < ht.segs[s].npass ? ht.segs[s].ntiles : 0);
        cp.pass_items[p] = pp[S];
    }
    ht.join_prefix.assign(F + 1, 0);
    for (int f = 0; f < F; ++f)
        ht.join_prefix[f + 1] = ht.join_prefix[f] + (b->frags[f].n_fact + BJCfg::TILE - 1) / BJCfg::TILE;
    cp.join_tiles = ht.join_prefix[F];
    (void)soff;
}

size_t scratch_bytes(const tqp_batch* b) {
    size_t soff = 0;
    auto stake = [&](size_t bytes) { soff = ((soff + 255) & ~size_t(255)) + bytes; };
    for (int f = 0; f < b->nf; ++f) {
        const tqp_flags_fragment& fr = b->frags[f];
        for (int side = 0; side < 2; ++side) {
            const int64_t n = side == 0 ? fr.n_fact : fr.n_dim;
            for (int q = 0; q < 4; ++q) stake((size_t)n * 4);
        }
        stake((size_t)(2 * ((fr.n_fact + BJCfg::TILE - 1) / BJCfg::TILE) + 2) * 8);
    }
    return (soff + 255) & ~size_t(255);
}

template <class F>
void for_each_cand(int c, F&& f) {
    switch (c) {
        case CAND_R4: f(CR4{}); break;
        case CAND_R8S: f(CR8S{}); break;
        case CAND_R11: f(CR11{}); break;
        default: f(CR8{}); break;
    }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t tables_bytes(int nf) {
    const int S = 2 * nf;
    return align256(sizeof(BatchSeg) * std::max(1, S)) + align256(sizeof(BatchFrag) * std::max(1, nf)) +
           align256(sizeof(int64_t) * (S + 1)) + align256(sizeof(int64_t) * 8 * (S + 1)) +
           align256(sizeof(int64_t) * (nf + 1));
}

// Workspace: shared scratch, then each planned configuration's zero region,
// then each planned configuration's descriptor tables.
size_t plan_all(tqp_batch* b, char* base, std::vector<HostTables>* tables) {
    const size_t scratch = scratch_bytes(b);
    size_t off = scratch;
    for (int c = 0; c < NCAND; ++c) {
        if (!(b->cand_mask & (1 << c))) continue;
        HostTables ht;
        for_each_cand(c, [&](auto cfg) { plan_candidate<decltype(cfg)>(b, c, base, off, 0, ht); });
        if (tables) (*tables)[c] = std::move(ht);
    }
    off = align256(off);
    for (int c = 0; c < NCAND; ++c) {
        if (!(b->cand_mask & (1 << c))) continue;
        CandPlan& cp = b->cand[c];
        const int S = 2 * b->nf, nf = b->nf;
        char* p = base ? base + off : nullptr;
        auto adv = [&](size_t bytes) { char* q = p; if (p) p += align256(bytes); off += align256(bytes); return q; };
        cp.d_segs = (BatchSeg*)adv(sizeof(BatchSeg) * std::max(1, S));
        cp.d_frags = (BatchFrag*)adv(sizeof(BatchFrag) * std::max(1, nf));
        cp.d_hist_prefix = (int64_t*)adv(sizeof(int64_t) * (S + 1));
        cp.d_pass_prefix = (int64_t*)adv(sizeof(int64_t) * 8 * (S + 1));
        cp.d_join_prefix = (int64_t*)adv(sizeof(int64_t) * (nf + 1));
    }
    return align256(off);
}

// Copies the planned descriptor tables to the workspace (asynchronously on
// `stream` when given; the host copies stay alive in the batch).
tqp_status upload_tables(tqp_batch* b, hipStream_t stream, bool sync) {
    const int S = 2 * b->nf, nf = b->nf;
    for (int c = 0; c < NCAND; ++c) {
        if (!(b->cand_mask & (1 << c))) continue;
        CandPlan& cp = b->cand[c];
        HostTables& ht = (*b->host)[c];
        struct { void* d; const void* h; size_t n; } cps[5] = {
            {cp.d_segs, ht.segs.data(), sizeof(BatchSeg) * S},
            {cp.d_frags, ht.frags.data(), sizeof(BatchFrag) * nf},
            {cp.d_hist_prefix, ht.hist_prefix.data(), sizeof(int64_t) * (S + 1)},
            {cp.d_pass_prefix, ht.pass_prefix.data(), sizeof(int64_t) * 8 * (S + 1)},
            {cp.d_join_prefix, ht.join_prefix.data(), sizeof(int64_t) * (nf + 1)}};
        for (auto& x : cps) {
            if (!x.n) continue;
            hipError_t e = sync ? hipMemcpy(x.d, x.h, x.n, hipMemcpyHostToDevice)
                                : hipMemcpyAsync(x.d, x.h, x.n, hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) return fail(TQP_ERR_HIP, "batch descriptor upload: %s", hipGetErrorString(e));
        }
    }
    return TQP_OK;
}

template <class Cfg>
tqp_status launch_candidate(tqp_batch* b, int c, hipStream_t s) {
    tqp_ctx* ctx = b->ctx;
    CandPlan& cp = b->cand[c];
    const int S = 2 * b->nf, F = b->nf;
    tqp_status st = fill_zero(b->ws + cp.zero_off, cp.zero_bytes, s, ctx);
    if (st != TQP_OK) return st;
    const int pgrid = (int)std::min<int64_t>(std::max<int64_t>(1, cp.hist_items), (int64_t)ctx->num_cus * 4);
    TQP_LAUNCH(ctx, s, "batch_hist",
               k_batch_hist<Cfg><<<pgrid, Cfg::BLOCK, 0, s>>>(cp.d_segs, S, cp.d_hist_prefix, cp.counters + 0, 0u,
                                                             ctx->d_err));
    for (int p = 0; p < cp.maxpass; ++p) {
        if (cp.pass_items[p] == 0) continue;
        const int g = (int)std::min<int64_t>(cp.pass_items[p], (int64_t)ctx->num_cus * 4);
        TQP_LAUNCH(ctx, s, "batch_pass",
                   k_batch_pass<Cfg><<<g, Cfg::BLOCK, 0, s>>>(cp.d_segs, S, cp.d_pass_prefix + (size_t)p * (S + 1), p,
                                                            cp.counters + 1 + p, ctx->d_err));
    }
    if (cp.join_tiles > 0) {
        TQP_LAUNCH(ctx, s, "batch_windows",
                   k_batch_windows<<<grid_for(cp.join_tiles, 256, 0), 256, 0, s>>>(cp.d_segs, cp.d_frags, F,
                                                                                   cp.d_join_prefix, BJCfg::TILE));
        const int g = (int)std::min<int64_t>(cp.join_tiles, (int64_t)ctx->num_cus * 4);
        TQP_LAUNCH(ctx, s, "batch_join",
                   k_batch_join<BJCfg><<<g, BJCfg::BLOCK, 0, s>>>(cp.d_segs, cp.d_frags, F, cp.d_join_prefix,
                                                                  cp.counters + 9, ctx->d_err));
    }
    TQP_LAUNCH(ctx, s, "batch_finalize", k_batch_finalize<<<grid_for(F, 64, 0), 64, 0, s>>>(cp.d_frags, F));
    return TQP_OK;
}

tqp_status run_candidate(tqp_batch* b, int c, hipStream_t s) {
    tqp_status st = TQP_OK;
    for_each_cand(c, [&](auto cfg) { st = launch_candidate<decltype(cfg)>(b, c, s); });
    return st;
}

void drop_graph(tqp_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

}  // namespace

namespace tqp {

tqp_status batch_prepare(tqp_ctx* ctx, const tqp_flags_fragment* frags, const tqp_flags_out* outs, int nf,
                         int cand_mask, int chosen, void* ws, size_t* ws_bytes, hipStream_t stream, bool sync,
                         tqp_batch** out) {
    if (!ctx || !ws_bytes || nf < 0 || (nf > 0 && (!frags || !outs)))
        return fail(TQP_ERR_INVALID, "batch: bad argument");
    for (int f = 0; f < nf; ++f) {
        tqp_status st = check_flags(&frags[f], &outs[f]);
        if (st != TQP_OK) return st;
    }
    tqp_batch* b = new tqp_batch;
    b->ctx = ctx;
    b->nf = nf;
    b->cand_mask = cand_mask;
    b->chosen = chosen;
    b->frags.assign(frags, frags + nf);
    b->outs.assign(outs, outs + nf);
    const size_t need = plan_all(b, nullptr, nullptr);
    if (!ws) {
        *ws_bytes = need;
        delete b;
        return TQP_OK;
    }
    tqp_status st = TQP_OK;
    if (!out) st = fail(TQP_ERR_INVALID, "batch: out is null");
    else if (*ws_bytes < need) st = fail(TQP_ERR_WORKSPACE, "batch workspace of %zu bytes, %zu needed", *ws_bytes, need);
    else if (reinterpret_cast<uintptr_t>(ws) & 255) st = fail(TQP_ERR_INVALID, "workspace not 256-byte aligned");
    if (st != TQP_OK) { delete b; return st; }
    b->ws = static_cast<char*>(ws);
    b->ws_bytes = *ws_bytes;
    b->host = new std::vector<HostTables>(NCAND);
    plan_all(b, b->ws, b->host);
    if ((st = upload_tables(b, stream, sync)) != TQP_OK) {
        delete b->host;
        delete b;
        return st;
    }
    *out = b;
    return TQP_OK;
}

tqp_status batch_launch(tqp_batch* b, hipStream_t stream) { return run_candidate(b, b->chosen, stream); }

void batch_free(tqp_batch* b) { tqp_batch_destroy(b); }

}  // namespace tqp

extern "C" {

tqp_status tqp_batch_create(tqp_ctx* ctx, const tqp_flags_fragment* frags, const tqp_flags_out* outs, int nf, void* ws,
                            size_t* ws_bytes, tqp_batch** out) {
    clear_error();
    return batch_prepare(ctx, frags, outs, nf, (1 << NCAND) - 1, CAND_R8, ws, ws_bytes, nullptr, true, out);
}

void tqp_batch_destroy(tqp_batch* b) {
    if (!b) return;
    drop_graph(b);
    delete b->host;
    delete b;
}

tqp_status tqp_batch_run(tqp_batch* b, hipStream_t stream) {
    clear_error();
    if (!b) return fail(TQP_ERR_INVALID, "null batch");
    return run_candidate(b, b->chosen, stream);
}

tqp_status tqp_batch_set_config(tqp_batch* b, int config) {
    clear_error();
    if (!b || config < 0 || config >= NCAND || !(b->cand_mask & (1 << config)))
        return fail(TQP_ERR_INVALID, "tqp_batch_set_config: config %d", config);
    if (config != b->chosen) drop_graph(b);
    b->chosen = config;
    return TQP_OK;
}

tqp_status tqp_batch_config(const tqp_batch* b, int* config, int* digit_bits, const char** name) {
    clear_error();
    if (!b) return fail(TQP_ERR_INVALID, "null batch");
    if (config) *config = b->chosen;
    if (digit_bits) *digit_bits = CAND_DIGITS[b->chosen];
    if (name) *name = CAND_NAMES[b->chosen];
    return TQP_OK;
}

tqp_status tqp_batch_autotune(tqp_batch* b, hipStream_t stream, int reps, float* times_ms) {
    clear_error();
    if (!b || reps < 1) return fail(TQP_ERR_INVALID, "tqp_batch_autotune: bad argument");
    const bool prof = b->ctx->prof;
    b->ctx->prof = false;
    hipEvent_t e0, e1;
    TQP_TRY_HIP(hipEventCreate(&e0));
    TQP_TRY_HIP(hipEventCreate(&e1));
    int best = b->chosen;
    float best_ms = 0.f;
    for (int c = 0; c < NCAND; ++c) {
        if (!(b->cand_mask & (1 << c))) continue;
        tqp_status st = run_candidate(b, c, stream);          // warm-up
        if (st != TQP_OK) { b->ctx->prof = prof; return st; }
        TQP_TRY_HIP(hipEventRecord(e0, stream));
        for (int r = 0; r < reps; ++r) {
            st = run_candidate(b, c, stream);
            if (st != TQP_OK) { b->ctx->prof = prof; return st; }
        }
        TQP_TRY_HIP(hipEventRecord(e1, stream));
        TQP_TRY_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        TQP_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
        ms /= reps;
        b->tuned_ms[c] = ms;
        if (times_ms) times_ms[c] = ms;
        if (best_ms == 0.f || ms < best_ms) { best_ms = ms; best = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->ctx->prof = prof;
    if (best != b->chosen) drop_graph(b);
    b->chosen = best;
    return TQP_OK;
}

tqp_status tqp_batch_capture(tqp_batch* b, hipStream_t stream) {
    clear_error();
    if (!b) return fail(TQP_ERR_INVALID, "null batch");
    if (!stream) return fail(TQP_ERR_INVALID, "graph capture needs a non-default stream");
    drop_graph(b);
    const bool prof = b->ctx->prof;
    b->ctx->prof = false;
    TQP_TRY_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    tqp_status st = run_candidate(b, b->chosen, stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(stream, &g);
    b->ctx->prof = prof;
    if (st != TQP_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return fail(TQP_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { drop_graph(b); return fail(TQP_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e)); }
    return TQP_OK;
}

tqp_status tqp_batch_replay(tqp_batch* b, hipStream_t stream) {
    clear_error();
    if (!b || !b->exec) return fail(TQP_ERR_INVALID, "tqp_batch_replay: no captured graph");
    TQP_TRY_HIP(hipGraphLaunch(b->exec, stream));
    return TQP_OK;
}

}  // extern "C"
