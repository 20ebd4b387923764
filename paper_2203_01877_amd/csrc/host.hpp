// Host-side plumbing shared by the C ABI entry points: the context, error
// reporting, the workspace arena and the radix-sort launch sequence.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <type_traits>
#include <vector>

#include "../../include/tqp.h"
#include "dev.hpp"
#include "radix.hpp"

struct tqp_prof_rec {
    const char* name;
    hipEvent_t a, b;
};

struct tqp_ctx {
    int device = 0;
    int num_cus = 256;
    uint32_t* d_err = nullptr;   // device error word (TQP_DEVERR_* bits)
    int digit_bits = 8;          // radix digit width of sorts
    bool prof = false;           // record a pair of events around every launch
    std::vector<tqp_prof_rec> recs;
    std::vector<hipEvent_t> pool;
    hipStream_t side = nullptr;  // second stream for independent work inside one call
    hipEvent_t fork = nullptr, join = nullptr;
};

namespace tqp {

tqp_status fail(tqp_status st, const char* fmt, ...);
void clear_error();

#define TQP_TRY_HIP(call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return ::tqp::fail(TQP_ERR_HIP, "%s: %s", #call,             \
                                                  hipGetErrorString(e_));                  \
    } while (0)

#define TQP_CHECK_LAUNCH() TQP_TRY_HIP(hipGetLastError())

// Per-launch timing (tqp_ctx_set_profiling): events recorded on the launch
// stream right before and after the kernel.
int prof_begin(tqp_ctx* c, hipStream_t s, const char* name);
void prof_end(tqp_ctx* c, hipStream_t s, int idx);

#define TQP_LAUNCH(ctx, s, name, ...)                                  \
    do {                                                               \
        const int pi_ = ::tqp::prof_begin((ctx), (s), (name));         \
        __VA_ARGS__;                                                   \
        TQP_CHECK_LAUNCH();                                            \
        ::tqp::prof_end((ctx), (s), pi_);                              \
    } while (0)

constexpr int64_t MAX_ELEMS = (int64_t(1) << 30) - 1;

// Two-region workspace: a region the library clears before use (counters,
// histograms, look-back status words) followed by plain scratch buffers.
// Planning runs twice with the same reservations: once without a base pointer
// to size both regions, once with the caller's buffer to place them.
struct Arena {
    char* base = nullptr;
    size_t zoff = 0, soff = 0, zsize = 0;
    static size_t align(size_t x) { return (x + 255) & ~size_t(255); }
    template <class T>
    T* zero(int64_t n) {
        size_t o = align(zoff);
        zoff = o + (size_t)(n > 0 ? n : 0) * sizeof(T);
        return base ? reinterpret_cast<T*>(base + o) : nullptr;
    }
    template <class T>
    T* scratch(int64_t n) {
        size_t o = align(soff);
        soff = o + (size_t)(n > 0 ? n : 0) * sizeof(T);
        return base ? reinterpret_cast<T*>(base + zsize + o) : nullptr;
    }
    size_t zero_bytes() const { return align(zoff); }
    size_t total() const { return align(zoff) + align(soff); }
};

// Runs plan(Arena&) once to size, checks or reports the workspace, then runs
// it again over the caller's buffer and clears the zero region.
template <class Plan>
tqp_status with_workspace(tqp_ctx* ctx, void* ws, size_t* ws_bytes, hipStream_t stream, Plan&& plan,
                          Arena& live) {
    if (!ws_bytes) return fail(TQP_ERR_INVALID, "ws_bytes is null");
    Arena sizing;
    plan(sizing);
    const size_t need = sizing.total();
    if (!ws) {
        *ws_bytes = need;
        return TQP_OK;
    }
    if (*ws_bytes < need)
        return fail(TQP_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", *ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(TQP_ERR_INVALID, "workspace not 256-byte aligned");
    live.base = static_cast<char*>(ws);
    live.zsize = sizing.zero_bytes();
    plan(live);
    (void)ctx;
    return TQP_OK;
}

tqp_status fill_zero(void* p, size_t bytes, hipStream_t stream, tqp_ctx* ctx = nullptr);

// Checks a postfix expression program over ncols columns and, for n > 0,
// evaluates it into out (n or *d_n rows) as out_mode says: int64 values; one
// byte per row, 1 where the value is nonzero (a predicate's keep column); or
// int32 values, a value outside int32 raising the value-range flag.  Column c
// is read at idx[c][row] when idx and idx[c] are given.  tqp_eval and the
// general fragments use it.
enum : int { XOUT_I64 = 0, XOUT_FLAG = 1, XOUT_I32 = 2 };
tqp_status eval_program(tqp_ctx* ctx, const tqp_column* cols, const int32_t* const* idx, int ncols, int64_t n,
                        const int64_t* d_n, const tqp_xinstr* prog, int nprog, void* out, hipStream_t stream,
                        const char* who, const char* label, int out_mode = XOUT_I64);

// Looks up this device's scratch array of tqp_filter_noalloc (the device must
// be current); done once per device, from tqp_ctx_create.
tqp_status noalloc_setup(int device);

// Fork: work launched on ctx->side after this call starts after everything
// already queued on s.  Join: s waits for everything queued on ctx->side.
inline tqp_status side_fork(tqp_ctx* ctx, hipStream_t s) {
    TQP_TRY_HIP(hipEventRecord(ctx->fork, s));
    TQP_TRY_HIP(hipStreamWaitEvent(ctx->side, ctx->fork, 0));
    return TQP_OK;
}
inline tqp_status side_join(tqp_ctx* ctx, hipStream_t s) {
    TQP_TRY_HIP(hipEventRecord(ctx->join, ctx->side));
    TQP_TRY_HIP(hipStreamWaitEvent(s, ctx->join, 0));
    return TQP_OK;
}

inline int grid_for(int64_t work, int64_t per_block, int64_t cap_blocks) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (cap_blocks > 0 && g > cap_blocks) g = cap_blocks;
    return (int)g;
}

// Digit passes for keys of key_bits bits with digits of at most rb bits,
// spread evenly (e.g. 25 bits at 8 -> 7, 6, 6, 6).
inline PassDesc make_passes(int key_bits, int rb) {
    PassDesc pd{};
    if (key_bits < 1) key_bits = 1;
    int np = (key_bits + rb - 1) / rb;
    if (np > 8) np = 8;
    int base = key_bits / np, rem = key_bits % np, sh = 0;
    for (int p = 0; p < np; ++p) {
        pd.bits[p] = base + (p < rem ? 1 : 0);
        pd.shift[p] = sh;
        sh += pd.bits[p];
    }
    pd.npass = np;
    return pd;
}

inline uint32_t key_mask_for(int key_bits) {
    return key_bits >= 32 ? 0xFFFFFFFFu : ((1u << key_bits) - 1);
}

inline int norm_key_bits(int key_bits) { return (key_bits <= 0 || key_bits > 31) ? 31 : key_bits; }

// ------------------------------------------------------------------ radix sort
template <class Cfg, class V>
struct RadixBufs {
    PassDesc pd{};
    int64_t ntiles = 0;
    uint32_t* hist = nullptr;       // npass * RADIX
    uint32_t* status = nullptr;     // per look-back pass: ntiles * RADIX
    uint32_t* counters = nullptr;   // npass tile counters
    // pre-counted first pass (when the histogram kernel runs): per tile and
    // chunk counts, chunk bases
    int64_t nchunks = 0;
    int tpc = 0;
    uint32_t* pre = nullptr;        // ntiles * RADIX
    uint32_t* ctot = nullptr;       // nchunks * RADIX
    uint32_t* cbase = nullptr;      // nchunks * RADIX
    int64_t* d_cnt = nullptr;       // elements that take part (from the histogram)
    uint32_t* ktmp = nullptr;
    V* vtmp = nullptr;
};

// skip_low: the lowest skip_low key bits are left unsorted (the passes cover
// bits [skip_low, key_bits)).  counted: the caller launches with the
// histogram kernel, whose tile counts spare the first pass its look-back
// (false when the histogram comes from elsewhere).
template <class Cfg0, class V>
RadixBufs<Cfg0, V> radix_reserve(Arena& a, int64_t n_upper, int key_bits, int skip_low = 0, bool counted = true) {
    using Cfg = typename Cfg0::template ForVal<V>;
    RadixBufs<Cfg0, V> b;
    b.pd = make_passes(key_bits - skip_low, Cfg::RADIX_BITS);
    for (int p = 0; p < b.pd.npass; ++p) b.pd.shift[p] += skip_low;
    b.ntiles = (n_upper + Cfg::TILE - 1) / Cfg::TILE;
    b.hist = a.zero<uint32_t>((int64_t)b.pd.npass * Cfg::RADIX);
    if (counted && b.ntiles > 0) {
        b.nchunks = b.ntiles < COUNT_CHUNKS ? b.ntiles : COUNT_CHUNKS;
        b.tpc = (int)((b.ntiles + b.nchunks - 1) / b.nchunks);
        b.nchunks = (b.ntiles + b.tpc - 1) / b.tpc;          // every chunk holds at least one tile
        b.pre = a.scratch<uint32_t>(b.ntiles * Cfg::RADIX);
        b.ctot = a.scratch<uint32_t>(b.nchunks * Cfg::RADIX);
        b.cbase = a.scratch<uint32_t>(b.nchunks * Cfg::RADIX);
    }
    const int look_passes = b.pd.npass - (b.pre ? 1 : 0);
    b.status = a.zero<uint32_t>((int64_t)look_passes * b.ntiles * Cfg::RADIX);
    b.counters = a.zero<uint32_t>(b.pd.npass);
    b.d_cnt = a.zero<int64_t>(1);
    if (b.pd.npass > 1) {
        b.ktmp = a.scratch<uint32_t>(n_upper);
        if constexpr (ValBytes<V>::value != 0) b.vtmp = a.scratch<V>(n_upper);
    }
    return b;
}

// Histogram (unless the caller accumulated it already) and one pass kernel per
// digit.  Pass 0 reads src0; later passes read the previous pass's output,
// bounded by the count of elements that took part (*count_src).
// first_label / pass_label (string literals, optional) name the first and the
// later pass kernels in the per-launch profile.  [p_begin, p_end) limits the
// call to those passes (the histogram runs with pass 0), so a sort can be
// split over two calls, e.g. around other work, with the same arguments.
template <class Cfg0, class V, int Tag = 0, class Src0>
tqp_status radix_launch(const RadixBufs<Cfg0, V>& b, const Src0& src0, int64_t n_upper, bool run_hist,
                        const int64_t* count_src, uint32_t key_mask, uint32_t* keys_out, V* vals_out,
                        tqp_ctx* ctx, hipStream_t s, const char* first_label = nullptr,
                        const char* pass_label = nullptr, int p_begin = 0, int p_end = 8) {
    using Cfg = typename Cfg0::template ForVal<V>;
    const int np = b.pd.npass;
    const int pe = p_end < np ? p_end : np;
    const int64_t tiles = b.ntiles;
    if (tiles == 0) return TQP_OK;
    const bool counted = run_hist && b.pre;
    if (run_hist) count_src = b.d_cnt;
    if (p_begin > 0) {
        // a later part of a split sort: the histogram has run with pass 0
    } else if (counted) {
        TQP_LAUNCH(ctx, s, "radix_hist",
                   k_radix_hist_tiles<Cfg, Src0><<<(unsigned)b.nchunks, Cfg::BLOCK, 0, s>>>(
                       src0, b.pd, key_mask, b.hist, b.d_cnt, ctx->d_err, b.pre, b.ctot, b.tpc, tiles));
        TQP_LAUNCH(ctx, s, "radix_chunk_scan",
                   k_radix_chunk_scan<<<1u << b.pd.bits[0], CHUNK_SCAN_BLOCK, 0, s>>>(
                       b.ctot, (int)b.nchunks, b.hist, Cfg::RADIX, b.cbase));
        count_src = b.d_cnt;
    } else if (run_hist) {
        const int g = grid_for(n_upper, (int64_t)Cfg::BLOCK * HIST_ITEMS * 4, (int64_t)ctx->num_cus * 2);
        TQP_LAUNCH(ctx, s, "radix_hist",
                   k_radix_hist<Cfg, Src0><<<g, Cfg::BLOCK, 0, s>>>(src0, b.pd, key_mask, b.hist, b.d_cnt,
                                                                    ctx->d_err));
        count_src = b.d_cnt;
    }
    constexpr int VB = ValBytes<V>::value;
    const char* pairs_name = VB == 8 ? "radix_pass_pairs_v8" : VB == 4 ? "radix_pass_pairs_v4" : "radix_pass_pairs_v0";
    const char* first_name = std::is_same<Src0, SrcPairs<V>>::value ? pairs_name
                             : VB == 8 ? "radix_pass_fused_v8" : VB == 4 ? "radix_pass_fused_v4" : "radix_pass_fused_v0";
    if (pass_label) pairs_name = pass_label;
    if (first_label) first_name = first_label;
    const uint32_t* in_k = nullptr;
    const V* in_v = nullptr;
    if (p_begin > 0) {                        // the output of the pass before p_begin
        const bool prev_final = ((np - p_begin) % 2) == 0;
        in_k = prev_final ? keys_out : b.ktmp;
        in_v = prev_final ? vals_out : b.vtmp;
    }
    for (int p = p_begin; p < pe; ++p) {
        const bool to_final = ((np - 1 - p) % 2) == 0;
        uint32_t* ok = to_final ? keys_out : b.ktmp;
        V* ov = to_final ? vals_out : b.vtmp;
        DstPairs<V> dst{ok, ov};
        const int sp = counted ? p - 1 : p;     // look-back passes only have status words
        uint32_t* st = sp >= 0 ? b.status + (int64_t)sp * tiles * Cfg::RADIX : nullptr;
        if (p == 0 && counted) {
            TQP_LAUNCH(ctx, s, first_name,
                       k_radix_pass_counted<Cfg, Src0, V, Tag><<<(unsigned)tiles, Cfg::BLOCK, 0, s>>>(
                           src0, dst, b.pd.shift[p], b.pd.bits[p], PassCounts{b.pre, b.cbase, b.tpc},
                           ctx->d_err));
        } else if (p == 0) {
            TQP_LAUNCH(ctx, s, first_name,
                       k_radix_pass<Cfg, Src0, V, Tag><<<(unsigned)tiles, Cfg::BLOCK, 0, s>>>(
                           src0, dst, b.pd.shift[p], b.pd.bits[p], b.hist + p * Cfg::RADIX, st, b.counters + p,
                           ctx->d_err));
        } else {
            SrcPairs<V> src{in_k, in_v, n_upper, count_src};
            TQP_LAUNCH(ctx, s, pairs_name,
                       k_radix_pass<Cfg, SrcPairs<V>, V, Tag><<<(unsigned)tiles, Cfg::BLOCK, 0, s>>>(
                           src, dst, b.pd.shift[p], b.pd.bits[p], b.hist + p * Cfg::RADIX, st, b.counters + p,
                           ctx->d_err));
        }
        in_k = ok;
        in_v = ov;
    }
    return TQP_OK;
}

// Digit-width dispatch: the context's digit width picks the configuration.
using R4 = RadixCfg<4, 256, 8, 8>;
using R8 = RadixCfg<8, 512, 12, 8, 16>;
using R11 = RadixCfg<11, 512, 8, 8>;

template <class F>
tqp_status with_radix_cfg(int digit_bits, F&& f) {
    switch (digit_bits) {
        case 4: return f(R4{});
        case 11: return f(R11{});
        default: return f(R8{});
    }
}

}  // namespace tqp
