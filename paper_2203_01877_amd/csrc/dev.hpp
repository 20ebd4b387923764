// Device primitives for CDNA4 (gfx950): 64-lane wavefront ballots and scans,
// agent-scope atomics for decoupled look-back, and small block-wide helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>

namespace tqp {

constexpr int WAVE = 64;

// Error bits OR-ed into the context's device flag word by kernels.
enum : uint32_t {
    FLAG_KEY_RANGE = 1u,      // a key had bits above the declared key width (or was negative)
    FLAG_SPIN_LIMIT = 2u,     // a look-back wait hit its bound (never expected)
    FLAG_CAPACITY = 4u,       // an output count exceeded the caller's capacity
    FLAG_VALUE_RANGE = 8u,    // a value was outside its declared width
};

__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (uint64_t(1) << lane_id()) - 1; }
__device__ __forceinline__ uint64_t lanemask_le() {
    return lane_id() == 63 ? ~uint64_t(0) : (uint64_t(2) << lane_id()) - 1;
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }

// ---------------------------------------------------------------- atomics
template <class T>
__device__ __forceinline__ T ld_relaxed(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_relaxed(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T atomic_add(T* p, T v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void set_flag(uint32_t* flags, uint32_t bit) {
    if (flags) __hip_atomic_fetch_or(flags, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bound on look-back polls of one predecessor.  A predecessor always holds a
// lower dynamic tile id, is already resident, and publishes without waiting on
// its successors, so the wait ends; the bound only turns a bug into an error
// flag instead of a hang.
constexpr uint32_t SPIN_LIMIT = 1u << 22;

// ---------------------------------------------------------------- wave scans
// Sums across the 64 lanes of a wave (all lanes active) on DPP lane moves:
// an ALU operand modifier, so a step costs a few cycles instead of an LDS
// permute round trip.  row_shr:n moves values n lanes up within each row of
// 16 lanes; row_bcast:15 / row_bcast:31 copy the last lane of a row into the
// rows selected by the row mask.  Lanes with no source (or outside the row
// mask) read 0.
namespace dpp {
constexpr int ROW_SHR1 = 0x111, ROW_SHR2 = 0x112, ROW_SHR4 = 0x114, ROW_SHR8 = 0x118;
constexpr int ROW_BCAST15 = 0x142, ROW_BCAST31 = 0x143;
// fill: what lanes with no source read
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t mov(uint32_t v, uint32_t fill = 0) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t mov(uint64_t v, uint64_t fill = 0) {
    return ((uint64_t)mov<CTRL, ROWS>((uint32_t)(v >> 32), (uint32_t)(fill >> 32)) << 32) |
           mov<CTRL, ROWS>((uint32_t)v, (uint32_t)fill);
}
// Inclusive scan with op (identity id) over the lanes of unsigned 4- or
// 8-byte words.
template <class U, class Op>
__device__ __forceinline__ U scan(U x, U id, Op op) {
    x = op(x, mov<ROW_SHR1, 0xF>(x, id));
    x = op(x, mov<ROW_SHR2, 0xF>(x, id));
    x = op(x, mov<ROW_SHR4, 0xF>(x, id));
    x = op(x, mov<ROW_SHR8, 0xF>(x, id));
    x = op(x, mov<ROW_BCAST15, 0xA>(x, id));
    x = op(x, mov<ROW_BCAST31, 0xC>(x, id));
    return x;
}
}  // namespace dpp

template <class T>
using lane_word_t = typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type;

// Inclusive prefix sum over the lanes (4- or 8-byte integers, wrapping).
template <class T>
__device__ __forceinline__ T wave_incl_sum(T v) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte integers");
    lane_word_t<T> x = (lane_word_t<T>)v;
    x += dpp::mov<dpp::ROW_SHR1, 0xF>(x);
    x += dpp::mov<dpp::ROW_SHR2, 0xF>(x);
    x += dpp::mov<dpp::ROW_SHR4, 0xF>(x);
    x += dpp::mov<dpp::ROW_SHR8, 0xF>(x);        // rows of 16 scanned
    x += dpp::mov<dpp::ROW_BCAST15, 0xA>(x);     // rows 1 and 3 add the last lane of rows 0 and 2
    x += dpp::mov<dpp::ROW_BCAST31, 0xC>(x);     // rows 2 and 3 add lane 31
    return (T)x;
}

// Value of lane `lane` (the same for every lane of the wave) in every lane.
template <class T>
__device__ __forceinline__ T wave_read(T v, int lane) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte values");
    if constexpr (sizeof(T) == 4) {
        return (T)(lane_word_t<T>)__builtin_amdgcn_readlane((int)(lane_word_t<T>)v, lane);
    } else {
        const uint64_t x = (uint64_t)v;
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
        return (T)(((uint64_t)hi << 32) | lo);
    }
}

// Value of lane `src` (its own for every lane) in every lane: the LDS
// crossbar permute, no LDS memory.
template <class T>
__device__ __forceinline__ T wave_shfl(T v, int src) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte values");
    if constexpr (sizeof(T) == 4) {
        return (T)(lane_word_t<T>)__builtin_amdgcn_ds_bpermute(src << 2, (int)(lane_word_t<T>)v);
    } else {
        const uint64_t x = (uint64_t)v;
        const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)x);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)(x >> 32));
        return (T)(((uint64_t)hi << 32) | lo);
    }
}

// The lane whose run holds item q of the wave's runs laid end to end, given
// every lane's exclusive start (non-decreasing over the lanes): the last lane
// whose start is <= q.  Every lane of the wave must take part.
__device__ __forceinline__ int wave_run_owner(int64_t excl, int64_t q) {
    int src = 0;
#pragma unroll
    for (int step = WAVE / 2; step >= 1; step >>= 1) {
        const int64_t e = wave_shfl(excl, src + step);
        if (e <= q) src += step;
    }
    return src;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
    return wave_read(wave_incl_sum(v), WAVE - 1);
}

// Maximum / minimum over the lanes of unsigned 4- or 8-byte words.
template <class U>
__device__ __forceinline__ U wave_max(U v) {
    static_assert(std::is_unsigned<U>::value && (sizeof(U) == 4 || sizeof(U) == 8), "unsigned words");
    return wave_read(dpp::scan<U>(v, U(0), [](U a, U b) { return a > b ? a : b; }), WAVE - 1);
}
template <class U>
__device__ __forceinline__ U wave_min(U v) {
    static_assert(std::is_unsigned<U>::value && (sizeof(U) == 4 || sizeof(U) == 8), "unsigned words");
    return wave_read(dpp::scan<U>(v, ~U(0), [](U a, U b) { return a < b ? a : b; }), WAVE - 1);
}

// Segmented inclusive scan across the wave: a lane with head=true starts a
// new segment.  Returns the running sum of the lane's segment up to the lane.
template <class T>
__device__ __forceinline__ T wave_seg_incl_sum(T v, uint64_t headmask) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte integers");
    // (sum, segment-started) pairs: a lane whose window already holds a head
    // keeps its sum, otherwise it adds the window before it
    lane_word_t<T> x = (lane_word_t<T>)v;
    uint32_t f = (uint32_t)(headmask >> lane_id()) & 1u;
    auto step = [&](auto xs, uint32_t fs) {
        x = f ? x : x + xs;
        f |= fs;
    };
    step(dpp::mov<dpp::ROW_SHR1, 0xF>(x), dpp::mov<dpp::ROW_SHR1, 0xF>(f));
    step(dpp::mov<dpp::ROW_SHR2, 0xF>(x), dpp::mov<dpp::ROW_SHR2, 0xF>(f));
    step(dpp::mov<dpp::ROW_SHR4, 0xF>(x), dpp::mov<dpp::ROW_SHR4, 0xF>(f));
    step(dpp::mov<dpp::ROW_SHR8, 0xF>(x), dpp::mov<dpp::ROW_SHR8, 0xF>(f));
    step(dpp::mov<dpp::ROW_BCAST15, 0xA>(x), dpp::mov<dpp::ROW_BCAST15, 0xA>(f));
    step(dpp::mov<dpp::ROW_BCAST31, 0xC>(x), dpp::mov<dpp::ROW_BCAST31, 0xC>(f));
    return (T)x;
}

// ---------------------------------------------------------------- block scans
// Exclusive scan of one value per thread over the block; *total receives the
// block sum.  lds must hold BLOCK/WAVE elements.
template <int BLOCK, class T>
__device__ __forceinline__ T block_excl_sum(T v, T* lds, T* total) {
    constexpr int W = BLOCK / WAVE;
    const int w = threadIdx.x / WAVE;
    T inc = wave_incl_sum(v);
    if (lane_id() == WAVE - 1) lds[w] = inc;
    __syncthreads();
    T wave_off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        T x = lds[i];
        if (i < w) wave_off += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return wave_off + inc - v;
}

// In-place exclusive scan of an LDS array of `count` elements (count a multiple
// of BLOCK or smaller than BLOCK); returns the total.  scratch holds BLOCK/WAVE.
template <int BLOCK, class T>
__device__ __forceinline__ T block_excl_scan_array(T* arr, int count, T* scratch) {
    const int per = (count + BLOCK - 1) / BLOCK;          // consecutive elements per thread
    const int base = threadIdx.x * per;
    T local = 0;
    for (int i = 0; i < per; ++i)
        if (base + i < count) local += arr[base + i];
    T total;
    T off = block_excl_sum<BLOCK>(local, scratch, &total);
    for (int i = 0; i < per; ++i) {
        if (base + i < count) {
            T x = arr[base + i];
            arr[base + i] = off;
            off += x;
        }
    }
    __syncthreads();
    return total;
}

// ---------------------------------------------------------------- look-back (64-bit)
// Status word of a tile in a single-value decoupled look-back: two flag bits
// over a 62-bit non-negative value.
constexpr uint64_t ST64_AGG = uint64_t(1) << 62;
constexpr uint64_t ST64_INC = uint64_t(2) << 62;
constexpr uint64_t ST64_VAL = (uint64_t(1) << 62) - 1;

// Called by all 64 lanes of one wave: publishes the tile's aggregate, reads
// the 64 preceding status words at once (one memory round trip), adds
// aggregates up to the nearest inclusive prefix, and repeats further back if
// none of the 64 had one.  Publishes the tile's inclusive prefix and returns
// the exclusive one (the same value in every lane).
__device__ __forceinline__ int64_t lookback64(uint64_t* status, int64_t tile, int64_t agg,
                                              uint32_t* flags) {
    const int l = lane_id();
    if (tile == 0) {
        if (l == 0) st_relaxed(status, ST64_INC | (uint64_t)agg);
        return 0;
    }
    if (l == 0) st_relaxed(status + tile, ST64_AGG | (uint64_t)agg);
    int64_t excl = 0;
    int64_t j = tile - 1;
    uint32_t spins = 0;
    while (j >= 0) {
        const int64_t idx = j - l;
        const uint64_t s = idx >= 0 ? ld_relaxed(status + idx) : ST64_INC;
        const uint64_t f = s & ~ST64_VAL;
        const uint64_t inc = ballot(f == ST64_INC);
        const uint64_t zero = ballot(f == 0);
        const int first_inc = inc ? __ffsll((unsigned long long)inc) - 1 : WAVE;
        const int first_zero = zero ? __ffsll((unsigned long long)zero) - 1 : WAVE;
        if (first_zero < first_inc) {          // a predecessor has not published yet
            excl += wave_sum(l < first_zero ? (int64_t)(s & ST64_VAL) : (int64_t)0);
            j -= first_zero;
            if (++spins > SPIN_LIMIT) { if (l == 0) set_flag(flags, FLAG_SPIN_LIMIT); break; }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        const int upto = first_inc < WAVE ? first_inc + 1 : WAVE;
        excl += wave_sum(l < upto ? (int64_t)(s & ST64_VAL) : (int64_t)0);
        j -= upto;
        if (first_inc < WAVE) break;
    }
    if (l == 0) st_relaxed(status + tile, ST64_INC | (uint64_t)(excl + agg));
    return excl;
}

// ---------------------------------------------------------------- wave search
// First index i in [0, n) with pred(a[i]) true, pred = (a[i] > key) when
// upper, else (a[i] >= key); n if none.  a is sorted ascending.  The whole
// wave takes part: each round probes 64 evenly spaced positions, so a search
// over n elements takes about log64(n) dependent loads.
__device__ __forceinline__ int64_t wave_bound(const uint32_t* a, int64_t n, uint32_t key, bool upper) {
    int64_t lo = 0, hi = n;   // the answer lies in [lo, hi]
    const int l = lane_id();
    while (lo < hi) {
        const int64_t span = hi - lo;
        const int64_t step = (span + WAVE - 1) / WAVE;
        const int64_t p = lo + (int64_t)l * step;
        bool t = true;
        if (p < hi) {
            const uint32_t x = a[p];
            t = upper ? (x > key) : (x >= key);
        }
        const uint64_t m = ballot(t);
        if (m == 0) {
            lo = lo + (int64_t)(WAVE - 1) * step + 1;
        } else {
            const int f = __ffsll((unsigned long long)m) - 1;
            const int64_t first_true = lo + (int64_t)f * step;
            if (f == 0) {
                hi = lo;
            } else {
                lo = lo + (int64_t)(f - 1) * step + 1;
                hi = first_true < hi ? first_true : hi;
            }
        }
    }
    return lo;
}

// Plain binary searches (one thread).
template <class T>
__device__ __forceinline__ int lower_bound_lds(const T* a, int n, T key) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}
template <class T>
__device__ __forceinline__ int upper_bound_lds(const T* a, int n, T key) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] <= key) lo = mid + 1; else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ int64_t lower_bound_glb(const uint32_t* a, int64_t lo, int64_t hi, uint32_t key) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ int64_t upper_bound_glb(const uint32_t* a, int64_t lo, int64_t hi, uint32_t key) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------- fill
__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v);

}  // namespace tqp
