// Context, error reporting and small utility kernels of the C ABI.
#include <cstring>
#include <string>

#include "host.hpp"
#include "join.hpp"
#include "radix.hpp"
#include "segreduce.hpp"
#include "topk.hpp"

namespace tqp {

static thread_local char g_err[512] = "";

tqp_status fail(tqp_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

void clear_error() { g_err[0] = 0; }

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ void k_copy_u128(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ void k_fill_u128(uint4* p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const uint4 z = make_uint4(0, 0, 0, 0);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = z;
}

int prof_begin(tqp_ctx* c, hipStream_t s, const char* name) {
    if (!c || !c->prof) return -1;
    hipEvent_t ev[2];
    for (int i = 0; i < 2; ++i) {
        if (!c->pool.empty()) {
            ev[i] = c->pool.back();
            c->pool.pop_back();
        } else if (hipEventCreate(&ev[i]) != hipSuccess) {
            return -1;
        }
    }
    if (hipEventRecord(ev[0], s) != hipSuccess) return -1;
    c->recs.push_back({name, ev[0], ev[1]});
    return (int)c->recs.size() - 1;
}

void prof_end(tqp_ctx* c, hipStream_t s, int idx) {
    if (!c || idx < 0 || idx >= (int)c->recs.size()) return;
    (void)hipEventRecord(c->recs[idx].b, s);
}

// Clears bytes (a multiple of 4) at p with a kernel (no memset node, so the
// sequence stays safe to capture and replay as a graph).
tqp_status fill_zero(void* p, size_t bytes, hipStream_t stream, tqp_ctx* ctx) {
    if (bytes == 0) return TQP_OK;
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    if ((a & 15) == 0 && (bytes & 15) == 0) {
        const int64_t n = (int64_t)(bytes / 16);
        TQP_LAUNCH(ctx, stream, "fill",
                   k_fill_u128<<<grid_for(n, 256 * 4, 2048), 256, 0, stream>>>(static_cast<uint4*>(p), n));
    } else {
        const int64_t n = (int64_t)(bytes / 4);
        TQP_LAUNCH(ctx, stream, "fill",
                   k_fill_u32<<<grid_for(n, 256 * 4, 2048), 256, 0, stream>>>(static_cast<uint32_t*>(p), n, 0u));
    }
    return TQP_OK;
}

__global__ void k_join_windows(const uint32_t* lkey, int64_t nl_upper, const int64_t* d_nl,
                               const uint32_t* rkey, int64_t nr_upper, const int64_t* d_nr, int tile_size,
                               int64_t* win, int lowb, const int64_t* rbstart, int64_t nbkt) {
    int64_t nl = nl_upper, nr = nr_upper;
    if (d_nl) { const int64_t t = *d_nl; nl = t < nl ? t : nl; }
    if (d_nr) { const int64_t t = *d_nr; nr = t < nr ? t : nr; }
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ntiles = (nl + tile_size - 1) / tile_size;
    if (t >= ntiles) return;
    const int64_t i0 = t * tile_size;
    const int64_t i1 = (i0 + tile_size < nl ? i0 + tile_size : nl) - 1;
    uint32_t kmin, kmax;
    tile_key_range(TileGeo{0, 0, lkey[i0], lkey[i1]}, lowb, kmin, kmax);
    if (rbstart) {
        // keys beyond the declared width (flagged elsewhere) are clamped, never indexed
        const int64_t b0 = kmin >> lowb, b1 = ((int64_t)kmax >> lowb) + 1;
        win[2 * t] = rbstart[b0 < nbkt ? b0 : nbkt];
        win[2 * t + 1] = rbstart[b1 < nbkt ? b1 : nbkt];
        return;
    }
    const int64_t lo = lower_bound_glb(rkey, 0, nr, kmin);
    win[2 * t] = lo;
    win[2 * t + 1] = upper_bound_glb(rkey, lo, nr, kmax);
}

__global__ void k_bucket_bounds(const uint32_t* keys, int64_t n_upper, const int64_t* d_n, int lowb,
                                int64_t nbuckets, int64_t* starts) {
    int64_t n = n_upper;
    if (d_n) { const int64_t t = *d_n; n = t < n ? t : n; }
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nbuckets) return;
    starts[b] = b == nbuckets ? n : lower_bound_glb(keys, 0, n, (uint32_t)(b << lowb));
}

__global__ void __launch_bounds__(CHUNK_SCAN_BLOCK)
k_radix_chunk_scan(const uint32_t* ctot, int nchunks, const uint32_t* hist0, int R, uint32_t* cbase) {
    __shared__ uint32_t scratch[CHUNK_SCAN_BLOCK / WAVE];
    const int d = blockIdx.x;
    const int c = threadIdx.x;
    uint32_t below = 0;
    for (int i = threadIdx.x; i < d; i += CHUNK_SCAN_BLOCK) below += hist0[i];
    uint32_t base;
    block_excl_sum<CHUNK_SCAN_BLOCK>(below, scratch, &base);
    const uint32_t v = c < nchunks ? ctot[(int64_t)c * R + d] : 0;
    uint32_t tot;
    const uint32_t excl = block_excl_sum<CHUNK_SCAN_BLOCK>(v, scratch, &tot);
    if (c < nchunks) cbase[(int64_t)c * R + d] = base + excl;
}

__global__ void __launch_bounds__(FINISH_BLOCK)
k_finish_sort(const uint32_t* kin, const uint32_t* vin, int64_t n, uint32_t* kout, uint32_t* vout, int lowb,
              int64_t* bstart, const int64_t* d_n) {
    if (d_n) {
        const int64_t t = *d_n;
        n = t < n ? t : n;
    }
    constexpr int U = 8;                              // loads in flight per thread
    constexpr int W = FINISH_BLOCK / WAVE;
    constexpr int SLICE = FINISH_SPAN / W;            // counters scanned by one wave
    __shared__ uint32_t cnt[FINISH_SPAN];
    __shared__ uint32_t s_wtot[W];
    __shared__ int64_t s_lo, s_hi;
    const int tid = threadIdx.x, w = tid / WAVE, l = lane_id();
    const uint32_t base = (uint32_t)blockIdx.x << FINISH_LOG2;
    if (w == 0) {
        const int64_t lo = wave_bound(kin, n, base, false);
        if (l == 0) s_lo = lo;
    } else if (w == 1) {
        const int64_t hi = wave_bound(kin, n, base + FINISH_SPAN, false);
        if (l == 0) s_hi = hi;
    }
    for (int i = tid; i < FINISH_SPAN; i += FINISH_BLOCK) cnt[i] = 0;
    __syncthreads();
    const int64_t lo = s_lo, hi = s_hi;
    const int nb_span = bstart ? 1 << (FINISH_LOG2 - lowb) : 0;          // buckets per span
    if (bstart && blockIdx.x == gridDim.x - 1 && tid == 0) bstart[(int64_t)gridDim.x * nb_span] = hi;
    if (lo >= hi) {
        for (int q = tid; q < nb_span; q += FINISH_BLOCK) bstart[(int64_t)blockIdx.x * nb_span + q] = lo;
        return;
    }
    // keys outside the span occur only in inputs that are not sorted on the
    // high bits (a broken key width): skipped, never indexed
    for (int64_t i0 = lo + tid; i0 < hi; i0 += (int64_t)FINISH_BLOCK * U) {
        uint32_t d[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {          // clamped index: no branch between the loads
            const int64_t i = i0 + (int64_t)j * FINISH_BLOCK;
            d[j] = kin[i < hi ? i : hi - 1] - base;
            if (i >= hi) d[j] = FINISH_SPAN;
        }
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (d[j] < FINISH_SPAN) atomicAdd(&cnt[d[j]], 1u);
    }
    __syncthreads();
    // exclusive scan of the counters: wave w scans its slice 64 entries at a
    // time (one per lane), then adds the totals of the slices before it
    uint32_t carry = 0;
    for (int c = w * SLICE; c < (w + 1) * SLICE; c += WAVE) {
        const uint32_t x = cnt[c + l];
        const uint32_t inc = wave_incl_sum(x);
        cnt[c + l] = carry + inc - x;
        carry += wave_read(inc, WAVE - 1);
    }
    if (l == 0) s_wtot[w] = carry;
    __syncthreads();
    uint32_t off = 0;
    for (int ww = 0; ww < w; ++ww) off += s_wtot[ww];
    if (off)
        for (int c = w * SLICE; c < (w + 1) * SLICE; c += WAVE) cnt[c + l] += off;
    __syncthreads();
    if (bstart) {
        for (int q = tid; q < nb_span; q += FINISH_BLOCK)
            bstart[(int64_t)blockIdx.x * nb_span + q] = lo + cnt[q << lowb];
        __syncthreads();                        // read before the scatter below advances the counters
    }
    for (int64_t i0 = lo + tid; i0 < hi; i0 += (int64_t)FINISH_BLOCK * U) {
        uint32_t k[U], v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int64_t i = i0 + (int64_t)j * FINISH_BLOCK;
            const int64_t ic = i < hi ? i : hi - 1;
            k[j] = kin[ic];
            v[j] = vin[ic];
            if (i >= hi) k[j] = base + FINISH_SPAN;
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint32_t d = k[j] - base;
            if (d < FINISH_SPAN) {
                const int64_t p = lo + atomicAdd(&cnt[d], 1u);
                kout[p] = k[j];
                vout[p] = v[j];
            }
        }
    }
}

__global__ void k_avg(const int64_t* sa, const int64_t* cnt, double* avg, const int64_t* d_ngroups,
                      int64_t gcap) {
    int64_t G = *d_ngroups;
    if (G > gcap) G = gcap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G; g += stride)
        avg[g] = (double)sa[g] / (double)cnt[g];
}

__global__ void k_topk_filter(const int32_t* gkey, const int64_t* gsum, int64_t n_upper, const int64_t* d_n,
                              const int64_t* thr, TopCand* out, int64_t* d_out) {
    // Survivors of a block's contiguous chunk are counted in LDS first, so the
    // shared output counter sees one atomic per block.
    constexpr int CHUNK_ITEMS = 8;
    __shared__ int32_t s_cnt;
    __shared__ int64_t s_base;
    int64_t n = n_upper;
    if (d_n) { const int64_t t = *d_n; n = t < n ? t : n; }
    const int64_t T = thr[0];
    const int64_t chunk = (int64_t)blockDim.x * CHUNK_ITEMS;
    for (int64_t c0 = (int64_t)blockIdx.x * chunk; c0 < n; c0 += (int64_t)gridDim.x * chunk) {
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        int64_t sm[CHUNK_ITEMS];
#pragma unroll
        for (int j = 0; j < CHUNK_ITEMS; ++j) {
            const int64_t g = c0 + (int64_t)j * blockDim.x + threadIdx.x;
            sm[j] = g < n ? gsum[g] : INT64_MIN;
        }
        bool keep[CHUNK_ITEMS];
        int32_t slot[CHUNK_ITEMS];
#pragma unroll
        for (int j = 0; j < CHUNK_ITEMS; ++j) {
            const int64_t g = c0 + (int64_t)j * blockDim.x + threadIdx.x;
            keep[j] = g < n && sm[j] >= T;
            const uint64_t m = ballot(keep[j]);
            int32_t wbase = 0;
            if (lane_id() == 0 && m) wbase = atomicAdd(&s_cnt, (int32_t)popc64(m));
            wbase = wave_read(wbase, 0);
            slot[j] = wbase + popc64(m & lanemask_lt());
        }
        __syncthreads();
        if (threadIdx.x == 0) s_base = s_cnt ? atomic_add(d_out, (int64_t)s_cnt) : 0;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CHUNK_ITEMS; ++j) {
            if (keep[j]) {
                const int64_t g = c0 + (int64_t)j * blockDim.x + threadIdx.x;
                TopCand x;
                x.sum = sm[j];
                x.key = gkey[g];
                x.idx = (int32_t)g;
                out[s_base + slot[j]] = x;
            }
        }
        __syncthreads();
    }
}

}  // namespace tqp

using namespace tqp;

extern "C" {

const char* tqp_last_error(void) { return g_err; }

tqp_status tqp_ctx_create(int device, tqp_ctx** out) {
    clear_error();
    if (!out) return fail(TQP_ERR_INVALID, "out is null");
    int ndev = 0;
    TQP_TRY_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(TQP_ERR_INVALID, "device %d of %d", device, ndev);
    TQP_TRY_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    TQP_TRY_HIP(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(TQP_ERR_UNSUPPORTED, "built for gfx950, device is %s", prop.gcnArchName);
    if (noalloc_setup(device) != TQP_OK) return TQP_ERR_HIP;
    tqp_ctx* c = new tqp_ctx;
    c->device = device;
    c->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    if (hipMalloc(&c->d_err, 256) != hipSuccess) {
        delete c;
        return fail(TQP_ERR_HIP, "hipMalloc of the error word failed");
    }
    if (hipMemset(c->d_err, 0, 256) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(c->d_err);
        delete c;
        return fail(TQP_ERR_HIP, "clearing the error word failed");
    }
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->join, hipEventDisableTiming) != hipSuccess) {
        (void)hipFree(c->d_err);
        delete c;
        return fail(TQP_ERR_HIP, "creating the side stream failed");
    }
    *out = c;
    return TQP_OK;
}

void tqp_ctx_destroy(tqp_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& r : ctx->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->join) (void)hipEventDestroy(ctx->join);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    (void)hipFree(ctx->d_err);
    delete ctx;
}

tqp_status tqp_ctx_set_profiling(tqp_ctx* ctx, int on) {
    clear_error();
    if (!ctx) return fail(TQP_ERR_INVALID, "null context");
    ctx->prof = on != 0;
    return TQP_OK;
}

tqp_status tqp_ctx_profile_read(tqp_ctx* ctx, hipStream_t stream, tqp_prof_entry* out, int cap, int* n) {
    clear_error();
    if (!ctx || !n || (cap > 0 && !out)) return fail(TQP_ERR_INVALID, "null argument");
    TQP_TRY_HIP(hipStreamSynchronize(stream));
    TQP_TRY_HIP(hipDeviceSynchronize());
    TQP_TRY_HIP(hipStreamSynchronize(ctx->side));
    int w = 0;
    for (auto& r : ctx->recs) {
        if (w < cap) {
            float ms = 0.f;
            TQP_TRY_HIP(hipEventElapsedTime(&ms, r.a, r.b));
            std::snprintf(out[w].name, sizeof out[w].name, "%s", r.name);
            out[w].ms = ms;
        }
        ++w;
        ctx->pool.push_back(r.a);
        ctx->pool.push_back(r.b);
    }
    ctx->recs.clear();
    *n = w;
    return TQP_OK;
}

tqp_status tqp_ctx_errors(tqp_ctx* ctx, hipStream_t stream, uint32_t* errors, int clear) {
    clear_error();
    if (!ctx || !errors) return fail(TQP_ERR_INVALID, "null argument");
    TQP_TRY_HIP(hipStreamSynchronize(stream));
    TQP_TRY_HIP(hipMemcpy(errors, ctx->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (clear) {
        TQP_TRY_HIP(hipMemset(ctx->d_err, 0, sizeof(uint32_t)));
        TQP_TRY_HIP(hipDeviceSynchronize());
    }
    return TQP_OK;
}

tqp_status tqp_copy(tqp_ctx* ctx, void* dst, const void* src, size_t bytes, hipStream_t stream) {
    clear_error();
    if (!ctx || (bytes && (!dst || !src))) return fail(TQP_ERR_INVALID, "tqp_copy: null argument");
    if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src) | bytes) & 15)
        return fail(TQP_ERR_INVALID, "tqp_copy: pointers and size must be multiples of 16 bytes");
    if (!bytes) return TQP_OK;
    const int64_t n = (int64_t)(bytes / 16);
    TQP_LAUNCH(ctx, stream, "copy",
               k_copy_u128<<<grid_for(n, 256 * 8, (int64_t)ctx->num_cus * 8), 256, 0, stream>>>(
                   static_cast<const uint4*>(src), static_cast<uint4*>(dst), n));
    return TQP_OK;
}

tqp_status tqp_ctx_set_digit_bits(tqp_ctx* ctx, int bits) {
    clear_error();
    if (!ctx) return fail(TQP_ERR_INVALID, "null context");
    if (bits == 0) bits = 8;
    if (bits != 4 && bits != 8 && bits != 11) return fail(TQP_ERR_UNSUPPORTED, "digit width %d", bits);
    ctx->digit_bits = bits;
    return TQP_OK;
}

}  // extern "C"
