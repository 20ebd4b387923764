// Gather by row position: the late materialisation step of Section 5.2.
// Joins return row positions; the columns a later operator needs (the next
// join's key in a chain of joins, an aggregated value) are read through them.
// Writes are coalesced, reads land where the positions point.
#include "dev.hpp"
#include "host.hpp"

namespace tqp {
namespace {

constexpr int GA_BLOCK = 256;
constexpr int GA_ITEMS = 4;

template <class T>
__global__ void __launch_bounds__(GA_BLOCK)
k_gather(const T* src, int64_t nsrc, const int32_t* idx, int64_t n_upper, const int64_t* d_n, T* out,
         uint32_t* flags) {
    int64_t n = n_upper;
    if (d_n) { const int64_t t = *d_n; n = t < n ? t : n; }
    const int64_t step = (int64_t)gridDim.x * GA_BLOCK * GA_ITEMS;
    for (int64_t base = (int64_t)blockIdx.x * GA_BLOCK * GA_ITEMS; base < n; base += step) {
        int32_t r[GA_ITEMS];
#pragma unroll
        for (int j = 0; j < GA_ITEMS; ++j) {
            const int64_t i = base + (int64_t)j * GA_BLOCK + threadIdx.x;
            r[j] = i < n ? idx[i] : -1;
        }
        T v[GA_ITEMS];
        bool bad = false;
#pragma unroll
        for (int j = 0; j < GA_ITEMS; ++j) {
            const bool ok = r[j] >= 0 && r[j] < nsrc;
            const int64_t i = base + (int64_t)j * GA_BLOCK + threadIdx.x;
            bad |= i < n && r[j] >= nsrc;
            v[j] = ok ? src[r[j]] : T(-1);
        }
        if (bad) set_flag(flags, FLAG_KEY_RANGE);
#pragma unroll
        for (int j = 0; j < GA_ITEMS; ++j) {
            const int64_t i = base + (int64_t)j * GA_BLOCK + threadIdx.x;
            if (i < n) out[i] = v[j];
        }
    }
}

}  // namespace
}  // namespace tqp

using namespace tqp;

extern "C" {

tqp_status tqp_gather(tqp_ctx* ctx, const void* src, int64_t nsrc, int elem_bytes, const int32_t* idx, int64_t n,
                      const int64_t* d_n, void* out, hipStream_t stream) {
    clear_error();
    if (!ctx || n < 0 || nsrc < 0 || (n > 0 && (!idx || !out)) || (nsrc > 0 && !src))
        return fail(TQP_ERR_INVALID, "tqp_gather: null pointer or negative size");
    if (elem_bytes != 4 && elem_bytes != 8) return fail(TQP_ERR_INVALID, "tqp_gather: elem_bytes must be 4 or 8");
    if (n > MAX_ELEMS) return fail(TQP_ERR_UNSUPPORTED, "tqp_gather: n = %lld", (long long)n);
    if (n == 0) return TQP_OK;
    const int grid = grid_for(n, (int64_t)GA_BLOCK * GA_ITEMS, (int64_t)ctx->num_cus * 16);
    if (elem_bytes == 4) {
        TQP_LAUNCH(ctx, stream, "gather",
                   k_gather<int32_t><<<grid, GA_BLOCK, 0, stream>>>(static_cast<const int32_t*>(src), nsrc, idx, n,
                                                                    d_n, static_cast<int32_t*>(out), ctx->d_err));
    } else {
        TQP_LAUNCH(ctx, stream, "gather",
                   k_gather<int64_t><<<grid, GA_BLOCK, 0, stream>>>(static_cast<const int64_t*>(src), nsrc, idx, n,
                                                                    d_n, static_cast<int64_t*>(out), ctx->d_err));
    }
    return TQP_OK;
}

}  // extern "C"
