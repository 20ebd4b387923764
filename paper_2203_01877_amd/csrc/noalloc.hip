// tqp_filter_noalloc: the filter of tqp_filter without any allocation and
// without a caller workspace, for callers that cannot allocate.
//
// tqp_filter's only scratch is one 64-bit look-back word per tile and a tile
// counter.  Here they live in a file-scope device array of a fixed size; its
// address on each device is looked up once, when a context is created on that
// device (hipGetSymbolAddress with the device current), and kept per device.
// Host code never passes the array's own name to a kernel or a copy: on the
// host that name is a stand-in, not a device address.
//
// Every call on a device uses that device's one array, and each call clears
// the part it uses with a fill kernel first (no memset node, so a caller may
// capture the call in a graph).  Calls that overlap in time on one device
// race on the array.
#include <mutex>

#include "filter.hpp"
#include "host.hpp"

namespace tqp {
namespace {

constexpr int NA_BLOCK = 256, NA_ITEMS = 16;
constexpr int64_t NA_TILE = NA_BLOCK * NA_ITEMS;
constexpr size_t NA_COUNTER_BYTES = 256;       // the tile counter, then the status words
constexpr int64_t NA_MAX_TILES = (TQP_NOALLOC_SCRATCH_BYTES - NA_COUNTER_BYTES) / 8;
static_assert(NA_MAX_TILES * NA_TILE == TQP_FILTER_NOALLOC_MAX_ROWS, "header limit matches the scratch layout");

__device__ __align__(256) unsigned char scratch[TQP_NOALLOC_SCRATCH_BYTES];

constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mu;
void* na_ptr[NA_MAX_DEVICES] = {};

}  // namespace

// Looks up this device's copy of the scratch array (the device must be
// current); later calls for the same device reuse the address.
tqp_status noalloc_setup(int device) {
    if (device < 0 || device >= NA_MAX_DEVICES) return fail(TQP_ERR_UNSUPPORTED, "device %d", device);
    std::lock_guard<std::mutex> lk(na_mu);
    if (na_ptr[device]) return TQP_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(TQP_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    na_ptr[device] = p;
    return TQP_OK;
}

static void* noalloc_scratch(int device) {
    if (device < 0 || device >= NA_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(na_mu);
    return na_ptr[device];
}

}  // namespace tqp

using namespace tqp;

extern "C" tqp_status tqp_filter_noalloc(tqp_ctx* ctx, const tqp_column* cols, int ncols, int64_t n,
                                         const tqp_pred* preds, int npreds, const int32_t* carry,
                                         int32_t* out_rowid, int32_t* out_carry, int64_t cap, int64_t* d_count,
                                         hipStream_t stream) {
    clear_error();
    if (!ctx || !d_count || (cap > 0 && !out_rowid) || n < 0 || cap < 0 || npreds < 0 || ncols < 0)
        return fail(TQP_ERR_INVALID, "tqp_filter_noalloc: null pointer or negative size");
    if (n > TQP_FILTER_NOALLOC_MAX_ROWS)
        return fail(TQP_ERR_UNSUPPORTED, "tqp_filter_noalloc: n = %lld is above the scratch limit of %lld rows",
                    (long long)n, (long long)TQP_FILTER_NOALLOC_MAX_ROWS);
    if (npreds > FILTER_MAX_PREDS) return fail(TQP_ERR_UNSUPPORTED, "tqp_filter_noalloc: %d predicates", npreds);
    if (n > 0 && cap > 0 && (carry == nullptr) != (out_carry == nullptr))
        return fail(TQP_ERR_INVALID, "tqp_filter_noalloc: carry and out_carry must both be given or both null");
    if (n == 0 || cap == 0) { carry = nullptr; out_carry = nullptr; }
    FilterPreds fp{};
    fp.np = npreds;
    for (int p = 0; p < npreds; ++p) {
        const tqp_pred& q = preds[p];
        if (q.col < 0 || q.col >= ncols || !cols || (n > 0 && !cols[q.col].data))
            return fail(TQP_ERR_INVALID, "tqp_filter_noalloc: predicate %d names column %d", p, q.col);
        if (q.op < TQP_LT || q.op > TQP_NE) return fail(TQP_ERR_INVALID, "tqp_filter_noalloc: op %d", q.op);
        const int t = cols[q.col].type;
        if (t != TQP_I8 && t != TQP_I32 && t != TQP_I64)
            return fail(TQP_ERR_INVALID, "tqp_filter_noalloc: type %d", t);
        fp.col[p] = cols[q.col].data;
        fp.type[p] = t;
        fp.op[p] = q.op;
        fp.k[p] = q.k;
    }
    char* base = static_cast<char*>(noalloc_scratch(ctx->device));
    if (!base) return fail(TQP_ERR_HIP, "tqp_filter_noalloc: no scratch address for device %d", ctx->device);
    const int64_t tiles = (n + NA_TILE - 1) / NA_TILE;
    uint32_t* counter = reinterpret_cast<uint32_t*>(base);
    uint64_t* status = reinterpret_cast<uint64_t*>(base + NA_COUNTER_BYTES);
    // counter and the status words of this call's tiles start at zero
    tqp_status st = fill_zero(base, NA_COUNTER_BYTES + (size_t)((tiles * 8 + 15) & ~int64_t(15)), stream, ctx);
    if (st != TQP_OK) return st;
    TQP_LAUNCH(ctx, stream, "filter_noalloc",
               k_filter<NA_BLOCK, NA_ITEMS><<<grid_for(n, NA_TILE, 0), NA_BLOCK, 0, stream>>>(
                   fp, n, carry, out_rowid, out_carry, cap, d_count, status, counter, ctx->d_err));
    return TQP_OK;
}
