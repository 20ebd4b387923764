// Request loop over device-resident tables (continuous batching).
//
// Requests are stamped when submitted and queued.  A background thread
// admits them first-come first-served into free slots as long as the
// in-flight working set (each launch's exact workspace and outputs) fits the
// budget, launches each admitted request (or a run of waiting flags requests
// as one batch) on the slot's own stream, so launches of different slots
// overlap on the device, and turns the slot's completion event into host
// results.  Latency is arrival -> result visible on the host.
//
// Every slot has a context of its own: its own side stream (the mid-table
// sort of a custkey request forks onto it) and its own device error word,
// which the slot's last kernel moves into the slot's result block, so errors
// come back with the request that raised them.  The mid table can be sorted
// once when the server starts: it never changes, and custkey requests then
// join against that order (the plan rule of skipping the sort of sorted
// data) instead of sorting 8 bytes per mid row each time.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "fragment.hpp"

namespace {

using Clock = std::chrono::steady_clock;
constexpr int MAX_BATCH = 256;
constexpr int MAX_SLOTS = 64;

// Small results of one slot, copied to pinned host memory in one piece.
struct ResultBlock {
    int32_t fkey[MAX_BATCH][8];
    int64_t fsum[MAX_BATCH][8];
    int64_t fcnt[MAX_BATCH][8];
    double favg[MAX_BATCH][8];
    int64_t fng[MAX_BATCH];
    int64_t fjoin[MAX_BATCH];
    int64_t cng;
    int64_t cjoin;
    int32_t tk;
    int32_t pad;
    int32_t tkey[TQP_TOPK_MAX];
    int64_t tsum[TQP_TOPK_MAX];
    int64_t tcnt[TQP_TOPK_MAX];
    uint32_t err;              // the slot's device error bits of this launch
    uint32_t pad2;
};

struct Pending {
    uint64_t id;
    tqp_request req;
    double t_arrival;
};

struct Slot {
    tqp_ctx* ctx = nullptr;              // own error word and side stream
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    ResultBlock* d_res = nullptr;
    ResultBlock* h_res = nullptr;
    int32_t* ckey = nullptr;
    int64_t* csum = nullptr;
    int64_t* ccnt = nullptr;
    bool busy = false;
    std::vector<Pending> reqs;
    size_t footprint = 0;
    tqp_batch* batch = nullptr;
    double t_admit = 0;
    int status = TQP_OK;
};

}  // namespace

struct tqp_server {
    tqp_ctx* ctx = nullptr;
    tqp_server_config cfg{};
    Clock::time_point t0;
    int64_t gcap = 0;
    size_t cust_ws = 0;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv;          // work arrived / stop
    std::condition_variable cv_done;     // a request finished
    std::deque<Pending> queue;
    std::vector<tqp_result> done;
    uint64_t next_id = 1, submitted = 0, finished = 0, launches = 0;
    size_t inflight = 0, peak = 0;
    bool stop = false;
    std::thread worker;
    void* dev_block = nullptr;           // all slot device memory
    void* host_block = nullptr;          // all slot pinned result blocks
    uint32_t* mid_keys = nullptr;        // the mid table sorted by pk (presort_mid), and its custkeys
    uint32_t* mid_cust = nullptr;
};

namespace {

double now_s(const tqp_server* s) {
    return std::chrono::duration<double>(Clock::now() - s->t0).count();
}

tqp_cust_fragment cust_desc(const tqp_server* s, const tqp_request& r) {
    tqp_cust_fragment f{};
    f.fk = s->cfg.fk_mid;
    f.date = s->cfg.date;
    f.price = s->cfg.price;
    f.disc = s->cfg.disc;
    f.n_fact = s->cfg.n_fact;
    f.pk = s->mid_keys ? reinterpret_cast<const int32_t*>(s->mid_keys) : s->cfg.mid_pk;
    f.custkey = s->mid_keys ? reinterpret_cast<const int32_t*>(s->mid_cust) : s->cfg.mid_custkey;
    f.mid_sorted = s->mid_keys ? 1 : 0;
    f.n_mid = s->cfg.n_mid;
    f.D = r.D;
    f.key_bits = s->cfg.key_bits_mid;
    f.cust_bits = s->cfg.cust_bits;
    f.k = r.k;
    f.join_cap = s->cfg.n_fact;
    f.revenue_bits = s->cfg.revenue_bits;
    return f;
}

tqp_flags_fragment flags_desc(const tqp_server* s, const tqp_request& r) {
    tqp_flags_fragment f{};
    f.fk = s->cfg.fk_dim;
    f.date = s->cfg.date;
    f.price = s->cfg.price;
    f.disc = s->cfg.disc;
    f.flagA = s->cfg.flagA;
    f.flagB = s->cfg.flagB;
    f.row0 = r.row0;
    f.n_fact = r.n_rows;
    f.pk = s->cfg.dim_pk;
    f.seg = s->cfg.dim_seg;
    f.n_dim = s->cfg.n_dim;
    f.D = r.D;
    f.c = r.c;
    f.key_bits = s->cfg.key_bits_dim;
    return f;
}

tqp_flags_out flags_out(ResultBlock* d, int i) {
    tqp_flags_out o{};
    o.key = d->fkey[i];
    o.sum = d->fsum[i];
    o.cnt = d->fcnt[i];
    o.avg = d->favg[i];
    o.d_ngroups = &d->fng[i];
    o.d_join = &d->fjoin[i];
    return o;
}

tqp_cust_out cust_out(const tqp_server* s, const Slot& sl) {
    tqp_cust_out o{};
    o.key = sl.ckey;
    o.sum = sl.csum;
    o.cnt = sl.ccnt;
    o.gcap = s->gcap;
    o.d_ngroups = &sl.d_res->cng;
    o.d_join = &sl.d_res->cjoin;
    o.top_key = sl.d_res->tkey;
    o.top_sum = sl.d_res->tsum;
    o.top_cnt = sl.d_res->tcnt;
    o.d_topk = &sl.d_res->tk;
    return o;
}

// Workspace of a launch of the given requests (one custkey request, or one or
// more flags requests); 0 on error.
size_t launch_bytes(tqp_server* s, const std::vector<Pending>& reqs, Slot& sl) {
    size_t bytes = 0;
    if (reqs[0].req.kind == TQP_REQ_CUST) return s->cust_ws;
    if (reqs.size() == 1) {
        tqp_flags_fragment f = flags_desc(s, reqs[0].req);
        tqp_flags_out o = flags_out(sl.d_res, 0);
        if (tqp_fragment_flags(s->ctx, &f, &o, nullptr, &bytes, nullptr) != TQP_OK) return 0;
        return bytes;
    }
    std::vector<tqp_flags_fragment> fs;
    std::vector<tqp_flags_out> os;
    for (size_t i = 0; i < reqs.size(); ++i) {
        fs.push_back(flags_desc(s, reqs[i].req));
        os.push_back(flags_out(sl.d_res, (int)i));
    }
    if (tqp::batch_prepare(s->ctx, fs.data(), os.data(), (int)fs.size(), 1 << tqp::BATCH_CONFIG_DEFAULT,
                           tqp::BATCH_CONFIG_DEFAULT, nullptr, &bytes, nullptr, false, nullptr) != TQP_OK)
        return 0;
    return bytes;
}

// Moves the slot context's error bits into the result block and clears them
// (one thread; runs after the slot's last kernel on the slot's stream).
__global__ void k_take_errors(uint32_t* err, uint32_t* dst) {
    *dst = *err;
    *err = 0;
}

int launch(tqp_server* s, Slot& sl) {
    const std::vector<Pending>& reqs = sl.reqs;
    size_t bytes = sl.ws_bytes;
    tqp_status st;
    if (reqs[0].req.kind == TQP_REQ_CUST) {
        tqp_cust_fragment f = cust_desc(s, reqs[0].req);
        tqp_cust_out o = cust_out(s, sl);
        st = tqp_fragment_cust(sl.ctx, &f, &o, sl.ws, &bytes, sl.stream);
    } else if (reqs.size() == 1) {
        tqp_flags_fragment f = flags_desc(s, reqs[0].req);
        tqp_flags_out o = flags_out(sl.d_res, 0);
        st = tqp_fragment_flags(sl.ctx, &f, &o, sl.ws, &bytes, sl.stream);
    } else {
        std::vector<tqp_flags_fragment> fs;
        std::vector<tqp_flags_out> os;
        for (size_t i = 0; i < reqs.size(); ++i) {
            fs.push_back(flags_desc(s, reqs[i].req));
            os.push_back(flags_out(sl.d_res, (int)i));
        }
        st = tqp::batch_prepare(sl.ctx, fs.data(), os.data(), (int)fs.size(), 1 << tqp::BATCH_CONFIG_DEFAULT,
                                tqp::BATCH_CONFIG_DEFAULT, sl.ws, &bytes, sl.stream, false, &sl.batch);
        if (st == TQP_OK) st = tqp::batch_launch(sl.batch, sl.stream);
    }
    k_take_errors<<<1, 1, 0, sl.stream>>>(sl.ctx->d_err, &sl.d_res->err);     // also after a failed launch
    if (st != TQP_OK) return st;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(sl.h_res, sl.d_res, sizeof(ResultBlock), hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
        hipEventRecord(sl.done, sl.stream) != hipSuccess)
        return TQP_ERR_HIP;
    return TQP_OK;
}

void complete(tqp_server* s, Slot& sl, double t_done) {
    const ResultBlock& h = *sl.h_res;
    std::vector<tqp_result> out;
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
        const Pending& p = sl.reqs[i];
        tqp_result r;
        std::memset(&r, 0, sizeof r);
        r.id = p.id;
        r.tag = p.req.tag;
        r.kind = p.req.kind;
        r.status = sl.status;
        r.t_arrival = p.t_arrival;
        r.t_admit = sl.t_admit;
        r.t_done = t_done;
        r.slot = (int32_t)(&sl - s->slots.data());
        r.batch_size = (int32_t)sl.reqs.size();
        if (sl.status == TQP_OK && h.err) {
            r.dev_errors = h.err;
            r.status = (h.err & TQP_DEVERR_CAPACITY) ? TQP_ERR_CAPACITY : TQP_ERR_INVALID;
        }
        if (sl.status == TQP_OK) {
            if (p.req.kind == TQP_REQ_CUST) {
                r.join_rows = h.cjoin;
                r.groups = h.cng;
                r.top_n = h.tk;
                for (int k = 0; k < h.tk && k < TQP_TOPK_MAX; ++k) {
                    r.top_key[k] = h.tkey[k];
                    r.top_sum[k] = h.tsum[k];
                    r.top_cnt[k] = h.tcnt[k];
                }
            } else {
                r.join_rows = h.fjoin[i];
                r.groups = h.fng[i];
                for (int g = 0; g < h.fng[i] && g < 8; ++g) {
                    r.key[g] = h.fkey[i][g];
                    r.sum[g] = h.fsum[i][g];
                    r.cnt[g] = h.fcnt[i][g];
                    r.avg[g] = h.favg[i][g];
                }
            }
        }
        out.push_back(r);
    }
    if (sl.batch) {
        tqp::batch_free(sl.batch);
        sl.batch = nullptr;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto& r : out) s->done.push_back(r);
    s->finished += out.size();
    s->inflight -= sl.footprint;
    sl.busy = false;
    sl.reqs.clear();
    s->cv_done.notify_all();
}

void worker_main(tqp_server* s) {
    (void)hipSetDevice(s->ctx->device);
    for (;;) {
        bool any_busy = false;
        // 1. completions
        for (auto& sl : s->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) complete(s, sl, now_s(s));
            else if (q == hipErrorNotReady) any_busy = true;
            else { sl.status = TQP_ERR_HIP; complete(s, sl, now_s(s)); }
        }
        // 2. admission
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop && s->queue.empty() && !any_busy) break;
        while (!s->queue.empty()) {
            Slot* free_slot = nullptr;
            for (auto& sl : s->slots)
                if (!sl.busy) { free_slot = &sl; break; }
            if (!free_slot) break;
            std::vector<Pending> take;
            take.push_back(s->queue.front());
            if (take[0].req.kind == TQP_REQ_FLAGS) {
                for (size_t i = 1; i < s->queue.size() && (int)take.size() < s->cfg.max_batch; ++i) {
                    if (s->queue[i].req.kind != TQP_REQ_FLAGS) break;
                    take.push_back(s->queue[i]);
                }
            }
            size_t bytes = launch_bytes(s, take, *free_slot);
            while (take.size() > 1 && (bytes == 0 || bytes > free_slot->ws_bytes ||
                                       s->inflight + bytes + sizeof(ResultBlock) > s->cfg.budget_bytes)) {
                take.resize(take.size() / 2);
                bytes = launch_bytes(s, take, *free_slot);
            }
            const size_t fp = bytes + sizeof(ResultBlock);
            const bool never = bytes == 0 || bytes > free_slot->ws_bytes || fp > s->cfg.budget_bytes;
            if (!never && s->inflight + fp > s->cfg.budget_bytes) break;      // wait for memory to free up
            for (size_t i = 0; i < take.size(); ++i) s->queue.pop_front();
            Slot& sl = *free_slot;
            sl.busy = true;
            sl.reqs = std::move(take);
            sl.footprint = never ? 0 : fp;
            sl.t_admit = now_s(s);
            sl.status = TQP_OK;
            s->inflight += sl.footprint;
            if (s->inflight > s->peak) s->peak = s->inflight;
            lk.unlock();
            int st = never ? TQP_ERR_CAPACITY : launch(s, sl);
            if (st == TQP_OK) {
                ++s->launches;
                any_busy = true;
            } else {
                sl.status = st;
                complete(s, sl, now_s(s));
            }
            lk.lock();
        }
        if (!any_busy) {
            if (s->queue.empty() && !s->stop) s->cv.wait_for(lk, std::chrono::milliseconds(50));
        } else {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(10));
        }
    }
}

// The mid table sorted by pk once, with its custkeys (the resident order
// custkey requests join against).  Uses the first slot's context; a key
// outside key_bits_mid fails the server's creation.
tqp_status presort_mid(tqp_server* s) {
    const int64_t m = s->cfg.n_mid;
    tqp_ctx* c = s->slots[0].ctx;
    if (hipMalloc(&s->mid_keys, (size_t)m * 8) != hipSuccess) {
        s->mid_keys = nullptr;
        return tqp::fail(TQP_ERR_HIP, "tqp_server_create: %lld bytes for the sorted mid table", (long long)m * 8);
    }
    s->mid_cust = s->mid_keys + m;
    size_t bytes = 0;
    tqp_status st = tqp_sort(c, s->cfg.mid_pk, s->cfg.mid_custkey, m, nullptr, s->cfg.key_bits_mid,
                             reinterpret_cast<int32_t*>(s->mid_keys), reinterpret_cast<int32_t*>(s->mid_cust),
                             nullptr, &bytes, nullptr);
    if (st != TQP_OK) return st;
    void* ws = nullptr;
    if (hipMalloc(&ws, bytes > 0 ? bytes : 256) != hipSuccess)
        return tqp::fail(TQP_ERR_HIP, "tqp_server_create: %zu bytes of sort workspace", bytes);
    hipStream_t stream = nullptr;      // the slots' streams do not exist yet
    st = tqp_sort(c, s->cfg.mid_pk, s->cfg.mid_custkey, m, nullptr, s->cfg.key_bits_mid,
                  reinterpret_cast<int32_t*>(s->mid_keys), reinterpret_cast<int32_t*>(s->mid_cust), ws, &bytes,
                  stream);
    uint32_t err = 0;
    const tqp_status es = tqp_ctx_errors(c, stream, &err, 1);
    (void)hipFree(ws);
    if (st != TQP_OK) return st;
    if (es != TQP_OK) return es;
    if (err) return tqp::fail(TQP_ERR_INVALID, "tqp_server_create: sorting the mid table raised device errors %#x", err);
    return TQP_OK;
}

}  // namespace

using namespace tqp;

extern "C" {

tqp_status tqp_server_create(tqp_ctx* ctx, const tqp_server_config* cfg, tqp_server** out) {
    clear_error();
    if (!ctx || !cfg || !out) return fail(TQP_ERR_INVALID, "tqp_server_create: null argument");
    if (cfg->slots < 1 || cfg->slots > MAX_SLOTS || cfg->max_batch < 1 || cfg->max_batch > MAX_BATCH)
        return fail(TQP_ERR_INVALID, "tqp_server_create: slots %d, max_batch %d", cfg->slots, cfg->max_batch);
    if (cfg->n_fact < 1 || cfg->n_mid < 1 || cfg->n_dim < 1 || cfg->max_flags_rows < 1 ||
        cfg->max_flags_rows > cfg->n_fact)
        return fail(TQP_ERR_INVALID, "tqp_server_create: table sizes");
    if (cfg->revenue_bits != 0 && cfg->revenue_bits != 32 && cfg->revenue_bits != 64)
        return fail(TQP_ERR_UNSUPPORTED, "tqp_server_create: revenue_bits = %d (0, 32 or 64)", cfg->revenue_bits);
    tqp_server* s = new tqp_server;
    s->ctx = ctx;
    s->cfg = *cfg;
    s->t0 = Clock::now();
    s->gcap = std::min<int64_t>(cfg->n_fact, int64_t(1) << norm_key_bits(cfg->cust_bits));
    s->slots.resize(cfg->slots);
    for (auto& sl : s->slots) {
        tqp_status cs = tqp_ctx_create(ctx->device, &sl.ctx);
        if (cs != TQP_OK) {
            tqp_server_destroy(s);
            return cs;
        }
        sl.ctx->digit_bits = ctx->digit_bits;
    }
    if (cfg->presort_mid) {
        tqp_status ps = presort_mid(s);
        if (ps != TQP_OK) {
            tqp_server_destroy(s);
            return ps;
        }
    }
    // Workspace of each kind of launch, from the library's own size queries.
    tqp_request rc{};
    rc.kind = TQP_REQ_CUST;
    rc.D = 0;
    rc.k = TQP_TOPK_MAX;
    tqp_cust_fragment cf = cust_desc(s, rc);
    Slot probe;
    ResultBlock fake;          // only addresses are taken during size queries
    probe.d_res = &fake;
    probe.ckey = reinterpret_cast<int32_t*>(&fake);
    probe.csum = reinterpret_cast<int64_t*>(&fake);
    probe.ccnt = reinterpret_cast<int64_t*>(&fake);
    tqp_cust_out co = cust_out(s, probe);
    size_t cb = 0;
    tqp_status st = tqp_fragment_cust(ctx, &cf, &co, nullptr, &cb, nullptr);
    if (st != TQP_OK) { tqp_server_destroy(s); return st; }
    s->cust_ws = cb;
    std::vector<Pending> big((size_t)cfg->max_batch);
    for (auto& p : big) {
        p.req.kind = TQP_REQ_FLAGS;
        p.req.row0 = 0;
        p.req.n_rows = cfg->max_flags_rows;
    }
    size_t fb = launch_bytes(s, big, probe);
    std::vector<Pending> one(big.begin(), big.begin() + 1);
    const size_t f1 = launch_bytes(s, one, probe);
    if (fb == 0 || f1 == 0) {
        tqp_server_destroy(s);
        return fail(TQP_ERR_INVALID, "tqp_server_create: flags size query failed");
    }
    const size_t ws = Arena::align(std::max(cb, std::max(fb, f1)));
    const size_t gbytes = Arena::align((size_t)s->gcap * 4) + 2 * Arena::align((size_t)s->gcap * 8);
    const size_t per_slot = ws + gbytes + Arena::align(sizeof(ResultBlock));
    if (hipMalloc(&s->dev_block, per_slot * cfg->slots) != hipSuccess) {
        s->dev_block = nullptr;
        tqp_server_destroy(s);
        return fail(TQP_ERR_HIP, "tqp_server_create: %zu bytes of slot memory", per_slot * cfg->slots);
    }
    if (hipHostMalloc(&s->host_block, sizeof(ResultBlock) * cfg->slots) != hipSuccess) {
        s->host_block = nullptr;
        tqp_server_destroy(s);
        return fail(TQP_ERR_HIP, "tqp_server_create: pinned result memory");
    }
    for (int i = 0; i < cfg->slots; ++i) {
        Slot& sl = s->slots[i];
        char* p = static_cast<char*>(s->dev_block) + per_slot * i;
        sl.ws = p;
        sl.ws_bytes = ws;
        p += ws;
        sl.ckey = reinterpret_cast<int32_t*>(p);
        p += Arena::align((size_t)s->gcap * 4);
        sl.csum = reinterpret_cast<int64_t*>(p);
        p += Arena::align((size_t)s->gcap * 8);
        sl.ccnt = reinterpret_cast<int64_t*>(p);
        p += Arena::align((size_t)s->gcap * 8);
        sl.d_res = reinterpret_cast<ResultBlock*>(p);
        sl.h_res = static_cast<ResultBlock*>(s->host_block) + i;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            tqp_server_destroy(s);
            return fail(TQP_ERR_HIP, "tqp_server_create: stream or event");
        }
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return TQP_OK;
}

void tqp_server_destroy(tqp_server* s) {
    if (!s) return;
    if (s->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv.notify_all();
        s->worker.join();
    }
    for (auto& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.batch) tqp::batch_free(sl.batch);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.ctx) tqp_ctx_destroy(sl.ctx);
    }
    if (s->mid_keys) (void)hipFree(s->mid_keys);
    if (s->dev_block) (void)hipFree(s->dev_block);
    if (s->host_block) (void)hipHostFree(s->host_block);
    delete s;
}

double tqp_server_now(const tqp_server* s) { return s ? now_s(s) : 0.0; }

tqp_status tqp_server_submit(tqp_server* s, const tqp_request* req, uint64_t* id) {
    clear_error();
    if (!s || !req) return fail(TQP_ERR_INVALID, "tqp_server_submit: null argument");
    if (req->kind == TQP_REQ_CUST) {
        if (req->k < 1 || req->k > TQP_TOPK_MAX) return fail(TQP_ERR_INVALID, "tqp_server_submit: k = %d", req->k);
    } else if (req->kind == TQP_REQ_FLAGS) {
        if (req->row0 < 0 || req->n_rows < 0 || req->n_rows > s->cfg.max_flags_rows ||
            req->row0 + req->n_rows > s->cfg.n_fact)
            return fail(TQP_ERR_INVALID, "tqp_server_submit: rows [%lld, +%lld)", (long long)req->row0,
                        (long long)req->n_rows);
    } else {
        return fail(TQP_ERR_INVALID, "tqp_server_submit: kind %d", req->kind);
    }
    Pending p;
    p.req = *req;
    p.t_arrival = now_s(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        p.id = s->next_id++;
        ++s->submitted;
        s->queue.push_back(p);
    }
    s->cv.notify_all();
    if (id) *id = p.id;
    return TQP_OK;
}

tqp_status tqp_server_poll(tqp_server* s, tqp_result* out, int cap, int* n) {
    clear_error();
    if (!s || !n || (cap > 0 && !out)) return fail(TQP_ERR_INVALID, "tqp_server_poll: null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    const int k = (int)std::min<size_t>((size_t)std::max(cap, 0), s->done.size());
    for (int i = 0; i < k; ++i) out[i] = s->done[i];
    s->done.erase(s->done.begin(), s->done.begin() + k);
    *n = k;
    return TQP_OK;
}

tqp_status tqp_server_drain(tqp_server* s) {
    clear_error();
    if (!s) return fail(TQP_ERR_INVALID, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->finished >= s->submitted; });
    return TQP_OK;
}

tqp_status tqp_server_stats(const tqp_server* s, uint64_t* submitted, uint64_t* finished, uint64_t* launches,
                            size_t* peak_bytes) {
    clear_error();
    if (!s) return fail(TQP_ERR_INVALID, "null server");
    tqp_server* m = const_cast<tqp_server*>(s);
    std::lock_guard<std::mutex> lk(m->mu);
    if (submitted) *submitted = s->submitted;
    if (finished) *finished = s->finished;
    if (launches) *launches = s->launches;
    if (peak_bytes) *peak_bytes = s->peak;
    return TQP_OK;
}

}  // extern "C"
