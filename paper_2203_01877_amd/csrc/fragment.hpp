// Workspace layouts of the fused fragments (shared by the single-fragment
// entry points and the batch runner).
#pragma once
#include "host.hpp"
#include "join.hpp"
#include "radix.hpp"
#include "segreduce.hpp"
#include "topk.hpp"

namespace tqp {

using JCfgFrag = JoinCfg<256, 4, 4096>;
using SCfgFrag = SegCfg<256, 16>;

template <class Cfg>
struct FlagsBufs {
    RadixBufs<Cfg, uint32_t> fact, dim;
    uint64_t* jstatus = nullptr;
    uint32_t* jcounter = nullptr;
    int64_t* d_join = nullptr;
    int64_t* acc = nullptr;
    uint32_t *fkeys = nullptr, *fvals = nullptr, *dkeys = nullptr, *dvals = nullptr;
};

// Levels of the top-k reduction: each keeps k of every CH candidates, so with
// k <= CH / 2 a level at least halves the set; 32 levels cover 2^30 groups.
constexpr int TOPK_MAX_LEVELS = 32;

struct TopkBufs {
    int levels = 0;
    int64_t n_in[TOPK_MAX_LEVELS] = {0};
    int64_t blocks[TOPK_MAX_LEVELS] = {0};
    TopCand* cand[TOPK_MAX_LEVELS] = {nullptr};
};

TopkBufs topk_reserve(Arena& a, int64_t n_upper, int k);
tqp_status topk_launch(const TopkBufs& t, const int32_t* key, const int64_t* sum, const int64_t* cnt,
                       const int64_t* d_n, int k, int32_t* out_key, int64_t* out_sum, int64_t* out_cnt,
                       int32_t* d_k, hipStream_t s, tqp_ctx* ctx);

template <class Cfg>
struct CustBufs {
    RadixBufs<Cfg, uint64_t> fact;
    RadixBufs<Cfg, uint32_t> mid;
    RadixBufs<Cfg, uint64_t> grp;
    uint64_t* jstatus = nullptr;
    uint32_t* jcounter = nullptr;
    int64_t* d_join = nullptr;
    uint64_t* sstatus = nullptr;
    uint32_t* scounter = nullptr;
    uint32_t *fkeys = nullptr, *mkeys = nullptr, *mvals = nullptr, *gkeys_in = nullptr, *gkeys = nullptr;
    uint64_t *fvals = nullptr, *gvals_in = nullptr, *gvals = nullptr;
    TopkBufs topk;
};

__global__ void k_copy_i64(const int64_t* src, int64_t* dst);
__global__ void k_flags_finalize(const int64_t* acc, const int64_t* d_join_in, tqp_flags_out o);

}  // namespace tqp
