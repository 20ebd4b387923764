"""ctypes declarations of the C ABI in include/tqp.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libtqp.so")

c_i32, c_i64, c_u32, c_vp, c_int = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int
c_size_p = ctypes.POINTER(ctypes.c_size_t)

TQP_OK, TQP_ERR_INVALID, TQP_ERR_WORKSPACE, TQP_ERR_CAPACITY, TQP_ERR_HIP, TQP_ERR_UNSUPPORTED = range(6)
STATUS_NAMES = {0: "TQP_OK", 1: "TQP_ERR_INVALID", 2: "TQP_ERR_WORKSPACE", 3: "TQP_ERR_CAPACITY",
                4: "TQP_ERR_HIP", 5: "TQP_ERR_UNSUPPORTED"}
TQP_I8, TQP_I32, TQP_I64 = 1, 2, 3
TQP_LT, TQP_LE, TQP_GT, TQP_GE, TQP_EQ, TQP_NE = range(6)
(TQP_X_COL, TQP_X_CONST, TQP_X_ADD, TQP_X_SUB, TQP_X_MUL, TQP_X_DIV, TQP_X_MOD, TQP_X_NEG, TQP_X_LT, TQP_X_LE,
 TQP_X_GT, TQP_X_GE, TQP_X_EQ, TQP_X_NE, TQP_X_AND, TQP_X_OR, TQP_X_NOT, TQP_X_SELECT) = range(18)
JOIN_INNER, JOIN_LEFT_SEMI, JOIN_LEFT_ANTI, JOIN_LEFT_OUTER = range(4)
DEVERR_KEY_RANGE, DEVERR_SPIN, DEVERR_CAPACITY, DEVERR_VALUE_RANGE = 1, 2, 4, 8


class ProfEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("ms", ctypes.c_double)]


class Column(ctypes.Structure):
    _fields_ = [("data", c_vp), ("type", c_i32), ("reserved", c_i32)]


class Pred(ctypes.Structure):
    _fields_ = [("col", c_i32), ("op", c_i32), ("k", c_i64)]


class XInstr(ctypes.Structure):
    _fields_ = [("op", c_i32), ("reserved", c_i32), ("arg", c_i64)]


class FlagsFragment(ctypes.Structure):
    _fields_ = [("fk", c_vp), ("date", c_vp), ("price", c_vp), ("disc", c_vp), ("flagA", c_vp),
                ("flagB", c_vp), ("row0", c_i64), ("n_fact", c_i64), ("pk", c_vp), ("seg", c_vp),
                ("n_dim", c_i64), ("D", c_i32), ("c", c_i32), ("key_bits", c_i32), ("reserved", c_i32)]


class FlagsOut(ctypes.Structure):
    _fields_ = [("key", c_vp), ("sum", c_vp), ("cnt", c_vp), ("avg", c_vp), ("d_ngroups", c_vp),
                ("d_join", c_vp)]


class CustFragment(ctypes.Structure):
    _fields_ = [("fk", c_vp), ("date", c_vp), ("price", c_vp), ("disc", c_vp), ("n_fact", c_i64),
                ("pk", c_vp), ("custkey", c_vp), ("n_mid", c_i64), ("D", c_i32), ("key_bits", c_i32),
                ("cust_bits", c_i32), ("k", c_i32), ("join_cap", c_i64), ("revenue_bits", c_i32),
                ("mid_sorted", c_i32)]


class CustOut(ctypes.Structure):
    _fields_ = [("key", c_vp), ("sum", c_vp), ("cnt", c_vp), ("gcap", c_i64), ("d_ngroups", c_vp),
                ("d_join", c_vp), ("top_key", c_vp), ("top_sum", c_vp), ("top_cnt", c_vp), ("d_topk", c_vp)]


TOPK_MAX = 128
FILTER_NOALLOC_MAX_ROWS = 536_739_840     # TQP_FILTER_NOALLOC_MAX_ROWS
REQ_CUST, REQ_FLAGS = 0, 1


class ServerConfig(ctypes.Structure):
    _fields_ = [("fk_mid", c_vp), ("fk_dim", c_vp), ("date", c_vp), ("price", c_vp), ("disc", c_vp),
                ("flagA", c_vp), ("flagB", c_vp), ("n_fact", c_i64), ("mid_pk", c_vp), ("mid_custkey", c_vp),
                ("n_mid", c_i64), ("dim_pk", c_vp), ("dim_seg", c_vp), ("n_dim", c_i64), ("key_bits_mid", c_i32),
                ("key_bits_dim", c_i32), ("cust_bits", c_i32), ("slots", c_i32), ("max_batch", c_i32),
                ("revenue_bits", c_i32), ("max_flags_rows", c_i64), ("budget_bytes", ctypes.c_size_t),
                ("presort_mid", c_i32), ("reserved", c_i32)]


AGG_COUNT, AGG_SUM, AGG_MIN, AGG_MAX, AGG_AVG, AGG_COUNT_DISTINCT = range(6)


class GroupCol(ctypes.Structure):
    _fields_ = [("col", c_i32), ("bits", c_i32)]


class Agg(ctypes.Structure):
    _fields_ = [("op", c_i32), ("nprog", c_i32), ("prog", c_vp), ("out", c_vp)]


class Fragment(ctypes.Structure):
    _fields_ = [("fact_cols", c_vp), ("n_fact_cols", c_i32), ("fact_key", c_i32), ("n_fact", c_i64),
                ("fact_pred", c_vp), ("n_fact_pred", c_i32), ("key_bits", c_i32), ("dim_cols", c_vp),
                ("n_dim_cols", c_i32), ("dim_key", c_i32), ("n_dim", c_i64), ("dim_pred", c_vp), ("n_dim_pred", c_i32),
                ("n_group", c_i32), ("group", c_vp), ("aggs", c_vp), ("n_agg", c_i32), ("topk", c_i32),
                ("join_cap", c_i64), ("value_bits", c_i32), ("reserved", c_i32)]


class FragmentOut(ctypes.Structure):
    _fields_ = [("key", c_vp), ("gcap", c_i64), ("d_ngroups", c_vp), ("d_join", c_vp), ("top_key", c_vp),
                ("top_val", c_vp), ("d_topk", c_vp)]


CHAIN_MAX_TABLES, CHAIN_PK_SORTED, CHAIN_PK_DENSE = 8, 1, 2


class ChainTable(ctypes.Structure):
    _fields_ = [("key_out", c_vp), ("key_pk", c_vp), ("n_rows", c_i64), ("cap", c_i64), ("key_bits", c_i32),
                ("rule", c_i32)]


class Request(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("D", c_i32), ("c", c_i32), ("k", c_i32), ("row0", c_i64), ("n_rows", c_i64),
                ("tag", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("kind", c_i32), ("status", c_i32),
                ("join_rows", c_i64), ("groups", c_i64), ("key", c_i32 * 8), ("sum", c_i64 * 8), ("cnt", c_i64 * 8),
                ("avg", ctypes.c_double * 8), ("top_n", c_i32), ("top_key", c_i32 * TOPK_MAX),
                ("top_sum", c_i64 * TOPK_MAX), ("top_cnt", c_i64 * TOPK_MAX), ("t_arrival", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("slot", c_i32), ("batch_size", c_i32),
                ("dev_errors", ctypes.c_uint32), ("reserved", c_i32)]


_lib = None


def load() -> ctypes.CDLL:
    """The HIP library.  There is no fallback: without libtqp.so nothing runs."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO):
        raise ImportError("libtqp.so is not built (run paper_2203_01877_amd.build.build()); "
                          "the library has no CPU fallback")
    lib = ctypes.CDLL(SO)
    S = c_int  # tqp_status
    lib.tqp_ctx_create.argtypes = [c_int, ctypes.POINTER(c_vp)]
    lib.tqp_ctx_create.restype = S
    lib.tqp_ctx_destroy.argtypes = [c_vp]
    lib.tqp_ctx_destroy.restype = None
    lib.tqp_last_error.argtypes = []
    lib.tqp_last_error.restype = ctypes.c_char_p
    lib.tqp_ctx_errors.argtypes = [c_vp, c_vp, ctypes.POINTER(c_u32), c_int]
    lib.tqp_ctx_errors.restype = S
    lib.tqp_ctx_set_digit_bits.argtypes = [c_vp, c_int]
    lib.tqp_ctx_set_digit_bits.restype = S
    lib.tqp_copy.argtypes = [c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]
    lib.tqp_copy.restype = S
    lib.tqp_ctx_set_profiling.argtypes = [c_vp, c_int]
    lib.tqp_ctx_set_profiling.restype = S
    lib.tqp_ctx_profile_read.argtypes = [c_vp, c_vp, ctypes.POINTER(ProfEntry), c_int, ctypes.POINTER(c_int)]
    lib.tqp_ctx_profile_read.restype = S
    lib.tqp_filter.argtypes = [c_vp, ctypes.POINTER(Column), c_int, c_i64, ctypes.POINTER(Pred), c_int, c_vp,
                               c_vp, c_vp, c_i64, c_vp, c_vp, c_size_p, c_vp]
    lib.tqp_filter.restype = S
    lib.tqp_filter_noalloc.argtypes = [c_vp, ctypes.POINTER(Column), c_int, c_i64, ctypes.POINTER(Pred), c_int,
                                       c_vp, c_vp, c_vp, c_i64, c_vp, c_vp]
    lib.tqp_filter_noalloc.restype = S
    lib.tqp_join_chain.argtypes = [c_vp, ctypes.POINTER(ChainTable), c_int, ctypes.POINTER(c_vp), c_vp, c_vp,
                                   c_size_p, c_vp]
    lib.tqp_join_chain.restype = S
    lib.tqp_fragment_run.argtypes = [c_vp, ctypes.POINTER(Fragment), ctypes.POINTER(FragmentOut), c_vp, c_size_p,
                                     c_vp]
    lib.tqp_fragment_run.restype = S
    lib.tqp_sort.argtypes = [c_vp, c_vp, c_vp, c_i64, c_vp, c_int, c_vp, c_vp, c_vp, c_size_p, c_vp]
    lib.tqp_sort.restype = S
    lib.tqp_join.argtypes = [c_vp, c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, c_i64, c_vp,
                             c_vp, c_size_p, c_vp]
    lib.tqp_join.restype = S
    lib.tqp_join_kind.argtypes = [c_vp, c_i32] + lib.tqp_join.argtypes[1:]
    lib.tqp_join_kind.restype = S
    lib.tqp_hash_join.argtypes = lib.tqp_join.argtypes
    lib.tqp_hash_join.restype = S
    lib.tqp_join_band.argtypes = lib.tqp_join.argtypes[:9] + [c_i64] + lib.tqp_join.argtypes[9:]
    lib.tqp_join_band.restype = S
    lib.tqp_pack_keys.argtypes = [c_vp, c_vp, c_vp, c_int, c_i64, c_vp, c_vp, c_vp]
    lib.tqp_pack_keys.restype = S
    lib.tqp_hash_groupby.argtypes = [c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
                                     c_i64, c_vp, c_vp, c_vp, c_vp]
    lib.tqp_hash_groupby.restype = S
    lib.tqp_gather.argtypes = [c_vp, c_vp, c_i64, c_int, c_vp, c_i64, c_vp, c_vp, c_vp]
    lib.tqp_gather.restype = S
    lib.tqp_eval.argtypes = [c_vp, c_vp, c_int, c_i64, c_vp, c_vp, c_int, c_vp, c_vp]
    lib.tqp_eval.restype = S
    lib.tqp_groupby_agg.argtypes = [c_vp, c_vp, c_i64, c_vp, c_int, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_i64,
                                    c_vp, c_vp, c_size_p, c_vp]
    lib.tqp_groupby_agg.restype = S
    lib.tqp_topk.argtypes = [c_vp, c_vp, c_vp, c_vp, c_i64, c_vp, c_int, c_vp, c_vp, c_vp, c_vp, c_vp,
                             c_size_p, c_vp]
    lib.tqp_topk.restype = S
    lib.tqp_fragment_flags.argtypes = [c_vp, ctypes.POINTER(FlagsFragment), ctypes.POINTER(FlagsOut), c_vp,
                                       c_size_p, c_vp]
    lib.tqp_fragment_flags.restype = S
    lib.tqp_fragment_cust.argtypes = [c_vp, ctypes.POINTER(CustFragment), ctypes.POINTER(CustOut), c_vp,
                                      c_size_p, c_vp]
    lib.tqp_fragment_cust.restype = S
    ip = ctypes.POINTER(c_int)
    lib.tqp_fragment_cust_plan.argtypes = [c_vp, ctypes.POINTER(CustFragment), ip, ip, ip, ip, ip]
    lib.tqp_fragment_cust_plan.restype = S
    lib.tqp_batch_create.argtypes = [c_vp, ctypes.POINTER(FlagsFragment), ctypes.POINTER(FlagsOut), c_int, c_vp,
                                     c_size_p, ctypes.POINTER(c_vp)]
    lib.tqp_batch_create.restype = S
    lib.tqp_batch_destroy.argtypes = [c_vp]
    lib.tqp_batch_destroy.restype = None
    lib.tqp_batch_run.argtypes = [c_vp, c_vp]
    lib.tqp_batch_run.restype = S
    lib.tqp_batch_set_config.argtypes = [c_vp, c_int]
    lib.tqp_batch_set_config.restype = S
    lib.tqp_batch_config.argtypes = [c_vp, ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                     ctypes.POINTER(ctypes.c_char_p)]
    lib.tqp_batch_config.restype = S
    lib.tqp_batch_autotune.argtypes = [c_vp, c_vp, c_int, ctypes.POINTER(ctypes.c_float)]
    lib.tqp_batch_autotune.restype = S
    lib.tqp_batch_capture.argtypes = [c_vp, c_vp]
    lib.tqp_batch_capture.restype = S
    lib.tqp_batch_replay.argtypes = [c_vp, c_vp]
    lib.tqp_batch_replay.restype = S
    lib.tqp_server_create.argtypes = [c_vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(c_vp)]
    lib.tqp_server_create.restype = S
    lib.tqp_server_destroy.argtypes = [c_vp]
    lib.tqp_server_destroy.restype = None
    lib.tqp_server_now.argtypes = [c_vp]
    lib.tqp_server_now.restype = ctypes.c_double
    lib.tqp_server_submit.argtypes = [c_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    lib.tqp_server_submit.restype = S
    lib.tqp_server_poll.argtypes = [c_vp, ctypes.POINTER(Result), c_int, ctypes.POINTER(c_int)]
    lib.tqp_server_poll.restype = S
    lib.tqp_server_drain.argtypes = [c_vp]
    lib.tqp_server_drain.restype = S
    lib.tqp_server_stats.argtypes = [c_vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                     ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_size_t)]
    lib.tqp_server_stats.restype = S
    _lib = lib
    return lib


class TQPError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = load().tqp_last_error().decode(errors="replace")
        super().__init__("%s: %s (%s)" % (where, STATUS_NAMES.get(status, status), msg))
        self.status = status


def check(status: int, where: str) -> None:
    if status != TQP_OK:
        raise TQPError(status, where)
