"""MI355X (gfx950) filter -> sort-based equi-join -> group-by, behind a C ABI.

The Python layer only marshals arguments: it allocates device buffers with
PyTorch (memory and streams are all PyTorch is used for), passes raw pointers
and the current HIP stream to libtqp.so, and wraps the results.  Every step of
the computation runs in the library's HIP kernels; there is no CPU fallback.

Operators (the paper's Section 5 and Algorithms 1-2):
    filter        predicate -> selection vector of row ids   (Section 3.1)
    sort          stable LSD radix sort of (key, payload)     (Algorithms 1-2)
    join          sort-based equi-join -> index pairs          (Section 5.2, Algorithm 1)
    join(kind=)   left semi / anti / outer joins; join_band: |l - r| <= w
    hash_join     open-addressing hash join                    (Section 5.3, Algorithm 3)
    pack_keys     composite keys packed into one key
    eval_expr     postfix expression programs, one kernel      (Section 5.1)
    gather        columns read through row positions           (late materialisation)
    join_chain    a chain of joins (a multi-join plan)
    groupby_agg   sort-based group-by with sum/count/avg       (Section 5.4, Algorithm 2)
    hash_groupby  hash-based group-by: sum/count/min/max/count distinct
    topk          ORDER BY sum DESC, key ASC LIMIT k
Fragments (whole queries in one launch sequence):
    FlagsFragmentRunner   date < D AND seg = c, fact.fk = dim.pk, group by (flagA, flagB)
    CustFragmentRunner    date < D, fact.fk = mid.pk, group by custkey, top-k
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (DEVERR_CAPACITY, DEVERR_KEY_RANGE, DEVERR_SPIN, DEVERR_VALUE_RANGE, JOIN_INNER, JOIN_LEFT_ANTI,
                   JOIN_LEFT_OUTER, JOIN_LEFT_SEMI, TQP_EQ, TQP_GE, TQP_GT, TQP_LE, TQP_LT, TQP_NE, TQPError, check)

__all__ = ["Context", "filter", "filter_noalloc", "fragment_run", "sort", "join", "hash_join", "join_band", "pack_keys", "eval_expr", "gather", "join_chain", "groupby_agg",
           "hash_groupby", "topk", "FlagsFragmentRunner",
           "CustFragmentRunner", "BatchRunner", "Server", "TQPError", "TQP_LT", "TQP_LE", "TQP_GT", "TQP_GE", "TQP_EQ", "TQP_NE",
           "DEVERR_KEY_RANGE", "DEVERR_SPIN", "DEVERR_CAPACITY", "DEVERR_VALUE_RANGE", "JOIN_INNER", "JOIN_LEFT_SEMI",
           "JOIN_LEFT_ANTI", "JOIN_LEFT_OUTER"]

_DTYPES = {torch.int8: _lib.TQP_I8, torch.int32: _lib.TQP_I32, torch.int64: _lib.TQP_I64}


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """A tqp_ctx on one device (error word + tuning)."""

    def __init__(self, device: int = 0):
        self.lib = _lib.load()
        self.device = device
        h = ctypes.c_void_p()
        with torch.cuda.device(device):
            check(self.lib.tqp_ctx_create(device, ctypes.byref(h)), "tqp_ctx_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.tqp_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def errors(self, clear: bool = True, stream=None) -> int:
        e = ctypes.c_uint32(0)
        check(self.lib.tqp_ctx_errors(self.h, _stream(stream), ctypes.byref(e), int(clear)), "tqp_ctx_errors")
        return int(e.value)

    def set_digit_bits(self, bits: int) -> None:
        check(self.lib.tqp_ctx_set_digit_bits(self.h, bits), "tqp_ctx_set_digit_bits")

    def copy(self, dst, src, nbytes: int, stream=None) -> None:
        """Device copy of nbytes (multiple of 16) with the library's streaming copy kernel."""
        check(self.lib.tqp_copy(self.h, _p(dst), _p(src), nbytes, _stream(stream)), "tqp_copy")

    def set_profiling(self, on: bool) -> None:
        check(self.lib.tqp_ctx_set_profiling(self.h, int(bool(on))), "tqp_ctx_set_profiling")

    def profile_read(self, stream=None, cap: int = 1 << 16) -> list:
        """[(kernel label, milliseconds)] of the launches since the last read, in launch order."""
        buf = (_lib.ProfEntry * cap)()
        n = ctypes.c_int(0)
        check(self.lib.tqp_ctx_profile_read(self.h, _stream(stream), buf, cap, ctypes.byref(n)),
              "tqp_ctx_profile_read")
        return [(buf[i].name.decode(), float(buf[i].ms)) for i in range(min(n.value, cap))]


def _workspace(call, where, device):
    """Size query (ws = NULL), then a device buffer of that size."""
    sz = ctypes.c_size_t(0)
    check(call(None, ctypes.byref(sz)), where + " (size query)")
    ws = torch.empty(max(int(sz.value), 256), dtype=torch.uint8, device=device)
    return ws, sz


def _run(call, where, device):
    ws, sz = _workspace(call, where, device)
    check(call(_p(ws), ctypes.byref(sz)), where)
    return ws


def _dev(ctx):
    return torch.device("cuda", ctx.device)


def filter(ctx: Context, cols: list, preds: list, carry=None, cap: int | None = None, stream=None):
    """Row ids where every (col_index, op, k) predicate holds.  Returns (rowid, carry_out, d_count)."""
    n = cols[0].numel() if cols else 0
    cap = n if cap is None else cap
    dev = _dev(ctx)
    carr = (_lib.Column * max(1, len(cols)))(*[_lib.Column(c.data_ptr(), _DTYPES[c.dtype], 0) for c in cols])
    parr = (_lib.Pred * max(1, len(preds)))(*[_lib.Pred(p[0], p[1], p[2]) for p in preds])
    out = torch.empty(max(1, cap), dtype=torch.int32, device=dev)
    outc = torch.empty(max(1, cap), dtype=torch.int32, device=dev) if carry is not None else None
    cnt = torch.empty(1, dtype=torch.int64, device=dev)
    s = _stream(stream)
    _run(lambda ws, sz: ctx.lib.tqp_filter(ctx.h, carr, len(cols), n, parr, len(preds), _p(carry), _p(out),
                                           _p(outc), cap, _p(cnt), ws, sz, s), "tqp_filter", dev)
    return out, outc, cnt


def filter_noalloc(ctx: Context, cols: list, preds: list, out, cnt, carry=None, out_carry=None, n: int | None = None,
                   stream=None):
    """tqp_filter_noalloc: the filter into caller-given outputs (out: int32 device tensor, its length is
    the capacity; cnt: one int64), with no workspace and no allocation.  n defaults to the column length."""
    n = (cols[0].numel() if cols else 0) if n is None else n
    carr = (_lib.Column * max(1, len(cols)))(*[_lib.Column(c.data_ptr(), _DTYPES[c.dtype], 0) for c in cols])
    parr = (_lib.Pred * max(1, len(preds)))(*[_lib.Pred(p[0], p[1], p[2]) for p in preds])
    check(ctx.lib.tqp_filter_noalloc(ctx.h, carr, len(cols), n, parr, len(preds), _p(carry), _p(out), _p(out_carry),
                                     out.numel(), _p(cnt), _stream(stream)), "tqp_filter_noalloc")


def sort(ctx: Context, keys, vals=None, key_bits: int = 0, perm: bool = False, d_n=None, stream=None):
    """Stable ascending sort.  vals given: (keys, vals) sorted together; perm=True: the
    permutation comes back as the payload; otherwise keys only."""
    n = keys.numel()
    dev = _dev(ctx)
    ko = torch.empty(max(1, n), dtype=torch.int32, device=dev)
    vo = torch.empty(max(1, n), dtype=torch.int32, device=dev) if (vals is not None or perm) else None
    s = _stream(stream)
    _run(lambda ws, sz: ctx.lib.tqp_sort(ctx.h, _p(keys), _p(vals), n, _p(d_n), key_bits, _p(ko), _p(vo), ws, sz,
                                         s), "tqp_sort", dev)
    return ko[:n], (vo[:n] if vo is not None else None)


def join(ctx: Context, lkey, rkey, lrow=None, rrow=None, cap: int | None = None, d_nl=None, d_nr=None,
         stream=None, kind: int = JOIN_INNER):
    """Sort-based join of key-sorted inputs: inner (default), or JOIN_LEFT_SEMI / JOIN_LEFT_ANTI /
    JOIN_LEFT_OUTER (-1 marks a missing right row).  Returns (out_l, out_r, d_count)."""
    nl, nr = lkey.numel(), rkey.numel()
    cap = nl if cap is None else cap
    dev = _dev(ctx)
    ol = torch.empty(max(1, cap), dtype=torch.int32, device=dev)
    orr = torch.empty(max(1, cap), dtype=torch.int32, device=dev)
    cnt = torch.empty(1, dtype=torch.int64, device=dev)
    s = _stream(stream)
    if kind == JOIN_INNER:
        _run(lambda ws, sz: ctx.lib.tqp_join(ctx.h, _p(lkey), _p(lrow), nl, _p(d_nl), _p(rkey), _p(rrow), nr,
                                             _p(d_nr), _p(ol), _p(orr), cap, _p(cnt), ws, sz, s), "tqp_join", dev)
    else:
        _run(lambda ws, sz: ctx.lib.tqp_join_kind(ctx.h, kind, _p(lkey), _p(lrow), nl, _p(d_nl), _p(rkey), _p(rrow),
                                                  nr, _p(d_nr), _p(ol), _p(orr), cap, _p(cnt), ws, sz, s),
             "tqp_join_kind", dev)
    return ol, orr, cnt


def eval_expr(ctx: Context, cols: list, prog: list, d_n=None, stream=None):
    """int64 values of a postfix expression program [(op, arg)] (TQP_X_* codes) over device columns."""
    n = cols[0].numel() if cols else 0
    carr = (_lib.Column * max(1, len(cols)))(*[_lib.Column(c.data_ptr(), _DTYPES[c.dtype], 0) for c in cols])
    parr = (_lib.XInstr * max(1, len(prog)))(*[_lib.XInstr(int(o), 0, int(a)) for o, a in prog])
    out = torch.empty(max(1, n), dtype=torch.int64, device=_dev(ctx))
    check(ctx.lib.tqp_eval(ctx.h, carr, len(cols), n, _p(d_n), parr, len(prog), _p(out), _stream(stream)),
          "tqp_eval")
    return out[:n]


def fragment_run(ctx: Context, fact: list, dim: list | None, fact_pred: list, dim_pred: list, fact_key: int,
                 dim_key: int, group: list, aggs: list, topk: int = 0, key_bits: int = 0, join_cap: int | None = None,
                 gcap: int | None = None, value_bits: int = 0, stream=None) -> dict:
    """A general fragment (tqp_fragment_run): fact / dim are lists of device columns; predicates and
    aggregate values are postfix programs [(op, arg)]; fact_key < 0 or dim None: no join; group =
    [(joined column, bits)]; aggs = [(AGG_* op, program)].  join_cap defaults to the fact rows (exact
    when dim keys are unique), gcap to join_cap; value_bits = 32 declares the one valued aggregate's
    values int32.  Returns device tensors: key, vals (one per aggregate, float64 for AVG), d_ngroups,
    d_join, top_key, top_val, d_topk."""
    join = dim is not None and fact_key >= 0
    dim = dim if join else []
    n_fact = fact[0].numel()
    n_dim = dim[0].numel() if dim else 0
    join_cap = max(1, n_fact if join_cap is None else join_cap)
    gcap = max(1, join_cap if gcap is None else gcap)
    dev = _dev(ctx)
    cols = lambda cs: (_lib.Column * max(1, len(cs)))(*[_lib.Column(c.data_ptr(), _DTYPES[c.dtype], 0) for c in cs])
    prog = lambda p: (_lib.XInstr * max(1, len(p)))(*[_lib.XInstr(int(o), 0, int(a)) for o, a in p])
    fc, dc, fp, dp = cols(fact), cols(dim), prog(fact_pred), prog(dim_pred if join else [])
    ga = (_lib.GroupCol * max(1, len(group)))(*[_lib.GroupCol(c, b) for c, b in group])
    vals = [torch.empty(gcap, dtype=torch.float64 if op == _lib.AGG_AVG else torch.int64, device=dev)
            for op, _ in aggs]
    progs = [prog(p) for _, p in aggs]
    aa = (_lib.Agg * max(1, len(aggs)))(*[_lib.Agg(op, 0 if op == _lib.AGG_COUNT else len(p), ctypes.addressof(pp),
                                                  v.data_ptr()) for (op, p), pp, v in zip(aggs, progs, vals)])
    f = _lib.Fragment(ctypes.addressof(fc), len(fact), fact_key if join else -1, n_fact, ctypes.addressof(fp),
                      len(fact_pred), key_bits, ctypes.addressof(dc), len(dim), dim_key, n_dim, ctypes.addressof(dp),
                      len(dim_pred) if join else 0, len(group), ctypes.addressof(ga), ctypes.addressof(aa), len(aggs),
                      topk, join_cap, value_bits, 0)
    out = {"key": torch.empty(gcap, dtype=torch.int32, device=dev), "vals": vals,
           "d_ngroups": torch.empty(1, dtype=torch.int64, device=dev), "d_join": torch.empty(1, dtype=torch.int64,
                                                                                             device=dev),
           "top_key": torch.empty(max(1, topk), dtype=torch.int32, device=dev),
           "top_val": torch.empty(max(1, topk), dtype=torch.int64, device=dev),
           "d_topk": torch.zeros(1, dtype=torch.int32, device=dev)}
    o = _lib.FragmentOut(out["key"].data_ptr(), gcap, out["d_ngroups"].data_ptr(), out["d_join"].data_ptr(),
                         out["top_key"].data_ptr(), out["top_val"].data_ptr(), out["d_topk"].data_ptr())
    s = _stream(stream)
    _run(lambda ws, sz: ctx.lib.tqp_fragment_run(ctx.h, ctypes.byref(f), ctypes.byref(o), ws, sz, s),
         "tqp_fragment_run", dev)
    return out


def gather(ctx: Context, src, idx, d_n=None, stream=None):
    """out[i] = src[idx[i]] for an int32 or int64 device column; a negative index gives -1."""
    n = idx.numel()
    out = torch.empty(max(1, n), dtype=src.dtype, device=_dev(ctx))
    check(ctx.lib.tqp_gather(ctx.h, _p(src), src.numel(), src.element_size(), _p(idx), n, _p(d_n), _p(out),
                             _stream(stream)), "tqp_gather")
    return out[:n]


def join_chain(ctx: Context, keys_out, keys_pk, pk_sorted=None, key_bits=0, caps=None, pk_dense=None,
               stream=None):
    """A chain of sort-based equi-joins (a multi-join plan) in one tqp_join_chain launch sequence: table
    0's column keys_out[0] joins table 1's keys_pk[0], table 1's keys_out[1] joins table 2's
    keys_pk[1], and so on.  Returns one int32 device tensor of row positions per table (the result
    tuples, in no fixed order) and their count.

    pk_sorted[t]: hop t's key column is already in order (its sort is skipped).  pk_dense[t]: it is
    exactly 0, 1, ..., M - 1 in row order (the hop is a filter of the keys in [0, M)).  key_bits: the
    key width of every hop, or one per hop.  caps[t] bounds hop t's tuples (default: the tuples
    entering the hop, exact for primary keys); when a hop overflows its bound the whole chain runs
    again with four times the bounds.  The hop sizes stay on the device; the only host reads are the
    final count and the error word, which is cleared; any other error raises."""
    hops = len(keys_pk)
    if len(keys_out) != hops or hops < 1 or hops + 1 > _lib.CHAIN_MAX_TABLES:
        raise ValueError("join_chain: one outgoing key column per hop, 1..%d hops" % (_lib.CHAIN_MAX_TABLES - 1))
    pk_sorted = pk_sorted or [False] * hops
    pk_dense = pk_dense or [False] * hops
    kbits = list(key_bits) if isinstance(key_bits, (list, tuple)) else [key_bits] * hops
    n0 = keys_out[0].numel()
    if caps is None:
        caps = []
        for t in range(hops):
            caps.append(max(1, n0 if t == 0 else caps[-1]))
    caps = [max(1, int(c)) for c in caps]
    dev = _dev(ctx)
    s = _stream(stream)
    while True:
        tabs = (_lib.ChainTable * (hops + 1))()
        tabs[0] = _lib.ChainTable(keys_out[0].data_ptr(), None, n0, 0, 0, 0)
        for t in range(hops):
            rule = _lib.CHAIN_PK_DENSE if pk_dense[t] else (_lib.CHAIN_PK_SORTED if pk_sorted[t] else 0)
            nxt = keys_out[t + 1].data_ptr() if t + 1 < hops else None
            tabs[t + 1] = _lib.ChainTable(nxt, keys_pk[t].data_ptr(), keys_pk[t].numel(), caps[t], kbits[t], rule)
        outs = [torch.empty(caps[-1], dtype=torch.int32, device=dev) for _ in range(hops + 1)]
        ptrs = (ctypes.c_void_p * (hops + 1))(*[o.data_ptr() for o in outs])
        cnt = torch.empty(1, dtype=torch.int64, device=dev)
        _run(lambda ws, sz: ctx.lib.tqp_join_chain(ctx.h, tabs, hops + 1, ptrs, _p(cnt), ws, sz, s),
             "tqp_join_chain", dev)
        err = ctx.errors(stream=stream)
        if err & DEVERR_CAPACITY and not err & ~DEVERR_CAPACITY:
            caps = [4 * c for c in caps]
            continue
        if err:
            raise RuntimeError("join_chain: device error flags 0x%x" % err)
        J = int(cnt.item())
        return [o[:J] for o in outs], J


def hash_join(ctx: Context, lkey, rkey, lrow=None, rrow=None, cap: int | None = None, d_nl=None, d_nr=None,
              stream=None):
    """Hash-based equi-join of unsorted inputs (rows of one left row in no fixed right order).
    Returns (out_l, out_r, d_count)."""
    nl, nr = lkey.numel(), rkey.numel()
    cap = nl if cap is None else cap
    dev = _dev(ctx)
    ol = torch.empty(max(1, cap), dtype=torch.int32, device=dev)
    orr = torch.empty(max(1, cap), dtype=torch.int32, device=dev)
    cnt = torch.empty(1, dtype=torch.int64, device=dev)
    s = _stream(stream)
    _run(lambda ws, sz: ctx.lib.tqp_hash_join(ctx.h, _p(lkey), _p(lrow), nl, _p(d_nl), _p(rkey), _p(rrow), nr,
                                              _p(d_nr), _p(ol), _p(orr), cap, _p(cnt), ws, sz, s), "tqp_hash_join",
         dev)
    return ol, orr, cnt


def join_band(ctx: Context, lkey, rkey, w: int, lrow=None, rrow=None, cap: int | None = None, d_nl=None, d_nr=None,
              stream=None):
    """Band join |lkey - rkey| <= w of key-sorted inputs.  Returns (out_l, out_r, d_count)."""
    nl, nr = lkey.numel(), rkey.numel()
    cap = nl if cap is None else cap
    dev = _dev(ctx)
    ol = torch.empty(max(1, cap), dtype=torch.int32, device=dev)
    orr = torch.empty(max(1, cap), dtype=torch.int32, device=dev)
    cnt = torch.empty(1, dtype=torch.int64, device=dev)
    s = _stream(stream)
    _run(lambda ws, sz: ctx.lib.tqp_join_band(ctx.h, _p(lkey), _p(lrow), nl, _p(d_nl), _p(rkey), _p(rrow), nr,
                                              _p(d_nr), w, _p(ol), _p(orr), cap, _p(cnt), ws, sz, s), "tqp_join_band",
         dev)
    return ol, orr, cnt


def pack_keys(ctx: Context, cols, bits, d_n=None, stream=None):
    """Composite key: the int32 device columns packed into one int32 key, first column most
    significant, column c taking bits[c] bits (sum <= 31)."""
    n = cols[0].numel()
    dev = _dev(ctx)
    out = torch.empty(max(1, n), dtype=torch.int32, device=dev)
    ptrs = (ctypes.c_void_p * len(cols))(*[c.data_ptr() for c in cols])
    b = (ctypes.c_int32 * len(bits))(*bits)
    check(ctx.lib.tqp_pack_keys(ctx.h, ctypes.cast(ptrs, ctypes.c_void_p), ctypes.cast(b, ctypes.c_void_p),
                                len(cols), n, _p(d_n), _p(out), _stream(stream)), "tqp_pack_keys")
    return out[:n]


def groupby_agg(ctx: Context, gkey, sum_in, avg_in=None, key_bits: int = 0, gcap: int | None = None, d_n=None,
                stream=None):
    """Sort-based group-by: dict of device tensors key/sum/cnt/avg (capacity gcap) and d_ngroups."""
    n = gkey.numel()
    gcap = max(1, n) if gcap is None else gcap
    dev = _dev(ctx)
    out = {"key": torch.empty(max(1, gcap), dtype=torch.int32, device=dev),
           "sum": torch.empty(max(1, gcap), dtype=torch.int64, device=dev),
           "cnt": torch.empty(max(1, gcap), dtype=torch.int64, device=dev),
           "avg": torch.empty(max(1, gcap), dtype=torch.float64, device=dev) if avg_in is not None else None,
           "d_ngroups": torch.empty(1, dtype=torch.int64, device=dev)}
    s = _stream(stream)
    _run(lambda ws, sz: ctx.lib.tqp_groupby_agg(ctx.h, _p(gkey), n, _p(d_n), key_bits, _p(sum_in), _p(avg_in),
                                                _p(out["key"]), _p(out["sum"]), _p(out["cnt"]), _p(out["avg"]),
                                                gcap, _p(out["d_ngroups"]), ws, sz, s), "tqp_groupby_agg", dev)
    return out


def hash_groupby(ctx: Context, gkey, val=None, dval=None, gcap: int | None = None, with_sum: bool = True,
                 minmax: bool = False, d_n=None, stream=None):
    """Hash-based group-by: dict of device tensors key/cnt and, as asked, sum/min/max (of val) and
    ndist (COUNT(DISTINCT dval)), capacity gcap, groups in no fixed order; and d_ngroups."""
    n = gkey.numel()
    gcap = max(1, n) if gcap is None else gcap
    dev = _dev(ctx)
    cap = max(1, gcap)
    i64 = lambda on: torch.empty(cap, dtype=torch.int64, device=dev) if on else None
    out = {"key": torch.empty(cap, dtype=torch.int32, device=dev), "cnt": i64(True),
           "sum": i64(with_sum and val is not None), "min": i64(minmax), "max": i64(minmax),
           "ndist": i64(dval is not None), "d_ngroups": torch.empty(1, dtype=torch.int64, device=dev)}
    s = _stream(stream)
    _run(lambda ws, sz: ctx.lib.tqp_hash_groupby(ctx.h, _p(gkey), n, _p(d_n), _p(val), _p(dval), _p(out["key"]),
                                                 _p(out["cnt"]), _p(out["sum"]), _p(out["min"]), _p(out["max"]),
                                                 _p(out["ndist"]), gcap, _p(out["d_ngroups"]), ws, sz, s),
         "tqp_hash_groupby", dev)
    return out


def topk(ctx: Context, key, sum_, cnt, k: int, d_n=None, stream=None):
    """ORDER BY sum DESC, key ASC LIMIT k: dict of key/sum/cnt (capacity k) and d_k."""
    n = key.numel()
    dev = _dev(ctx)
    out = {"key": torch.empty(k, dtype=torch.int32, device=dev), "sum": torch.empty(k, dtype=torch.int64, device=dev),
           "cnt": torch.empty(k, dtype=torch.int64, device=dev), "d_k": torch.empty(1, dtype=torch.int32, device=dev)}
    s = _stream(stream)
    _run(lambda ws, sz: ctx.lib.tqp_topk(ctx.h, _p(key), _p(sum_), _p(cnt), n, _p(d_n), k, _p(out["key"]),
                                         _p(out["sum"]), _p(out["cnt"]), _p(out["d_k"]), ws, sz, s), "tqp_topk", dev)
    return out


class FlagsFragmentRunner:
    """Prepared flags fragment over device-resident columns: outputs and workspace are
    allocated once; run() only launches."""

    def __init__(self, ctx: Context, fact: dict, dim: dict, D: int, c: int, key_bits: int = 0,
                 row0: int = 0, n_fact: int | None = None):
        self.ctx = ctx
        dev = _dev(ctx)
        self.fact, self.dim = fact, dim
        n_fact = fact["fk"].numel() - row0 if n_fact is None else n_fact
        self.desc = _lib.FlagsFragment(fact["fk"].data_ptr(), fact["date"].data_ptr(), fact["price"].data_ptr(),
                                       fact["disc"].data_ptr(), fact["flagA"].data_ptr(), fact["flagB"].data_ptr(),
                                       row0, n_fact, dim["pk"].data_ptr(), dim["seg"].data_ptr(), dim["pk"].numel(),
                                       D, c, key_bits, 0)
        self.out = {"key": torch.empty(8, dtype=torch.int32, device=dev),
                    "sum": torch.empty(8, dtype=torch.int64, device=dev),
                    "cnt": torch.empty(8, dtype=torch.int64, device=dev),
                    "avg": torch.empty(8, dtype=torch.float64, device=dev),
                    "d_ngroups": torch.empty(1, dtype=torch.int64, device=dev),
                    "d_join": torch.empty(1, dtype=torch.int64, device=dev)}
        o = self.out
        self.odesc = _lib.FlagsOut(o["key"].data_ptr(), o["sum"].data_ptr(), o["cnt"].data_ptr(), o["avg"].data_ptr(),
                                   o["d_ngroups"].data_ptr(), o["d_join"].data_ptr())
        sz = ctypes.c_size_t(0)
        check(ctx.lib.tqp_fragment_flags(ctx.h, ctypes.byref(self.desc), ctypes.byref(self.odesc), None,
                                         ctypes.byref(sz), None), "tqp_fragment_flags (size query)")
        self.ws = torch.empty(max(256, sz.value), dtype=torch.uint8, device=dev)
        self.ws_bytes = ctypes.c_size_t(sz.value)

    def run(self, stream=None):
        check(self.ctx.lib.tqp_fragment_flags(self.ctx.h, ctypes.byref(self.desc), ctypes.byref(self.odesc),
                                              _p(self.ws), ctypes.byref(self.ws_bytes), _stream(stream)),
              "tqp_fragment_flags")

    def result(self) -> dict:
        """Host copy of the result (synchronises)."""
        o = {k: v.cpu() for k, v in self.out.items()}
        G = int(o["d_ngroups"][0])
        return {"key": o["key"][:G].numpy(), "sum": o["sum"][:G].numpy(), "cnt": o["cnt"][:G].numpy(),
                "avg": o["avg"][:G].numpy(), "join_rows": int(o["d_join"][0])}


class CustFragmentRunner:
    """Prepared custkey fragment (join to the mid table, group by custkey, top-k)."""

    def __init__(self, ctx: Context, fact: dict, mid: dict, D: int, k: int = 100, key_bits: int = 0,
                 cust_bits: int = 0, gcap: int | None = None, join_cap: int | None = None, revenue_bits: int = 0,
                 mid_sorted: bool = False):
        """mid_sorted: mid["pk"] is already ascending (custkey row-aligned), so the mid sort is skipped."""
        self.ctx = ctx
        dev = _dev(ctx)
        self.fact, self.mid = fact, mid
        n, m = fact["fk"].numel(), mid["pk"].numel()
        join_cap = n if join_cap is None else join_cap
        if gcap is None:
            gcap = min(max(1, join_cap), 1 << (cust_bits if cust_bits else 31))
        self.k = k
        self.desc = _lib.CustFragment(fact["fk"].data_ptr(), fact["date"].data_ptr(), fact["price"].data_ptr(),
                                      fact["disc"].data_ptr(), n, mid["pk"].data_ptr(), mid["custkey"].data_ptr(),
                                      m, D, key_bits, cust_bits, k, join_cap, revenue_bits, int(bool(mid_sorted)))
        self.out = {"key": torch.empty(gcap, dtype=torch.int32, device=dev),
                    "sum": torch.empty(gcap, dtype=torch.int64, device=dev),
                    "cnt": torch.empty(gcap, dtype=torch.int64, device=dev),
                    "d_ngroups": torch.empty(1, dtype=torch.int64, device=dev),
                    "d_join": torch.empty(1, dtype=torch.int64, device=dev),
                    "top_key": torch.empty(k, dtype=torch.int32, device=dev),
                    "top_sum": torch.empty(k, dtype=torch.int64, device=dev),
                    "top_cnt": torch.empty(k, dtype=torch.int64, device=dev),
                    "d_topk": torch.empty(1, dtype=torch.int32, device=dev)}
        o = self.out
        self.odesc = _lib.CustOut(o["key"].data_ptr(), o["sum"].data_ptr(), o["cnt"].data_ptr(), gcap,
                                  o["d_ngroups"].data_ptr(), o["d_join"].data_ptr(), o["top_key"].data_ptr(),
                                  o["top_sum"].data_ptr(), o["top_cnt"].data_ptr(), o["d_topk"].data_ptr())
        sz = ctypes.c_size_t(0)
        check(ctx.lib.tqp_fragment_cust(ctx.h, ctypes.byref(self.desc), ctypes.byref(self.odesc), None,
                                        ctypes.byref(sz), None), "tqp_fragment_cust (size query)")
        self.ws = torch.empty(max(256, sz.value), dtype=torch.uint8, device=dev)
        self.ws_bytes = ctypes.c_size_t(sz.value)

    def plan(self) -> dict:
        """Radix passes and low-bit choices of this fragment (host only)."""
        v = [ctypes.c_int(0) for _ in range(5)]
        check(self.ctx.lib.tqp_fragment_cust_plan(self.ctx.h, ctypes.byref(self.desc), *[ctypes.byref(x) for x in v]),
              "tqp_fragment_cust_plan")
        return dict(zip(("fact_passes", "fact_lowb", "mid_passes", "group_passes", "group_lowb"),
                        [x.value for x in v]))

    def run(self, stream=None):
        check(self.ctx.lib.tqp_fragment_cust(self.ctx.h, ctypes.byref(self.desc), ctypes.byref(self.odesc),
                                             _p(self.ws), ctypes.byref(self.ws_bytes), _stream(stream)),
              "tqp_fragment_cust")

    def result(self, all_groups: bool = True) -> dict:
        o = {k: v.cpu() for k, v in self.out.items()}
        G = int(o["d_ngroups"][0])
        kk = int(o["d_topk"][0])
        r = {"groups": G, "join_rows": int(o["d_join"][0]), "top_key": o["top_key"][:kk].numpy(),
             "top_sum": o["top_sum"][:kk].numpy(), "top_cnt": o["top_cnt"][:kk].numpy()}
        if all_groups:
            w = min(G, o["key"].numel())
            r.update(key=o["key"][:w].numpy(), sum=o["sum"][:w].numpy(), cnt=o["cnt"][:w].numpy())
        return r


class BatchRunner:
    """Many flags fragments in one launch sequence (persistent kernels over a device work queue),
    with an autotuner and hipGraph capture / replay.

    fragments: list of dicts with device columns fact / dim and D, c, key_bits (optional row0, n_fact).
    Outputs for all fragments live in one set of device tensors [nf, 8]."""

    CONFIGS = ("digit4_tile2048", "digit8_tile2048", "digit8_tile4096", "digit11_tile4096")

    def __init__(self, ctx: Context, fragments: list):
        self.ctx = ctx
        dev = _dev(ctx)
        nf = len(fragments)
        self.nf = nf
        self.fragments = fragments
        self.out = {"key": torch.empty((max(1, nf), 8), dtype=torch.int32, device=dev),
                    "sum": torch.empty((max(1, nf), 8), dtype=torch.int64, device=dev),
                    "cnt": torch.empty((max(1, nf), 8), dtype=torch.int64, device=dev),
                    "avg": torch.empty((max(1, nf), 8), dtype=torch.float64, device=dev),
                    "d_ngroups": torch.empty(max(1, nf), dtype=torch.int64, device=dev),
                    "d_join": torch.empty(max(1, nf), dtype=torch.int64, device=dev)}
        descs = (_lib.FlagsFragment * max(1, nf))()
        outs = (_lib.FlagsOut * max(1, nf))()
        o = self.out
        for i, fr in enumerate(fragments):
            fact, dim = fr["fact"], fr["dim"]
            row0 = fr.get("row0", 0)
            n_fact = fr.get("n_fact", fact["fk"].numel() - row0)
            descs[i] = _lib.FlagsFragment(fact["fk"].data_ptr(), fact["date"].data_ptr(), fact["price"].data_ptr(),
                                          fact["disc"].data_ptr(), fact["flagA"].data_ptr(),
                                          fact["flagB"].data_ptr(), row0, n_fact, dim["pk"].data_ptr(),
                                          dim["seg"].data_ptr(), dim["pk"].numel(), fr["D"], fr["c"],
                                          fr.get("key_bits", 0), 0)
            outs[i] = _lib.FlagsOut(o["key"][i].data_ptr(), o["sum"][i].data_ptr(), o["cnt"][i].data_ptr(),
                                    o["avg"][i].data_ptr(), o["d_ngroups"][i:].data_ptr(),
                                    o["d_join"][i:].data_ptr())
        self._descs, self._outs = descs, outs
        sz = ctypes.c_size_t(0)
        check(ctx.lib.tqp_batch_create(ctx.h, descs, outs, nf, None, ctypes.byref(sz), None),
              "tqp_batch_create (size query)")
        self.ws = torch.empty(max(256, sz.value), dtype=torch.uint8, device=dev)
        h = ctypes.c_void_p()
        check(ctx.lib.tqp_batch_create(ctx.h, descs, outs, nf, _p(self.ws), ctypes.byref(sz), ctypes.byref(h)),
              "tqp_batch_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            torch.cuda.synchronize()
            self.ctx.lib.tqp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, stream=None):
        check(self.ctx.lib.tqp_batch_run(self.h, _stream(stream)), "tqp_batch_run")

    def set_config(self, config: int):
        check(self.ctx.lib.tqp_batch_set_config(self.h, config), "tqp_batch_set_config")

    def config(self) -> tuple:
        c, d, name = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_char_p()
        check(self.ctx.lib.tqp_batch_config(self.h, ctypes.byref(c), ctypes.byref(d), ctypes.byref(name)),
              "tqp_batch_config")
        return c.value, d.value, name.value.decode()

    def autotune(self, reps: int = 3, stream=None) -> dict:
        t = (ctypes.c_float * 4)()
        check(self.ctx.lib.tqp_batch_autotune(self.h, _stream(stream), reps, t), "tqp_batch_autotune")
        return {name: float(t[i]) for i, name in enumerate(self.CONFIGS)}

    def capture(self, stream):
        """Record the launch sequence into a hipGraph (stream must not be the default stream)."""
        check(self.ctx.lib.tqp_batch_capture(self.h, _stream(stream)), "tqp_batch_capture")

    def replay(self, stream=None):
        check(self.ctx.lib.tqp_batch_replay(self.h, _stream(stream)), "tqp_batch_replay")

    def results(self) -> list:
        o = {k: v.cpu() for k, v in self.out.items()}
        res = []
        for i in range(self.nf):
            G = int(o["d_ngroups"][i])
            res.append({"key": o["key"][i, :G].numpy(), "sum": o["sum"][i, :G].numpy(),
                        "cnt": o["cnt"][i, :G].numpy(), "avg": o["avg"][i, :G].numpy(),
                        "join_rows": int(o["d_join"][i])})
        return res


class Server:
    """Request loop over device-resident tables (tqp_server_*): requests are stamped on submit,
    admitted into slots under an HBM budget, launched on per-slot streams (waiting flags requests
    coalesced into one batch), and finished results are polled.  The server uses its own context
    from a background thread."""

    def __init__(self, tables: dict, slots: int = 8, max_batch: int = 32, max_flags_rows: int = 4_000_000,
                 budget_bytes: int = 200 << 30, key_bits_mid: int = 0, key_bits_dim: int = 0, cust_bits: int = 0,
                 revenue_bits: int = 0, presort_mid: bool = False, device: int = 0):
        self.ctx = Context(device)
        self.tables = tables
        f, m, d = tables["fact"], tables["mid"], tables["dim"]
        cfg = _lib.ServerConfig(f["fk"].data_ptr(), f["fk_dim"].data_ptr(), f["date"].data_ptr(),
                                f["price"].data_ptr(), f["disc"].data_ptr(), f["flagA"].data_ptr(),
                                f["flagB"].data_ptr(), f["fk"].numel(), m["pk"].data_ptr(), m["custkey"].data_ptr(),
                                m["pk"].numel(), d["pk"].data_ptr(), d["seg"].data_ptr(), d["pk"].numel(),
                                key_bits_mid, key_bits_dim, cust_bits, slots, max_batch, revenue_bits,
                                min(max_flags_rows, f["fk"].numel()), budget_bytes, int(bool(presort_mid)), 0)
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        check(self.ctx.lib.tqp_server_create(self.ctx.h, ctypes.byref(cfg), ctypes.byref(h)), "tqp_server_create")
        self.h = h
        self._buf = (_lib.Result * 1024)()

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.tqp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def now(self) -> float:
        return float(self.ctx.lib.tqp_server_now(self.h))

    def submit(self, kind: int, D: int, c: int = 0, k: int = 100, row0: int = 0, n_rows: int = 0,
               tag: int = 0) -> int:
        rid = ctypes.c_uint64(0)
        req = _lib.Request(kind, D, c, k, row0, n_rows, tag)
        check(self.ctx.lib.tqp_server_submit(self.h, ctypes.byref(req), ctypes.byref(rid)), "tqp_server_submit")
        return int(rid.value)

    def poll(self) -> list:
        out = []
        while True:
            n = ctypes.c_int(0)
            check(self.ctx.lib.tqp_server_poll(self.h, self._buf, len(self._buf), ctypes.byref(n)), "tqp_server_poll")
            for i in range(n.value):
                r = self._buf[i]
                d = {"id": r.id, "tag": r.tag, "kind": r.kind, "status": r.status, "join_rows": r.join_rows,
                     "groups": r.groups, "t_arrival": r.t_arrival, "t_admit": r.t_admit, "t_done": r.t_done,
                     "slot": r.slot, "batch_size": r.batch_size, "dev_errors": r.dev_errors}
                if r.kind == _lib.REQ_FLAGS:
                    G = max(0, min(8, r.groups))
                    d.update(key=list(r.key[:G]), sum=list(r.sum[:G]), cnt=list(r.cnt[:G]), avg=list(r.avg[:G]))
                else:
                    T = max(0, min(_lib.TOPK_MAX, r.top_n))
                    d.update(top_key=list(r.top_key[:T]), top_sum=list(r.top_sum[:T]), top_cnt=list(r.top_cnt[:T]))
                out.append(d)
            if n.value < len(self._buf):
                return out

    def drain(self):
        check(self.ctx.lib.tqp_server_drain(self.h), "tqp_server_drain")

    def stats(self) -> dict:
        a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        p = ctypes.c_size_t()
        check(self.ctx.lib.tqp_server_stats(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(p)),
              "tqp_server_stats")
        return {"submitted": a.value, "finished": b.value, "launches": c.value, "peak_bytes": p.value}


def to_device(table: dict, device="cuda") -> dict:
    """Copy a dict of numpy columns to device tensors (the resident columnar layout)."""
    return {k: torch.from_numpy(v).to(device) for k, v in table.items()}
