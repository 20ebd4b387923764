"""CPU oracle (plain C++, exact int64) for filter -> sort-based equi-join -> group-by.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library and imports nothing from it.

Each wrapper takes and returns numpy arrays; see ``oracle.cpp`` for the
definition each function computes and the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

I8, I32, I64 = 1, 2, 3
LT, LE, GT, GE, EQ, NE = 0, 1, 2, 3, 4, 5
_TYPES = {np.dtype(np.int8): I8, np.dtype(np.int32): I32, np.dtype(np.int64): I64}


def build(force: bool = False) -> str:
    """Compile oracle.cpp with g++ (-O2, IEEE arithmetic, no fast-math)."""
    src = os.path.join(_HERE, "oracle.cpp")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fno-fast-math",
                               "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.orc_filter.argtypes = [i64, ctypes.c_int, vp, vp, ctypes.c_int, vp, vp, vp, vp]
        lib.orc_filter.restype = i64
        lib.orc_sort_pairs.argtypes = [vp, vp, i64, vp, vp]
        lib.orc_sort_pairs.restype = None
        lib.orc_join.argtypes = [vp, vp, i64, vp, vp, i64, vp, vp, i64]
        lib.orc_join.restype = i64
        lib.orc_join_kind.argtypes = [ctypes.c_int, vp, vp, i64, vp, vp, i64, vp, vp, i64]
        lib.orc_join_kind.restype = i64
        lib.orc_join_band.argtypes = [vp, vp, i64, vp, vp, i64, i64, vp, vp, i64]
        lib.orc_join_band.restype = i64
        lib.orc_pack_keys.argtypes = [vp, vp, ctypes.c_int, i64, vp]
        lib.orc_pack_keys.restype = i64
        lib.orc_groupby.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, i64]
        lib.orc_groupby.restype = i64
        lib.orc_group_minmax.argtypes = [vp, i64, vp, vp, vp, vp, vp, i64]
        lib.orc_group_minmax.restype = i64
        lib.orc_join_chain.argtypes = [ctypes.c_int, vp, vp, vp, vp, i64]
        lib.orc_join_chain.restype = i64
        lib.orc_eval.argtypes = [vp, ctypes.c_int, i64, vp, vp, ctypes.c_int, vp]
        lib.orc_eval.restype = i64
        lib.orc_fragment_flags.argtypes = [vp, vp, vp, vp, vp, vp, i64, vp, vp, i64, i32, i32,
                                           vp, vp, vp, vp, i64, vp]
        lib.orc_fragment_flags.restype = i64
        lib.orc_fragment_cust.argtypes = [vp, vp, vp, vp, i64, vp, vp, i64, i32, vp, vp, vp, i64,
                                          i32, vp, vp, vp, vp, vp]
        lib.orc_fragment_cust.restype = i64
        lib.orc_fragment_general.argtypes = [ctypes.c_int, vp, vp, i64, ctypes.c_int, vp, vp, i64, vp, vp,
                                             ctypes.c_int, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, vp, vp, ctypes.c_int, vp, vp, vp, vp, vp, vp, i64, i32,
                                             vp, vp, vp, vp, vp]
        lib.orc_fragment_general.restype = i64
        lib.orc_overflow_flag.restype = ctypes.c_int
        lib.orc_clear_overflow.restype = None
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _check_overflow():
    if _L().orc_overflow_flag():
        _L().orc_clear_overflow()
        raise OverflowError("oracle: exact int64 accumulation overflowed")


def filter_rows(cols: list, preds: list) -> np.ndarray:
    """Row ids (int32, increasing) where every predicate (col_index, op, k) holds."""
    cols = [np.ascontiguousarray(c) for c in cols]
    n = len(cols[0]) if cols else 0
    ptrs = (ctypes.c_void_p * max(1, len(cols)))(*[c.ctypes.data for c in cols])
    types = np.array([_TYPES[c.dtype] for c in cols] or [0], dtype=np.int32)
    pc = np.array([p[0] for p in preds] or [0], dtype=np.int32)
    po = np.array([p[1] for p in preds] or [0], dtype=np.int32)
    pk = np.array([p[2] for p in preds] or [0], dtype=np.int64)
    out = np.empty(max(1, n), dtype=np.int32)
    w = _L().orc_filter(n, len(cols), ptrs, types.ctypes.data, len(preds), pc.ctypes.data,
                        po.ctypes.data, pk.ctypes.data, out.ctypes.data)
    return out[:w].copy()


def sort_pairs(keys, vals=None):
    keys = _c(keys, np.int32)
    vals = None if vals is None else _c(vals, np.int32)
    n = len(keys)
    ko, vo = np.empty(n, np.int32), np.empty(n, np.int32)
    if n:
        _L().orc_sort_pairs(keys.ctypes.data, _p(vals), n, ko.ctypes.data, vo.ctypes.data)
    return ko, vo


def join(lkey, rkey, lrow=None, rrow=None, cap=None):
    """Equi-join pairs (left payload, right payload) and the true count."""
    lkey, rkey = _c(lkey, np.int32), _c(rkey, np.int32)
    lrow = None if lrow is None else _c(lrow, np.int32)
    rrow = None if rrow is None else _c(rrow, np.int32)
    if cap is None:
        cap = _L().orc_join(lkey.ctypes.data, _p(lrow), len(lkey), rkey.ctypes.data, _p(rrow),
                            len(rkey), None, None, 0)
    ol, orr = np.empty(max(1, cap), np.int32), np.empty(max(1, cap), np.int32)
    J = _L().orc_join(lkey.ctypes.data, _p(lrow), len(lkey), rkey.ctypes.data, _p(rrow), len(rkey),
                      ol.ctypes.data, orr.ctypes.data, cap)
    w = min(J, cap)
    return ol[:w].copy(), orr[:w].copy(), J


JOIN_INNER, JOIN_LEFT_SEMI, JOIN_LEFT_ANTI, JOIN_LEFT_OUTER = 0, 1, 2, 3


def join_kind(kind, lkey, rkey, lrow=None, rrow=None, cap=None):
    """Inner (0), left semi (1), left anti (2) or left outer (3) join: rows (left payload,
    right payload or -1) in left order, then right order, and the true count."""
    lkey, rkey = _c(lkey, np.int32), _c(rkey, np.int32)
    lrow = None if lrow is None else _c(lrow, np.int32)
    rrow = None if rrow is None else _c(rrow, np.int32)
    if cap is None:
        cap = _L().orc_join_kind(kind, lkey.ctypes.data, _p(lrow), len(lkey), rkey.ctypes.data, _p(rrow),
                                 len(rkey), None, None, 0)
    ol, orr = np.empty(max(1, cap), np.int32), np.empty(max(1, cap), np.int32)
    J = _L().orc_join_kind(kind, lkey.ctypes.data, _p(lrow), len(lkey), rkey.ctypes.data, _p(rrow), len(rkey),
                           ol.ctypes.data, orr.ctypes.data, cap)
    w = min(J, cap)
    return ol[:w].copy(), orr[:w].copy(), J


def join_band(lkey, rkey, w, lrow=None, rrow=None, cap=None):
    """Band join |lkey - rkey| <= w: pairs (left payload, right payload) in left order, then right
    order, and the true count (all pairs compared: small inputs only)."""
    lkey, rkey = _c(lkey, np.int32), _c(rkey, np.int32)
    lrow = None if lrow is None else _c(lrow, np.int32)
    rrow = None if rrow is None else _c(rrow, np.int32)
    if cap is None:
        cap = _L().orc_join_band(lkey.ctypes.data, _p(lrow), len(lkey), rkey.ctypes.data, _p(rrow), len(rkey), w,
                                 None, None, 0)
    ol, orr = np.empty(max(1, cap), np.int32), np.empty(max(1, cap), np.int32)
    J = _L().orc_join_band(lkey.ctypes.data, _p(lrow), len(lkey), rkey.ctypes.data, _p(rrow), len(rkey), w,
                           ol.ctypes.data, orr.ctypes.data, cap)
    w_ = min(J, cap)
    return ol[:w_].copy(), orr[:w_].copy(), J


def pack_keys(cols, bits):
    """Columns packed into one int32 key, first column most significant; (keys, values outside
    their width)."""
    cols = [_c(c, np.int32) for c in cols]
    n = len(cols[0]) if cols else 0
    ptrs = (ctypes.c_void_p * max(1, len(cols)))(*[c.ctypes.data for c in cols])
    b = np.asarray(bits, np.int32)
    out = np.empty(max(1, n), np.int32)
    bad = _L().orc_pack_keys(ctypes.cast(ptrs, ctypes.c_void_p), b.ctypes.data, len(cols), n, out.ctypes.data)
    return out[:n].copy(), int(bad)


def groupby(gkey, val, avg_in=None):
    """(keys, sums, counts, avgs or None) with one row per distinct key, keys ascending."""
    gkey, val = _c(gkey, np.int32), _c(val, np.int64)
    avg_in = None if avg_in is None else _c(avg_in, np.int64)
    n = len(gkey)
    cap = max(1, n)
    k, s, c, a = (np.empty(cap, np.int32), np.empty(cap, np.int64), np.empty(cap, np.int64),
                  np.empty(cap, np.float64))
    G = _L().orc_groupby(gkey.ctypes.data, n, val.ctypes.data, _p(avg_in), k.ctypes.data,
                         s.ctypes.data, c.ctypes.data, a.ctypes.data, cap)
    _check_overflow()
    return k[:G].copy(), s[:G].copy(), c[:G].copy(), (a[:G].copy() if avg_in is not None else None)


def group_minmax(gkey, val):
    """(keys, mins, maxs, ndistinct) with one row per distinct key, keys ascending."""
    gkey, val = _c(gkey, np.int32), _c(val, np.int64)
    n = len(gkey)
    cap = max(1, n)
    k, lo, hi, nd = (np.empty(cap, np.int32), np.empty(cap, np.int64), np.empty(cap, np.int64),
                     np.empty(cap, np.int64))
    G = _L().orc_group_minmax(gkey.ctypes.data, n, val.ctypes.data, k.ctypes.data, lo.ctypes.data,
                              hi.ctypes.data, nd.ctypes.data, cap)
    return k[:G].copy(), lo[:G].copy(), hi[:G].copy(), nd[:G].copy()


# expression operator codes (postfix programs of (op, arg) pairs)
X_COL, X_CONST, X_ADD, X_SUB, X_MUL, X_DIV, X_MOD, X_NEG = range(8)
X_LT, X_LE, X_GT, X_GE, X_EQ, X_NE, X_AND, X_OR, X_NOT, X_SELECT = range(8, 18)


def eval_expr(cols, prog):
    """Values of a postfix expression program [(op, arg)] over int columns (as int64), and the number
    of zero divisors met; raises ValueError for a malformed program."""
    cs = [_c(np.asarray(c).astype(np.int64), np.int64) for c in cols]
    n = len(cs[0]) if cs else 0
    ptr = (ctypes.c_void_p * max(1, len(cs)))(*[c.ctypes.data for c in cs])
    ops = np.array([p[0] for p in prog], np.int32)
    args = np.array([p[1] for p in prog], np.int64)
    out = np.empty(max(1, n), np.int64)
    z = _L().orc_eval(ctypes.cast(ptr, ctypes.c_void_p), len(cs), n, ops.ctypes.data, args.ctypes.data, len(prog),
                      out.ctypes.data)
    if z < 0:
        raise ValueError("malformed expression program")
    return out[:n].copy(), int(z)


def join_chain(keys_out, keys_pk):
    """Tuples (r0, ..., r_hops) of a chain of equi-joins: keys_out[t] of table t against keys_pk[t]
    (the matched column of table t + 1).  Returns an int32 array of shape (count, hops + 1), nested
    in input order."""
    hops = len(keys_pk)
    outs = [_c(k, np.int32) for k in keys_out]
    pks = [np.zeros(1, np.int32)] + [_c(k, np.int32) for k in keys_pk]
    nrows = np.array([len(outs[0])] + [len(k) for k in keys_pk], np.int64)
    optr = (ctypes.c_void_p * hops)(*[o.ctypes.data for o in outs])
    pptr = (ctypes.c_void_p * (hops + 1))(*[p.ctypes.data for p in pks])
    args = (hops, ctypes.cast(optr, ctypes.c_void_p), nrows.ctypes.data, ctypes.cast(pptr, ctypes.c_void_p))
    cnt = _L().orc_join_chain(*args, None, 0)
    out = np.empty((max(1, cnt), hops + 1), np.int32)
    _L().orc_join_chain(*args, out.ctypes.data, cnt)
    return out[:cnt].copy()


def fragment_flags(fact: dict, dim: dict, D: int, c: int) -> dict:
    """The flags fragment (date < D, seg == c, fk = pk, group by flagA*2 + flagB)."""
    f = {k: np.ascontiguousarray(v) for k, v in fact.items()}
    d = {k: np.ascontiguousarray(v) for k, v in dim.items()}
    cap = 8
    k, s, cn, a = np.empty(cap, np.int32), np.empty(cap, np.int64), np.empty(cap, np.int64), np.empty(cap)
    J = np.zeros(1, np.int64)
    G = _L().orc_fragment_flags(f["fk"].ctypes.data, f["date"].ctypes.data, f["price"].ctypes.data,
                                f["disc"].ctypes.data, f["flagA"].ctypes.data, f["flagB"].ctypes.data,
                                len(f["fk"]), d["pk"].ctypes.data, d["seg"].ctypes.data, len(d["pk"]),
                                D, c, k.ctypes.data, s.ctypes.data, cn.ctypes.data, a.ctypes.data, cap,
                                J.ctypes.data)
    _check_overflow()
    return {"key": k[:G].copy(), "sum": s[:G].copy(), "cnt": cn[:G].copy(), "avg": a[:G].copy(),
            "join_rows": int(J[0])}


def fragment_cust(fact: dict, mid: dict, D: int, k: int = 100, gcap: int | None = None) -> dict:
    """The custkey fragment (date < D, fk = pk, group by custkey, top-k by sum desc, key asc)."""
    f = {kk: np.ascontiguousarray(v) for kk, v in fact.items()}
    m = {kk: np.ascontiguousarray(v) for kk, v in mid.items()}
    if gcap is None:
        gcap = max(1, min(len(m["pk"]), int(m["custkey"].max()) + 1 if len(m["custkey"]) else 1))
    key, s, cn = np.empty(gcap, np.int32), np.empty(gcap, np.int64), np.empty(gcap, np.int64)
    tk, ts, tc = np.empty(max(1, k), np.int32), np.empty(max(1, k), np.int64), np.empty(max(1, k), np.int64)
    kout = np.zeros(1, np.int32)
    J = np.zeros(1, np.int64)
    G = _L().orc_fragment_cust(f["fk"].ctypes.data, f["date"].ctypes.data, f["price"].ctypes.data,
                               f["disc"].ctypes.data, len(f["fk"]), m["pk"].ctypes.data,
                               m["custkey"].ctypes.data, len(m["pk"]), D, key.ctypes.data,
                               s.ctypes.data, cn.ctypes.data, gcap, k, tk.ctypes.data, ts.ctypes.data,
                               tc.ctypes.data, kout.ctypes.data, J.ctypes.data)
    _check_overflow()
    kk = int(kout[0])
    w = min(G, gcap)
    return {"key": key[:w].copy(), "sum": s[:w].copy(), "cnt": cn[:w].copy(), "groups": int(G),
            "top_key": tk[:kk].copy(), "top_sum": ts[:kk].copy(), "top_cnt": tc[:kk].copy(),
            "join_rows": int(J[0])}


AGG_COUNT, AGG_SUM, AGG_MIN, AGG_MAX, AGG_AVG, AGG_COUNT_DISTINCT = range(6)


def fragment_general(fact: list, dim: list | None, fpred: list, dpred: list, fkey: int, dkey: int, group: list,
                     aggs: list, topk: int = 0, gcap: int | None = None) -> dict:
    """A general fragment by its definition: the fact rows whose predicate program is nonzero, joined on
    fact column fkey = dim column dkey to the dim rows whose predicate is nonzero (no join when dim is
    None or fkey < 0), grouped by the packed columns group = [(joined column, bits)], with aggregates
    aggs = [(op, program)] (op AGG_*; the program over the joined row's columns, fact first, is
    ignored for AGG_COUNT).  Returns keys ascending, one array per aggregate (float64 for AVG), the
    group and joined-row counts, the count of group values outside their width, and the first topk
    groups by (aggregate 0 desc, key asc)."""
    join = dim is not None and fkey >= 0
    fc = [np.ascontiguousarray(c) for c in fact]
    dc = [np.ascontiguousarray(c) for c in (dim or [])] if join else []
    n_fact = len(fc[0]) if fc else 0
    n_dim = len(dc[0]) if dc else 0
    fptr = (ctypes.c_void_p * max(1, len(fc)))(*[c.ctypes.data for c in fc])
    dptr = (ctypes.c_void_p * max(1, len(dc)))(*[c.ctypes.data for c in dc])
    ftyp = np.array([_TYPES[c.dtype] for c in fc] or [0], np.int32)
    dtyp = np.array([_TYPES[c.dtype] for c in dc] or [0], np.int32)
    prog = lambda p: (np.array([x[0] for x in p] or [0], np.int32), np.array([x[1] for x in p] or [0], np.int64))
    fo, fa = prog(fpred)
    do, da = prog(dpred if join else [])
    gcol = np.array([g[0] for g in group] or [0], np.int32)
    gbits = np.array([g[1] for g in group] or [0], np.int32)
    aop = np.array([a[0] for a in aggs] or [0], np.int32)
    alen = np.array([0 if a[0] == AGG_COUNT else len(a[1]) for a in aggs] or [0], np.int32)
    flat = [x for a in aggs if a[0] != AGG_COUNT for x in a[1]]
    ao, aa = prog(flat)
    if gcap is None:
        gcap = max(1, n_fact * max(1, n_dim) if join else n_fact)
        gcap = min(gcap, 1 << 22)
    key = np.empty(gcap, np.int32)
    vals = np.empty((max(1, len(aggs)), gcap), np.int64)
    tk, tv = np.empty(max(1, topk), np.int32), np.empty(max(1, topk), np.int64)
    kout, J, bad = np.zeros(1, np.int32), np.zeros(1, np.int64), np.zeros(1, np.int64)
    G = _L().orc_fragment_general(len(fc), ctypes.cast(fptr, ctypes.c_void_p), ftyp.ctypes.data, n_fact, len(dc),
                                  ctypes.cast(dptr, ctypes.c_void_p), dtyp.ctypes.data, n_dim, fo.ctypes.data,
                                  fa.ctypes.data, len(fpred), do.ctypes.data, da.ctypes.data,
                                  len(dpred) if join else 0, fkey if join else -1, dkey, len(group), gcol.ctypes.data,
                                  gbits.ctypes.data, len(aggs), aop.ctypes.data, alen.ctypes.data, ao.ctypes.data,
                                  aa.ctypes.data, key.ctypes.data, vals.ctypes.data, gcap, topk, tk.ctypes.data,
                                  tv.ctypes.data, kout.ctypes.data, J.ctypes.data, bad.ctypes.data)
    if G < 0:
        raise ValueError("malformed program")
    _check_overflow()
    w = min(G, gcap)
    out_vals = []
    for a, (op, _) in enumerate(aggs):
        v = vals[a, :w].copy()
        out_vals.append(v.view(np.float64) if op == AGG_AVG else v)
    kk = int(kout[0])
    return {"key": key[:w].copy(), "vals": out_vals, "groups": int(G), "join_rows": int(J[0]), "bad": int(bad[0]),
            "top_key": tk[:kk].copy(), "top_val": tv[:kk].copy()}
