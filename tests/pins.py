"""Checks that pin the oracle to something other than itself.

Each check compares one oracle function with a library routine (numpy's
flatnonzero / stable argsort / intersect1d / bincount, Python's correctly
rounded int division), with brute force over all pairs on small inputs, or
with a closed-form identity.  The checks raise AssertionError; they are run
against the real oracle (test_oracle.py) and against planted mistakes
(test_oracle_mutants.py), where at least one of them must fail.
"""
from __future__ import annotations

import itertools

import numpy as np

import datagen
import oracle

REV = lambda price, disc: int(price) * (100 - int(disc))  # noqa: E731  (price*(100-disc), cent*percent)


def _rng(seed):
    return np.random.default_rng(seed)


# --------------------------------------------------------------------------- filter

def check_filter():
    rng = _rng(1)
    n = 3000
    date = rng.integers(0, 2557, n).astype(np.int32)
    seg = rng.integers(0, 5, n).astype(np.int8)
    big = rng.integers(-2**40, 2**40, n).astype(np.int64)
    cols = [date, seg, big]
    ops = {oracle.LT: np.less, oracle.LE: np.less_equal, oracle.GT: np.greater,
           oracle.GE: np.greater_equal, oracle.EQ: np.equal, oracle.NE: np.not_equal}
    for D in (0, 1, 1200, 2556, 2557, 2**31 - 1):
        for op, fn in ops.items():
            got = oracle.filter_rows(cols, [(0, op, D)])
            want = np.flatnonzero(fn(date, D)).astype(np.int32)
            assert np.array_equal(got, want), ("filter", D, op)
    got = oracle.filter_rows(cols, [(0, oracle.LT, 2400), (1, oracle.EQ, 1), (2, oracle.GE, 0)])
    want = np.flatnonzero((date < 2400) & (seg == 1) & (big >= 0)).astype(np.int32)
    assert np.array_equal(got, want), "filter conjunction"
    assert len(oracle.filter_rows([date[:0]], [(0, oracle.LT, 5)])) == 0
    got = oracle.filter_rows([seg], [(0, oracle.EQ, 7)])      # a value that never occurs
    assert len(got) == 0


# --------------------------------------------------------------------------- sort

def check_sort():
    rng = _rng(2)
    cases = [rng.integers(0, 50, 5000), rng.integers(0, 2**31 - 1, 4000), np.zeros(300, np.int64),
             np.arange(1000)[::-1], np.array([7]), np.array([], np.int64),
             np.array([2**31 - 1, 0, 2**31 - 1, 5, 0])]
    for keys in cases:
        keys = keys.astype(np.int32)
        vals = rng.integers(-2**31, 2**31 - 1, len(keys)).astype(np.int32)
        ko, vo = oracle.sort_pairs(keys, vals)
        order = np.argsort(keys, kind="stable")
        assert np.array_equal(ko, keys[order]), "sort keys"
        assert np.array_equal(vo, vals[order]), "sort payload (stability)"
        ko2, io = oracle.sort_pairs(keys)                  # payload = input index
        assert np.array_equal(io, order.astype(np.int32)), "sort permutation"


# --------------------------------------------------------------------------- join

def _brute_join(lkey, rkey, lrow, rrow):
    out = []
    for i in range(len(lkey)):
        for j in range(len(rkey)):
            if lkey[i] == rkey[j]:
                out.append((int(lrow[i]), int(rrow[j])))
    return out


def check_join():
    rng = _rng(3)
    for trial in range(12):
        nl, nr = int(rng.integers(0, 300)), int(rng.integers(0, 120))
        hi = int(rng.integers(1, 40))
        lkey = np.sort(rng.integers(0, hi, nl)).astype(np.int32)
        rkey = np.sort(rng.integers(0, hi, nr)).astype(np.int32)
        lrow = rng.permutation(max(nl, 1))[:nl].astype(np.int32)
        rrow = rng.permutation(max(nr, 1))[:nr].astype(np.int32)
        ol, orr, J = oracle.join(lkey, rkey, lrow, rrow)
        want = _brute_join(lkey, rkey, lrow, rrow)
        assert J == len(want), ("join size", trial)
        assert list(zip(ol.tolist(), orr.tolist())) == want, ("join pairs / order", trial)
        # closed form of Algorithm 1: outSize = sum_k leftHist[k] * rightHist[k]
        if nl and nr:
            L = max(int(lkey.max()), int(rkey.max())) + 1
            assert J == int(np.dot(np.bincount(lkey, minlength=L).astype(np.int64),
                                   np.bincount(rkey, minlength=L).astype(np.int64)))
    # every row on one key: J = n * m
    ol, orr, J = oracle.join(np.full(70, 3, np.int32), np.full(40, 3, np.int32))
    assert J == 70 * 40 and np.array_equal(ol, np.repeat(np.arange(70), 40)) \
        and np.array_equal(orr, np.tile(np.arange(40), 70))
    # unique keys on both sides: the matches are the set intersection
    a = np.sort(rng.choice(5000, 800, replace=False)).astype(np.int32)
    b = np.sort(rng.choice(5000, 900, replace=False)).astype(np.int32)
    ol, orr, J = oracle.join(a, b)
    inter = np.intersect1d(a, b)
    assert J == len(inter) and np.array_equal(a[ol], inter) and np.array_equal(b[orr], inter)
    # no matches, empty sides
    assert oracle.join(np.arange(10, dtype=np.int32), np.arange(10, 20, dtype=np.int32))[2] == 0
    assert oracle.join(np.zeros(0, np.int32), np.arange(5, dtype=np.int32))[2] == 0
    assert oracle.join(np.arange(5, dtype=np.int32), np.zeros(0, np.int32))[2] == 0
    # capacity: the first cap pairs of the canonical order, true count still returned
    lk = np.array([1, 1, 2], np.int32)
    rk = np.array([1, 1, 2, 2], np.int32)
    ol, orr, J = oracle.join(lk, rk, cap=3)
    assert J == 6 and list(zip(ol, orr)) == [(0, 0), (0, 1), (1, 0)]


def _brute_join_kind(kind, lkey, rkey, lrow, rrow):
    """Join kinds written out from their definitions, one left row at a time."""
    out = []
    for i in range(len(lkey)):
        hits = [int(rrow[j]) for j in range(len(rkey)) if rkey[j] == lkey[i]]
        if kind == oracle.JOIN_INNER:
            out += [(int(lrow[i]), r) for r in hits]
        elif kind == oracle.JOIN_LEFT_SEMI:
            out += [(int(lrow[i]), -1)] if hits else []
        elif kind == oracle.JOIN_LEFT_ANTI:
            out += [] if hits else [(int(lrow[i]), -1)]
        else:
            out += [(int(lrow[i]), r) for r in hits] if hits else [(int(lrow[i]), -1)]
    return out


def check_join_kinds():
    rng = _rng(31)
    kinds = (oracle.JOIN_INNER, oracle.JOIN_LEFT_SEMI, oracle.JOIN_LEFT_ANTI, oracle.JOIN_LEFT_OUTER)
    for trial in range(10):
        nl, nr = int(rng.integers(0, 200)), int(rng.integers(0, 80))
        hi = int(rng.integers(1, 50))
        lkey = np.sort(rng.integers(0, hi, nl)).astype(np.int32)
        rkey = np.sort(rng.integers(0, hi, nr)).astype(np.int32)
        lrow = rng.permutation(max(nl, 1))[:nl].astype(np.int32)
        rrow = rng.permutation(max(nr, 1))[:nr].astype(np.int32)
        got = {}
        for kind in kinds:
            ol, orr, J = oracle.join_kind(kind, lkey, rkey, lrow, rrow)
            want = _brute_join_kind(kind, lkey, rkey, lrow, rrow)
            assert J == len(want), ("join kind size", kind, trial)
            assert list(zip(ol.tolist(), orr.tolist())) == want, ("join kind rows", kind, trial)
            got[kind] = (ol, orr)
        # semi and anti split the left rows: membership by np.isin, in order
        member = np.isin(lkey, rkey)
        assert np.array_equal(got[oracle.JOIN_LEFT_SEMI][0], lrow[member])
        assert np.array_equal(got[oracle.JOIN_LEFT_ANTI][0], lrow[~member])
        # inner equals the plain join; outer is inner plus one row per unmatched left row
        ol, orr, _ = oracle.join(lkey, rkey, lrow, rrow)
        assert np.array_equal(got[oracle.JOIN_INNER][0], ol) and np.array_equal(got[oracle.JOIN_INNER][1], orr)
        o_l, o_r = got[oracle.JOIN_LEFT_OUTER]
        assert len(o_l) == len(ol) + int((~member).sum())
        assert np.array_equal(o_l[o_r != -1], ol) and np.array_equal(o_r[o_r != -1], orr)
        assert np.array_equal(o_l[o_r == -1], lrow[~member])
    # capacity: the first cap rows, true count returned
    ol, orr, J = oracle.join_kind(oracle.JOIN_LEFT_OUTER, np.array([1, 2, 3], np.int32),
                                  np.array([2, 2], np.int32), cap=2)
    assert J == 4 and list(zip(ol, orr)) == [(0, -1), (1, 0)]


def check_join_band():
    rng = _rng(37)
    for trial in range(8):
        nl, nr = int(rng.integers(0, 120)), int(rng.integers(0, 90))
        hi = int(rng.integers(1, 200))
        w = int(rng.integers(0, 12))
        lkey = np.sort(rng.integers(0, hi, nl)).astype(np.int32)
        rkey = np.sort(rng.integers(0, hi, nr)).astype(np.int32)
        lrow = rng.permutation(max(nl, 1))[:nl].astype(np.int32)
        rrow = rng.permutation(max(nr, 1))[:nr].astype(np.int32)
        ol, orr, J = oracle.join_band(lkey, rkey, w, lrow, rrow)
        want = [(int(lrow[i]), int(rrow[j])) for i in range(nl) for j in range(nr)
                if abs(int(lkey[i]) - int(rkey[j])) <= w]
        assert J == len(want) and list(zip(ol.tolist(), orr.tolist())) == want, ("band rows", trial)
        # closed form on sorted keys: per left key, the right keys in [k - w, k + w]
        assert J == int((np.searchsorted(rkey, lkey.astype(np.int64) + w, "right")
                         - np.searchsorted(rkey, lkey.astype(np.int64) - w, "left")).sum())
        # w = 0 is the equi-join; widening the band never loses a row
        e_l, e_r, e_J = oracle.join(lkey, rkey, lrow, rrow)
        z_l, z_r, z_J = oracle.join_band(lkey, rkey, 0, lrow, rrow)
        assert z_J == e_J and np.array_equal(z_l, e_l) and np.array_equal(z_r, e_r)
        assert oracle.join_band(lkey, rkey, w + 1)[2] >= J


def check_pack_keys():
    rng = _rng(41)
    bits = [7, 11, 5]
    cols = [rng.integers(0, 1 << b, 5000).astype(np.int32) for b in bits]
    packed, bad = oracle.pack_keys(cols, bits)
    assert bad == 0
    # the packed order is the tuples' lexicographic order (numpy lexsort, last key primary)
    assert np.array_equal(np.argsort(packed, kind="stable"), np.lexsort(cols[::-1]))
    # unpacking by shifts returns every column
    assert np.array_equal(packed >> 16, cols[0]) and np.array_equal((packed >> 5) & 2047, cols[1])
    assert np.array_equal(packed & 31, cols[2])
    # a composite-key join is the join of the packed keys: brute force over tuples
    a = [rng.integers(0, 4, 60).astype(np.int32), rng.integers(0, 3, 60).astype(np.int32)]
    b = [rng.integers(0, 4, 40).astype(np.int32), rng.integers(0, 3, 40).astype(np.int32)]
    ka, _ = oracle.pack_keys(a, [2, 2])
    kb, _ = oracle.pack_keys(b, [2, 2])
    ol, orr, J = oracle.join(ka, kb)
    want = [(i, j) for i in range(60) for j in range(40) if a[0][i] == b[0][j] and a[1][i] == b[1][j]]
    assert J == len(want) and list(zip(ol.tolist(), orr.tolist())) == want
    # values outside their width are counted
    assert oracle.pack_keys([np.array([3, 4, -1], np.int32)], [2])[1] == 2


# --------------------------------------------------------------------------- group-by

def _random_expr(rng, ncols, depth):
    """A random expression tree as a postfix program, and the same tree as a numpy evaluator."""
    O = oracle
    if depth == 0 or rng.random() < 0.25:
        if rng.random() < 0.6:
            c = int(rng.integers(0, ncols))
            return [(O.X_COL, c)], lambda cols, c=c: cols[c].astype(np.int64)
        k = int(rng.integers(-50, 50))
        return [(O.X_CONST, k)], lambda cols, k=k: np.full(len(cols[0]), k, np.int64)
    op = int(rng.choice([O.X_ADD, O.X_SUB, O.X_MUL, O.X_NEG, O.X_LT, O.X_LE, O.X_GT, O.X_GE, O.X_EQ, O.X_NE,
                         O.X_AND, O.X_OR, O.X_NOT, O.X_SELECT]))
    ar = 1 if op in (O.X_NEG, O.X_NOT) else 3 if op == O.X_SELECT else 2
    kids = [_random_expr(rng, ncols, depth - 1) for _ in range(ar)]
    prog = [i for k in kids for i in k[0]] + [(op, 0)]
    f = [k[1] for k in kids]
    with np.errstate(over="ignore"):
        ev = {O.X_ADD: lambda c: f[0](c) + f[1](c), O.X_SUB: lambda c: f[0](c) - f[1](c),
              O.X_MUL: lambda c: f[0](c) * f[1](c), O.X_NEG: lambda c: -f[0](c),
              O.X_LT: lambda c: (f[0](c) < f[1](c)).astype(np.int64),
              O.X_LE: lambda c: (f[0](c) <= f[1](c)).astype(np.int64),
              O.X_GT: lambda c: (f[0](c) > f[1](c)).astype(np.int64),
              O.X_GE: lambda c: (f[0](c) >= f[1](c)).astype(np.int64),
              O.X_EQ: lambda c: (f[0](c) == f[1](c)).astype(np.int64),
              O.X_NE: lambda c: (f[0](c) != f[1](c)).astype(np.int64),
              O.X_AND: lambda c: np.logical_and(f[0](c), f[1](c)).astype(np.int64),
              O.X_OR: lambda c: np.logical_or(f[0](c), f[1](c)).astype(np.int64),
              O.X_NOT: lambda c: np.logical_not(f[0](c)).astype(np.int64),
              O.X_SELECT: lambda c: np.where(f[0](c) != 0, f[1](c), f[2](c))}[op]
    return prog, ev


def check_eval():
    O = oracle
    rng = _rng(16)
    for trial in range(40):
        n = int(rng.integers(1, 300))
        cols = [rng.integers(-10**6, 10**6, n).astype(np.int64), rng.integers(-3, 4, n).astype(np.int32),
                rng.integers(0, 2, n).astype(np.int8), rng.integers(-2**62, 2**62, n).astype(np.int64)]
        prog, ev = _random_expr(rng, len(cols), int(rng.integers(1, 5)))
        got, z = O.eval_expr(cols, prog)
        with np.errstate(over="ignore"):
            want = ev(cols)              # numpy's int64 arithmetic wraps the same way
        assert z == 0 and np.array_equal(got, want), ("expression", trial, prog)
    # division and remainder truncate toward zero (C), against hand-computed values
    a = np.array([7, -7, 7, -7, 0, 5, np.iinfo(np.int64).min, np.iinfo(np.int64).min], np.int64)
    b = np.array([2, 2, -2, -2, 3, 0, -1, 1], np.int64)
    q, z = O.eval_expr([a, b], [(O.X_COL, 0), (O.X_COL, 1), (O.X_DIV, 0)])
    assert q.tolist() == [3, -3, -3, 3, 0, 0, np.iinfo(np.int64).min, np.iinfo(np.int64).min] and z == 1
    r, z = O.eval_expr([a, b], [(O.X_COL, 0), (O.X_COL, 1), (O.X_MOD, 0)])
    assert r.tolist() == [1, -1, 1, -1, 0, 0, 0, 0] and z == 1
    nz = b != 0
    assert np.array_equal((q * b + r)[nz], a[nz])           # a = q * b + r wherever b != 0
    # identities: SELECT(c, x, x) = x, NOT NOT x = (x != 0), x - y = x + (-y)
    x = rng.integers(-5, 5, 100).astype(np.int64)
    y = rng.integers(-5, 5, 100).astype(np.int64)
    s1, _ = O.eval_expr([x, y], [(O.X_COL, 1), (O.X_COL, 0), (O.X_COL, 0), (O.X_SELECT, 0)])
    s2, _ = O.eval_expr([x, y], [(O.X_COL, 0), (O.X_NOT, 0), (O.X_NOT, 0)])
    s3, _ = O.eval_expr([x, y], [(O.X_COL, 0), (O.X_COL, 1), (O.X_SUB, 0)])
    s4, _ = O.eval_expr([x, y], [(O.X_COL, 0), (O.X_COL, 1), (O.X_NEG, 0), (O.X_ADD, 0)])
    assert np.array_equal(s1, x) and np.array_equal(s2, (x != 0).astype(np.int64)) and np.array_equal(s3, s4)
    # malformed programs are refused
    for bad in ([(O.X_ADD, 0)], [(O.X_CONST, 1), (O.X_CONST, 2)], [(O.X_COL, 5)], [(99, 0)], []):
        try:
            O.eval_expr([x], bad)
        except ValueError:
            continue
        raise AssertionError(("malformed program accepted", bad))


def check_join_chain():
    rng = _rng(15)
    for trial in range(8):
        hops = int(rng.integers(1, 4))
        sizes = [int(rng.integers(0, 40)) for _ in range(hops + 1)]
        doms = [int(rng.integers(1, 12)) for _ in range(hops)]
        outs = [rng.integers(0, doms[t], sizes[t]).astype(np.int32) for t in range(hops)]
        pks = [rng.integers(0, doms[t], sizes[t + 1]).astype(np.int32) for t in range(hops)]
        got = oracle.join_chain(outs, pks)
        # brute force: grow the tuples hop by hop with Python loops, in input order
        tuples = [(i,) for i in range(sizes[0])]
        for t in range(hops):
            tuples = [tp + (j,) for tp in tuples for j in range(sizes[t + 1]) if outs[t][tp[-1]] == pks[t][j]]
        assert got.shape == (len(tuples), hops + 1), ("chain shape", trial)
        assert [tuple(r) for r in got.tolist()] == tuples, ("chain tuples", trial)
        # closed form for the count: path counts carried back with bincount
        c = np.ones(sizes[hops], np.int64)
        for t in range(hops - 1, -1, -1):
            per_key = np.bincount(pks[t], weights=c, minlength=doms[t]).astype(np.int64)
            c = per_key[outs[t]]
        assert len(got) == int(c.sum()), ("chain count", trial)
    # one hop is the plain join, in the same order
    lk = rng.integers(0, 30, 500).astype(np.int32)
    rk = rng.integers(0, 30, 200).astype(np.int32)
    wl, wr, _ = oracle.join(lk, rk)
    got = oracle.join_chain([lk], [rk])
    assert np.array_equal(got[:, 0], wl) and np.array_equal(got[:, 1], wr)
    # two hops equal a join, a gather of the next key through its right rows, and a second join
    pk1 = rng.integers(0, 30, 300).astype(np.int32)
    k1 = rng.integers(0, 50, 300).astype(np.int32)
    pk2 = rng.integers(0, 50, 80).astype(np.int32)
    a, b, _ = oracle.join(lk, pk1)
    i, c, _ = oracle.join(k1[b], pk2)
    got = oracle.join_chain([lk, k1], [pk1, pk2])
    assert np.array_equal(got, np.stack([a[i], b[i], c], axis=1).reshape(-1, 3))


def check_groupby():
    rng = _rng(4)
    for trial in range(10):
        n = int(rng.integers(0, 2000))
        keys = rng.integers(0, int(rng.integers(1, 60)), n).astype(np.int32)
        val = rng.integers(-10**9, 10**9, n).astype(np.int64)
        price = rng.integers(0, 10**7, n).astype(np.int64)
        k, s, c, a = oracle.groupby(keys, val, price)
        ref = {}
        for key, v, p in zip(keys.tolist(), val.tolist(), price.tolist()):
            e = ref.setdefault(key, [0, 0, 0])
            e[0] += v; e[1] += 1; e[2] += p
        assert k.tolist() == sorted(ref), ("group keys", trial)
        for i, key in enumerate(k.tolist()):
            assert s[i] == ref[key][0] and c[i] == ref[key][1], ("group aggregates", trial)
            # Python's int / int is correctly rounded: the exact average, rounded once
            assert a[i] == ref[key][2] / ref[key][1], ("avg rounding", trial)
        assert int(c.sum()) == n and int(s.sum()) == int(val.sum())   # conservation
    # one group: reduces to a plain sum and mean
    val = rng.integers(0, 10**9, 777).astype(np.int64)
    k, s, c, a = oracle.groupby(np.full(777, 5, np.int32), val, val)
    assert k.tolist() == [5] and s[0] == int(val.sum()) and c[0] == 777
    assert a[0] == int(val.sum()) / 777
    # empty input: no groups
    k, s, c, a = oracle.groupby(np.zeros(0, np.int32), np.zeros(0, np.int64), np.zeros(0, np.int64))
    assert len(k) == 0


def check_group_minmax():
    rng = _rng(14)
    for trial in range(10):
        n = int(rng.integers(1, 3000))
        keys = rng.integers(0, int(rng.integers(1, 80)), n).astype(np.int32)
        # few distinct values so that repeats inside a group are common
        val = rng.integers(-int(rng.integers(1, 50)), int(rng.integers(1, 50)), n).astype(np.int64)
        k, lo, hi, nd = oracle.group_minmax(keys, val)
        # library routines: sort by key, reduce each run
        o = np.argsort(keys, kind="stable")
        sk, sv = keys[o], val[o]
        heads = np.flatnonzero(np.r_[True, sk[1:] != sk[:-1]])
        assert np.array_equal(k, sk[heads]), ("keys", trial)
        assert np.array_equal(lo, np.minimum.reduceat(sv, heads)), ("min", trial)
        assert np.array_equal(hi, np.maximum.reduceat(sv, heads)), ("max", trial)
        pairs = np.unique(np.stack([keys.astype(np.int64), val]), axis=1)
        assert np.array_equal(nd, np.unique(pairs[0], return_counts=True)[1]), ("distinct", trial)
    # brute force on a tiny input, with Python sets
    keys = np.array([3, 1, 3, 3, 1, 7, 3], np.int32)
    val = np.array([5, -2, 5, -9, -2, 0, 4], np.int64)
    k, lo, hi, nd = oracle.group_minmax(keys, val)
    assert k.tolist() == [1, 3, 7] and lo.tolist() == [-2, -9, 0] and hi.tolist() == [-2, 5, 0]
    assert nd.tolist() == [1, 3, 1]
    # extremes of int64 survive; one constant group has min = max and one distinct value
    big = np.array([np.iinfo(np.int64).min, np.iinfo(np.int64).max, 0], np.int64)
    k, lo, hi, nd = oracle.group_minmax(np.zeros(3, np.int32), big)
    assert lo[0] == big[0] and hi[0] == big[1] and nd[0] == 3
    k, lo, hi, nd = oracle.group_minmax(np.full(50, 9, np.int32), np.full(50, 4, np.int64))
    assert k.tolist() == [9] and lo[0] == hi[0] == 4 and nd[0] == 1
    k, lo, hi, nd = oracle.group_minmax(np.zeros(0, np.int32), np.zeros(0, np.int64))
    assert len(k) == 0


# --------------------------------------------------------------------------- fragments

def brute_flags(fact, dim, D, c):
    """All fact x dim pairs, compared directly; aggregates in Python integers."""
    eq = fact["fk"][:, None] == dim["pk"][None, :]
    eq &= (fact["date"] < D)[:, None]
    eq &= (dim["seg"] == c)[None, :]
    fi, di = np.nonzero(eq)
    ref = {}
    for f in fi.tolist():
        g = int(fact["flagA"][f]) * 2 + int(fact["flagB"][f])
        e = ref.setdefault(g, [0, 0, 0])
        e[0] += REV(fact["price"][f], fact["disc"][f]); e[1] += 1; e[2] += int(fact["price"][f])
    return ref, len(fi)


def check_fragment_flags():
    for seed, n, m, fk_hi, D, c, dup in [(11, 2000, 200, 200, 2400, 1, False),
                                         (12, 1500, 150, 260, 1000, 3, False),
                                         (13, 1000, 300, 50, 2557, 0, True),
                                         (14, 500, 40, 40, 0, 1, False),
                                         (15, 0, 40, 40, 2400, 1, False),
                                         (16, 800, 90, 90, 2400, 9, False)]:
        fr = datagen.random_flags_fragment(seed, n, m, fk_hi, D, c, dup_dim=dup)
        got = oracle.fragment_flags(fr.fact, fr.dim, D, c)
        ref, J = brute_flags(fr.fact, fr.dim, D, c)
        assert got["join_rows"] == J, ("flags join size", seed)
        assert got["key"].tolist() == sorted(ref), ("flags groups", seed)
        for i, g in enumerate(got["key"].tolist()):
            s, cn, sp = ref[g]
            assert got["sum"][i] == s and got["cnt"][i] == cn, ("flags aggregates", seed)
            assert got["avg"][i] == sp / cn, ("flags avg", seed)


def check_fragment_flags_invariants():
    fr = datagen.config0()
    got = oracle.fragment_flags(fr.fact, fr.dim, fr.D, fr.c)
    f, d = fr.fact, fr.dim
    # J from histograms: sum over qualifying fact rows of the number of qualifying dim rows per key
    hits = np.bincount(d["pk"][d["seg"] == fr.c], minlength=1500)
    keep = f["date"] < fr.D
    w = hits[f["fk"]] * keep
    J = int(w.sum())
    assert got["join_rows"] == J and int(got["cnt"].sum()) == J
    v = f["price"] * (100 - f["disc"])
    assert int(got["sum"].sum()) == int((v * w).sum())                     # sum conservation
    g = f["flagA"].astype(np.int64) * 2 + f["flagB"]
    for i, key in enumerate(got["key"].tolist()):
        sel = w * (g == key)
        assert got["cnt"][i] == int(sel.sum()) and got["sum"][i] == int((v * sel).sum())
        assert got["avg"][i] == int((f["price"] * sel).sum()) / int(sel.sum())
    assert len(got["key"]) == 6                       # all six (flagA, flagB) groups occur


def brute_cust(fact, mid, D):
    eq = (fact["fk"][:, None] == mid["pk"][None, :]) & (fact["date"] < D)[:, None]
    fi, ri = np.nonzero(eq)
    ref = {}
    for f, r in zip(fi.tolist(), ri.tolist()):
        e = ref.setdefault(int(mid["custkey"][r]), [0, 0])
        e[0] += REV(fact["price"][f], fact["disc"][f]); e[1] += 1
    return ref, len(fi)


def check_fragment_cust():
    for seed, n, m, cust, D, k in [(21, 2000, 300, 40, 2400, 10), (22, 1200, 100, 500, 1800, 100),
                                    (23, 900, 200, 3, 2557, 5), (24, 0, 50, 10, 2400, 100)]:
        fr = datagen.config2(seed=seed, n=n, m=m, cust_hi=cust)
        got = oracle.fragment_cust(fr.fact, fr.mid, D, k)
        ref, J = brute_cust(fr.fact, fr.mid, D)
        assert got["join_rows"] == J and got["groups"] == len(ref), ("cust sizes", seed)
        assert got["key"].tolist() == sorted(ref), ("cust groups", seed)
        for i, g in enumerate(got["key"].tolist()):
            assert got["sum"][i] == ref[g][0] and got["cnt"][i] == ref[g][1], ("cust aggs", seed)
        order = sorted(ref, key=lambda g: (-ref[g][0], g))[:k]
        assert got["top_key"].tolist() == order, ("cust top-k", seed)
        assert got["top_sum"].tolist() == [ref[g][0] for g in order]
        assert got["top_cnt"].tolist() == [ref[g][1] for g in order]
    # mid keys with repeats: a many-to-many join
    fr = datagen.config2(seed=25, n=1500, m=200, cust_hi=30)
    mid = {"pk": datagen.uniform(25, datagen.COL_MID_PK, 200, 0, 120, np.int32),
           "custkey": fr.mid["custkey"]}
    got = oracle.fragment_cust(fr.fact, mid, 2400, 50)
    ref, J = brute_cust(fr.fact, mid, 2400)
    assert got["join_rows"] == J and got["key"].tolist() == sorted(ref), "cust many-to-many"
    for i, g in enumerate(got["key"].tolist()):
        assert got["sum"][i] == ref[g][0] and got["cnt"][i] == ref[g][1], "cust many-to-many aggs"


def check_topk_ties():
    # equal sums: custkey ascending decides
    fact = {"fk": np.array([0, 1, 2, 3], np.int32), "date": np.zeros(4, np.int32),
            "price": np.full(4, 100, np.int64), "disc": np.zeros(4, np.int64)}
    mid = {"pk": np.array([3, 2, 1, 0], np.int32), "custkey": np.array([9, 4, 7, 1], np.int32)}
    got = oracle.fragment_cust(fact, mid, 10, 3)
    assert got["top_key"].tolist() == [1, 4, 7] and got["top_sum"].tolist() == [10000] * 3


# --------------------------------------------------------------------------- general fragments

def _general_tables(rng, n, m, fk_hi, dup):
    fact = [rng.integers(0, fk_hi, n).astype(np.int32), rng.integers(-1000, 1000, n).astype(np.int32),
            rng.integers(-1000, 1000, n).astype(np.int64), rng.integers(0, 4, n).astype(np.int8)]
    pk = rng.integers(0, fk_hi, m) if dup else rng.permutation(max(m, fk_hi))[:m]
    dim = [pk.astype(np.int32), rng.integers(0, 4, m).astype(np.int8), rng.integers(-500, 500, m).astype(np.int32)]
    return fact, dim


def brute_general(fact, dim, fpred, dpred, fkey, dkey, group, aggs, topk):
    """Every fact x dim pair compared directly (numpy evaluators of the programs), groups in a dict,
    aggregates in Python integers; AVG by Python's correctly rounded integer division."""
    n = len(fact[0])
    keep_f = fpred(fact) != 0 if fpred else np.ones(n, bool)
    if dim is not None:
        keep_d = dpred(dim) != 0 if dpred else np.ones(len(dim[0]), bool)
        eq = (fact[fkey].astype(np.int64)[:, None] == dim[dkey].astype(np.int64)[None, :])
        eq &= keep_f[:, None] & keep_d[None, :]
        fi, di = np.nonzero(eq)
        cols = [c[fi] for c in fact] + [c[di] for c in dim]
    else:
        fi = np.flatnonzero(keep_f)
        cols = [c[fi] for c in fact]
    J = len(fi)
    keys = np.zeros(J, np.int64)
    for col, bits in group:
        keys = keys * (1 << bits) + (cols[col].astype(np.int64) & ((1 << bits) - 1))
    vals = [None if op == oracle.AGG_COUNT else ev(cols) for op, ev in aggs] if J else [None] * len(aggs)
    ref = {}
    for i in range(J):
        ref.setdefault(int(keys[i]), []).append(i)
    out = {}
    for k, rows in ref.items():
        res = []
        for (op, _), v in zip(aggs, vals):
            if op == oracle.AGG_COUNT:
                res.append(len(rows))
                continue
            xs = [int(v[i]) for i in rows]
            res.append({oracle.AGG_SUM: sum(xs), oracle.AGG_MIN: min(xs), oracle.AGG_MAX: max(xs),
                        oracle.AGG_AVG: sum(xs) / len(xs), oracle.AGG_COUNT_DISTINCT: len(set(xs))}[op])
        out[k] = res
    top = sorted(out, key=lambda k: (-out[k][0], k))[:topk] if topk and aggs else []
    return out, J, top


def _value_expr(rng, ncols):
    """An arithmetic value over the columns (a postfix program and its numpy evaluator): a*k + b,
    a - b, SELECT(a > k, b, c), -a + k or a*b, with random columns a, b, c and a small constant k."""
    O = oracle
    a, b, c = (int(x) for x in rng.integers(0, ncols, 3))
    k = int(rng.integers(-20, 20))
    i64 = lambda cols, i: cols[i].astype(np.int64)
    forms = [([(O.X_COL, a), (O.X_CONST, k), (O.X_MUL, 0), (O.X_COL, b), (O.X_ADD, 0)],
              lambda cols: i64(cols, a) * k + i64(cols, b)),
             ([(O.X_COL, a), (O.X_COL, b), (O.X_SUB, 0)], lambda cols: i64(cols, a) - i64(cols, b)),
             ([(O.X_COL, a), (O.X_CONST, k), (O.X_GT, 0), (O.X_COL, b), (O.X_COL, c), (O.X_SELECT, 0)],
              lambda cols: np.where(i64(cols, a) > k, i64(cols, b), i64(cols, c))),
             ([(O.X_COL, a), (O.X_NEG, 0), (O.X_CONST, k), (O.X_ADD, 0)], lambda cols: -i64(cols, a) + k),
             ([(O.X_COL, a), (O.X_COL, b), (O.X_MUL, 0)], lambda cols: i64(cols, a) * i64(cols, b))]
    return forms[int(rng.integers(0, len(forms)))]


def _pred_expr(rng, cols):
    """A predicate keeping a fair share of rows: a < k, or (a < k1) AND (b >= k2), or (a != k1) OR
    (b < k2), with thresholds drawn from the columns' own values."""
    O = oracle
    a, b = (int(x) for x in rng.integers(0, len(cols), 2))
    pick = lambda i: int(cols[i][int(rng.integers(0, len(cols[i])))]) if len(cols[i]) else 0
    k1, k2 = pick(a), pick(b)
    i64 = lambda cs, i: cs[i].astype(np.int64)
    forms = [([(O.X_COL, a), (O.X_CONST, k1), (O.X_LT, 0)], lambda cs: (i64(cs, a) < k1).astype(np.int64)),
             ([(O.X_COL, a), (O.X_CONST, k1), (O.X_LT, 0), (O.X_COL, b), (O.X_CONST, k2), (O.X_GE, 0), (O.X_AND, 0)],
              lambda cs: ((i64(cs, a) < k1) & (i64(cs, b) >= k2)).astype(np.int64)),
             ([(O.X_COL, a), (O.X_CONST, k1), (O.X_NE, 0), (O.X_COL, b), (O.X_CONST, k2), (O.X_LT, 0), (O.X_OR, 0)],
              lambda cs: ((i64(cs, a) != k1) | (i64(cs, b) < k2)).astype(np.int64))]
    return forms[int(rng.integers(0, len(forms)))]


def check_fragment_general():
    O = oracle
    rng = _rng(31)
    for trial in range(30):
        n, m = int(rng.integers(0, 400)), int(rng.integers(1, 120))
        fact, dim = _general_tables(rng, n, m, int(rng.integers(1, 150)), trial % 3 == 0)
        join = trial % 5 != 4
        nf, nd = len(fact), len(dim)
        ncol = nf + (nd if join else 0)
        fp, fev = (_random_expr(rng, nf, 2) if trial % 8 == 1 else _pred_expr(rng, fact)) if trial % 4 else ([], None)
        dp, dev_ = _pred_expr(rng, dim) if trial % 3 else ([], None)
        group = [(3, 2), (nf + 1, 2)] if join else [(3, 2)]
        if trial % 7 == 6:
            group = []
        aggs_p, aggs_e = [], []
        for op in (O.AGG_SUM, O.AGG_COUNT, O.AGG_MIN, O.AGG_MAX, O.AGG_AVG, O.AGG_COUNT_DISTINCT):
            prog, ev = _random_expr(rng, ncol, 2) if trial % 6 == 5 else _value_expr(rng, ncol)
            aggs_p.append((op, prog))
            aggs_e.append((op, ev))
        topk = int(rng.integers(0, 6))
        got = O.fragment_general(fact, dim if join else None, fp, dp if join else [], 0, 0, group, aggs_p, topk=topk)
        ref, J, top = brute_general(fact, dim if join else None, fev, dev_ if join else None, 0, 0, group, aggs_e,
                                    topk)
        assert got["join_rows"] == J, ("general join size", trial)
        assert got["key"].tolist() == sorted(ref), ("general groups", trial)
        for a in range(len(aggs_p)):
            want = [ref[k][a] for k in sorted(ref)]
            assert got["vals"][a].tolist() == want, ("general aggregate", trial, a)
        assert got["top_key"].tolist() == top, ("general top-k", trial)
        assert got["top_val"].tolist() == [ref[k][0] for k in top], ("general top-k values", trial)
    # the flags fragment written as a general one equals the flags fragment (pinned by brute force)
    fr = datagen.random_flags_fragment(77, 3000, 300, 300, 1500, 2, dup_dim=True)
    f, d = fr.fact, fr.dim
    fact = [f["fk"], f["date"], f["price"], f["disc"], f["flagA"], f["flagB"]]
    dim = [d["pk"], d["seg"]]
    rev = [(O.X_COL, 2), (O.X_CONST, 100), (O.X_COL, 3), (O.X_SUB, 0), (O.X_MUL, 0)]
    got = O.fragment_general(fact, dim, [(O.X_COL, 1), (O.X_CONST, fr.D), (O.X_LT, 0)],
                             [(O.X_COL, 1), (O.X_CONST, fr.c), (O.X_EQ, 0)], 0, 0, [(4, 2), (5, 1)],
                             [(O.AGG_SUM, rev), (O.AGG_COUNT, []), (O.AGG_AVG, [(O.X_COL, 2)])])
    want = O.fragment_flags(f, d, fr.D, fr.c)
    assert got["join_rows"] == want["join_rows"] and np.array_equal(got["key"], want["key"])
    assert np.array_equal(got["vals"][0], want["sum"]) and np.array_equal(got["vals"][1], want["cnt"])
    assert np.array_equal(got["vals"][2].view(np.int64), want["avg"].view(np.int64))
    # no join, no group: one group, COUNT = the kept rows, SUM = their plain sum
    x = _rng(32).integers(-100, 100, 1000).astype(np.int64)
    got = O.fragment_general([x], None, [(O.X_COL, 0), (O.X_CONST, 0), (O.X_GT, 0)], [], -1, 0, [],
                             [(O.AGG_COUNT, []), (O.AGG_SUM, [(O.X_COL, 0)])])
    assert got["key"].tolist() == [0] and got["vals"][0][0] == int((x > 0).sum())
    assert got["vals"][1][0] == int(x[x > 0].sum())
    # group values outside their width are counted; a malformed program is refused
    got = O.fragment_general([np.array([0, 5, 9], np.int32)], None, [], [], -1, 0, [(0, 3)], [(O.AGG_COUNT, [])])
    assert got["bad"] == 1 and got["key"].tolist() == [0, 1, 5]
    try:
        O.fragment_general([x], None, [(O.X_ADD, 0)], [], -1, 0, [], [(O.AGG_COUNT, [])])
    except ValueError:
        pass
    else:
        raise AssertionError("malformed predicate accepted")


ALL_CHECKS = [check_filter, check_sort, check_join, check_join_kinds, check_join_band, check_pack_keys,
              check_join_chain, check_eval, check_groupby, check_group_minmax, check_fragment_flags,
              check_fragment_flags_invariants, check_fragment_cust, check_topk_ties, check_fragment_general]
