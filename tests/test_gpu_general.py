"""General fragments (tqp_fragment_run) against the oracle's general fragment: random descriptors
(predicate programs on both sides, an equi-join or none, one or two packed group columns or none,
COUNT / SUM / MIN / MAX / AVG / COUNT(DISTINCT) over random value programs, an optional top-k) at
sizes that span many tiles with ragged tails; and the two fixed workloads written as descriptors
(the flags fragment of configs 0 / 1 and a scaled custkey fragment) against their own oracles."""
import numpy as np
import pytest

import datagen
import oracle
import pins

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(hip):
    return hip.Context(0)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(t, n=None):
    a = t.cpu().numpy()
    return a if n is None else a[:n]


def _check(got, want, topk):
    G = int(_np(got["d_ngroups"])[0])
    assert G == want["groups"]
    assert int(_np(got["d_join"])[0]) == want["join_rows"]
    assert np.array_equal(_np(got["key"], G), want["key"])
    for g, w in zip(got["vals"], want["vals"]):
        assert np.array_equal(_np(g, G).view(np.int64), np.asarray(w).view(np.int64))
    if topk:
        k = int(_np(got["d_topk"])[0])
        assert k == len(want["top_key"])
        assert np.array_equal(_np(got["top_key"], k), want["top_key"])
        assert np.array_equal(_np(got["top_val"], k), want["top_val"])


def _tables(rng, n, m, fk_hi, dup):
    fact = [rng.integers(0, fk_hi, n).astype(np.int32), rng.integers(-1000, 1000, n).astype(np.int32),
            rng.integers(-1000, 1000, n).astype(np.int64), rng.integers(0, 4, n).astype(np.int8),
            rng.integers(0, 2557, n).astype(np.int32)]
    pk = rng.integers(0, fk_hi, m) if dup else rng.permutation(max(m, fk_hi))[:m]
    dim = [pk.astype(np.int32), rng.integers(0, 5, m).astype(np.int8), rng.integers(-500, 500, m).astype(np.int32)]
    return fact, dim


def _random_case(trial):
    O = oracle
    rng = np.random.default_rng(9000 + trial)
    n = int(rng.choice([1000, 4097, 60_001, 250_003]))
    m = int(rng.choice([300, 20_011]))
    fk_hi = int(m * rng.choice([1.0, 1.25, 4.0]))              # match rates 1, 0.8 and 0.25
    dup = trial % 3 == 0                                          # repeated dim keys: a many-to-many join
    fact, dim = _tables(rng, n, m, fk_hi, dup)
    join = trial % 5 != 4
    nf, nd = len(fact), len(dim)
    ncol = nf + (nd if join else 0)
    fp = pins._pred_expr(rng, fact)[0] if trial % 4 else []
    dp = pins._pred_expr(rng, dim)[0] if join and trial % 3 == 1 else []
    if join:
        group = [[(3, 2)], [(3, 2), (nf + 1, 3)], [(nf + 1, 3), (4, 12)], [(nf + 2, 10)], []][trial % 5]
    else:
        group = [(3, 2), (1, 11)]                                 # fact column 1 holds negative values
    ops = [O.AGG_SUM, O.AGG_COUNT, O.AGG_MIN, O.AGG_MAX, O.AGG_AVG]
    if trial % 2 == 0:
        ops.append(O.AGG_COUNT_DISTINCT)
    aggs = [(op, [] if op == O.AGG_COUNT else pins._value_expr(rng, ncol)[0]) for op in ops]
    topk = int(rng.choice([0, 1, 10, 100]))
    kb = datagen.bits_for(max(fk_hi, m, 2))
    return fact, dim if join else None, fp, dp, group, aggs, topk, kb


@pytest.mark.parametrize("trial", range(16))
def test_general_random(hip, ctx, trial):
    """Random descriptors; a group column with values outside its width (dim column 2, fact column 1
    hold negative values) is masked into the key and raises the key-range flag, as in the oracle."""
    fact, dim, fp, dp, group, aggs, topk, kb = _random_case(trial)
    want = oracle.fragment_general(fact, dim, fp, dp, 0, 0, group, aggs, topk=topk, gcap=1 << 20)
    got = hip.fragment_run(ctx, [_dev(c) for c in fact], [_dev(c) for c in dim] if dim is not None else None, fp, dp,
                           0, 0, group, aggs, topk=topk, key_bits=kb, join_cap=max(1, want["join_rows"]),
                           gcap=max(1, want["groups"]))
    assert ctx.errors() == (hip.DEVERR_KEY_RANGE if want["bad"] else 0)
    _check(got, want, topk)


@pytest.mark.parametrize("trial", range(12))
def test_general_pushdown(hip, ctx, trial):
    """Descriptors that take the plan rules carrying values through the join sorts instead of row
    ids: one valued aggregate over fact columns (and COUNTs) grouped by one int32 dim column (both
    carried: here the dim key itself), the same with no group columns (the fact value alone), and
    several fact aggregates grouped by an int32 dim column holding negative values (the dim column
    alone; masked into the key, key-range flag).  Predicates on both sides, repeated dim keys,
    match rates 1 to 0.25; equal to the oracle's general fragment."""
    O = oracle
    rng = np.random.default_rng(9100 + trial)
    n = int(rng.choice([4097, 60_001, 250_003]))
    m = int(rng.choice([300, 20_011]))
    fk_hi = int(m * rng.choice([1.0, 1.25, 4.0]))
    fact, dim = _tables(rng, n, m, fk_hi, trial % 4 == 0)
    nf = len(fact)
    kb = datagen.bits_for(max(fk_hi, m, 2))
    fp = pins._pred_expr(rng, fact)[0] if trial % 2 else []
    dp = pins._pred_expr(rng, dim)[0] if trial % 4 == 1 else []
    shape = trial % 3
    if shape == 0:
        group = [(nf + 0, kb)]
        aggs = [(O.AGG_SUM, pins._value_expr(rng, nf)[0]), (O.AGG_COUNT, [])]
    elif shape == 1:
        group = []
        aggs = [(O.AGG_COUNT, []), (O.AGG_MAX, pins._value_expr(rng, nf)[0])]
    else:
        group = [(nf + 2, 10)]
        aggs = [(O.AGG_SUM, pins._value_expr(rng, nf)[0]), (O.AGG_MIN, pins._value_expr(rng, nf)[0]),
                (O.AGG_AVG, pins._value_expr(rng, nf)[0]), (O.AGG_COUNT, [])]
    topk = int(rng.choice([0, 10]))
    want = oracle.fragment_general(fact, dim, fp, dp, 0, 0, group, aggs, topk=topk, gcap=1 << 20)
    got = hip.fragment_run(ctx, [_dev(c) for c in fact], [_dev(c) for c in dim], fp, dp, 0, 0, group, aggs,
                           topk=topk, key_bits=kb, join_cap=max(1, want["join_rows"]), gcap=max(1, want["groups"]))
    assert ctx.errors() == (hip.DEVERR_KEY_RANGE if want["bad"] else 0)
    _check(got, want, topk)


@pytest.mark.parametrize("trial", range(12))
def test_general_bucket(hip, ctx, trial):
    """Descriptors that take the bucket group-by (one valued aggregate, SUM / MIN / MAX / AVG, with
    COUNTs; packed group keys of 19 to 27 bits, so one or two passes over the bits above the bucket
    and 2^8 to 2^13 keys per bucket): none, one or two COUNTs, a top-k ordered by the value or by a
    COUNT; equal to the oracle's general fragment."""
    O = oracle
    rng = np.random.default_rng(9300 + trial)
    n = [60_001, 250_003, 400_000][trial % 3]
    m = 20_011
    fact, dim = _tables(rng, n, m, int(m * [1.0, 1.25][trial % 2]), trial % 4 == 0)
    gb = [16, 18, 21, 24][trial % 4]
    fact.append(rng.integers(0, 1 << gb, n).astype(np.int32))
    nf = len(fact)
    group = [(nf + 1, 3), (nf - 1, gb)]
    vop = [O.AGG_SUM, O.AGG_MIN, O.AGG_MAX, O.AGG_AVG][(trial // 3) % 4]
    prog = pins._value_expr(rng, nf + len(dim))[0]
    shape = trial % 3
    aggs = [[(vop, prog), (O.AGG_COUNT, [])], [(O.AGG_COUNT, []), (vop, prog), (O.AGG_COUNT, [])],
            [(vop, prog)]][shape]
    topk = 0 if aggs[0][0] == O.AGG_AVG else [10, 100, 0, 1][trial % 4]
    fp = pins._pred_expr(rng, fact)[0] if trial % 2 else []
    kb = datagen.bits_for(int(m * 1.25))
    want = oracle.fragment_general(fact, dim, fp, [], 0, 0, group, aggs, topk=topk, gcap=1 << 20)
    got = hip.fragment_run(ctx, [_dev(c) for c in fact], [_dev(c) for c in dim], fp, [], 0, 0, group, aggs,
                           topk=topk, key_bits=kb, join_cap=max(1, want["join_rows"]), gcap=max(1, want["groups"]))
    assert ctx.errors() == (hip.DEVERR_KEY_RANGE if want["bad"] else 0)
    _check(got, want, topk)


@pytest.mark.parametrize("neg,vb", [(False, 0), (True, 0), (False, 32), (True, 32), (False, 64)])
def test_general_bucket_carried_key(hip, ctx, neg, vb):
    """The keyed bucket group-by: the fact value program rides the fact sort (int64, or int32 under
    value_bits = 32), the one int32 dim group column rides the dim sort, and the join emits (group
    key, value) with the group sort's digit counts: keys in range (18 bits), or with negative values
    (16 bits: masked into the key, key-range flag); equal to the oracle."""
    O = oracle
    rng = np.random.default_rng(9400 + neg)
    fact, dim = _tables(rng, 300_007, 20_011, 25_000, False)
    if not neg:
        dim[2] = rng.integers(0, 1 << 18, len(dim[2])).astype(np.int32)
    nf = len(fact)
    group = [(nf + 2, 16 if neg else 18)]
    aggs = [(O.AGG_SUM, [(O.X_COL, 2), (O.X_COL, 1), (O.X_MUL, 0)]), (O.AGG_COUNT, [])]
    fp = [(O.X_COL, 4), (O.X_CONST, 2000), (O.X_LT, 0)]
    want = O.fragment_general(fact, dim, fp, [], 0, 0, group, aggs, topk=10, gcap=1 << 20)
    got = hip.fragment_run(ctx, [_dev(c) for c in fact], [_dev(c) for c in dim], fp, [], 0, 0, group, aggs, topk=10,
                           key_bits=15, join_cap=max(1, want["join_rows"]), gcap=max(1, want["groups"]), value_bits=vb)
    assert ctx.errors() == (hip.DEVERR_KEY_RANGE if neg else 0)
    assert bool(want["bad"]) == neg
    _check(got, want, 10)


@pytest.mark.parametrize("op", [oracle.AGG_SUM, oracle.AGG_MIN, oracle.AGG_MAX, oracle.AGG_AVG])
def test_general_value32(hip, ctx, op):
    """value_bits = 32 with values spanning the whole int32 range (negative and positive extremes)
    for every valued aggregate, a COUNT first for the top-k (AVG) or the value (the others); equal
    to the oracle.  A value outside int32 raises the value-range flag."""
    O = oracle
    rng = np.random.default_rng(9500 + op)
    fact, dim = _tables(rng, 250_003, 20_011, 20_011, False)
    fact[2] = rng.integers(-(1 << 31), 1 << 31, len(fact[2])).astype(np.int64)
    dim[2] = rng.integers(0, 1 << 17, len(dim[2])).astype(np.int32)
    nf = len(fact)
    aggs = [(op, [(O.X_COL, 2)]), (O.AGG_COUNT, [])]
    if op == O.AGG_AVG:
        aggs = aggs[::-1]
    want = O.fragment_general(fact, dim, [], [], 0, 0, [(nf + 2, 17)], aggs, topk=20, gcap=1 << 20)
    got = hip.fragment_run(ctx, [_dev(c) for c in fact], [_dev(c) for c in dim], [], [], 0, 0, [(nf + 2, 17)], aggs,
                           topk=20, key_bits=15, join_cap=max(1, want["join_rows"]), gcap=max(1, want["groups"]),
                           value_bits=32)
    assert ctx.errors() == 0
    _check(got, want, 20)
    if op == O.AGG_SUM:
        big = [(O.X_COL, 2), (O.X_CONST, 2), (O.X_MUL, 0)]
        hip.fragment_run(ctx, [_dev(c) for c in fact], [_dev(c) for c in dim], [], [], 0, 0, [(nf + 2, 17)],
                         [(O.AGG_SUM, big), (O.AGG_COUNT, [])], key_bits=15, gcap=1 << 17, value_bits=32)
        assert ctx.errors() == hip.DEVERR_VALUE_RANGE


@pytest.mark.parametrize("trial", range(6))
def test_general_direct(hip, ctx, trial):
    """Descriptors that take the direct group-by (packed keys of at most 9 bits, no COUNT(DISTINCT)):
    every aggregate, MIN / MAX over values of both signs up to 2^52, several valued
    aggregates, with and without a join, a top-k; fewer group slots than groups (capacity flag,
    the first gcap groups exact); equal to the oracle's general fragment."""
    O = oracle
    rng = np.random.default_rng(9600 + trial)
    n = [60_001, 250_003, 4097][trial % 3]
    fact, dim = _tables(rng, n, 20_011, 20_011, trial % 2 == 0)
    ext = np.array([-(1 << 52), 1 << 52, -1, 0, 1], np.int64)      # large, and the oracle's sums stay exact
    fact.append(np.where(rng.random(n) < 0.01, rng.choice(ext, n), fact[2]).astype(np.int64))
    nf = len(fact)
    join = trial % 3 != 2
    group = [[(3, 2), (nf + 1, 3)], [(4, 9)], [(3, 2)], [(nf + 1, 3), (3, 2), (3, 1)], [], [(1, 5)]][trial]
    if not join:
        group = [g for g in group if g[0] < nf]
    ops = [O.AGG_SUM, O.AGG_COUNT, O.AGG_MIN, O.AGG_MAX, O.AGG_AVG]
    src = {O.AGG_SUM: 2, O.AGG_MIN: 5, O.AGG_MAX: 5, O.AGG_AVG: 1}      # column 5: values of +-2^52 mixed in
    aggs = [(op, [] if op == O.AGG_COUNT else [(O.X_COL, src[op])]) for op in ops]
    if trial % 2:
        aggs = aggs[1:] + aggs[:1]
    topk = [0, 5, 100][trial % 3] if aggs[0][0] != O.AGG_AVG else 0
    fp = pins._pred_expr(rng, fact)[0] if trial % 2 else []
    want = O.fragment_general(fact, dim if join else None, fp, [], 0, 0, group, aggs, topk=topk, gcap=1 << 20)
    kw = dict(topk=topk, key_bits=15, join_cap=max(1, want["join_rows"]), gcap=max(1, want["groups"]))
    got = hip.fragment_run(ctx, [_dev(c) for c in fact], [_dev(c) for c in dim] if join else None, fp, [],
                           0 if join else -1, 0, group, aggs, **kw)
    assert ctx.errors() == (hip.DEVERR_KEY_RANGE if want["bad"] else 0)
    _check(got, want, topk)
    if want["groups"] > 3:
        cap = want["groups"] // 2
        kw["gcap"] = cap
        got = hip.fragment_run(ctx, [_dev(c) for c in fact], [_dev(c) for c in dim] if join else None, fp, [],
                               0 if join else -1, 0, group, aggs, **kw)
        assert ctx.errors() & hip.DEVERR_CAPACITY
        assert int(_np(got["d_ngroups"])[0]) == want["groups"]
        assert np.array_equal(_np(got["key"], cap), want["key"][:cap])
        for g, w in zip(got["vals"], want["vals"]):
            assert np.array_equal(_np(g, cap).view(np.int64), np.asarray(w)[:cap].view(np.int64))


def test_general_fact_order(hip, ctx):
    """A flags-style descriptor over 16M fact rows whose columns read through the pairs (flags,
    price, disc: 18 B a row, 288 MB) outgrow the last-level cache, so the joined pairs are first
    sorted by fact row; every aggregate, equal to the oracle's general fragment."""
    O = oracle
    fact = datagen.fact_table(4242, 16_000_000, 400_000)
    dim = datagen.dim_table(4242, 400_000)
    fc = [fact[k] for k in ("fk", "date", "price", "disc", "flagA", "flagB")]
    dc = [dim["pk"], dim["seg"]]
    rev = [(O.X_COL, 2), (O.X_CONST, 100), (O.X_COL, 3), (O.X_SUB, 0), (O.X_MUL, 0)]
    aggs = [(O.AGG_SUM, rev), (O.AGG_COUNT, []), (O.AGG_AVG, [(O.X_COL, 2)]), (O.AGG_MIN, [(O.X_COL, 3)]),
            (O.AGG_MAX, [(O.X_COL, 2)])]
    fp = [(O.X_COL, 1), (O.X_CONST, 2400), (O.X_LT, 0)]
    dp = [(O.X_COL, 1), (O.X_CONST, 1), (O.X_EQ, 0)]
    group = [(4, 2), (5, 1)]
    want = O.fragment_general(fc, dc, fp, dp, 0, 0, group, aggs, topk=3, gcap=8)
    got = hip.fragment_run(ctx, [_dev(c) for c in fc], [_dev(c) for c in dc], fp, dp, 0, 0, group, aggs, topk=3,
                           key_bits=datagen.bits_for(400_000), gcap=8)
    assert ctx.errors() == 0
    _check(got, want, 3)


@pytest.mark.parametrize("n,m", [(0, 1000), (1000, 0), (1, 1)])
def test_general_keyed_empty(hip, ctx, n, m):
    """The keyed bucket group-by and the direct group-by with an empty or one-row side: no joined
    rows and no groups (or the single match), with and without a top-k."""
    O = oracle
    rng = np.random.default_rng(n + 7 * m)
    fact, dim = _tables(rng, n, max(m, 1), 5, False)
    dim = [c[:m] for c in dim]
    dim[2] = rng.integers(0, 1 << 18, m).astype(np.int32)
    if n and m:
        dim[0][:] = fact[0][0]                     # the one row matches
    nf = len(fact)
    for group, aggs, vb in (([(nf + 2, 18)], [(O.AGG_SUM, [(O.X_COL, 2)]), (O.AGG_COUNT, [])], 32),
                            ([(3, 2)], [(O.AGG_SUM, [(O.X_COL, 2)]), (O.AGG_MAX, [(O.X_COL, 1)])], 0)):
        for topk in (0, 5):
            want = O.fragment_general(fact, dim, [], [], 0, 0, group, aggs, topk=topk, gcap=4)
            got = hip.fragment_run(ctx, [_dev(c) for c in fact], [_dev(c) for c in dim], [], [], 0, 0, group, aggs,
                                   topk=topk, key_bits=10, gcap=4, value_bits=vb)
            assert ctx.errors() == 0
            _check(got, want, topk)


@pytest.mark.parametrize("digit_bits", [4, 11])
def test_general_digit_widths(hip, ctx, digit_bits):
    """The plan rules under 4- and 11-bit radix digits (other pass counts, bucket widths and join
    low bits): the keyed bucket group-by (32-bit value), the bucket group-by through the pairs,
    the direct group-by and the fact-sorted pairs, each equal to the oracle."""
    O = oracle
    rng = np.random.default_rng(9700 + digit_bits)
    fact, dim = _tables(rng, 250_003, 20_011, 25_000, False)
    dim[2] = rng.integers(0, 1 << 19, len(dim[2])).astype(np.int32)
    nf = len(fact)
    cases = [([(nf + 2, 19)], [(O.AGG_SUM, [(O.X_COL, 2), (O.X_COL, 1), (O.X_MUL, 0)]), (O.AGG_COUNT, [])], 10, 32),
             ([(nf + 1, 3), (nf + 2, 19)], [(O.AGG_MAX, [(O.X_COL, 2), (O.X_COL, nf + 1), (O.X_ADD, 0)])], 5, 0),
             ([(3, 2), (nf + 1, 3)], [(O.AGG_SUM, [(O.X_COL, 2)]), (O.AGG_MIN, [(O.X_COL, 1)]), (O.AGG_COUNT, [])], 3, 0)]
    ctx.set_digit_bits(digit_bits)
    try:
        for group, aggs, topk, vb in cases:
            want = O.fragment_general(fact, dim, [(O.X_COL, 4), (O.X_CONST, 2000), (O.X_LT, 0)], [], 0, 0, group, aggs,
                                      topk=topk, gcap=1 << 20)
            got = hip.fragment_run(ctx, [_dev(c) for c in fact], [_dev(c) for c in dim],
                                   [(O.X_COL, 4), (O.X_CONST, 2000), (O.X_LT, 0)], [], 0, 0, group, aggs, topk=topk,
                                   key_bits=15, join_cap=max(1, want["join_rows"]), gcap=max(1, want["groups"]),
                                   value_bits=vb)
            assert ctx.errors() == 0
            _check(got, want, topk)
    finally:
        ctx.set_digit_bits(8)


def test_general_bucket_capacity_and_empty(hip, ctx):
    """The bucket group-by with fewer group slots than groups (capacity flag, the true group count,
    the first gcap groups exact, top-k over the written groups as the oracle's) and with no joined
    rows (an empty dim table)."""
    O = oracle
    rng = np.random.default_rng(78)
    fact, dim = _tables(rng, 200_000, 5000, 5000, False)
    fact.append(rng.integers(0, 1 << 20, 200_000).astype(np.int32))
    aggs = [(O.AGG_SUM, [(O.X_COL, 2)]), (O.AGG_COUNT, [])]
    group = [(len(fact) - 1, 20)]
    want = O.fragment_general(fact, dim, [], [], 0, 0, group, aggs, gcap=1000)
    got = hip.fragment_run(ctx, [_dev(c) for c in fact], [_dev(c) for c in dim], [], [], 0, 0, group, aggs,
                           key_bits=13, gcap=1000)
    assert ctx.errors() == hip.DEVERR_CAPACITY
    assert int(_np(got["d_ngroups"])[0]) == want["groups"] > 1000
    assert np.array_equal(_np(got["key"], 1000), want["key"][:1000])
    assert np.array_equal(_np(got["vals"][0], 1000), want["vals"][0][:1000])
    assert np.array_equal(_np(got["vals"][1], 1000), want["vals"][1][:1000])
    empty = [c[:0] for c in dim]
    want = O.fragment_general(fact, empty, [], [], 0, 0, group, aggs, topk=5, gcap=4)
    got = hip.fragment_run(ctx, [_dev(c) for c in fact], [_dev(c) for c in empty], [], [], 0, 0, group, aggs, topk=5,
                           key_bits=13, gcap=4)
    assert ctx.errors() == 0
    _check(got, want, 5)


@pytest.mark.parametrize("n,m", [(0, 10), (1, 1), (10, 0), (250_003, 0)])
def test_general_empty(hip, ctx, n, m):
    """Empty and one-row sides: no joined rows and no groups (or the single match); 250,003 fact
    rows against an empty dim table (the fact sort leaves low bits to the join)."""
    O = oracle
    rng = np.random.default_rng(n + 3 * m)
    fact, dim = _tables(rng, n, max(m, 1), 5, False)
    dim = [c[:m] for c in dim]
    aggs = [(O.AGG_SUM, [(O.X_COL, 2)]), (O.AGG_COUNT, []), (O.AGG_COUNT_DISTINCT, [(O.X_COL, 1)])]
    want = O.fragment_general(fact, dim, [], [], 0, 0, [(3, 2)], aggs, topk=5, gcap=4)
    got = hip.fragment_run(ctx, [_dev(c) for c in fact], [_dev(c) for c in dim], [], [], 0, 0, [(3, 2)], aggs,
                           topk=5, key_bits=4, gcap=4)
    assert ctx.errors() == 0
    _check(got, want, 5)


def test_general_flags_descriptor(hip, ctx):
    """Config 1's flags fragment (6M fact rows) as a descriptor equals the flags fragment's oracle."""
    O = oracle
    fr = datagen.config1()
    f, d = fr.fact, fr.dim
    fact = [f["fk"], f["date"], f["price"], f["disc"], f["flagA"], f["flagB"]]
    dim = [d["pk"], d["seg"]]
    rev = [(O.X_COL, 2), (O.X_CONST, 100), (O.X_COL, 3), (O.X_SUB, 0), (O.X_MUL, 0)]
    got = hip.fragment_run(ctx, [_dev(c) for c in fact], [_dev(c) for c in dim],
                           [(O.X_COL, 1), (O.X_CONST, fr.D), (O.X_LT, 0)], [(O.X_COL, 1), (O.X_CONST, fr.c), (O.X_EQ, 0)],
                           0, 0, [(4, 2), (5, 1)], [(O.AGG_SUM, rev), (O.AGG_COUNT, []), (O.AGG_AVG, [(O.X_COL, 2)])],
                           key_bits=fr.key_bits, gcap=8)
    want = O.fragment_flags(f, d, fr.D, fr.c)
    assert ctx.errors() == 0
    G = int(_np(got["d_ngroups"])[0])
    assert G == len(want["key"]) and int(_np(got["d_join"])[0]) == want["join_rows"]
    assert np.array_equal(_np(got["key"], G), want["key"])
    assert np.array_equal(_np(got["vals"][0], G), want["sum"]) and np.array_equal(_np(got["vals"][1], G), want["cnt"])
    assert np.array_equal(_np(got["vals"][2], G).view(np.int64), want["avg"].view(np.int64))


def test_general_custkey_descriptor(hip, ctx):
    """A scaled custkey fragment (1.5M fact rows, 400k mid rows, 50k custkeys) as a descriptor: group
    by a dim column, SUM and COUNT, top-100 by the sum; equals the custkey fragment's oracle."""
    O = oracle
    fr = datagen.config2(seed=71, n=1_500_000, m=400_000, cust_hi=50_000)
    f, m = fr.fact, fr.mid
    rev = [(O.X_COL, 2), (O.X_CONST, 100), (O.X_COL, 3), (O.X_SUB, 0), (O.X_MUL, 0)]
    got = hip.fragment_run(ctx, [_dev(f[k]) for k in ("fk", "date", "price", "disc")], [_dev(m["pk"]), _dev(m["custkey"])],
                           [(O.X_COL, 1), (O.X_CONST, fr.D), (O.X_LT, 0)], [], 0, 0, [(5, 16)],
                           [(O.AGG_SUM, rev), (O.AGG_COUNT, [])], topk=100,
                           key_bits=datagen.bits_for(int(f["fk"].max()) + 1), gcap=fr.cust_hi)
    want = O.fragment_cust(f, m, fr.D, 100, gcap=fr.cust_hi)
    assert ctx.errors() == 0
    G = int(_np(got["d_ngroups"])[0])
    assert G == want["groups"] and int(_np(got["d_join"])[0]) == want["join_rows"]
    assert np.array_equal(_np(got["key"], G), want["key"])
    assert np.array_equal(_np(got["vals"][0], G), want["sum"]) and np.array_equal(_np(got["vals"][1], G), want["cnt"])
    k = int(_np(got["d_topk"])[0])
    assert np.array_equal(_np(got["top_key"], k), want["top_key"])
    assert np.array_equal(_np(got["top_val"], k), want["top_sum"])


def test_general_capacity_and_refusals(hip, ctx):
    """Fewer group slots than groups: the capacity flag, the true group count, the first gcap groups
    exact; malformed descriptors are refused before any launch."""
    O = oracle
    rng = np.random.default_rng(77)
    fact, dim = _tables(rng, 50_000, 2000, 2000, False)
    aggs = [(O.AGG_SUM, [(O.X_COL, 2)]), (O.AGG_COUNT, [])]
    want = O.fragment_general(fact, dim, [], [], 0, 0, [(0, 11)], aggs)
    got = hip.fragment_run(ctx, [_dev(c) for c in fact], [_dev(c) for c in dim], [], [], 0, 0, [(0, 11)], aggs,
                           key_bits=11, gcap=100)
    assert ctx.errors() == hip.DEVERR_CAPACITY
    assert int(_np(got["d_ngroups"])[0]) == want["groups"] > 100
    assert np.array_equal(_np(got["key"], 100), want["key"][:100])
    assert np.array_equal(_np(got["vals"][0], 100), want["vals"][0][:100])
    d = [_dev(c) for c in fact]
    for bad in (dict(fact_pred=[(O.X_ADD, 0)]), dict(group=[(0, 20), (1, 20)]),
                dict(aggs=[(O.AGG_SUM, [])]), dict(aggs=[(O.AGG_COUNT_DISTINCT, [(O.X_COL, 1)])] * 2),
                dict(topk=5, aggs=[(O.AGG_AVG, [(O.X_COL, 1)])])):
        kw = dict(fact_pred=[], group=[(3, 2)], aggs=[(O.AGG_COUNT, [])], topk=0)
        kw.update(bad)
        with pytest.raises(hip.TQPError):
            hip.fragment_run(ctx, d, None, kw["fact_pred"], [], -1, 0, kw["group"], kw["aggs"], topk=kw["topk"])
    assert ctx.errors() == 0
