"""HIP operators against the oracle, element by element, on the same seeded inputs.

Sizes span several tiles and a ragged tail (tiles are 4096 rows for the
filter, sort and group-by kernels, 1024 left rows for the join), plus the
empty and one-element cases.  Integer and index outputs must match bit for
bit; averages are one IEEE division of exact integers on both sides and must
match bit for bit too.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 63, 4095, 4096, 4097, 70_001, 300_007]


def _rng(seed):
    return np.random.default_rng(seed)


@pytest.fixture(scope="module")
def ctx(hip):
    return hip.Context(0)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(t, n=None):
    a = t.cpu().numpy()
    return a if n is None else a[:n]


# ------------------------------------------------------------------ filter
@pytest.mark.parametrize("n", SIZES)
def test_filter_parity(hip, ctx, n):
    rng = _rng(n + 1)
    date = rng.integers(0, 2557, n).astype(np.int32)
    seg = rng.integers(0, 5, n).astype(np.int8)
    price = rng.integers(90_000, 10_500_000, n).astype(np.int64)
    carry = rng.integers(-2**31, 2**31 - 1, n).astype(np.int32)
    cols = [date, seg, price]
    for preds in ([(0, oracle.LT, 2400)], [(0, oracle.LT, 2400), (1, oracle.EQ, 1)],
                  [(2, oracle.GE, 5_000_000), (0, oracle.NE, 7), (1, oracle.LE, 2)], [(0, oracle.LT, 0)]):
        want = oracle.filter_rows(cols, preds)
        rows, cout, cnt = hip.filter(ctx, [_dev(c) for c in cols], preds, carry=_dev(carry))
        k = int(_np(cnt)[0])
        assert k == len(want)
        assert np.array_equal(_np(rows, k), want)
        assert np.array_equal(_np(cout, k), carry[want])
    assert ctx.errors() == 0


def test_filter_capacity(hip, ctx):
    date = np.arange(10_000, dtype=np.int32) % 2557
    rows, _, cnt = hip.filter(ctx, [_dev(date)], [(0, oracle.LT, 2400)], cap=1000)
    want = oracle.filter_rows([date], [(0, oracle.LT, 2400)])
    assert int(_np(cnt)[0]) == len(want)
    assert np.array_equal(_np(rows, 1000), want[:1000])
    assert ctx.errors() == hip.DEVERR_CAPACITY


# ------------------------------------------------------------------ sort
@pytest.mark.parametrize("digit_bits", [4, 8, 11])
@pytest.mark.parametrize("key_bits", [1, 11, 18, 25, 31])
@pytest.mark.parametrize("n", [0, 1, 4097, 300_007])
def test_sort_parity(hip, ctx, digit_bits, key_bits, n):
    rng = _rng(key_bits * 7 + n)
    hi = min(2**key_bits, 2**31 - 1)
    keys = rng.integers(0, hi, n).astype(np.int32)
    if n > 10:
        keys[: n // 3] = keys[0]          # long runs of one key
    vals = rng.integers(-2**31, 2**31 - 1, n).astype(np.int32)
    ctx.set_digit_bits(digit_bits)
    try:
        wk, wv = oracle.sort_pairs(keys, vals)
        ko, vo = hip.sort(ctx, _dev(keys), _dev(vals), key_bits=key_bits)
        assert np.array_equal(_np(ko), wk) and np.array_equal(_np(vo), wv)
        wk2, perm = oracle.sort_pairs(keys)
        ko, po = hip.sort(ctx, _dev(keys), key_bits=key_bits, perm=True)
        assert np.array_equal(_np(ko), wk2) and np.array_equal(_np(po), perm)
        ko, _ = hip.sort(ctx, _dev(keys), key_bits=key_bits)
        assert np.array_equal(_np(ko), wk)
    finally:
        ctx.set_digit_bits(8)
    assert ctx.errors() == 0


@pytest.mark.parametrize("digit_bits", [4, 8, 11])
def test_sort_many_tiles_per_chunk(hip, ctx, digit_bits):
    """5M keys: the histogram kernel's chunks hold several tiles each (the
    first pass's pre-counted offsets span chunks), with a ragged last tile."""
    n = 5_000_003
    rng = _rng(811 + digit_bits)
    keys = rng.integers(0, 1 << 25, n).astype(np.int32)
    keys[1000:400_000] = 77            # a digit run across many tiles
    vals = np.arange(n, dtype=np.int32)
    ctx.set_digit_bits(digit_bits)
    try:
        wk, wv = oracle.sort_pairs(keys, vals)
        ko, vo = hip.sort(ctx, _dev(keys), _dev(vals), key_bits=25)
        assert np.array_equal(_np(ko), wk) and np.array_equal(_np(vo), wv)
    finally:
        ctx.set_digit_bits(8)
    assert ctx.errors() == 0


def test_sort_one_first_digit(hip, ctx):
    """16M keys whose first-pass digit is the same for every key (multiples of 256, 8-bit digits):
    every count of the histogram kernel lands on one counter per chunk.  Regression test for the
    histogram kernel clearing its counters between the tiles of a chunk, where the clearing store
    could land after the next tile's first increments (lost counts shift every later chunk by a
    wave's 64 rows).  Three calls, each against a stable sort."""
    n = 16_000_001
    rng = _rng(907)
    keys = (rng.integers(0, 25, n) * 256).astype(np.int32)
    vals = np.arange(n, dtype=np.int32)
    order = np.argsort(keys, kind="stable")
    wk, wv = keys[order], vals[order]
    dk, dv = _dev(keys), _dev(vals)
    for _ in range(3):
        ko, vo = hip.sort(ctx, dk, dv, key_bits=13)
        assert np.array_equal(_np(ko), wk) and np.array_equal(_np(vo), wv)
    assert ctx.errors() == 0


def test_sort_device_count(hip, ctx):
    import torch
    rng = _rng(5)
    keys = rng.integers(0, 1 << 20, 50_000).astype(np.int32)
    d_n = torch.tensor([33_333], dtype=torch.int64, device="cuda")
    ko, vo = hip.sort(ctx, _dev(keys), key_bits=20, perm=True, d_n=d_n)
    wk, wp = oracle.sort_pairs(keys[:33_333])
    assert np.array_equal(_np(ko, 33_333), wk) and np.array_equal(_np(vo, 33_333), wp)


def test_sort_key_range_flag(hip, ctx):
    keys = np.array([1, 2, 3, 1 << 12], dtype=np.int32)
    hip.sort(ctx, _dev(keys), key_bits=12)
    assert ctx.errors() & hip.DEVERR_KEY_RANGE


# ------------------------------------------------------------------ join
def _join_case(hip, ctx, lkey, rkey, cap=None):
    lkey = np.sort(lkey).astype(np.int32)
    rkey = np.sort(rkey).astype(np.int32)
    rng = _rng(len(lkey) + 3 * len(rkey))
    lrow = rng.permutation(max(1, len(lkey)))[: len(lkey)].astype(np.int32)
    rrow = rng.permutation(max(1, len(rkey)))[: len(rkey)].astype(np.int32)
    wl, wr, J = oracle.join(lkey, rkey, lrow, rrow, cap=cap)
    ol, orr, cnt = hip.join(ctx, _dev(lkey), _dev(rkey), _dev(lrow), _dev(rrow),
                            cap=cap if cap is not None else J)
    assert int(_np(cnt)[0]) == J
    w = len(wl)
    assert np.array_equal(_np(ol, w), wl) and np.array_equal(_np(orr, w), wr)


def _pairs_sorted(l, r):
    o = np.lexsort((r, l))
    return l[o], r[o]


@pytest.mark.parametrize("nl,nr,hi,sort", [(0, 10, 5, False), (10, 0, 5, False), (1, 1, 1, False),
                                           (5000, 300, 1500, False), (300_007, 40_000, 150_000, False),
                                           (200_000, 150_000, 150_000, True), (4097, 5, 3, False),
                                           (20_000, 20_000, 1_000_000, False), (100_000, 64_000, 1_000, False),
                                           (1_000_003, 3_000_000, 3_500_000, False),
                                           (400_000, 1_500_000, 25_000, False)])
def test_hash_join(hip, ctx, nl, nr, hi, sort):
    """Partitioned hash join of unsorted inputs against the oracle's join: the
    same set of (lrow, rrow) pairs (rows come in no fixed order, so both sides
    are compared sorted; the row ids are permutations, so the pairs are
    unique).  (100000, 64000, 1000): 64 right rows per key; (1000003,
    3000000, ...): 2048 partitions of about 1500 right rows; (400000,
    1500000, 25000): 60 right rows per key and partitions over the LDS
    table's row capacity (several table builds per partition)."""
    rng = _rng(nl * 5 + nr + hi)
    lkey = rng.integers(0, hi, nl).astype(np.int32)
    rkey = rng.integers(0, hi, nr).astype(np.int32)
    if sort:
        lkey, rkey = np.sort(lkey), np.sort(rkey)
    lrow = rng.permutation(max(1, nl))[:nl].astype(np.int32)
    rrow = rng.permutation(max(1, nr))[:nr].astype(np.int32)
    wl, wr, J = oracle.join(lkey, rkey, lrow, rrow)
    ol, orr, cnt = hip.hash_join(ctx, _dev(lkey), _dev(rkey), _dev(lrow), _dev(rrow), cap=max(J, 1))
    assert int(_np(cnt)[0]) == J
    gl, gr = _pairs_sorted(_np(ol, J), _np(orr, J))
    wl, wr = _pairs_sorted(wl, wr)
    assert np.array_equal(gl, wl) and np.array_equal(gr, wr)
    assert ctx.errors() == 0


def test_hash_join_hot_key_and_edges(hip, ctx):
    """One key on 10000 right rows (its partition takes several table builds) and
    on 300 left rows; element indexes as payloads (no row columns); a
    negative key (flagged, its row left out); the device row counts below the
    host bounds; an output capacity below the join size (capacity flag, the
    true count, only cap rows written)."""
    rng = _rng(4242)
    nl, nr = 50_000, 40_000
    lkey = rng.integers(0, 20_000, nl).astype(np.int32)
    rkey = rng.integers(0, 20_000, nr).astype(np.int32)
    rkey[:10_000] = 777
    lkey[rng.integers(0, nl, 300)] = 777
    wl, wr, J = oracle.join(lkey, rkey)
    ol, orr, cnt = hip.hash_join(ctx, _dev(lkey), _dev(rkey), cap=J)
    assert int(_np(cnt)[0]) == J and J > 2_500_000
    gl, gr = _pairs_sorted(_np(ol, J), _np(orr, J))
    wl, wr = _pairs_sorted(wl, wr)
    assert np.array_equal(gl, wl) and np.array_equal(gr, wr)
    assert ctx.errors() == 0
    # device counts: only the first 30000 left and 25000 right rows take part
    d_nl, d_nr = _dev(np.array([30_000], np.int64)), _dev(np.array([25_000], np.int64))
    wl, wr, J = oracle.join(lkey[:30_000], rkey[:25_000])
    ol, orr, cnt = hip.hash_join(ctx, _dev(lkey), _dev(rkey), cap=J, d_nl=d_nl, d_nr=d_nr)
    assert int(_np(cnt)[0]) == J
    gl, gr = _pairs_sorted(_np(ol, J), _np(orr, J))
    wl, wr = _pairs_sorted(wl, wr)
    assert np.array_equal(gl, wl) and np.array_equal(gr, wr)
    assert ctx.errors() == 0
    # a negative key
    lbad = lkey.copy()
    lbad[5] = -3
    keep = np.flatnonzero(lbad >= 0).astype(np.int32)
    wl, wr, J = oracle.join(lbad[keep], rkey, keep)
    ol, orr, cnt = hip.hash_join(ctx, _dev(lbad), _dev(rkey), cap=J)
    assert ctx.errors() == hip.DEVERR_KEY_RANGE
    assert int(_np(cnt)[0]) == J
    gl, gr = _pairs_sorted(_np(ol, J), _np(orr, J))
    wl, wr = _pairs_sorted(wl, wr)
    assert np.array_equal(gl, wl) and np.array_equal(gr, wr)
    # capacity below the join size: the true count, cap rows that are all join rows
    _, _, J = oracle.join(lkey, rkey)
    cap = J // 3
    ol, orr, cnt = hip.hash_join(ctx, _dev(lkey), _dev(rkey), cap=cap)
    assert int(_np(cnt)[0]) == J
    assert ctx.errors() == hip.DEVERR_CAPACITY
    gl, gr = _np(ol, cap), _np(orr, cap)
    assert np.array_equal(lkey[gl], rkey[gr])                  # every written row is a join row
    assert len(np.unique(gl.astype(np.int64) * nr + gr)) == cap     # no row written twice


@pytest.mark.parametrize("nl,nr,hi,w", [(0, 10, 5, 1), (10, 0, 5, 1), (1, 1, 1, 0), (5000, 300, 1500, 3),
                                        (300_007, 40_000, 150_000, 2), (200_000, 150_000, 150_000, 0),
                                        (4097, 5, 3, 1), (20_000, 20_000, 1_000_000, 40), (60_000, 50_000, 3_000, 5)])
def test_join_band(hip, ctx, nl, nr, hi, w):
    """Band join against the oracle (all pairs compared on the CPU, so the
    sizes stay small): rows, order and count; windows that fit the LDS
    staging and ones that do not (few distinct keys, wide bands)."""
    rng = _rng(nl * 3 + nr + w)
    lkey = np.sort(rng.integers(0, hi, nl)).astype(np.int32)
    rkey = np.sort(rng.integers(0, hi, nr)).astype(np.int32)
    lrow = rng.permutation(max(1, nl))[:nl].astype(np.int32)
    rrow = rng.permutation(max(1, nr))[:nr].astype(np.int32)
    # the rows from the contiguous ranges of the sorted right side (exact at any size) ...
    lo = np.searchsorted(rkey, lkey.astype(np.int64) - w, "left")
    cnt_ = np.searchsorted(rkey, lkey.astype(np.int64) + w, "right") - lo
    J = int(cnt_.sum())
    wl = np.repeat(lrow, cnt_)
    wr = rrow[np.repeat(lo, cnt_) + np.arange(J) - np.repeat(np.cumsum(cnt_) - cnt_, cnt_)]
    if nl * nr <= 2e9:
        # ... and, where all pairs can be compared, the oracle's
        ol_, or_, J2 = oracle.join_band(lkey, rkey, w, lrow, rrow)
        assert J2 == J and np.array_equal(ol_, wl) and np.array_equal(or_, wr)
    ol, orr, cnt = hip.join_band(ctx, _dev(lkey), _dev(rkey), w, _dev(lrow), _dev(rrow), cap=max(J, 1))
    assert int(_np(cnt)[0]) == J
    assert np.array_equal(_np(ol, J), wl) and np.array_equal(_np(orr, J), wr)
    assert ctx.errors() == 0


@pytest.mark.parametrize("bits", [[7, 11, 5], [3, 28], [31], [2, 2, 2, 2]])
def test_pack_keys(hip, ctx, bits):
    """Composite keys packed on the GPU equal the oracle's packing."""
    rng = _rng(sum(bits) * 13 + len(bits))
    n = 300_007
    cols = [rng.integers(0, 1 << b, n).astype(np.int32) for b in bits]
    want, bad = oracle.pack_keys(cols, bits)
    assert bad == 0
    got = hip.pack_keys(ctx, [_dev(c) for c in cols], bits)
    assert np.array_equal(_np(got), want)
    assert ctx.errors() == 0


def test_composite_key_join(hip, ctx):
    """A two-column equi-join: both sides packed, sorted and joined on the GPU,
    against the oracle's join of its own packed keys (brute force over tuples
    pins that the packed join is the tuple join)."""
    rng = _rng(99)
    a = [rng.integers(0, 500, 100_000).astype(np.int32), rng.integers(0, 64, 100_000).astype(np.int32)]
    b = [rng.integers(0, 500, 30_000).astype(np.int32), rng.integers(0, 64, 30_000).astype(np.int32)]
    ka, _ = oracle.pack_keys(a, [9, 6])
    kb, _ = oracle.pack_keys(b, [9, 6])
    sa, sb = np.argsort(ka, kind="stable"), np.argsort(kb, kind="stable")
    wl, wr, J = oracle.join(ka[sa], kb[sb], sa.astype(np.int32), sb.astype(np.int32))
    pa = hip.pack_keys(ctx, [_dev(c) for c in a], [9, 6])
    pb = hip.pack_keys(ctx, [_dev(c) for c in b], [9, 6])
    ka_s, pa_perm = hip.sort(ctx, pa, key_bits=15, perm=True)
    kb_s, pb_perm = hip.sort(ctx, pb, key_bits=15, perm=True)
    ol, orr, cnt = hip.join(ctx, ka_s, kb_s, pa_perm, pb_perm, cap=max(J, 1))
    assert int(_np(cnt)[0]) == J
    assert np.array_equal(_np(ol, J), wl) and np.array_equal(_np(orr, J), wr)
    assert ctx.errors() == 0


def test_pack_keys_range_flag(hip, ctx):
    cols = [np.array([1, 2, 3], np.int32), np.array([0, 8, 1], np.int32)]
    hip.pack_keys(ctx, [_dev(c) for c in cols], [4, 3])
    assert ctx.errors() & hip.DEVERR_KEY_RANGE


def _random_program(rng, ncols, length):
    """A valid postfix program of about `length` instructions, every operator included."""
    prog, sp = [], 0
    while len(prog) < length or sp != 1:
        can = [0, 1] if sp < 12 else []
        if sp >= 1:
            can += [oracle.X_NEG, oracle.X_NOT]
        if sp >= 2:
            can += list(range(2, 7)) + list(range(8, 16))
        if sp >= 3:
            can += [oracle.X_SELECT]
        if len(prog) >= length and sp > 1:
            can = [c for c in can if c not in (0, 1, oracle.X_NEG, oracle.X_NOT)]
        op = int(rng.choice(can))
        arg = int(rng.integers(0, ncols)) if op == 0 else int(rng.integers(-9, 10)) if op == 1 else 0
        prog.append((op, arg))
        sp += 1 if op in (0, 1) else 0 if op in (oracle.X_NEG, oracle.X_NOT) else -2 if op == oracle.X_SELECT else -1
    return prog


@pytest.mark.parametrize("n", [0, 1, 255, 4097, 300_007])
def test_eval(hip, ctx, n):
    """Random postfix programs (every operator, nested selects, divisions by columns that hold zeros)
    over int8 / int32 / int64 columns against the oracle's tree evaluation, element by element."""
    rng = _rng(n + 3)
    cols = [rng.integers(-10**6, 10**6, n).astype(np.int64), rng.integers(-3, 4, n).astype(np.int32),
            rng.integers(-2, 3, n).astype(np.int8), rng.integers(-2**62, 2**62, n).astype(np.int64)]
    dc = [_dev(c) for c in cols]
    for trial in range(12):
        prog = _random_program(rng, len(cols), int(rng.integers(1, 40)))
        want, z = oracle.eval_expr(cols, prog)
        got = _np(hip.eval_expr(ctx, dc, prog))
        assert np.array_equal(got, want), (trial, prog)
        assert ctx.errors() == (hip.DEVERR_VALUE_RANGE if z else 0), (trial, prog)


@pytest.mark.parametrize("n", [1, 513, 4097, 250_003])
def test_eval_wide(hip, ctx, n):
    """Programs reading 5 to 7 of seven columns (the 8-column kernel), each column a view that
    starts 1 to 3 elements into its allocation (so int8 and int32 columns begin off an 8-byte
    boundary), against the oracle element by element."""
    rng = _rng(n + 11)
    kinds = [np.int8, np.int32, np.int64, np.int8, np.int32, np.int64, np.int32]
    full = [rng.integers(-100, 100, n + 3).astype(k) for k in kinds]
    offs = [1, 3, 2, 1, 1, 3, 2]
    cols = [f[o:o + n] for f, o in zip(full, offs)]
    dc = [_dev(f)[o:o + n] for f, o in zip(full, offs)]
    for trial in range(8):
        want_cols = int(rng.integers(5, 8))
        prog = [(oracle.X_COL, c) for c in range(want_cols)] + [(oracle.X_ADD, 0)] * (want_cols - 1)
        mid = _random_program(rng, want_cols, int(rng.integers(3, 20)))
        prog = prog + mid + [(oracle.X_ADD, 0)]
        want, z = oracle.eval_expr(cols, prog)
        got = _np(hip.eval_expr(ctx, dc, prog))
        assert np.array_equal(got, want), (trial, prog)
        assert ctx.errors() == (hip.DEVERR_VALUE_RANGE if z else 0), (trial, prog)


@pytest.mark.parametrize("kinds", [[np.int64] * 2, [np.int64] * 4, [np.int32] * 2, [np.int32] * 4, [np.int8]])
def test_eval_one_type(hip, ctx, kinds):
    """Programs over columns of one element type (the kernels that load only that type), 70,001
    rows (a ragged last tile), against the oracle element by element."""
    n = 70_001
    rng = _rng(len(kinds) * 7 + np.dtype(kinds[0]).itemsize)
    cols = [rng.integers(-50, 50, n).astype(k) for k in kinds]
    dc = [_dev(c) for c in cols]
    for trial in range(6):
        prog = [(oracle.X_COL, c) for c in range(len(cols))] + [(oracle.X_SUB, 0)] * (len(cols) - 1)
        prog = prog + _random_program(rng, len(cols), int(rng.integers(1, 16))) + [(oracle.X_MUL, 0)]
        want, z = oracle.eval_expr(cols, prog)
        got = _np(hip.eval_expr(ctx, dc, prog))
        assert np.array_equal(got, want), (trial, prog)
        assert ctx.errors() == (hip.DEVERR_VALUE_RANGE if z else 0), (trial, prog)


def test_eval_edges(hip, ctx):
    X = oracle
    a = np.array([7, -7, 7, -7, 0, 5, np.iinfo(np.int64).min, np.iinfo(np.int64).min, np.iinfo(np.int64).max],
                 np.int64)
    b = np.array([2, 2, -2, -2, 3, 0, -1, 1, -1], np.int64)
    for op in (X.X_DIV, X.X_MOD, X.X_MUL, X.X_ADD, X.X_SUB):
        prog = [(X.X_COL, 0), (X.X_COL, 1), (op, 0)]
        want, z = oracle.eval_expr([a, b], prog)
        assert np.array_equal(_np(hip.eval_expr(ctx, [_dev(a), _dev(b)], prog)), want)
        assert ctx.errors() == (hip.DEVERR_VALUE_RANGE if z else 0)
    dn = _dev(np.array([4], np.int64))
    out = _np(hip.eval_expr(ctx, [_dev(a)], [(X.X_COL, 0), (X.X_CONST, 1), (X.X_ADD, 0)], d_n=dn))
    assert np.array_equal(out[:4], a[:4] + 1)
    for bad in ([(X.X_ADD, 0)], [(X.X_CONST, 1), (X.X_CONST, 2)], [(X.X_COL, 1)], [(99, 0)],
                [(X.X_CONST, 1)] * 17 + [(X.X_ADD, 0)] * 16):
        with pytest.raises(hip.TQPError):
            hip.eval_expr(ctx, [_dev(a)], bad)


@pytest.mark.parametrize("n,nsrc", [(0, 5), (1, 1), (4097, 100), (300_007, 2_000_000)])
def test_gather(hip, ctx, n, nsrc):
    rng = _rng(n + nsrc)
    idx = rng.integers(-1, nsrc, n).astype(np.int32)
    for dt in (np.int32, np.int64):
        src = rng.integers(-(1 << 30), 1 << 30, nsrc).astype(dt)
        out = _np(hip.gather(ctx, _dev(src), _dev(idx)))
        want = np.where(idx >= 0, src[np.maximum(idx, 0)], -1).astype(dt)
        assert out.dtype == dt and np.array_equal(out, want)
    assert ctx.errors() == 0
    if n:
        dn = _dev(np.array([n // 2], np.int64))
        src = rng.integers(0, 9, nsrc).astype(np.int32)
        out = _np(hip.gather(ctx, _dev(src), _dev(idx), d_n=dn))
        assert np.array_equal(out[:n // 2], np.where(idx >= 0, src[np.maximum(idx, 0)], -1)[:n // 2])


def test_gather_out_of_range(hip, ctx):
    src = np.arange(10, dtype=np.int32)
    out = _np(hip.gather(ctx, _dev(src), _dev(np.array([3, 10, 9], np.int32))))
    assert out.tolist() == [3, -1, 9]
    assert ctx.errors() == hip.DEVERR_KEY_RANGE


def _lex(rows):
    return rows[np.lexsort(rows.T[::-1])] if len(rows) else rows


@pytest.mark.parametrize("sizes,doms,pk_sorted", [
    ([1000, 300], [50], [False]),
    ([20_000, 5000, 800], [3000, 500], [False, False]),
    ([50_000, 20_000, 3000, 40], [20_000, 3000, 40], [True, False, True]),
    ([0, 100, 10], [10, 5], [False, False]),
    ([300_007, 100_000, 25], [100_000, 25], [True, True]),
])
def test_join_chain(hip, ctx, sizes, doms, pk_sorted):
    """Chains of one to three sort-based joins (sorted inputs where pk_sorted says so, so that
    hop skips its sort) against the oracle's nested chain, compared as sets of row tuples."""
    rng = _rng(sum(sizes) + len(doms))
    hops = len(doms)
    outs = [rng.integers(0, doms[t], sizes[t]).astype(np.int32) for t in range(hops)]
    pks = []
    for t in range(hops):
        k = rng.integers(0, doms[t], sizes[t + 1]).astype(np.int32)
        pks.append(np.sort(k) if pk_sorted[t] else k)
    want = oracle.join_chain(outs, pks)
    kb = [int(d - 1).bit_length() or 1 for d in doms] if hops > 1 else 0      # per hop, or the full width
    cols, J = hip.join_chain(ctx, [_dev(o) for o in outs], [_dev(p) for p in pks], pk_sorted=pk_sorted,
                             key_bits=kb, caps=[max(1, sizes[0] // 3)] * hops)  # small caps: hops rerun at their size
    assert J == len(want)
    got = np.stack([_np(c, J) for c in cols], axis=1) if J else np.zeros((0, hops + 1), np.int32)
    assert np.array_equal(_lex(got), _lex(want))


def test_join_chain_dense(hip, ctx):
    """Hops whose key column is 0..M-1 in order take the dense rule (a filter, no sort or join);
    left keys at or above M drop out; mixed with ordinary hops."""
    rng = _rng(93)
    outs = [rng.integers(0, 12_000, 200_000).astype(np.int32), rng.integers(0, 3000, 10_000).astype(np.int32),
            rng.integers(0, 40, 3000).astype(np.int32)]
    pks = [np.arange(10_000, dtype=np.int32), rng.integers(0, 3000, 3000).astype(np.int32),
           np.arange(40, dtype=np.int32)]
    want = oracle.join_chain(outs, pks)
    for dense in ([True, False, True], [False, False, False]):
        cols, J = hip.join_chain(ctx, [_dev(o) for o in outs], [_dev(p) for p in pks], pk_dense=dense,
                                 pk_sorted=[True, False, True])
        assert J == len(want)
        got = np.stack([_np(c, J) for c in cols], axis=1)
        assert np.array_equal(_lex(got), _lex(want))


def test_join_chain_dense_edges(hip, ctx):
    """The one-pass dense hop at its edges: negative keys and keys at or above M drop out, a dense
    table with no rows keeps no tuple (the next key is never read), and a dense last hop carries
    three earlier position columns."""
    rng = _rng(95)
    outs = [rng.integers(-50, 1100, 100_000).astype(np.int32), rng.integers(0, 700, 1000).astype(np.int32),
            rng.integers(-3, 30, 700).astype(np.int32)]
    pks = [np.arange(1000, dtype=np.int32), rng.permutation(700).astype(np.int32), np.arange(25, dtype=np.int32)]
    want = oracle.join_chain(outs, pks)
    cols, J = hip.join_chain(ctx, [_dev(o) for o in outs], [_dev(p) for p in pks], pk_dense=[True, False, True],
                             pk_sorted=[True, False, True])
    assert J == len(want) > 0
    got = np.stack([_np(c, J) for c in cols], axis=1)
    assert np.array_equal(_lex(got), _lex(want))
    empty = [outs[0], np.zeros(0, np.int32), outs[2]]
    pk0 = [np.zeros(0, np.int32), pks[1], pks[2]]
    cols, J = hip.join_chain(ctx, [_dev(o) for o in empty], [_dev(p) for p in pk0], pk_dense=[True, False, True],
                             pk_sorted=[True, False, True])
    assert J == 0 == len(oracle.join_chain(empty, pk0))
    assert ctx.errors() == 0


@pytest.mark.parametrize("digit_bits", [8, 4, 11])
def test_join_chain_dense_partitioned(hip, ctx, digit_bits):
    """The first dense hop into a table of at least 2^20 rows, entered by at least 2^20 tuples: a
    radix pass over the keys' top digit partitions the tuples (keys below 0 or at or above M take no
    part), then the dense pass reads them in that order.  Against the oracle, with a sort-based
    hop after it."""
    rng = _rng(131 + digit_bits)
    M, C = 1_200_000, 40_000
    outs = [rng.integers(-2000, M + 3000, 1_500_000).astype(np.int32), rng.integers(0, C, M).astype(np.int32)]
    pks = [np.arange(M, dtype=np.int32), rng.permutation(C).astype(np.int32)]
    want = oracle.join_chain(outs, pks)
    ctx.set_digit_bits(digit_bits)
    try:
        cols, J = hip.join_chain(ctx, [_dev(o) for o in outs], [_dev(p) for p in pks], pk_dense=[True, False],
                                 pk_sorted=[True, False])
    finally:
        ctx.set_digit_bits(8)
    assert J == len(want) > 1_400_000
    got = np.stack([_np(c, J) for c in cols], axis=1)
    assert np.array_equal(_lex(got), _lex(want))
    assert ctx.errors() == 0


@pytest.mark.parametrize("digit_bits", [4, 11])
def test_join_chain_digit_widths(hip, ctx, digit_bits):
    """A three-join chain (a dense hop, a sorted one, a shuffled one) under 4- and 11-bit radix
    digits, where the left sorts leave other low-bit widths to the join tiles; against the oracle."""
    rng = _rng(97 + digit_bits)
    outs = [rng.integers(0, 60_000, 400_000).astype(np.int32), rng.integers(0, 9000, 50_000).astype(np.int32),
            rng.integers(0, 700, 9000).astype(np.int32)]
    pks = [np.arange(50_000, dtype=np.int32), np.sort(rng.integers(0, 9000, 9000)).astype(np.int32),
           rng.permutation(700).astype(np.int32)]
    want = oracle.join_chain(outs, pks)
    ctx.set_digit_bits(digit_bits)
    try:
        cols, J = hip.join_chain(ctx, [_dev(o) for o in outs], [_dev(p) for p in pks], pk_dense=[True, False, False],
                                 pk_sorted=[True, True, False])
    finally:
        ctx.set_digit_bits(8)
    assert J == len(want) > 0
    got = np.stack([_np(c, J) for c in cols], axis=1)
    assert np.array_equal(_lex(got), _lex(want))
    assert ctx.errors() == 0


@pytest.mark.parametrize("rules", ["none", "mixed"])
def test_join_chain_six_hops(hip, ctx, rules):
    """Six joins over seven tables (the shape of Section 6.3's six-join query) in one launch
    sequence with every hop's size on the device, against the oracle's chain.  About 9% of each
    hop's keys find no match.  mixed: hops 0 and 3 take the dense rule, hop 1 (a sorted key column
    with duplicate keys) the sorted rule; its duplicates can push the tuples past the default
    bounds, so the chain may run again with larger ones."""
    rng = _rng(606 + len(rules))
    sizes = [400_000, 150_000, 60_000, 30_000, 10_000, 2_000, 25]
    outs = [rng.integers(0, int(sizes[t + 1] * 1.1), sizes[t]).astype(np.int32) for t in range(6)]
    pks, dense, srt = [], [], []
    for t in range(6):
        M = sizes[t + 1]
        if rules == "mixed" and t in (0, 3):
            pks.append(np.arange(M, dtype=np.int32))
        elif rules == "mixed" and t == 1:
            pks.append(np.sort(rng.integers(0, M, M)).astype(np.int32))
        else:
            pks.append(rng.permutation(M).astype(np.int32))
        dense.append(rules == "mixed" and t in (0, 3))
        srt.append(rules == "mixed" and t in (0, 1, 3))
    want = oracle.join_chain(outs, pks)
    kb = [int(int(sizes[t + 1] * 1.1) - 1).bit_length() for t in range(6)]
    cols, J = hip.join_chain(ctx, [_dev(o) for o in outs], [_dev(p) for p in pks], pk_sorted=srt, pk_dense=dense,
                             key_bits=kb)
    assert J == len(want) and J > 100_000
    got = np.stack([_np(c, J) for c in cols], axis=1)
    assert np.array_equal(_lex(got), _lex(want))
    assert ctx.errors() == 0


_KINDS = {"semi": 1, "anti": 2, "outer": 3, "inner": 0}


@pytest.mark.parametrize("kind", list(_KINDS))
@pytest.mark.parametrize("nl,nr,hi", [(0, 10, 5), (10, 0, 5), (1, 1, 1), (5000, 300, 1500), (300_007, 40_000, 150_000),
                                      (4097, 5, 3), (250_000, 60_000, 400_000), (20_000, 20_000, 1_000_000)])
def test_join_kinds(hip, ctx, kind, nl, nr, hi):
    """Left semi / anti / outer joins against the oracle: the rows, their
    order and the count, over windows that fit the LDS table and ones that
    do not (few distinct keys), with empty sides and partial tiles."""
    k = _KINDS[kind]
    rng = _rng(nl * 7 + nr + k)
    lkey = np.sort(rng.integers(0, hi, nl)).astype(np.int32)
    rkey = np.sort(rng.integers(0, hi, nr)).astype(np.int32)
    lrow = rng.permutation(max(1, nl))[:nl].astype(np.int32)
    rrow = rng.permutation(max(1, nr))[:nr].astype(np.int32)
    wl, wr, J = oracle.join_kind(k, lkey, rkey, lrow, rrow)
    ol, orr, cnt = hip.join(ctx, _dev(lkey), _dev(rkey), _dev(lrow), _dev(rrow), cap=max(J, 1), kind=k)
    assert int(_np(cnt)[0]) == J
    assert np.array_equal(_np(ol, J), wl)
    assert np.array_equal(_np(orr, J), wr)
    assert ctx.errors() == 0


def test_join_kind_capacity(hip, ctx):
    """Past the capacity only the count is exact and the flag is raised."""
    lkey = np.sort(_rng(3).integers(0, 100, 5000)).astype(np.int32)
    rkey = np.arange(0, 100, 2, dtype=np.int32)
    wl, wr, J = oracle.join_kind(3, lkey, rkey)
    ol, orr, cnt = hip.join(ctx, _dev(lkey), _dev(rkey), cap=1000, kind=3)
    assert int(_np(cnt)[0]) == J
    assert np.array_equal(_np(ol, 1000), wl[:1000]) and np.array_equal(_np(orr, 1000), wr[:1000])
    assert ctx.errors() == hip.DEVERR_CAPACITY


@pytest.mark.parametrize("nl,nr,hi", [(0, 10, 5), (10, 0, 5), (1, 1, 1), (5000, 300, 1500), (300_007, 40_000, 150_000),
                                      (200_000, 150_000, 150_000), (4097, 5, 3), (20_000, 20_000, 1_000_000)])
def test_join_parity(hip, ctx, nl, nr, hi):
    rng = _rng(nl * 31 + nr)
    _join_case(hip, ctx, rng.integers(0, hi, nl), rng.integers(0, hi, nr))
    assert ctx.errors() == 0


def test_join_pk_fk(hip, ctx):
    rng = _rng(11)
    pk = rng.permutation(100_000)
    fk = rng.integers(0, 125_000, 400_000)
    _join_case(hip, ctx, fk, pk)


def test_join_one_key_everywhere(hip, ctx):
    _join_case(hip, ctx, np.full(3000, 7), np.full(250, 7))     # J = 750,000 from one bucket


def test_join_wide_window(hip, ctx):
    # sparse left keys against a dense right side: each left tile spans far more
    # right rows than the LDS window holds (global binary-search path)
    rng = _rng(12)
    _join_case(hip, ctx, rng.integers(0, 2_000_000, 3000), rng.integers(0, 2_000_000, 1_500_000))


def test_join_capacity(hip, ctx):
    rng = _rng(13)
    _join_case(hip, ctx, rng.integers(0, 50, 20_000), rng.integers(0, 50, 2_000), cap=12_345)
    assert ctx.errors() == hip.DEVERR_CAPACITY


# ------------------------------------------------------------------ group-by
@pytest.mark.parametrize("n,domain", [(0, 5), (1, 5), (4097, 1), (70_001, 6), (300_007, 5000),
                                      (300_007, 1 << 20), (65_536, 65_536)])
def test_groupby_parity(hip, ctx, n, domain):
    rng = _rng(n + domain)
    keys = rng.integers(0, domain, n).astype(np.int32)
    val = rng.integers(0, 1_050_000_000, n).astype(np.int64)
    price = rng.integers(90_000, 10_500_000, n).astype(np.int64)
    wk, ws, wc, wa = oracle.groupby(keys, val, price)
    kb = max(1, int(domain - 1).bit_length())
    out = hip.groupby_agg(ctx, _dev(keys), _dev(val), _dev(price), key_bits=kb, gcap=max(1, len(wk)))
    G = int(_np(out["d_ngroups"])[0])
    assert G == len(wk)
    assert np.array_equal(_np(out["key"], G), wk)
    assert np.array_equal(_np(out["sum"], G), ws) and np.array_equal(_np(out["cnt"], G), wc)
    assert np.array_equal(_np(out["avg"], G).view(np.int64), wa.view(np.int64))   # bit-exact
    assert ctx.errors() == 0


@pytest.mark.parametrize("digit_bits", [4, 8, 11])
@pytest.mark.parametrize("n,domain", [(0, 5), (1, 5), (70_001, 6), (300_007, 5000), (300_007, 1 << 20),
                                      (1_000_003, 1 << 31)])
def test_groupby_sum_only(hip, ctx, n, domain, digit_bits):
    """Without an averaged column the values are sorted alongside the keys
    (8-byte payload) instead of gathered through the permutation; every
    digit width, and a device row count below the host bound."""
    rng = _rng(n + domain + digit_bits)
    keys = rng.integers(0, domain, n).astype(np.int32)
    val = rng.integers(-(1 << 50), 1 << 50, n).astype(np.int64)
    dn = n - n // 5
    wk, ws, wc, _ = oracle.groupby(keys[:dn], val[:dn])
    kb = max(1, int(domain - 1).bit_length())
    ctx.set_digit_bits(digit_bits)
    try:
        out = hip.groupby_agg(ctx, _dev(keys), _dev(val), key_bits=kb, gcap=max(1, len(wk)),
                              d_n=_dev(np.array([dn], np.int64)))
    finally:
        ctx.set_digit_bits(8)
    G = int(_np(out["d_ngroups"])[0])
    assert G == len(wk)
    assert np.array_equal(_np(out["key"], G), wk)
    assert np.array_equal(_np(out["sum"], G), ws) and np.array_equal(_np(out["cnt"], G), wc)
    assert ctx.errors() == 0


@pytest.mark.parametrize("digit_bits", [4, 8, 11])
@pytest.mark.parametrize("n,domain", [(5_000_003, 1 << 24), (2_000_000, 1 << 17)])
def test_groupby_bucket(hip, ctx, n, domain, digit_bits):
    """The sort-based group-by's bucket form (wide keys over many rows: the sort covers the key
    bits above the bucket, one or two passes, and each bucket of keys is summed and counted in LDS),
    a device row count below the host bound, and fewer group slots than groups (capacity flag, the
    first gcap groups exact)."""
    rng = _rng(n + digit_bits)
    keys = rng.integers(0, domain, n).astype(np.int32)
    val = rng.integers(-(1 << 40), 1 << 40, n).astype(np.int64)
    dn = n - 12345
    wk, ws, wc, _ = oracle.groupby(keys[:dn], val[:dn])
    kb = int(domain - 1).bit_length()
    ctx.set_digit_bits(digit_bits)
    try:
        out = hip.groupby_agg(ctx, _dev(keys), _dev(val), key_bits=kb, gcap=len(wk), d_n=_dev(np.array([dn], np.int64)))
        G = int(_np(out["d_ngroups"])[0])
        assert G == len(wk) and ctx.errors() == 0
        assert np.array_equal(_np(out["key"], G), wk)
        assert np.array_equal(_np(out["sum"], G), ws) and np.array_equal(_np(out["cnt"], G), wc)
        cap = len(wk) // 3
        out = hip.groupby_agg(ctx, _dev(keys), _dev(val), key_bits=kb, gcap=cap, d_n=_dev(np.array([dn], np.int64)))
        assert int(_np(out["d_ngroups"])[0]) == len(wk) and ctx.errors() == hip.DEVERR_CAPACITY
        assert np.array_equal(_np(out["key"], cap), wk[:cap]) and np.array_equal(_np(out["sum"], cap), ws[:cap])
    finally:
        ctx.set_digit_bits(8)


def _hash_groupby_case(hip, ctx, keys, val, dval, gcap=None, d_n=None):
    """Hash group-by with every aggregate against the oracle's group-by and
    min / max / count distinct.  The hash output has no fixed order: it is
    sorted by key (keys are unique) before the element-wise comparison."""
    n = len(keys) if d_n is None else d_n
    wk, ws, wc, _ = oracle.groupby(keys[:n], val[:n])
    mk, mlo, mhi, mnd = oracle.group_minmax(keys[:n], val[:n])
    dk, _, _, dnd = oracle.group_minmax(keys[:n], dval[:n].astype(np.int64))
    assert np.array_equal(wk, mk) and np.array_equal(wk, dk)
    dn = None if d_n is None else _dev(np.array([d_n], np.int64))
    out = hip.hash_groupby(ctx, _dev(keys), _dev(val), _dev(dval), minmax=True,
                           gcap=max(1, len(wk)) if gcap is None else gcap, d_n=dn)
    G = int(_np(out["d_ngroups"])[0])
    assert G == len(wk)
    o = np.argsort(_np(out["key"], G), kind="stable")
    assert np.array_equal(_np(out["key"], G)[o], wk)
    assert np.array_equal(_np(out["cnt"], G)[o], wc)
    assert np.array_equal(_np(out["sum"], G)[o], ws)
    assert np.array_equal(_np(out["min"], G)[o], mlo)
    assert np.array_equal(_np(out["max"], G)[o], mhi)
    assert np.array_equal(_np(out["ndist"], G)[o], dnd)
    assert ctx.errors() == 0


# few groups take the per-block LDS table (gcap <= 512), the rest the global table
@pytest.mark.parametrize("n,domain", [(0, 5), (1, 5), (4097, 1), (70_001, 6), (300_007, 500), (300_007, 1000),
                                      (300_007, 5000),
                                      (300_007, 1 << 20), (65_536, 65_536), (1_000_003, 1 << 31)])
def test_hash_groupby_parity(hip, ctx, n, domain):
    rng = _rng(n + domain + 5)
    keys = rng.integers(0, domain, n).astype(np.int32)
    val = rng.integers(-(1 << 40), 1 << 40, n).astype(np.int64)
    dval = rng.integers(0, 37, n).astype(np.int32)       # repeats inside every group
    _hash_groupby_case(hip, ctx, keys, val, dval)


def test_hash_groupby_paths(hip, ctx):
    """The same 300 groups through the LDS path (gcap = 300) and the global
    path (gcap = 10_000); the value extremes of int64 for min and max; the
    device row count below the host bound."""
    rng = _rng(77)
    keys = rng.integers(0, 300, 200_000).astype(np.int32)
    val = rng.integers(-5, 5, 200_000).astype(np.int64)
    val[rng.integers(0, 200_000, 50)] = np.iinfo(np.int64).max
    val[rng.integers(0, 200_000, 50)] = np.iinfo(np.int64).min + 1
    dval = rng.integers(-3, 3, 200_000).astype(np.int32)
    # sums would overflow with both extremes in one group: take min and max only from this input
    wk, mlo, mhi, _ = oracle.group_minmax(keys, val)
    for gcap in (300, 10_000):
        out = hip.hash_groupby(ctx, _dev(keys), _dev(val), minmax=True, with_sum=False, gcap=gcap)
        G = int(_np(out["d_ngroups"])[0])
        assert G == len(wk)
        o = np.argsort(_np(out["key"], G))
        assert np.array_equal(_np(out["min"], G)[o], mlo) and np.array_equal(_np(out["max"], G)[o], mhi)
        assert out["sum"] is None
        assert ctx.errors() == 0
        _hash_groupby_case(hip, ctx, keys, val % 1000, dval, gcap=gcap, d_n=150_001)


@pytest.mark.parametrize("domain,gcap", [(1500, 1500), (2048, 2048), (2048, 2049), (3000, 4000)])
def test_hash_groupby_sum_count(hip, ctx, domain, gcap):
    """SUM and COUNT only: the LDS table grows to 4096 slots (gcap <= 2048);
    gcap 2049 and 4000 take the global table."""
    rng = _rng(domain + gcap)
    keys = rng.integers(0, domain, 400_001).astype(np.int32)
    val = rng.integers(-10**12, 10**12, 400_001).astype(np.int64)
    wk, ws, wc, _ = oracle.groupby(keys, val)
    out = hip.hash_groupby(ctx, _dev(keys), _dev(val), gcap=gcap)
    G = int(_np(out["d_ngroups"])[0])
    o = np.argsort(_np(out["key"], G))
    assert G == len(wk) and np.array_equal(_np(out["key"], G)[o], wk)
    assert np.array_equal(_np(out["sum"], G)[o], ws) and np.array_equal(_np(out["cnt"], G)[o], wc)
    assert ctx.errors() == 0


@pytest.mark.parametrize("n,domain,minmax", [(1, 1, False), (5000, 3000, True), (300_007, 150_000, False),
                                             (1_000_003, 1 << 20, True), (1_000_003, 1 << 31, False),
                                             (2_000_000, 40_000_000, True)])
def test_hash_groupby_partitioned(hip, ctx, n, domain, minmax):
    """Many groups with sum (and min / max): the radix-partitioned path, one
    LDS table per partition; gcap = the key domain bound (2^20 partitions
    and more for the widest), a device row count below the host bound."""
    rng = _rng(n + domain)
    keys = rng.integers(0, domain, n).astype(np.int32)
    val = rng.integers(-(1 << 40), 1 << 40, n).astype(np.int64)
    dn = n - n // 7
    wk, ws, wc, _ = oracle.groupby(keys[:dn], val[:dn])
    _, mlo, mhi, _ = oracle.group_minmax(keys[:dn], val[:dn])
    gcap = max(3000, min(domain, 2 * n))
    out = hip.hash_groupby(ctx, _dev(keys), _dev(val), gcap=gcap, minmax=minmax,
                           d_n=_dev(np.array([dn], np.int64)))
    G = int(_np(out["d_ngroups"])[0])
    assert G == len(wk)
    o = np.argsort(_np(out["key"], G))
    assert np.array_equal(_np(out["key"], G)[o], wk)
    assert np.array_equal(_np(out["cnt"], G)[o], wc) and np.array_equal(_np(out["sum"], G)[o], ws)
    if minmax:
        assert np.array_equal(_np(out["min"], G)[o], mlo) and np.array_equal(_np(out["max"], G)[o], mhi)
    assert ctx.errors() == 0


def test_hash_groupby_partitioned_negative_key(hip, ctx):
    rng = _rng(91)
    keys = rng.integers(0, 100_000, 200_000).astype(np.int32)
    val = rng.integers(0, 1000, 200_000).astype(np.int64)
    keys[[3, 99_999]] = [-1, -(1 << 31)]
    wk, ws, wc, _ = oracle.groupby(keys[keys >= 0], val[keys >= 0])
    out = hip.hash_groupby(ctx, _dev(keys), _dev(val), gcap=100_000)
    assert ctx.errors() == hip.DEVERR_KEY_RANGE
    G = int(_np(out["d_ngroups"])[0])
    o = np.argsort(_np(out["key"], G))
    assert G == len(wk) and np.array_equal(_np(out["key"], G)[o], wk)
    assert np.array_equal(_np(out["sum"], G)[o], ws) and np.array_equal(_np(out["cnt"], G)[o], wc)


def test_hash_groupby_distinct_skewed(hip, ctx):
    """COUNT(DISTINCT) with many groups (the partitioned path) where one key holds half the rows and
    tens of thousands of distinct values: its partition's LDS pair set fills and the rest of its
    pairs go to the global set."""
    rng = _rng(92)
    n = 400_000
    keys = rng.integers(0, 100_000, n).astype(np.int32)
    keys[: n // 2] = 7
    keys = keys[rng.permutation(n)]
    val = rng.integers(-1000, 1000, n).astype(np.int64)
    dval = rng.integers(0, 60_000, n).astype(np.int32)
    _hash_groupby_case(hip, ctx, keys, val, dval, gcap=100_000)


@pytest.mark.parametrize("groups", [1, 6, 64])
def test_hash_groupby_distinct_set_overflow(hip, ctx, groups):
    """At most 64 groups with about a million distinct values: every block's
    LDS pair set fills, so most pairs take the global-set fallback after a
    full probe run; about a third of the rows repeat a value already drawn.
    No pair may be counted twice or lost."""
    rng = _rng(1000 + groups)
    n = 1_000_003
    keys = rng.integers(0, groups, n).astype(np.int32)
    val = rng.integers(-1000, 1000, n).astype(np.int64)
    dval = rng.integers(0, 1_000_000, n).astype(np.int32)
    _hash_groupby_case(hip, ctx, keys, val, dval, gcap=64)


@pytest.mark.parametrize("domain,gcap", [(3000, 4000), (30_000, 50_000)])
def test_hash_groupby_count_only(hip, ctx, domain, gcap):
    """COUNT(*) and COUNT(DISTINCT) with no value column at all: a per-block LDS table (gcap 4000)
    and the partitioned path that carries the distinct column as the payload (gcap 50000)."""
    rng = _rng(78 + domain)
    keys = rng.integers(0, domain, 100_000).astype(np.int32)
    dval = rng.integers(-50, 50, 100_000).astype(np.int32)
    wk, _, wc, _ = oracle.groupby(keys, np.zeros(len(keys), np.int64))
    _, _, _, wnd = oracle.group_minmax(keys, dval.astype(np.int64))
    out = hip.hash_groupby(ctx, _dev(keys), dval=_dev(dval), gcap=gcap)
    G = int(_np(out["d_ngroups"])[0])
    o = np.argsort(_np(out["key"], G))
    assert G == len(wk) and np.array_equal(_np(out["key"], G)[o], wk)
    assert np.array_equal(_np(out["cnt"], G)[o], wc) and np.array_equal(_np(out["ndist"], G)[o], wnd)
    assert ctx.errors() == 0


@pytest.mark.parametrize("gcap", [0, 100, 600, 5000])
def test_hash_groupby_errors(hip, ctx, gcap):
    """More groups than gcap: the capacity flag, and no more than gcap rows;
    a negative key: the key-range flag and its row left out."""
    rng = _rng(79)
    keys = rng.integers(0, 8000, 50_000).astype(np.int32)
    val = rng.integers(0, 100, 50_000).astype(np.int64)
    dval = rng.integers(0, 10, 50_000).astype(np.int32)
    hip.hash_groupby(ctx, _dev(keys), _dev(val), gcap=gcap)
    assert ctx.errors() & hip.DEVERR_CAPACITY
    hip.hash_groupby(ctx, _dev(keys), _dev(val), _dev(dval), minmax=True, gcap=gcap)
    assert ctx.errors() & hip.DEVERR_CAPACITY
    keys[[5, 7]] = -4
    wk, ws, wc, _ = oracle.groupby(keys[keys >= 0], val[keys >= 0])
    out = hip.hash_groupby(ctx, _dev(keys), _dev(val), gcap=8000)
    assert ctx.errors() == hip.DEVERR_KEY_RANGE
    G = int(_np(out["d_ngroups"])[0])
    o = np.argsort(_np(out["key"], G))
    assert G == len(wk) and np.array_equal(_np(out["sum"], G)[o], ws) and np.array_equal(_np(out["cnt"], G)[o], wc)


# ------------------------------------------------------------------ top-k
@pytest.mark.parametrize("n,k", [(0, 10), (5, 10), (100, 100), (2048, 100), (2049, 7), (1_500_000, 100),
                                 (300_000, 1024)])
@pytest.mark.parametrize("dist", ["random", "equal", "signed", "ascending"])
def test_topk_parity(hip, ctx, n, k, dist):
    """Sum distributions: many ties; all equal (every group passes the
    threshold, so the chunk levels and the final merge rounds all run);
    negative and positive sums; sums growing with the key (the strided
    sample still bounds the threshold)."""
    rng = _rng(n + k)
    key = rng.permutation(max(1, 2 * n))[:n].astype(np.int32)       # unique keys
    if dist == "random":
        s = rng.integers(0, 1000, n).astype(np.int64) * 1_000_003   # many equal sums
    elif dist == "equal":
        s = np.full(n, 777, dtype=np.int64)
    elif dist == "signed":
        s = rng.integers(-10**15, 10**15, n).astype(np.int64)
    else:
        s = key.astype(np.int64) * 3 - n
    c = rng.integers(1, 50, n).astype(np.int64)
    order = np.lexsort((key, -s))[:k]
    out = hip.topk(ctx, _dev(key), _dev(s), _dev(c), k)
    kk = int(_np(out["d_k"])[0])
    assert kk == min(k, n)
    assert np.array_equal(_np(out["key"], kk), key[order])
    assert np.array_equal(_np(out["sum"], kk), s[order]) and np.array_equal(_np(out["cnt"], kk), c[order])
