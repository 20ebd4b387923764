"""The request loop: every result of a concurrent, micro-batched mix equals the oracle and the
same request run alone; a tight HBM budget serialises the work without changing any result; a
request that can never fit is rejected."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def resident(hip):
    t = datagen.config4_tables(seed=31337, n=2_000_000, m_mid=500_000, m_dim=20_000, cust_hi=40_000)
    dev = {"fact": hip.to_device(t["fact"]), "mid": hip.to_device(t["mid"]), "dim": hip.to_device(t["dim"])}
    return t, dev


def _requests(n_fact, count, seed):
    reqs = datagen.config4_requests(seed, count, n_fact, p_cust=0.25, len_lo=1e3, len_hi=4e5)
    return reqs


def _want(t, r):
    f = t["fact"]
    if r["kind"] == "cust":
        fact = {"fk": f["fk"], "date": f["date"], "price": f["price"], "disc": f["disc"]}
        w = oracle.fragment_cust(fact, t["mid"], r["D"], 100)
        return w
    sl = slice(r["start"], r["start"] + r["len"])
    fact = {"fk": f["fk_dim"][sl], "date": f["date"][sl], "price": f["price"][sl], "disc": f["disc"][sl],
            "flagA": f["flagA"][sl], "flagB": f["flagB"][sl]}
    return oracle.fragment_flags(fact, t["dim"], r["D"], r["c"])


def _check(got, want, kind):
    assert got["status"] == 0 and got["dev_errors"] == 0
    assert got["join_rows"] == want["join_rows"]
    if kind == "cust":
        assert got["groups"] == want["groups"]
        assert got["top_key"] == want["top_key"].tolist() and got["top_sum"] == want["top_sum"].tolist()
        assert got["top_cnt"] == want["top_cnt"].tolist()
    else:
        assert got["key"] == want["key"].tolist() and got["sum"] == want["sum"].tolist()
        assert got["cnt"] == want["cnt"].tolist()
        assert np.array_equal(np.array(got["avg"]).view(np.int64), want["avg"].view(np.int64))


def _run(hip, dev, reqs, **kw):
    srv = hip.Server(dev, key_bits_mid=20, key_bits_dim=15, cust_bits=16, max_flags_rows=400_000, **kw)
    for i, r in enumerate(reqs):
        srv.submit(0 if r["kind"] == "cust" else 1, r["D"], c=r["c"], k=100, row0=r["start"], n_rows=r["len"],
                   tag=i)
    srv.drain()
    out = {r["tag"]: r for r in srv.poll()}
    stats = srv.stats()
    srv.close()
    return out, stats


@pytest.mark.parametrize("presort,revenue_bits", [(False, 0), (True, 32), (True, 64)])
def test_mix_equals_oracle_and_alone(hip, resident, presort, revenue_bits):
    """The mix, with the mid table sorted per request or once at start-up, and the revenue carried in
    64 or 32 bits, equals the oracle and the serial server's results."""
    t, dev = resident
    reqs = _requests(len(t["fact"]["fk"]), 48, seed=5)
    wants = [_want(t, r) for r in reqs]
    mixed, stats = _run(hip, dev, reqs, slots=4, max_batch=8, presort_mid=presort, revenue_bits=revenue_bits)
    assert stats["finished"] == len(reqs) and stats["launches"] <= len(reqs)
    assert max(r["batch_size"] for r in mixed.values()) > 1        # some flags requests ran batched
    serial, _ = _run(hip, dev, reqs, slots=1, max_batch=1)
    for i, r in enumerate(reqs):
        _check(mixed[i], wants[i], r["kind"])
        _check(serial[i], wants[i], r["kind"])
        assert serial[i]["batch_size"] == 1


def test_budget_serialises(hip, resident):
    t, dev = resident
    reqs = _requests(len(t["fact"]["fk"]), 12, seed=6)
    wants = [_want(t, r) for r in reqs]
    # room for about one custkey request at a time
    out, stats = _run(hip, dev, reqs, slots=4, max_batch=4, budget_bytes=160 << 20)
    assert stats["peak_bytes"] <= 160 << 20
    for i, r in enumerate(reqs):
        _check(out[i], wants[i], r["kind"])


def test_request_larger_than_budget_is_rejected(hip, resident):
    t, dev = resident
    srv = hip.Server(dev, key_bits_mid=20, key_bits_dim=15, cust_bits=16, max_flags_rows=400_000, slots=2,
                     max_batch=2, budget_bytes=1 << 20)
    srv.submit(0, 2400, k=10, tag=1)
    srv.drain()
    res = srv.poll()
    srv.close()
    assert len(res) == 1 and res[0]["status"] == 3     # TQP_ERR_CAPACITY


def test_errors_come_back_with_their_request(hip, resident):
    """A server whose declared custkey width is too small: every custkey request comes back with the
    key-range bit and a non-OK status, while the flags requests served beside them (other slots,
    other launches) come back clean and exact."""
    t, dev = resident
    reqs = _requests(len(t["fact"]["fk"]), 24, seed=8)
    assert {r["kind"] for r in reqs} == {"cust", "flags"}
    srv = hip.Server(dev, key_bits_mid=20, key_bits_dim=15, cust_bits=8, max_flags_rows=400_000, slots=4,
                     max_batch=1)
    for i, r in enumerate(reqs):
        srv.submit(0 if r["kind"] == "cust" else 1, r["D"], c=r["c"], k=100, row0=r["start"], n_rows=r["len"],
                   tag=i)
    srv.drain()
    out = {r["tag"]: r for r in srv.poll()}
    srv.close()
    for i, r in enumerate(reqs):
        if r["kind"] == "cust":
            assert out[i]["status"] != 0 and out[i]["dev_errors"] & hip.DEVERR_KEY_RANGE
        else:
            _check(out[i], _want(t, r), "flags")
