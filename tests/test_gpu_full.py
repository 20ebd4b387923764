"""The batched and served workloads at their stated sizes.

Batched: the 256 config-3 fragments (fact sizes log-uniform in [1e3, 4e6],
about 117M fact rows in all, dim = fact / 40, own D and c each), run as one
batch with the default configuration, after autotuning and on repeated
hipGraph replays; every fragment must equal the oracle and its own plain
single-fragment run bit for bit.
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(hip):
    return hip.Context(0)


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def cfg3(hip):
    spec = datagen.config3_spec()
    assert len(spec.n_fact) == 256
    dev, wants = [], []
    for i in range(len(spec.n_fact)):
        fr = datagen.config3_fragment(spec, i)
        wants.append(oracle.fragment_flags(fr.fact, fr.dim, fr.D, fr.c))
        dev.append({"fact": hip.to_device(fr.fact), "dim": hip.to_device(fr.dim), "D": fr.D, "c": fr.c,
                    "key_bits": fr.key_bits})
    _say("config 3: %d fragments, %d fact rows" % (len(dev), sum(spec.n_fact)))
    return dev, wants


def _check(got, want):
    assert got["join_rows"] == want["join_rows"]
    assert np.array_equal(got["key"], want["key"])
    assert np.array_equal(got["sum"], want["sum"]) and np.array_equal(got["cnt"], want["cnt"])
    assert np.array_equal(got["avg"].view(np.int64), want["avg"].view(np.int64))


@pytest.mark.timeout(600)
def test_config3_batch_and_alone(hip, ctx, cfg3):
    dev, wants = cfg3
    b = hip.BatchRunner(ctx, dev)
    _say("config 3: batch run, default configuration")
    b.run()
    res = b.results()
    for got, want in zip(res, wants):
        _check(got, want)
    assert ctx.errors() == 0
    b.close()
    _say("config 3: 256 plain single-fragment runs")
    for fr, got in zip(dev, res):
        r = hip.FlagsFragmentRunner(ctx, fr["fact"], fr["dim"], fr["D"], fr["c"], fr["key_bits"])
        r.run()
        _check(r.result(), got)
    assert ctx.errors() == 0


@pytest.mark.timeout(600)
def test_config3_autotune_and_graph_replay(hip, ctx, cfg3):
    import torch
    dev, wants = cfg3
    b = hip.BatchRunner(ctx, dev)
    _say("config 3: autotune")
    times = b.autotune(reps=1)
    cfg, digits, name = b.config()
    assert times[name] == min(times.values())
    b.run()
    for got, want in zip(b.results(), wants):
        _check(got, want)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        _say("config 3: capture and replay (%s)" % name)
        b.capture(s)
        for _ in range(3):
            b.out["sum"].fill_(-1)             # eager work between replays
            b.out["d_ngroups"].fill_(-1)
            b.replay(s)
            s.synchronize()
            for got, want in zip(b.results(), wants):
                _check(got, want)
    assert ctx.errors() == 0
    b.close()


# ------------------------------------------------------------------ served, config 4
# Resident 60M-row fact (keys into the mid and the dim table), 15M-row mid,
# 150k-row dim; a burst of requests drawn from the config-2 / config-3 mix
# (half custkey fragments over the whole fact table, each with its own D; half
# flags fragments over log-uniform fact row ranges in [1e3, 4e6], own D and c).
# Every request must equal the same request run alone with plain launches;
# every flags request and three custkey requests at different D also equal
# the oracle.

def _cust_view(f):
    return {"fk": f["fk"], "date": f["date"], "price": f["price"], "disc": f["disc"]}


def _flags_view(f):
    return {"fk": f["fk_dim"], "date": f["date"], "price": f["price"], "disc": f["disc"],
            "flagA": f["flagA"], "flagB": f["flagB"]}


@pytest.fixture(scope="module")
def cfg4(hip):
    t = datagen.config4_tables()
    f = t["fact"]
    n = len(f["fk"])
    assert n == 60_000_000 and len(t["mid"]["pk"]) == 15_000_000 and len(t["dim"]["pk"]) == 150_000
    dev = {"fact": hip.to_device(f), "mid": hip.to_device(t["mid"]), "dim": hip.to_device(t["dim"])}
    reqs = datagen.config4_requests(t["seed"] + 1, 48, n, p_cust=0.5)
    bits = {"key_bits_mid": datagen.bits_for(int(f["fk"].max()) + 1),
            "key_bits_dim": datagen.bits_for(len(t["dim"]["pk"])), "cust_bits": datagen.bits_for(t["cust_hi"])}
    wants = {}
    cust_checked = []
    for i, r in enumerate(reqs):
        if r["kind"] == "flags":
            sl = slice(r["start"], r["start"] + r["len"])
            wants[i] = oracle.fragment_flags({k: v[sl] for k, v in _flags_view(f).items()}, t["dim"], r["D"], r["c"])
        elif len(cust_checked) < 3 and all(reqs[j]["D"] != r["D"] for j in cust_checked):
            _say("config 4: oracle for custkey request %d (D = %d)" % (i, r["D"]))
            wants[i] = oracle.fragment_cust(_cust_view(f), t["mid"], r["D"], 100)
            cust_checked.append(i)
    assert len(cust_checked) == 3
    ctx = hip.Context(0)
    _say("config 4: plain single-request runs")
    alone = [_alone(hip, ctx, dev, r, bits) for r in reqs]
    assert ctx.errors() == 0
    for i, w in wants.items():
        _same(alone[i], w, reqs[i]["kind"])
    return dev, reqs, bits, alone


def _alone(hip, ctx, dev, r, bits):
    """The request as one plain fragment launch sequence (64-bit revenue, the mid table sorted in the
    fragment), in the server's result form."""
    f = dev["fact"]
    if r["kind"] == "cust":
        run = hip.CustFragmentRunner(ctx, _cust_view(f), dev["mid"], r["D"], 100, key_bits=bits["key_bits_mid"],
                                     cust_bits=bits["cust_bits"])
        run.run()
        res = run.result(all_groups=False)
        lists = ("top_key", "top_sum", "top_cnt")
    else:
        run = hip.FlagsFragmentRunner(ctx, _flags_view(f), dev["dim"], r["D"], r["c"], bits["key_bits_dim"],
                                      row0=r["start"], n_fact=r["len"])
        run.run()
        res = run.result()
        lists = ("key", "sum", "cnt", "avg")
    res.update({k: np.asarray(res[k]).tolist() for k in lists}, status=0, dev_errors=0)
    return res


def _same(got, want, kind):
    """got: a result in the server's form; want: the same, or the oracle's arrays."""
    assert got["status"] == 0 and got["dev_errors"] == 0
    assert got["join_rows"] == want["join_rows"]
    eq = lambda a, b: np.array_equal(np.asarray(a, np.int64), np.asarray(b, np.int64))
    if kind == "cust":
        assert got["groups"] == want["groups"]
        assert eq(got["top_key"], want["top_key"]) and eq(got["top_sum"], want["top_sum"])
        assert eq(got["top_cnt"], want["top_cnt"])
    else:
        assert eq(got["key"], want["key"]) and eq(got["sum"], want["sum"]) and eq(got["cnt"], want["cnt"])
        assert np.array_equal(np.asarray(got["avg"], np.float64).view(np.int64),
                              np.asarray(want["avg"], np.float64).view(np.int64))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("presort,revenue_bits", [(True, 32), (False, 64)])
def test_config4_served_mix(hip, cfg4, presort, revenue_bits):
    dev, reqs, bits, alone = cfg4
    _say("config 4: served burst, presort_mid=%s, revenue_bits=%d" % (presort, revenue_bits))
    srv = hip.Server(dev, slots=8, max_batch=32, presort_mid=presort, revenue_bits=revenue_bits, **bits)
    for i, r in enumerate(reqs):
        srv.submit(0 if r["kind"] == "cust" else 1, r["D"], c=r["c"], k=100, row0=r["start"], n_rows=r["len"], tag=i)
    srv.drain()
    got = {r["tag"]: r for r in srv.poll()}
    stats = srv.stats()
    srv.close()
    assert stats["finished"] == len(reqs)
    assert max(g["batch_size"] for g in got.values()) > 1           # flags requests were batched
    for i, r in enumerate(reqs):
        _same(got[i], alone[i], r["kind"])
