"""Batched flags fragments: every fragment's result equals the oracle and the same fragment
run alone, under every digit-width / tile configuration, after autotuning, and on
repeated hipGraph replays with eager work in between."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(hip):
    return hip.Context(0)


@pytest.fixture(scope="module")
def batch_case(hip):
    """40 fragments of uneven size (0 .. 400k fact rows), each with its own D and c, plus two
    fragments over row ranges of one shared fact table (the served form)."""
    spec = datagen.config3_spec(count=40, seed=777, n_lo=1, n_hi=4e5)
    frags, wants, host = [], [], []
    for i in range(40):
        fr = datagen.config3_fragment(spec, i)
        if i == 3:                      # an empty fact side
            fr.fact = {k: v[:0] for k, v in fr.fact.items()}
        host.append(fr)
    big = datagen.random_flags_fragment(4242, 300_000, 7_500, 7_500, 2000, 2)
    for (row0, n, D, c) in [(1000, 120_000, 2000, 2), (150_000, 149_000, 900, 4)]:
        sub = {k: v[row0:row0 + n] for k, v in big.fact.items()}
        wants.append(None)
        host.append(("range", big, row0, n, D, c, sub))
    dev_frags = []
    big_dev = None
    for item in host:
        if isinstance(item, tuple):
            _, bg, row0, n, D, c, sub = item
            if big_dev is None:
                big_dev = (hip.to_device(bg.fact), hip.to_device(bg.dim))
            dev_frags.append({"fact": big_dev[0], "dim": big_dev[1], "D": D, "c": c, "key_bits": bg.key_bits,
                              "row0": row0, "n_fact": n})
            wants_i = oracle.fragment_flags(sub, bg.dim, D, c)
        else:
            dev_frags.append({"fact": hip.to_device(item.fact), "dim": hip.to_device(item.dim), "D": item.D,
                              "c": item.c, "key_bits": item.key_bits})
            wants_i = oracle.fragment_flags(item.fact, item.dim, item.D, item.c)
        frags.append(wants_i)
    return dev_frags, frags


def _check(got, want):
    assert got["join_rows"] == want["join_rows"]
    assert np.array_equal(got["key"], want["key"])
    assert np.array_equal(got["sum"], want["sum"]) and np.array_equal(got["cnt"], want["cnt"])
    assert np.array_equal(got["avg"].view(np.int64), want["avg"].view(np.int64))


@pytest.mark.parametrize("config", [0, 1, 2, 3])
def test_batch_configs(hip, ctx, batch_case, config):
    dev_frags, wants = batch_case
    b = hip.BatchRunner(ctx, dev_frags)
    b.set_config(config)
    for _ in range(2):
        b.run()
        for got, want in zip(b.results(), wants):
            _check(got, want)
    assert ctx.errors() == 0
    b.close()


def test_batch_matches_single_fragment_runs(hip, ctx, batch_case):
    dev_frags, wants = batch_case
    b = hip.BatchRunner(ctx, dev_frags)
    b.run()
    res = b.results()
    for fr, got in zip(dev_frags[:12], res[:12]):
        r = hip.FlagsFragmentRunner(ctx, fr["fact"], fr["dim"], fr["D"], fr["c"], fr["key_bits"],
                                    row0=fr.get("row0", 0), n_fact=fr.get("n_fact"))
        r.run()
        alone = r.result()
        _check(got, alone)
    b.close()


def test_batch_autotune_and_graph_replay(hip, ctx, batch_case):
    import torch
    dev_frags, wants = batch_case
    b = hip.BatchRunner(ctx, dev_frags)
    times = b.autotune(reps=2)
    assert set(times) == set(hip.BatchRunner.CONFIGS) and all(t > 0 for t in times.values())
    cfg, digits, name = b.config()
    assert times[name] == min(times.values())
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.capture(s)
        for rep in range(3):
            b.out["sum"].fill_(-1)             # eager work between replays
            b.out["d_ngroups"].fill_(-1)
            b.replay(s)
            s.synchronize()
            for got, want in zip(b.results(), wants):
                _check(got, want)
    assert ctx.errors() == 0
    b.close()
