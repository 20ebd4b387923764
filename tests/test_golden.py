"""The oracle and the generator still reproduce the stored regression fixture."""
import json
import os

import datagen
import oracle

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_small.json")


def test_config0_fixture():
    g = json.load(open(GOLD))["config0"]
    fr = datagen.config0()
    r = oracle.fragment_flags(fr.fact, fr.dim, fr.D, fr.c)
    assert r["join_rows"] == g["join_rows"]
    assert r["key"].tolist() == g["key"] and r["sum"].tolist() == g["sum"] and r["cnt"].tolist() == g["cnt"]
    assert [float(a).hex() for a in r["avg"]] == g["avg"]


def test_cust_fixture():
    g = json.load(open(GOLD))["cust_small"]
    fr = datagen.config2(seed=datagen.SEED_BASE + 2, n=g["n"], m=g["m"], cust_hi=g["cust_hi"])
    r = oracle.fragment_cust(fr.fact, fr.mid, g["D"], 100)
    assert r["groups"] == g["groups"] and r["join_rows"] == g["join_rows"]
    assert r["top_key"].tolist() == g["top_key"] and r["top_sum"].tolist() == g["top_sum"]
    assert r["top_cnt"].tolist() == g["top_cnt"]
