"""Write the stored expected results under tests/golden/.

The paper prints no worked example with values (its join illustration is a
figure without numbers), so the stored values here are regression fixtures:
the oracle's results on the small seeded workloads, written by this script,
which calls only oracle/ and datagen/.  Run from the repository root:

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import datagen  # noqa: E402
import oracle  # noqa: E402


def flags_record(fr):
    r = oracle.fragment_flags(fr.fact, fr.dim, fr.D, fr.c)
    return {"D": fr.D, "c": fr.c, "join_rows": r["join_rows"], "key": r["key"].tolist(),
            "sum": r["sum"].tolist(), "cnt": r["cnt"].tolist(), "avg": [float(a).hex() for a in r["avg"]]}


def main():
    out = {"config0": flags_record(datagen.config0())}
    fr = datagen.config2(seed=datagen.SEED_BASE + 2, n=200_000, m=50_000, cust_hi=5_000)
    r = oracle.fragment_cust(fr.fact, fr.mid, fr.D, 100)
    out["cust_small"] = {"n": 200_000, "m": 50_000, "cust_hi": 5_000, "D": fr.D, "groups": r["groups"],
                         "join_rows": r["join_rows"], "top_key": r["top_key"].tolist(),
                         "top_sum": r["top_sum"].tolist(), "top_cnt": r["top_cnt"].tolist()}
    with open(os.path.join(HERE, "oracle_small.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
