"""The seeded generator: ranges, determinism, permutations, workload recipes."""
import numpy as np

import datagen


def test_ranges_and_determinism():
    f = datagen.fact_table(7, 50_000, 1_500)
    assert f["fk"].min() >= 0 and f["fk"].max() < 1_500
    assert f["date"].min() >= 0 and f["date"].max() < 2557
    assert f["price"].min() >= 90_000 and f["price"].max() < 10_500_000
    assert set(np.unique(f["disc"]).tolist()) == set(range(11))
    assert set(np.unique(f["flagA"]).tolist()) == {0, 1, 2}
    assert set(np.unique(f["flagB"]).tolist()) == {0, 1}
    g = datagen.fact_table(7, 50_000, 1_500)
    for k in f:
        assert np.array_equal(f[k], g[k])
    # slices of a column are the same values (counter-based)
    part = datagen.uniform(7, datagen.COL_FK, 100, 0, 1_500, np.int32, row0=1000)
    assert np.array_equal(part, f["fk"][1000:1100])


def test_permutation():
    p = datagen.permutation(3, datagen.COL_DIM_PK, 10_000)
    assert np.array_equal(np.sort(p), np.arange(10_000))
    assert not np.array_equal(p, np.arange(10_000))


def test_config_recipes():
    c0 = datagen.config0()
    assert len(c0.fact["fk"]) == 60_000 and len(c0.dim["pk"]) == 1_500 and c0.D == 2400 and c0.c == 1
    s = datagen.config3_spec()
    assert len(s.n_fact) == 256
    assert min(s.n_fact) >= 1_000 and max(s.n_fact) <= 4_000_000
    assert all(m == max(1, n // 40) for n, m in zip(s.n_fact, s.n_dim))
    assert all(0 <= d <= 2557 for d in s.D) and all(0 <= c < 5 for c in s.c)
    # log-uniform sizes: the median is near the geometric mean of the bounds (63k)
    med = sorted(s.n_fact)[128]
    assert 20_000 < med < 200_000
