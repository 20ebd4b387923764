"""Seeded synthetic star-schema inputs (shared by the HIP path and the oracle).

The module draws columns and nothing else; it contains none of the filter,
join or aggregation arithmetic.  Values come from a counter-based SplitMix64
(see ``gen.c``), so every (seed, column, row) maps to one fixed value.

The workloads stand in for the paper's TPC-H runs (Section 6, experimental
setup): fact / dimension / mid tables whose sizes follow TPC-H cardinalities
(60k / 6M / 60M fact rows are the line-item-sized table at SF 0.01 / 1 / 10,
1.5k / 150k dimension rows the customer-sized table, 15M mid rows the SF10
order-sized table) and a 2,557-day date range.  No benchmark data or query
text is used.  Decimals are int64 fixed point (price in cents, discount in
percent) instead of the doubles the paper stores (Section 6).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libtqpgen.so")

SEED_BASE = 20220301

# Column ids of the generator streams.
COL_FK, COL_DATE, COL_PRICE, COL_DISC, COL_FLAGA, COL_FLAGB, COL_FK_DIM = 1, 2, 3, 4, 5, 6, 7
COL_DIM_PK, COL_DIM_SEG = 11, 12
COL_MID_PK, COL_MID_CUST = 21, 22
COL_P_N, COL_P_D, COL_P_C = 31, 32, 33
COL_S_KIND, COL_S_START, COL_S_LEN, COL_S_D, COL_S_C, COL_S_GAP = 41, 42, 43, 44, 45, 46

DATE_DAYS = 2557          # dates are day numbers in [0, 2557)
PRICE_LO, PRICE_HI = 90_000, 10_500_000   # cents, half-open
DISC_LO, DISC_HI = 0, 11                  # percent, 0..10 inclusive
FLAGA_HI, FLAGB_HI = 3, 2
SEG_HI = 5


def build(force: bool = False) -> str:
    """Compile gen.c into libtqpgen.so (gcc, OpenMP)."""
    src = os.path.join(_HERE, "gen.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        u64, i64 = ctypes.c_uint64, ctypes.c_int64
        vp = ctypes.c_void_p
        for name in ("tqpgen_i32", "tqpgen_i64", "tqpgen_i8"):
            getattr(lib, name).argtypes = [u64, u64, i64, i64, i64, i64, vp]
            getattr(lib, name).restype = None
        lib.tqpgen_perm_i32.argtypes = [u64, u64, i64, vp]
        lib.tqpgen_perm_i32.restype = None
        lib.tqpgen_unit.argtypes = [u64, u64, i64]
        lib.tqpgen_unit.restype = ctypes.c_double
        lib.tqpgen_draw.argtypes = [u64, u64, i64]
        lib.tqpgen_draw.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def uniform(seed: int, col: int, n: int, lo: int, hi: int, dtype=np.int32, row0: int = 0) -> np.ndarray:
    """Column of n integers uniform in [lo, hi)."""
    out = np.empty(int(n), dtype=dtype)
    if n == 0:
        return out
    fn = {np.dtype(np.int32): "tqpgen_i32", np.dtype(np.int64): "tqpgen_i64",
          np.dtype(np.int8): "tqpgen_i8"}[np.dtype(dtype)]
    getattr(_L(), fn)(seed, col, row0, int(n), int(lo), int(hi), out.ctypes.data)
    return out


def permutation(seed: int, col: int, n: int) -> np.ndarray:
    out = np.empty(int(n), dtype=np.int32)
    if n:
        _L().tqpgen_perm_i32(seed, col, int(n), out.ctypes.data)
    return out


def unit(seed: int, col: int, row: int) -> float:
    return float(_L().tqpgen_unit(seed, col, row))


def draw(seed: int, col: int, row: int) -> int:
    return int(_L().tqpgen_draw(seed, col, row))


def draw_range(seed: int, col: int, row: int, lo: int, hi: int) -> int:
    """One integer uniform in [lo, hi) at (seed, col, row) (same mapping as the columns)."""
    r = draw(seed, col, row)
    return lo + ((r * (hi - lo)) >> 64)


# ---------------------------------------------------------------------------
# Tables
# ---------------------------------------------------------------------------

def fact_table(seed: int, n: int, fk_hi: int, fk_dim_hi: int | None = None) -> dict:
    """Fact table: fk i32 U[0,fk_hi), date i32 U[0,2557), price i64 U[90000,10500000),
    disc i64 U[0,10], flagA i8 U{0,1,2}, flagB i8 U{0,1}; optional second key fk_dim."""
    t = {
        "fk": uniform(seed, COL_FK, n, 0, fk_hi, np.int32),
        "date": uniform(seed, COL_DATE, n, 0, DATE_DAYS, np.int32),
        "price": uniform(seed, COL_PRICE, n, PRICE_LO, PRICE_HI, np.int64),
        "disc": uniform(seed, COL_DISC, n, DISC_LO, DISC_HI, np.int64),
        "flagA": uniform(seed, COL_FLAGA, n, 0, FLAGA_HI, np.int8),
        "flagB": uniform(seed, COL_FLAGB, n, 0, FLAGB_HI, np.int8),
    }
    if fk_dim_hi is not None:
        t["fk_dim"] = uniform(seed, COL_FK_DIM, n, 0, fk_dim_hi, np.int32)
    return t


def dim_table(seed: int, m: int) -> dict:
    """Dimension table: pk = seeded permutation of 0..m-1 (unique, unsorted), seg i8 U[0,5)."""
    return {"pk": permutation(seed, COL_DIM_PK, m), "seg": uniform(seed, COL_DIM_SEG, m, 0, SEG_HI, np.int8)}


def mid_table(seed: int, m: int, cust_hi: int) -> dict:
    """Mid table: pk = seeded permutation of 0..m-1, custkey i32 U[0,cust_hi)."""
    return {"pk": permutation(seed, COL_MID_PK, m), "custkey": uniform(seed, COL_MID_CUST, m, 0, cust_hi, np.int32)}


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

@dataclass
class FlagsFragment:
    """date < D AND seg == c, fact.fk = dim.pk, group by (flagA, flagB)."""
    fact: dict
    dim: dict
    D: int = 2400
    c: int = 1
    seed: int = 0
    key_bits: int = 0      # bits needed by the join keys (0: derive from the dim size)


@dataclass
class CustFragment:
    """date < D, fact.fk = mid.pk, group by mid.custkey, sum and count, top-k by sum desc."""
    fact: dict
    mid: dict
    D: int = 2400
    k: int = 100
    seed: int = 0
    cust_hi: int = 1_500_000


def bits_for(n_values: int) -> int:
    """Bits needed for keys in [0, n_values)."""
    return max(1, int(n_values - 1).bit_length()) if n_values > 1 else 1


def config0(seed: int | None = None) -> FlagsFragment:
    s = SEED_BASE + 0 if seed is None else seed
    return FlagsFragment(fact_table(s, 60_000, 1_500), dim_table(s, 1_500), 2400, 1, s, bits_for(1_500))


def config1(seed: int | None = None) -> FlagsFragment:
    s = SEED_BASE + 1 if seed is None else seed
    return FlagsFragment(fact_table(s, 6_000_000, 150_000), dim_table(s, 150_000), 2400, 1, s, bits_for(150_000))


CFG2_N, CFG2_M, CFG2_CUST = 60_000_000, 15_000_000, 1_500_000
CFG2_FK_HI = CFG2_M * 5 // 4   # 80% of fact keys fall in the mid pk range: 4 matched to 1 unmatched


def config2(seed: int | None = None, n: int = CFG2_N, m: int = CFG2_M, cust_hi: int = CFG2_CUST) -> CustFragment:
    """60M fact rows against a 15M-row mid table; fk uniform in [0, 1.25*M) so that four of
    five fact rows find their key among the mid pks (the 4:1 match-rate skew)."""
    s = SEED_BASE + 2 if seed is None else seed
    return CustFragment(fact_table(s, n, m * 5 // 4), mid_table(s, m, cust_hi), 2400, 100, s, cust_hi)


@dataclass
class BatchSpec:
    seeds: list = field(default_factory=list)
    n_fact: list = field(default_factory=list)
    n_dim: list = field(default_factory=list)
    D: list = field(default_factory=list)
    c: list = field(default_factory=list)


def config3_spec(count: int = 256, seed: int | None = None, n_lo: float = 1e3, n_hi: float = 4e6) -> BatchSpec:
    """256 fragments; fragment i: N_i = floor(10^U(log10 n_lo, log10 n_hi)), M_i = max(1, N_i // 40),
    fk U[0, M_i), D_i uniform in [0, 2557] (closed), c_i uniform in [0, 5)."""
    s = SEED_BASE + 3 if seed is None else seed
    spec = BatchSpec()
    a, b = math.log10(n_lo), math.log10(n_hi)
    for i in range(count):
        u = unit(s, COL_P_N, i)
        n = int(math.floor(10 ** (a + u * (b - a))))
        n = max(1, min(n, int(n_hi)))
        spec.seeds.append(s * 4096 + i)
        spec.n_fact.append(n)
        spec.n_dim.append(max(1, n // 40))
        spec.D.append(draw_range(s, COL_P_D, i, 0, DATE_DAYS + 1))
        spec.c.append(draw_range(s, COL_P_C, i, 0, SEG_HI))
    return spec


def config3_fragment(spec: BatchSpec, i: int) -> FlagsFragment:
    s = spec.seeds[i]
    n, m = spec.n_fact[i], spec.n_dim[i]
    return FlagsFragment(fact_table(s, n, m), dim_table(s, m), spec.D[i], spec.c[i], s, bits_for(m))


CFG4_N, CFG4_MID, CFG4_DIM = 60_000_000, 15_000_000, 150_000


def config4_tables(seed: int | None = None, n: int = CFG4_N, m_mid: int = CFG4_MID, m_dim: int = CFG4_DIM,
                   cust_hi: int = CFG2_CUST) -> dict:
    """Resident tables of the served workload: one fact table with two keys (fk into the mid
    table as in the 60M-row join, fk_dim uniform over the dimension pks), the mid and the dim."""
    s = SEED_BASE + 4 if seed is None else seed
    fact = fact_table(s, n, m_mid * 5 // 4, fk_dim_hi=m_dim)
    return {"seed": s, "fact": fact, "mid": mid_table(s, m_mid, cust_hi), "dim": dim_table(s, m_dim),
            "cust_hi": cust_hi}


def config4_requests(seed: int, count: int, n_fact: int, p_cust: float = 0.5,
                     len_lo: float = 1e3, len_hi: float = 4e6) -> list:
    """Served request mix: with probability p_cust a 60M-row custkey fragment (its own D), else a
    flags fragment over a contiguous fact row range of log-uniform length in [len_lo, len_hi]
    joined to the dimension with its own (D, c)."""
    reqs = []
    a, b = math.log10(len_lo), math.log10(len_hi)
    for i in range(count):
        kind = "cust" if unit(seed, COL_S_KIND, i) < p_cust else "flags"
        D = draw_range(seed, COL_S_D, i, 0, DATE_DAYS + 1)
        if kind == "cust":
            reqs.append({"kind": kind, "start": 0, "len": n_fact, "D": D, "c": 0})
        else:
            ln = int(math.floor(10 ** (a + unit(seed, COL_S_LEN, i) * (b - a))))
            ln = max(1, min(ln, n_fact))
            start = draw_range(seed, COL_S_START, i, 0, n_fact - ln + 1)
            reqs.append({"kind": kind, "start": start, "len": ln, "D": D,
                         "c": draw_range(seed, COL_S_C, i, 0, SEG_HI)})
    return reqs


def poisson_gaps(seed: int, count: int, rate: float) -> np.ndarray:
    """Inter-arrival gaps (seconds) of a Poisson process of the given rate."""
    return np.array([-math.log(1.0 - unit(seed, COL_S_GAP, i)) / rate for i in range(count)])


def random_flags_fragment(seed: int, n: int, m: int, fk_hi: int | None = None, D: int = 2400, c: int = 1,
                          dup_dim: bool = False) -> FlagsFragment:
    """Small fragments for edge-case tests.  dup_dim draws dim pks with repeats instead of a
    permutation (a many-to-many join)."""
    fk_hi = m if fk_hi is None else fk_hi
    fact = fact_table(seed, n, max(1, fk_hi))
    if dup_dim:
        dim = {"pk": uniform(seed, COL_DIM_PK, m, 0, max(1, fk_hi), np.int32),
               "seg": uniform(seed, COL_DIM_SEG, m, 0, SEG_HI, np.int8)}
    else:
        dim = dim_table(seed, m)
    bits = bits_for(max(fk_hi, m, 2))
    return FlagsFragment(fact, dim, D, c, seed, bits)
