"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check that
at least one pin catches each of them."""
import os
import shutil
import subprocess

import pytest

import oracle
import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.cpp")

# (name, original text, mutated text): a dropped term, a wrong sign, a wrong
# comparison, a transposed operand, a wrong index, a dropped tie-break ...
MUTANTS = [
    ("revenue_sign", "mul_checked(price, 100 - disc)", "mul_checked(price, 100 + disc)"),
    ("revenue_dropped_term", "mul_checked(price, 100 - disc)", "mul_checked(price, 100)"),
    ("lt_as_le", "case ORC_LT: return x < k;", "case ORC_LT: return x <= k;"),
    ("fragment_filter_off_by_one", "if (!(date[f] < D)) continue;\n        auto range = dim",
     "if (!(date[f] <= D)) continue;\n        auto range = dim"),
    ("sort_unstable", "return keys[a] != keys[b] ? keys[a] < keys[b] : a < b;",
     "return keys[a] != keys[b] ? keys[a] < keys[b] : a > b;"),
    ("join_transposed", "out_l[w] = lrow ? lrow[i] : static_cast<int32_t>(i);",
     "out_l[w] = lrow ? lrow[i ? i - 1 : 0] : static_cast<int32_t>(i);"),
    ("group_key_transposed", "groups[flagA[f] * 2 + flagB[f]]", "groups[flagB[f] * 2 + flagA[f]]"),
    ("avg_wrong_divisor", "static_cast<double>(kv.second.sum_avg) / static_cast<double>(kv.second.cnt);\n        }\n        ++g;\n    }\n    return g;\n}\n\n// The remaining aggregates",
     "static_cast<double>(kv.second.sum_avg) / static_cast<double>(kv.second.cnt + 1);\n        }\n        ++g;\n    }\n    return g;\n}\n\n// The remaining aggregates"),
    ("count_dropped", "a.cnt += 1;\n            a.sum_avg = add_checked(a.sum_avg, price[f]);",
     "a.sum_avg = add_checked(a.sum_avg, price[f]);"),
    ("topk_tiebreak", "return a.first < b.first;\n              });\n    const int64_t kk",
     "return a.first > b.first;\n              });\n    const int64_t kk"),
    ("semi_as_anti", "if (kind == 1) {\n            if (matched) put(l, -1);", "if (kind == 1) {\n            if (!matched) put(l, -1);"),
    ("outer_drops_unmatched", "} else if (kind == 3) {\n            put(l, -1);", "} else if (kind == 3) {\n            (void)l;"),
    ("band_one_sided", "if (d <= w && -d <= w) {", "if (d <= w) {"),
    ("pack_reversed", "v = v * lim + (x & (lim - 1));", "v = v + (x & (lim - 1)) * (lim - 1);"),
    ("min_is_max", "out_min[g] = *kv.second.begin();", "out_min[g] = *kv.second.rbegin();"),
    ("distinct_counts_rows", "std::map<int32_t, std::set<int64_t>> groups;",
     "std::map<int32_t, std::multiset<int64_t>> groups;"),
    ("chain_first_match_only", "for (int32_t next : it->second) self(self, t + 1, next);",
     "self(self, t + 1, it->second.front());"),
    ("expr_sub_swapped", "case 3: return wrap(static_cast<uint64_t>(a) - static_cast<uint64_t>(b));",
     "case 3: return wrap(static_cast<uint64_t>(b) - static_cast<uint64_t>(a));"),
    ("expr_div_floor", "            return a / b;", "            return a / b - ((a % b != 0) && ((a < 0) != (b < 0)));"),
    ("cust_uses_fact_key", "Agg& a = groups[custkey[it->second]];", "Agg& a = groups[fk[f]];"),
    ("general_dim_pred_ignored", "if (x_eval(dpt, dpr, cp.data() + nf, 0, zdiv) == 0) continue;",
     "if (x_eval(dpt, dpr, cp.data() + nf, 0, zdiv) == 0) {}"),
    ("general_group_first_column_low", "key = key * lim + (x & (lim - 1));", "key = key + (x & (lim - 1)) * lim;"),
    ("general_distinct_counts_rows", "if (agg_op[a] == 5) g.dist[i].insert(v);",
     "if (agg_op[a] == 5) g.dist[i].insert(v + g.cnt);"),
    ("general_min_starts_at_zero", "g.mn.assign(static_cast<size_t>(nagg), INT64_MAX);",
     "g.mn.assign(static_cast<size_t>(nagg), 0);"),
    ("mid_first_match_only", "for (auto it = range.first; it != range.second; ++it) {\n            Agg& a = groups[custkey",
     "for (auto it = range.first; it != range.second; it = range.second) {\n            Agg& a = groups[custkey"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, orig, mut):
    text = open(SRC).read()
    assert text.count(orig) == 1, "mutation anchor must match exactly once: " + name
    src = tmp_path / "oracle_mut.cpp"
    src.write_text(text.replace(orig, mut))
    so = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-o", str(so), str(src)])
    saved = (oracle._lib, oracle._SO)
    oracle._lib, oracle._SO = None, str(so)
    failed = []
    try:
        for check in pins.ALL_CHECKS:
            try:
                check()
            except AssertionError:
                failed.append(check.__name__)
    finally:
        oracle._lib, oracle._SO = saved
    assert failed, "no pin caught mutant " + name
