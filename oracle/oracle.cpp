// CPU oracle for the filter -> sort-based equi-join -> group-by path.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this code:
// only the tests, the smoke check and the CPU-baseline leg of the benchmark
// load it.  It shares no code, header, table or helper with the HIP library.
//
// Every function computes the plain relational definition of its operator,
// one row at a time, with exact 64-bit integer arithmetic (overflow checked)
// and the C++ standard library only.  The paper's operators (Section 5 and
// Algorithms 1-2) reach these definitions exactly: sorting, histogram-based
// joins and sort-based grouping reorder work but do not change the result.
//
//   filter      Section 3.1 (Listing 1 and the selection-vector variant):
//               the rows whose predicate holds, in input order.
//   sort        Algorithm 1 (sort of the key columns), Algorithm 2 (sort of
//               the group keys), Section 5.4 (radix sort): ascending by key,
//               stable, payload carried along.
//   join        Section 5.2 / Algorithm 1: the pairs (left row, right row)
//               whose keys are equal; late materialisation returns index
//               pairs.  Canonical order: left input order, then right input
//               order (for key-sorted inputs this is the left-major order of
//               the quotient / remainder step of Algorithm 1).  Left semi,
//               left anti and left outer joins (Section 5) mark a missing
//               right row with -1.
//   group-by    Section 5.4 / Algorithm 2: one output row per distinct key,
//               in ascending key order, with sum, count and average; the
//               other aggregates listed in the introduction of Section 5
//               (min, max, count distinct) by the same definition.
//   fragments   the whole filter -> join -> group-by query of the workloads,
//               as a hash join followed by a hash aggregation.
//
// Parity status: every function here is pinned by tests against library
// routines, brute force on small inputs and closed-form invariants.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <set>
#include <unordered_map>
#include <vector>

namespace {

enum { ORC_I8 = 1, ORC_I32 = 2, ORC_I64 = 3 };
enum { ORC_LT = 0, ORC_LE = 1, ORC_GT = 2, ORC_GE = 3, ORC_EQ = 4, ORC_NE = 5 };

int g_overflow = 0;   // set when an exact int64 accumulation would overflow

inline int64_t add_checked(int64_t a, int64_t b) {
    int64_t r;
    if (__builtin_add_overflow(a, b, &r)) g_overflow = 1;
    return r;
}

inline int64_t mul_checked(int64_t a, int64_t b) {
    int64_t r;
    if (__builtin_mul_overflow(a, b, &r)) g_overflow = 1;
    return r;
}

int64_t load_value(const void* col, int type, int64_t i) {
    switch (type) {
        case ORC_I8: return static_cast<const int8_t*>(col)[i];
        case ORC_I32: return static_cast<const int32_t*>(col)[i];
        default: return static_cast<const int64_t*>(col)[i];
    }
}

bool compare(int64_t x, int op, int64_t k) {
    switch (op) {
        case ORC_LT: return x < k;
        case ORC_LE: return x <= k;
        case ORC_GT: return x > k;
        case ORC_GE: return x >= k;
        case ORC_EQ: return x == k;
        default: return x != k;
    }
}

// Revenue expression of the workloads, price * (100 - disc), in the exact
// fixed-point unit cent * percent (the paper evaluates the same expression on
// doubles, Section 5.1).
inline int64_t revenue(int64_t price, int64_t disc) {
    return mul_checked(price, 100 - disc);
}

struct Agg {
    int64_t sum = 0, cnt = 0, sum_avg = 0;
};

}  // namespace

extern "C" {

int orc_overflow_flag(void) { return g_overflow; }
void orc_clear_overflow(void) { g_overflow = 0; }

// Filter (Section 3.1): rows i in [0, n) for which every predicate
// cols[pred_col[p]][i] <op> k[p] holds, written in increasing order.
// Returns the number of rows written.
int64_t orc_filter(int64_t n, int ncols, const void* const* cols, const int32_t* types, int np,
                   const int32_t* pred_col, const int32_t* pred_op, const int64_t* pred_k,
                   int32_t* out_rows) {
    (void)ncols;
    int64_t w = 0;
    for (int64_t i = 0; i < n; ++i) {
        bool keep = true;
        for (int p = 0; p < np && keep; ++p)
            keep = compare(load_value(cols[pred_col[p]], types[pred_col[p]], i), pred_op[p], pred_k[p]);
        if (keep) out_rows[w++] = static_cast<int32_t>(i);
    }
    return w;
}

// Sort (Algorithms 1-2): the pairs ordered by key ascending; equal keys keep
// their input order.  vals may be null (the payload is then the input index).
void orc_sort_pairs(const int32_t* keys, const int32_t* vals, int64_t n, int32_t* keys_out,
                    int32_t* vals_out) {
    std::vector<int64_t> idx(static_cast<size_t>(n));
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
        return keys[a] != keys[b] ? keys[a] < keys[b] : a < b;
    });
    for (int64_t i = 0; i < n; ++i) {
        keys_out[i] = keys[idx[i]];
        vals_out[i] = vals ? vals[idx[i]] : static_cast<int32_t>(idx[i]);
    }
}

// Equi-join (Section 5.2): every (lrow[i], rrow[j]) with lkey[i] == rkey[j],
// ordered by i, then j.  Writes at most cap pairs; returns the true count.
int64_t orc_join(const int32_t* lkey, const int32_t* lrow, int64_t nl, const int32_t* rkey,
                 const int32_t* rrow, int64_t nr, int32_t* out_l, int32_t* out_r, int64_t cap) {
    std::unordered_map<int32_t, std::vector<int64_t>> right;  // key -> right positions, in order
    right.reserve(static_cast<size_t>(nr));
    for (int64_t j = 0; j < nr; ++j) right[rkey[j]].push_back(j);
    int64_t w = 0;
    for (int64_t i = 0; i < nl; ++i) {
        auto it = right.find(lkey[i]);
        if (it == right.end()) continue;
        for (int64_t j : it->second) {
            if (w < cap) {
                out_l[w] = lrow ? lrow[i] : static_cast<int32_t>(i);
                out_r[w] = rrow ? rrow[j] : static_cast<int32_t>(j);
            }
            ++w;
        }
    }
    return w;
}

// Expressions (Section 5.1: arithmetic, comparisons and logic over columns,
// CASE as a select).  The program is postfix; here it is first turned into a
// tree (each operator node takes the subtrees left on the stack) and every row
// is evaluated by recursion over the tree.  Values are int64 with wrap-around
// (two's complement) for +, - and *, and for unary minus; / and % truncate
// toward zero as in C, a zero divisor gives 0 (and is counted), INT64_MIN / -1
// gives INT64_MIN and INT64_MIN % -1 gives 0; comparisons, AND, OR and NOT give
// 0 or 1 (nonzero is true); SELECT(c, t, f) = c ? t : f.  Operator codes:
// 0 column, 1 constant, 2 +, 3 -, 4 *, 5 /, 6 %, 7 unary -, 8 <, 9 <=, 10 >,
// 11 >=, 12 ==, 13 !=, 14 AND, 15 OR, 16 NOT, 17 SELECT.  Returns the number of
// zero divisors met, or -1 for a malformed program.
namespace {
struct XNode {
    int op;
    int64_t arg;
    int kid[3];
};
int x_arity(int op) {
    if (op == 0 || op == 1) return 0;
    if (op == 7 || op == 16) return 1;
    if (op == 17) return 3;
    return (op >= 2 && op <= 15) ? 2 : -1;
}
int64_t x_eval(const std::vector<XNode>& t, int at, const int64_t* const* cols, int64_t row, int64_t& zdiv) {
    const XNode& nd = t[static_cast<size_t>(at)];
    auto kid = [&](int i) { return x_eval(t, nd.kid[i], cols, row, zdiv); };
    auto wrap = [](uint64_t v) { return static_cast<int64_t>(v); };
    switch (nd.op) {
        case 0: return cols[nd.arg][row];
        case 1: return nd.arg;
        case 7: return wrap(0u - static_cast<uint64_t>(kid(0)));
        case 16: return kid(0) == 0 ? 1 : 0;
        case 17: {
            const int64_t c = kid(0), a = kid(1), b = kid(2);
            return c != 0 ? a : b;
        }
        default: break;
    }
    const int64_t a = kid(0), b = kid(1);
    switch (nd.op) {
        case 2: return wrap(static_cast<uint64_t>(a) + static_cast<uint64_t>(b));
        case 3: return wrap(static_cast<uint64_t>(a) - static_cast<uint64_t>(b));
        case 4: return wrap(static_cast<uint64_t>(a) * static_cast<uint64_t>(b));
        case 5:
            if (b == 0) { ++zdiv; return 0; }
            if (a == INT64_MIN && b == -1) return INT64_MIN;
            return a / b;
        case 6:
            if (b == 0) { ++zdiv; return 0; }
            if (b == -1) return 0;
            return a % b;
        case 8: return a < b;
        case 9: return a <= b;
        case 10: return a > b;
        case 11: return a >= b;
        case 12: return a == b;
        case 13: return a != b;
        case 14: return (a != 0) && (b != 0);
        default: return (a != 0) || (b != 0);
    }
}
}  // namespace

namespace {
// The tree of a postfix program over ncols columns; false if malformed.
bool x_build(const int32_t* ops, const int64_t* args, int nprog, int ncols, std::vector<XNode>& tree, int& root) {
    std::vector<int> stack;
    for (int pc = 0; pc < nprog; ++pc) {
        const int ar = x_arity(ops[pc]);
        if (ar < 0 || static_cast<int>(stack.size()) < ar) return false;
        if (ops[pc] == 0 && (args[pc] < 0 || args[pc] >= ncols)) return false;
        XNode nd{ops[pc], args[pc], {-1, -1, -1}};
        for (int i = ar - 1; i >= 0; --i) {
            nd.kid[i] = stack.back();
            stack.pop_back();
        }
        tree.push_back(nd);
        stack.push_back(static_cast<int>(tree.size()) - 1);
    }
    if (stack.size() != 1) return false;
    root = stack[0];
    return true;
}
}  // namespace

int64_t orc_eval(const int64_t* const* cols, int ncols, int64_t n, const int32_t* ops,
                 const int64_t* args, int nprog, int64_t* out) {
    std::vector<XNode> tree;
    int root = 0;
    if (!x_build(ops, args, nprog, ncols, tree, root)) return -1;
    int64_t zdiv = 0;
    for (int64_t r = 0; r < n; ++r) out[r] = x_eval(tree, root, cols, r, zdiv);
    return zdiv;
}

// A chain of equi-joins, the shape of the multi-join plans of Section 6
// (hand-optimized plans, the six-join query): tables 0..hops; table t < hops
// has the key column outk[t] into table t + 1, whose matched column is pk[t + 1]
// (pk[0] is unused).  Every tuple (r0, ..., r_hops) of row positions with
// outk[t][r_t] == pk[t + 1][r_{t + 1}] for every t, nested in input order (r0
// ascending, then r1 in input order, ...).  Tuples row-major in out_rows
// (hops + 1 ints each); at most cap tuples written; returns the true count.
int64_t orc_join_chain(int hops, const int32_t* const* outk, const int64_t* nrows, const int32_t* const* pk,
                       int32_t* out_rows, int64_t cap) {
    std::vector<std::unordered_map<int32_t, std::vector<int32_t>>> index(static_cast<size_t>(hops) + 1);
    for (int t = 1; t <= hops; ++t)
        for (int64_t j = 0; j < nrows[t]; ++j) index[t][pk[t][j]].push_back(static_cast<int32_t>(j));
    std::vector<int32_t> tuple(static_cast<size_t>(hops) + 1);
    int64_t w = 0;
    // depth-first: extend a partial tuple ending at table t, row r
    auto extend = [&](auto&& self, int t, int32_t r) -> void {
        tuple[t] = r;
        if (t == hops) {
            if (w < cap)
                for (int u = 0; u <= hops; ++u) out_rows[w * (hops + 1) + u] = tuple[u];
            ++w;
            return;
        }
        auto it = index[t + 1].find(outk[t][r]);
        if (it == index[t + 1].end()) return;
        for (int32_t next : it->second) self(self, t + 1, next);
    };
    for (int64_t i = 0; i < nrows[0]; ++i) extend(extend, 0, static_cast<int32_t>(i));
    return w;
}

// Join kinds (the operator list at the start of Section 5 names left-outer,
// left-semi and left-anti joins beside the natural join; Section 5.2 reaches
// them by small changes to the sort-based join).  kind 0: inner, as orc_join.  kind 1, left semi: one row
// (lrow[i], -1) for every left row with at least one match.  kind 2, left
// anti: (lrow[i], -1) for every left row with none.  kind 3, left outer: the
// inner pairs of every left row, or (lrow[i], -1) when it has none.  Left
// input order, then right input order.  At most cap rows written; returns
// the true count.
int64_t orc_join_kind(int kind, const int32_t* lkey, const int32_t* lrow, int64_t nl, const int32_t* rkey,
                      const int32_t* rrow, int64_t nr, int32_t* out_l, int32_t* out_r, int64_t cap) {
    std::unordered_map<int32_t, std::vector<int64_t>> right;
    right.reserve(static_cast<size_t>(nr));
    for (int64_t j = 0; j < nr; ++j) right[rkey[j]].push_back(j);
    int64_t w = 0;
    auto put = [&](int32_t l, int32_t r) {
        if (w < cap) {
            out_l[w] = l;
            out_r[w] = r;
        }
        ++w;
    };
    for (int64_t i = 0; i < nl; ++i) {
        const int32_t l = lrow ? lrow[i] : static_cast<int32_t>(i);
        auto it = right.find(lkey[i]);
        const bool matched = it != right.end();
        if (kind == 1) {
            if (matched) put(l, -1);
        } else if (kind == 2) {
            if (!matched) put(l, -1);
        } else if (matched) {
            for (int64_t j : it->second) put(l, rrow ? rrow[j] : static_cast<int32_t>(j));
        } else if (kind == 3) {
            put(l, -1);
        }
    }
    return w;
}

// Band join, the non-equi join of Section 5.2's list of variants: every
// (lrow[i], rrow[j]) with |lkey[i] - rkey[j]| <= w (w >= 0; w = 0 is the
// equi-join), ordered by i, then j.  At most cap rows written; returns the
// true count.
int64_t orc_join_band(const int32_t* lkey, const int32_t* lrow, int64_t nl, const int32_t* rkey,
                      const int32_t* rrow, int64_t nr, int64_t w, int32_t* out_l, int32_t* out_r, int64_t cap) {
    int64_t n = 0;
    for (int64_t i = 0; i < nl; ++i) {
        for (int64_t j = 0; j < nr; ++j) {
            const int64_t d = static_cast<int64_t>(lkey[i]) - static_cast<int64_t>(rkey[j]);
            if (d <= w && -d <= w) {
                if (n < cap) {
                    out_l[n] = lrow ? lrow[i] : static_cast<int32_t>(i);
                    out_r[n] = rrow ? rrow[j] : static_cast<int32_t>(j);
                }
                ++n;
            }
        }
    }
    return n;
}

// Composite keys (Section 5.4: the group-by columns are concatenated into one
// key before the sort; Algorithm 3 matches several join-key columns): the
// columns packed into one integer, the first column most significant, column
// c taking bits[c] bits, so the packed order is the lexicographic order of
// the tuples.  Returns the number of values outside their width (negative or
// >= 2^bits[c]); those rows are packed from their masked values.
int64_t orc_pack_keys(const int32_t* const* cols, const int32_t* bits, int ncols, int64_t n, int32_t* out) {
    int64_t bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t v = 0;
        for (int c = 0; c < ncols; ++c) {
            const int64_t x = cols[c][i];
            const int64_t lim = int64_t(1) << bits[c];
            if (x < 0 || x >= lim) ++bad;
            v = v * lim + (x & (lim - 1));
        }
        out[i] = static_cast<int32_t>(v);
    }
    return bad;
}

// Group-by aggregation (Section 5.4, Algorithm 2): one row per distinct key in
// ascending order with sum(val), count and avg(avg_in) = (double)sum(avg_in) /
// (double)count.  avg_in may be null (out_avg is then not written).  Writes at
// most gcap groups; returns the number of groups.
int64_t orc_groupby(const int32_t* gkey, int64_t n, const int64_t* val, const int64_t* avg_in,
                    int32_t* out_key, int64_t* out_sum, int64_t* out_cnt, double* out_avg,
                    int64_t gcap) {
    std::map<int32_t, Agg> groups;
    for (int64_t i = 0; i < n; ++i) {
        Agg& a = groups[gkey[i]];
        a.sum = add_checked(a.sum, val[i]);
        a.cnt += 1;
        if (avg_in) a.sum_avg = add_checked(a.sum_avg, avg_in[i]);
    }
    int64_t g = 0;
    for (const auto& kv : groups) {
        if (g < gcap) {
            out_key[g] = kv.first;
            out_sum[g] = kv.second.sum;
            out_cnt[g] = kv.second.cnt;
            if (avg_in && out_avg)
                out_avg[g] = static_cast<double>(kv.second.sum_avg) / static_cast<double>(kv.second.cnt);
        }
        ++g;
    }
    return g;
}

// The remaining aggregates of Section 5's introduction (min, max and count
// with DISTINCT), per distinct key in ascending order: min(val), max(val) and the number of
// different values of val in the group.  Writes at most gcap groups; returns
// the number of groups.
int64_t orc_group_minmax(const int32_t* gkey, int64_t n, const int64_t* val, int32_t* out_key,
                         int64_t* out_min, int64_t* out_max, int64_t* out_ndist, int64_t gcap) {
    std::map<int32_t, std::set<int64_t>> groups;
    for (int64_t i = 0; i < n; ++i) groups[gkey[i]].insert(val[i]);
    int64_t g = 0;
    for (const auto& kv : groups) {
        if (g < gcap) {
            out_key[g] = kv.first;
            out_min[g] = *kv.second.begin();
            out_max[g] = *kv.second.rbegin();
            out_ndist[g] = static_cast<int64_t>(kv.second.size());
        }
        ++g;
    }
    return g;
}

// Flags fragment: date < D on the fact table, seg == c on the dimension,
// fact.fk = dim.pk, group by the packed key flagA * 2 + flagB, aggregates
// sum(price * (100 - disc)), count and avg(price).  Groups in ascending key
// order; returns the number of groups (at most 6, never more than gcap
// written).  out_join (nullable) receives the join cardinality.
int64_t orc_fragment_flags(const int32_t* fk, const int32_t* date, const int64_t* price,
                           const int64_t* disc, const int8_t* flagA, const int8_t* flagB,
                           int64_t n_fact, const int32_t* pk, const int8_t* seg, int64_t n_dim,
                           int32_t D, int32_t c, int32_t* out_key, int64_t* out_sum,
                           int64_t* out_cnt, double* out_avg, int64_t gcap, int64_t* out_join) {
    std::unordered_multimap<int32_t, int64_t> dim;   // build side: filtered dimension rows
    dim.reserve(static_cast<size_t>(n_dim));
    for (int64_t d = 0; d < n_dim; ++d)
        if (seg[d] == c) dim.emplace(pk[d], d);
    std::map<int32_t, Agg> groups;
    int64_t joined = 0;
    for (int64_t f = 0; f < n_fact; ++f) {           // probe side: filtered fact rows
        if (!(date[f] < D)) continue;
        auto range = dim.equal_range(fk[f]);
        for (auto it = range.first; it != range.second; ++it) {
            Agg& a = groups[flagA[f] * 2 + flagB[f]];
            a.sum = add_checked(a.sum, revenue(price[f], disc[f]));
            a.cnt += 1;
            a.sum_avg = add_checked(a.sum_avg, price[f]);
            ++joined;
        }
    }
    if (out_join) *out_join = joined;
    int64_t g = 0;
    for (const auto& kv : groups) {
        if (g < gcap) {
            out_key[g] = kv.first;
            out_sum[g] = kv.second.sum;
            out_cnt[g] = kv.second.cnt;
            out_avg[g] = static_cast<double>(kv.second.sum_avg) / static_cast<double>(kv.second.cnt);
        }
        ++g;
    }
    return g;
}

// Custkey fragment: date < D on the fact table, fact.fk = mid.pk, group by
// mid.custkey, aggregates sum(price * (100 - disc)) and count.  All groups go
// out in ascending custkey order (at most gcap written); the first k rows of
// the order (sum descending, custkey ascending) go to the top_* arrays and
// *out_k receives min(k, groups).  Returns the number of groups.
int64_t orc_fragment_cust(const int32_t* fk, const int32_t* date, const int64_t* price,
                          const int64_t* disc, int64_t n_fact, const int32_t* pk,
                          const int32_t* custkey, int64_t n_mid, int32_t D, int32_t* out_key,
                          int64_t* out_sum, int64_t* out_cnt, int64_t gcap, int32_t k,
                          int32_t* top_key, int64_t* top_sum, int64_t* top_cnt, int32_t* out_k,
                          int64_t* out_join) {
    std::unordered_multimap<int32_t, int64_t> mid;
    mid.reserve(static_cast<size_t>(n_mid));
    for (int64_t r = 0; r < n_mid; ++r) mid.emplace(pk[r], r);
    std::unordered_map<int32_t, Agg> groups;
    int64_t joined = 0;
    for (int64_t f = 0; f < n_fact; ++f) {
        if (!(date[f] < D)) continue;
        auto range = mid.equal_range(fk[f]);
        for (auto it = range.first; it != range.second; ++it) {
            Agg& a = groups[custkey[it->second]];
            a.sum = add_checked(a.sum, revenue(price[f], disc[f]));
            a.cnt += 1;
            ++joined;
        }
    }
    if (out_join) *out_join = joined;
    std::vector<std::pair<int32_t, Agg>> rows(groups.begin(), groups.end());
    std::sort(rows.begin(), rows.end(),
              [](const std::pair<int32_t, Agg>& a, const std::pair<int32_t, Agg>& b) {
                  return a.first < b.first;
              });
    const int64_t G = static_cast<int64_t>(rows.size());
    for (int64_t g = 0; g < G && g < gcap; ++g) {
        out_key[g] = rows[g].first;
        out_sum[g] = rows[g].second.sum;
        out_cnt[g] = rows[g].second.cnt;
    }
    // ORDER BY sum DESC, custkey ASC, first k rows (Section 5: sort operator).
    std::sort(rows.begin(), rows.end(),
              [](const std::pair<int32_t, Agg>& a, const std::pair<int32_t, Agg>& b) {
                  if (a.second.sum != b.second.sum) return a.second.sum > b.second.sum;
                  return a.first < b.first;
              });
    const int64_t kk = std::min<int64_t>(k, G);
    for (int64_t i = 0; i < kk; ++i) {
        top_key[i] = rows[i].first;
        top_sum[i] = rows[i].second.sum;
        top_cnt[i] = rows[i].second.cnt;
    }
    *out_k = static_cast<int32_t>(kk);
    return G;
}

// A general query fragment (the operators of Section 5 composed: filters,
// an equi-join, a group-by over several columns and a list of aggregates,
// ORDER BY ... LIMIT k), by its relational definition:
//
//   SELECT pack(g_1, ..., g_q), agg_1, ..., agg_m
//   FROM fact [JOIN dim ON fact.col[fkey] = dim.col[dkey]]
//   WHERE fpred(fact row) [AND dpred(dim row)]
//   GROUP BY pack(g_1, ..., g_q) ORDER BY the packed key
//   [then, separately, ORDER BY agg_1 DESC, key ASC LIMIT topk]
//
// Columns are int8 / int32 / int64 (types 1 / 2 / 3), widened to int64.  A
// joined row numbers the fact columns 0..nf-1 and the dim columns nf..nf+nd-1
// (without a join, fkey < 0: the kept fact rows, fact columns only).
// Predicates and aggregate values are postfix programs (the operator codes of
// orc_eval) over the row's columns; an empty predicate keeps every row, a row
// is kept when the predicate is nonzero.  The group key packs the columns
// gcol[0..q-1] (joined numbering), column i taking gbits[i] bits, the first
// most significant (a value outside [0, 2^bits) enters masked and is counted
// in *out_bad); q = 0 puts every row in group 0.  Aggregates: 0 COUNT(*), 1
// SUM(v), 2 MIN(v), 3 MAX(v), 4 AVG(v) = (double)SUM / (double)COUNT, 5
// COUNT(DISTINCT v).  Output per group, keys ascending: out_key[g] and
// out_vals[a * gcap + g] (int64, or the bits of the double for AVG).  At most
// gcap groups written; returns the number of groups (-1: malformed
// program).  topk > 0: the first topk groups in the order (agg_1 desc, key
// asc) go to top_key / top_val, *out_k = their number.  *out_join = the
// number of joined rows (rows of the join that pass both predicates).
int64_t orc_fragment_general(int nf, const void* const* fcols, const int32_t* ftypes, int64_t n_fact, int nd,
                             const void* const* dcols, const int32_t* dtypes, int64_t n_dim,
                             const int32_t* fp_ops, const int64_t* fp_args, int n_fp, const int32_t* dp_ops,
                             const int64_t* dp_args, int n_dp, int fkey, int dkey, int ngroup, const int32_t* gcol,
                             const int32_t* gbits, int nagg, const int32_t* agg_op, const int32_t* agg_len,
                             const int32_t* agg_ops, const int64_t* agg_args, int32_t* out_key, int64_t* out_vals,
                             int64_t gcap, int32_t topk, int32_t* top_key, int64_t* top_val, int32_t* out_k,
                             int64_t* out_join, int64_t* out_bad) {
    const bool join = fkey >= 0;
    const int ncol = nf + (join ? nd : 0);
    // the programs as trees
    std::vector<XNode> fpt, dpt;
    int fpr = 0, dpr = 0;
    if (n_fp > 0 && !x_build(fp_ops, fp_args, n_fp, nf, fpt, fpr)) return -1;
    if (join && n_dp > 0 && !x_build(dp_ops, dp_args, n_dp, nd, dpt, dpr)) return -1;
    std::vector<std::vector<XNode>> at(static_cast<size_t>(nagg));
    std::vector<int> ar(static_cast<size_t>(nagg), 0);
    int off = 0;
    for (int a = 0; a < nagg; ++a) {
        if (agg_op[a] != 0 && !x_build(agg_ops + off, agg_args + off, agg_len[a], ncol, at[a], ar[a])) return -1;
        off += agg_len[a];
    }
    // one row's columns as int64 values; the programs read cols[c][0]
    std::vector<int64_t> val(static_cast<size_t>(ncol > 0 ? ncol : 1));
    std::vector<const int64_t*> cp(val.size());
    for (size_t c = 0; c < val.size(); ++c) cp[c] = &val[c];
    int64_t zdiv = 0;
    // build side: the dim rows that pass their predicate, by key
    std::unordered_multimap<int64_t, int64_t> dim;
    if (join) {
        for (int64_t d = 0; d < n_dim; ++d) {
            for (int c = 0; c < nd; ++c) val[static_cast<size_t>(nf + c)] = load_value(dcols[c], dtypes[c], d);
            if (n_dp > 0) {
                // the dim predicate reads the dim columns as its columns 0..nd-1
                if (x_eval(dpt, dpr, cp.data() + nf, 0, zdiv) == 0) continue;
            }
            dim.emplace(load_value(dcols[dkey], dtypes[dkey], d), d);
        }
    }
    struct G {
        int64_t cnt = 0;
        std::vector<int64_t> sum, mn, mx;
        std::vector<std::set<int64_t>> dist;
    };
    std::map<int32_t, G> groups;
    int64_t joined = 0, bad = 0;
    auto emit = [&]() {
        int64_t key = 0;
        for (int i = 0; i < ngroup; ++i) {
            const int64_t x = val[static_cast<size_t>(gcol[i])];
            const int64_t lim = int64_t(1) << gbits[i];
            if (x < 0 || x >= lim) ++bad;
            key = key * lim + (x & (lim - 1));
        }
        G& g = groups[static_cast<int32_t>(key)];
        if (g.sum.empty()) {
            g.sum.assign(static_cast<size_t>(nagg), 0);
            g.mn.assign(static_cast<size_t>(nagg), INT64_MAX);
            g.mx.assign(static_cast<size_t>(nagg), INT64_MIN);
            g.dist.resize(static_cast<size_t>(nagg));
        }
        g.cnt += 1;
        for (int a = 0; a < nagg; ++a) {
            if (agg_op[a] == 0) continue;
            const int64_t v = x_eval(at[a], ar[a], cp.data(), 0, zdiv);
            const size_t i = static_cast<size_t>(a);
            g.sum[i] = add_checked(g.sum[i], v);
            g.mn[i] = std::min(g.mn[i], v);
            g.mx[i] = std::max(g.mx[i], v);
            if (agg_op[a] == 5) g.dist[i].insert(v);
        }
        ++joined;
    };
    // probe side: the fact rows that pass their predicate
    for (int64_t f = 0; f < n_fact; ++f) {
        for (int c = 0; c < nf; ++c) val[static_cast<size_t>(c)] = load_value(fcols[c], ftypes[c], f);
        if (n_fp > 0 && x_eval(fpt, fpr, cp.data(), 0, zdiv) == 0) continue;
        if (!join) {
            emit();
            continue;
        }
        auto range = dim.equal_range(val[static_cast<size_t>(fkey)]);
        for (auto it = range.first; it != range.second; ++it) {
            for (int c = 0; c < nd; ++c) val[static_cast<size_t>(nf + c)] = load_value(dcols[c], dtypes[c], it->second);
            emit();
        }
    }
    if (out_join) *out_join = joined;
    if (out_bad) *out_bad = bad;
    auto result = [&](const G& g, int a) -> int64_t {
        const size_t i = static_cast<size_t>(a);
        switch (agg_op[a]) {
            case 0: return g.cnt;
            case 1: return g.sum[i];
            case 2: return g.mn[i];
            case 3: return g.mx[i];
            case 4: {
                const double d = static_cast<double>(g.sum[i]) / static_cast<double>(g.cnt);
                int64_t bits;
                std::memcpy(&bits, &d, sizeof bits);
                return bits;
            }
            default: return static_cast<int64_t>(g.dist[i].size());
        }
    };
    std::vector<std::pair<int32_t, int64_t>> order;     // (key, agg_1) for the top rows
    int64_t w = 0;
    for (const auto& kv : groups) {
        if (w < gcap) {
            out_key[w] = kv.first;
            for (int a = 0; a < nagg; ++a) out_vals[a * gcap + w] = result(kv.second, a);
        }
        if (topk > 0 && nagg > 0) order.emplace_back(kv.first, result(kv.second, 0));
        ++w;
    }
    if (topk > 0) {
        std::sort(order.begin(), order.end(), [](const std::pair<int32_t, int64_t>& x, const std::pair<int32_t, int64_t>& y) {
            if (x.second != y.second) return x.second > y.second;
            return x.first < y.first;
        });
        const int64_t kk = std::min<int64_t>(topk, static_cast<int64_t>(order.size()));
        for (int64_t i = 0; i < kk; ++i) {
            top_key[i] = order[static_cast<size_t>(i)].first;
            top_val[i] = order[static_cast<size_t>(i)].second;
        }
        *out_k = static_cast<int32_t>(kk);
    }
    return w;
}

}  // extern "C"
