/*
 * tqp.h — C ABI of the MI355X (gfx950) filter -> sort-based equi-join ->
 * group-by library.
 *
 * The operators follow "Query Processing on Tensor Computation Runtimes"
 * (Section 5 and Algorithms 1-2): a filter that turns a predicate into a
 * selection of rows (Section 3.1), a sort-based equi-join that returns pairs
 * of row indexes (Section 5.2, Algorithm 1), a sort-based group-by
 * aggregation (Section 5.4, Algorithm 2) and an ORDER BY ... LIMIT k sort
 * (Section 5, operator list).  Inputs are columns: one contiguous device
 * buffer per column (Section 4.1).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Pointers named d_* and every column / output pointer are DEVICE pointers,
 *   owned by the caller.  The library keeps none of them after the call
 *   returns.  Structures passed by pointer (tqp_column, tqp_pred, fragment
 *   descriptors) live in HOST memory and are read during the call only.
 * - Calls are asynchronous on `stream`; argument errors are reported
 *   synchronously through the return value and tqp_last_error().
 * - Workspace: every call that needs scratch memory takes (ws, ws_bytes).
 *   With ws == NULL the call only writes the number of bytes it needs to
 *   *ws_bytes and returns TQP_OK.  Otherwise ws must be a device buffer of at
 *   least *ws_bytes bytes, 256-byte aligned, not used by any other call until
 *   this call's work on `stream` has completed.  The library clears what it
 *   needs inside the workspace with its own kernels.
 * - Data-dependent sizes (rows kept by a filter, join rows, groups) are
 *   written to device counters (d_count, d_ngroups ...); the host is never
 *   synchronised.  When a true size exceeds the caller's capacity, only
 *   `cap` rows are written, the true size is still stored, and the context's
 *   device error word gets TQP_DEVERR_CAPACITY (see tqp_ctx_errors).
 * - Keys of sorts and joins are non-negative int32.  `key_bits` declares that
 *   every key is < 2^key_bits (1..31; 0 means 31).  A key outside that range
 *   sets TQP_DEVERR_KEY_RANGE and leaves the output unspecified.
 * - Element counts are limited to 2^30 - 1 per call (TQP_ERR_UNSUPPORTED
 *   beyond).
 * - All integer aggregates are exact int64; averages are one IEEE double
 *   division of the exact sum by the count.
 */
#ifndef TQP_H
#define TQP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TQP_OK = 0,
    TQP_ERR_INVALID = 1,      /* bad argument (null pointer, negative size, bad enum) */
    TQP_ERR_WORKSPACE = 2,    /* ws_bytes smaller than the size query returned */
    TQP_ERR_CAPACITY = 3,     /* reported by tqp_ctx_errors when an output overflowed */
    TQP_ERR_HIP = 4,          /* a HIP runtime call or kernel launch failed */
    TQP_ERR_UNSUPPORTED = 5   /* size or option outside what the library implements */
} tqp_status;

typedef enum { TQP_I8 = 1, TQP_I32 = 2, TQP_I64 = 3 } tqp_dtype;

/* Comparison of a column with a constant (Section 5.1 expressions). */
typedef enum { TQP_LT = 0, TQP_LE = 1, TQP_GT = 2, TQP_GE = 3, TQP_EQ = 4, TQP_NE = 5 } tqp_cmp;

/* Device error bits (OR-ed by kernels into the context's error word). */
#define TQP_DEVERR_KEY_RANGE 1u   /* a key was negative or >= 2^key_bits */
#define TQP_DEVERR_SPIN 2u        /* an inter-tile wait hit its safety bound */
#define TQP_DEVERR_CAPACITY 4u    /* an output count exceeded its capacity */
#define TQP_DEVERR_VALUE_RANGE 8u /* a value was outside its declared width or domain */

/* One column: device pointer to n contiguous values of `type`. */
typedef struct {
    const void* data;
    int32_t type;             /* tqp_dtype */
    int32_t reserved;
} tqp_column;

/* One conjunct of a filter: cols[col] <op> k. */
typedef struct {
    int32_t col;
    int32_t op;               /* tqp_cmp */
    int64_t k;
} tqp_pred;

typedef struct tqp_ctx tqp_ctx;

/* ---------------------------------------------------------------- context
 * A context binds the library to one device and owns a small device error
 * word and the tuning table (radix digit width, tile shape per workload).
 * It is not thread-safe: use one context per host thread. */
tqp_status tqp_ctx_create(int device, tqp_ctx** out);
void tqp_ctx_destroy(tqp_ctx* ctx);

/* Thread-local description of the last error returned on this thread. */
const char* tqp_last_error(void);

/* Synchronises `stream`, copies the device error word to *errors (a bitmask
 * of TQP_DEVERR_*) and clears it when `clear` is non-zero. */
tqp_status tqp_ctx_errors(tqp_ctx* ctx, hipStream_t stream, uint32_t* errors, int clear);

/* Radix digit width used by sorts: 4, 8 or 11 bits (0 restores the default
 * of 8).  The batch autotuner sets it per workload. */
tqp_status tqp_ctx_set_digit_bits(tqp_ctx* ctx, int bits);

/* Plain device-to-device copy of `bytes` (a multiple of 16, 16-byte aligned
 * pointers) with one streaming kernel: moves columns, and is the reference
 * kernel of known size against which hardware traffic counters are read. */
tqp_status tqp_copy(tqp_ctx* ctx, void* dst, const void* src, size_t bytes, hipStream_t stream);

/* Per-launch timing.  While profiling is on, every kernel the library
 * launches is bracketed by two events recorded on the launch stream (this
 * adds a little host work per launch).  tqp_ctx_profile_read synchronises
 * `stream` and the device, writes up to `cap` records (kernel label and
 * duration in milliseconds, in launch order) to `out`, the number of records
 * to *n, and clears them. */
typedef struct {
    char name[40];
    double ms;
} tqp_prof_entry;

tqp_status tqp_ctx_set_profiling(tqp_ctx* ctx, int on);
tqp_status tqp_ctx_profile_read(tqp_ctx* ctx, hipStream_t stream, tqp_prof_entry* out, int cap, int* n);

/* ---------------------------------------------------------------- filter
 * Section 3.1 (Listing 1 and the selection-vector form): the row ids i in
 * [0, n) for which every predicate cols[p.col][i] <p.op> p.k holds, in
 * increasing order, written to out_rowid; carry (nullable, int32[n]) is
 * compacted the same way into out_carry.  At most 4 predicates.  The number
 * of selected rows goes to *d_count (device int64). */
tqp_status tqp_filter(tqp_ctx* ctx, const tqp_column* cols, int ncols, int64_t n,
                      const tqp_pred* preds, int npreds, const int32_t* carry,
                      int32_t* out_rowid, int32_t* out_carry, int64_t cap, int64_t* d_count,
                      void* ws, size_t* ws_bytes, hipStream_t stream);

/* The filter above without allocation or workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, semantics and results
 * as tqp_filter, minus (ws, ws_bytes).  Its scratch (a tile counter and one
 * look-back word per 4096 rows) is a fixed device array of
 * TQP_NOALLOC_SCRATCH_BYTES per device, held until the process ends, so n is
 * limited to TQP_FILTER_NOALLOC_MAX_ROWS (TQP_ERR_UNSUPPORTED above; checked
 * before anything is launched).  The array's address is looked up when a
 * context is created on the device.  Every call clears the part it uses with
 * a kernel (no memset).  All calls on one device share the one array: calls
 * that overlap in time on the same device (other streams, other host
 * threads) race and give wrong results; serialise them. */
#define TQP_NOALLOC_SCRATCH_BYTES 1048576
#define TQP_FILTER_NOALLOC_MAX_ROWS 536739840LL   /* (1 MiB - 256 B) / 8 B per tile x 4096 rows per tile */
tqp_status tqp_filter_noalloc(tqp_ctx* ctx, const tqp_column* cols, int ncols, int64_t n,
                              const tqp_pred* preds, int npreds, const int32_t* carry,
                              int32_t* out_rowid, int32_t* out_carry, int64_t cap, int64_t* d_count,
                              hipStream_t stream);

/* ---------------------------------------------------------------- sort
 * Algorithm 1 (sort of each join-key column with its index) and Algorithm 2
 * (sort of the group keys): stable ascending LSD radix sort of the pairs
 * (keys[i], vals[i]).  vals == NULL sorts the pairs (keys[i], i), so vals_out
 * receives the sorting permutation; vals_out == NULL sorts keys only.  The
 * element count is n, or *d_n (device int64, <= n) when d_n is not NULL.
 * Outputs must not alias inputs. */
tqp_status tqp_sort(tqp_ctx* ctx, const int32_t* keys, const int32_t* vals, int64_t n,
                    const int64_t* d_n, int key_bits, int32_t* keys_out, int32_t* vals_out,
                    void* ws, size_t* ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- join
 * Section 5.2, Algorithm 1: equi-join of two inputs already sorted by key
 * (ascending).  For every pair i, j with lkey[i] == rkey[j] one output row
 * (lrow[i], rrow[j]) — the index pairs of late materialisation — in the order
 * (i, j) ascending, i.e. key ascending and, within a key, left-major as in
 * the quotient / remainder step of Algorithm 1.  lrow / rrow may be NULL
 * (the positions i / j are emitted).  Sizes nl / nr, or the device counts
 * *d_nl / *d_nr when given.  The true number of output rows goes to
 * *d_count; at most cap rows are written. */
tqp_status tqp_join(tqp_ctx* ctx, const int32_t* lkey, const int32_t* lrow, int64_t nl,
                    const int64_t* d_nl, const int32_t* rkey, const int32_t* rrow, int64_t nr,
                    const int64_t* d_nr, int32_t* out_l, int32_t* out_r, int64_t cap,
                    int64_t* d_count, void* ws, size_t* ws_bytes, hipStream_t stream);

/* Join kinds (the operator list at the start of Section 5; Section 5.2 gets
 * them from Algorithm 1 by changing the number of output rows per left row):
 *   TQP_JOIN_INNER       as tqp_join;
 *   TQP_JOIN_LEFT_SEMI   one row (lrow[i], -1) per left row with a match;
 *   TQP_JOIN_LEFT_ANTI   one row (lrow[i], -1) per left row without one;
 *   TQP_JOIN_LEFT_OUTER  the inner rows of every left row, or (lrow[i], -1)
 *                        when it has no match.
 * Rows in left order, then right order.  Arguments, sizes, sortedness and
 * capacity as tqp_join; out_r may be NULL for the semi and anti joins (it
 * would hold only -1).  An unknown kind returns TQP_ERR_INVALID. */
/* Section 5.3, Algorithm 3: the hash-based equi-join, partitioned.  Same
 * rows as tqp_join (every (lrow[i], rrow[j]) with lkey[i] == rkey[j]), but
 * the inputs need not be sorted.  Both sides are split into 2^P partitions
 * (P <= 16, up to about 2000 right rows each) by the top bits of a
 * multiplicative hash of the key, one or two radix passes per side; then
 * every partition is joined
 * in LDS: a table of its right rows (one slot per distinct key, the rows of a
 * key stored as one run from a count and a scan, so duplicates cost O(1) per
 * insert), probed once per left row.  Output rows come in no fixed order; the
 * set of rows is exact.  A negative key sets TQP_DEVERR_KEY_RANGE and its row
 * is left out.  Arguments, device counts and capacity as tqp_join (with an
 * overflow, which cap rows are written is not fixed). */
tqp_status tqp_hash_join(tqp_ctx* ctx, const int32_t* lkey, const int32_t* lrow, int64_t nl,
                         const int64_t* d_nl, const int32_t* rkey, const int32_t* rrow, int64_t nr,
                         const int64_t* d_nr, int32_t* out_l, int32_t* out_r, int64_t cap,
                         int64_t* d_count, void* ws, size_t* ws_bytes, hipStream_t stream);

/* Band join, the non-equi join of Section 5.2's variants: every
 * (lrow[i], rrow[j]) with |lkey[i] - rkey[j]| <= w, w >= 0 (w = 0 is
 * tqp_join).  Both inputs sorted by key (ascending); the matches of left row i
 * are one contiguous range of the right side, emitted in the order (i, j)
 * ascending.  Keys non-negative int32.  Arguments, device counts and capacity
 * as tqp_join; w < 0 returns TQP_ERR_INVALID. */
tqp_status tqp_join_band(tqp_ctx* ctx, const int32_t* lkey, const int32_t* lrow, int64_t nl,
                         const int64_t* d_nl, const int32_t* rkey, const int32_t* rrow, int64_t nr,
                         const int64_t* d_nr, int64_t w, int32_t* out_l, int32_t* out_r, int64_t cap,
                         int64_t* d_count, void* ws, size_t* ws_bytes, hipStream_t stream);

#define TQP_JOIN_INNER 0
#define TQP_JOIN_LEFT_SEMI 1
#define TQP_JOIN_LEFT_ANTI 2
#define TQP_JOIN_LEFT_OUTER 3
tqp_status tqp_join_kind(tqp_ctx* ctx, int kind, const int32_t* lkey, const int32_t* lrow, int64_t nl,
                         const int64_t* d_nl, const int32_t* rkey, const int32_t* rrow, int64_t nr,
                         const int64_t* d_nr, int32_t* out_l, int32_t* out_r, int64_t cap,
                         int64_t* d_count, void* ws, size_t* ws_bytes, hipStream_t stream);

/* Composite keys (Section 5.4 concatenates the group-by columns into one key
 * before the sort; Algorithm 3 compares several join-key columns): out[i]
 * packs cols[0][i], ..., cols[ncols-1][i], the first column most significant
 * and column c taking bits[c] bits, so sorting or joining the packed keys
 * sorts or joins the tuples.  1 <= ncols <= 4, each bits[c] >= 1, their sum
 * <= 31.  Values must lie in [0, 2^bits[c]); others set
 * TQP_DEVERR_KEY_RANGE (their row is packed from the masked value).  cols and
 * bits are host arrays of device column pointers and widths; n or *d_n rows.
 * No workspace. */
tqp_status tqp_pack_keys(tqp_ctx* ctx, const int32_t* const* cols, const int32_t* bits, int ncols, int64_t n,
                         const int64_t* d_n, int32_t* out, hipStream_t stream);

/* Expression programs (Section 5.1: arithmetic, comparisons, logic and CASE
 * over columns), as a postfix program of at most 64 instructions over int64
 * values, with at most 16 values on the stack and at most 8 columns (int8,
 * int32 or int64, widened).  Binary operators pop b, then a, and push a op b;
 * SELECT pops f, t, c and pushes c ? t : f.  +, -, * and unary minus wrap
 * (two's complement); / and % truncate toward zero; a zero divisor gives 0
 * and sets TQP_DEVERR_VALUE_RANGE; INT64_MIN / -1 = INT64_MIN, INT64_MIN %
 * -1 = 0; comparisons, AND, OR and NOT give 0 or 1 (nonzero is true).  out[i]
 * = the program's value on row i, for n or *d_n rows.  A malformed program
 * (unknown operator, missing operands, a column out of range, not exactly
 * one value left) is refused with TQP_ERR_INVALID before any launch.  No
 * workspace. */
typedef enum {
    TQP_X_COL = 0, TQP_X_CONST = 1, TQP_X_ADD = 2, TQP_X_SUB = 3, TQP_X_MUL = 4, TQP_X_DIV = 5,
    TQP_X_MOD = 6, TQP_X_NEG = 7, TQP_X_LT = 8, TQP_X_LE = 9, TQP_X_GT = 10, TQP_X_GE = 11,
    TQP_X_EQ = 12, TQP_X_NE = 13, TQP_X_AND = 14, TQP_X_OR = 15, TQP_X_NOT = 16, TQP_X_SELECT = 17
} tqp_xop;
typedef struct {
    int32_t op;               /* tqp_xop */
    int32_t reserved;
    int64_t arg;              /* column index (TQP_X_COL) or constant (TQP_X_CONST) */
} tqp_xinstr;
tqp_status tqp_eval(tqp_ctx* ctx, const tqp_column* cols, int ncols, int64_t n, const int64_t* d_n,
                    const tqp_xinstr* prog, int nprog, int64_t* out, hipStream_t stream);

/* Gather by row position, the late materialisation of Section 5.2 (joins
 * return row positions; the columns a later operator needs, such as the next
 * join's key in a chain of joins, are read through them): out[i] =
 * src[idx[i]] for i < n (or *d_n), elements of elem_bytes = 4 or 8 bytes.  A
 * negative idx[i] (the missing right row of an outer join) gives -1; an
 * index >= nsrc gives -1 and sets TQP_DEVERR_KEY_RANGE.  No workspace. */
tqp_status tqp_gather(tqp_ctx* ctx, const void* src, int64_t nsrc, int elem_bytes, const int32_t* idx, int64_t n,
                      const int64_t* d_n, void* out, hipStream_t stream);

/* Chains of equi-joins (a multi-join plan, such as the six-join query of
 * Section 6.3): table 0's key column key_out joins table 1's key_pk, table
 * 1's key_out joins table 2's key_pk, and so on.  Each hop sorts the current
 * tuples' keys, sorts table t's key column (unless its rule says otherwise)
 * and runs the sort-based join of tqp_join, then reads the earlier row
 * positions and the next key through the join's output (late
 * materialisation).  Rules (Section 6.6's hand-optimised plans; asserted by
 * the caller, not checked): TQP_CHAIN_PK_SORTED, key_pk is already ascending
 * (its sort is skipped); TQP_CHAIN_PK_DENSE, key_pk is exactly 0..n_rows-1
 * in row order (no sort and no join: the tuples whose key lies in
 * [0, n_rows) are kept, the key being the row position; key_pk may be NULL).
 * Every hop's size stays on the device; the hop into table t writes at most
 * tables[t].cap tuples (a larger true size sets TQP_DEVERR_CAPACITY and the
 * later hops work on the written ones).  Output: out_rows[u] (device, at
 * least tables[ntables-1].cap entries each) receives the final tuples' row
 * positions in table u, *d_count (device) the final tuple count.  Tuples come
 * in no fixed order.  2 <= ntables <= TQP_CHAIN_MAX_TABLES; keys are
 * non-negative int32 below 2^key_bits of their hop (TQP_DEVERR_KEY_RANGE
 * otherwise). */
#define TQP_CHAIN_MAX_TABLES 8
#define TQP_CHAIN_PK_SORTED 1
#define TQP_CHAIN_PK_DENSE 2
typedef struct {
    const int32_t* key_out;   /* n_rows keys into the next table (unused for the last table) */
    const int32_t* key_pk;    /* n_rows keys joined by the previous table's key_out (unused for table 0) */
    int64_t n_rows;
    int64_t cap;              /* tuples the hop into this table may write (unused for table 0) */
    int32_t key_bits;         /* key width of the hop into this table (0: 31) */
    int32_t rule;             /* 0, TQP_CHAIN_PK_SORTED or TQP_CHAIN_PK_DENSE */
} tqp_chain_table;
tqp_status tqp_join_chain(tqp_ctx* ctx, const tqp_chain_table* tables, int ntables, int32_t* const* out_rows,
                          int64_t* d_count, void* ws, size_t* ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- group-by
 * Section 5.4, Algorithm 2: sort the group keys, permute the value columns
 * by the sorted order, find the runs of equal keys and evaluate the
 * aggregates per run.  Output: one row per distinct key in ascending key
 * order: out_key, out_sum = sum(sum_in), out_cnt = count, and (when avg_in
 * and out_avg are not NULL) out_avg = (double)sum(avg_in) / (double)count.
 * Keys are non-negative int32 < 2^key_bits.  n or *d_n elements.  The
 * number of groups goes to *d_ngroups; at most gcap groups are written. */
tqp_status tqp_groupby_agg(tqp_ctx* ctx, const int32_t* gkey, int64_t n, const int64_t* d_n,
                           int key_bits, const int64_t* sum_in, const int64_t* avg_in,
                           int32_t* out_key, int64_t* out_sum, int64_t* out_cnt, double* out_avg,
                           int64_t gcap, int64_t* d_ngroups, void* ws, size_t* ws_bytes,
                           hipStream_t stream);

/* Hash-based group-by (the hash aggregation Section 6 contrasts with the
 * sort-based one of Section 5.4) with the aggregates listed in the
 * introduction of Section 5:
 * one row per distinct key of gkey, in no fixed order: out_key, out_cnt =
 * count, and, for each of these outputs that is not NULL, out_sum =
 * sum(val), out_min = min(val), out_max = max(val), out_ndist = the number
 * of different values of dval in the group (COUNT(DISTINCT dval)).  val is
 * needed for sum, min and max, dval for out_ndist.  Keys must be >= 0; a
 * negative key sets TQP_DEVERR_KEY_RANGE and its row is skipped.  gcap:
 * the caller's bound on groups, which sizes the table (2 * gcap slots of 32
 * bytes, plus 2 * n slots of 8 bytes when out_ndist is given); groups beyond
 * it, or a probe of more than 4096 slots, set TQP_DEVERR_CAPACITY and leave
 * those rows out.  The group count goes to *d_ngroups (after an overflow:
 * the groups that were taken in, which may be more or fewer than gcap); at
 * most gcap rows are written.  n or *d_n rows. */
tqp_status tqp_hash_groupby(tqp_ctx* ctx, const int32_t* gkey, int64_t n, const int64_t* d_n,
                            const int64_t* val, const int32_t* dval, int32_t* out_key, int64_t* out_cnt,
                            int64_t* out_sum, int64_t* out_min, int64_t* out_max, int64_t* out_ndist,
                            int64_t gcap, int64_t* d_ngroups, void* ws, size_t* ws_bytes,
                            hipStream_t stream);

/* ---------------------------------------------------------------- top-k
 * ORDER BY sum DESC, key ASC LIMIT k over aggregated groups (keys must be
 * unique, as group-by output is): rows (key, sum, cnt) of the first min(k, n)
 * groups; the row count goes to *d_k (device int32).  1 <= k <= 1024. */
tqp_status tqp_topk(tqp_ctx* ctx, const int32_t* key, const int64_t* sum, const int64_t* cnt,
                    int64_t n, const int64_t* d_n, int k, int32_t* out_key, int64_t* out_sum,
                    int64_t* out_cnt, int32_t* d_k, void* ws, size_t* ws_bytes,
                    hipStream_t stream);

/* ---------------------------------------------------------------- fragments
 * Whole query fragments: filter -> sort-based join -> group-by in one launch
 * sequence on one stream, with every intermediate in the workspace and the
 * filters, the revenue expression and (for few groups) the aggregation fused
 * into the neighbouring kernels. */

/* Flags fragment:
 *   SELECT flagA*2+flagB AS g, SUM(price*(100-disc)), COUNT(*), AVG(price)
 *   FROM fact JOIN dim ON fact.fk = dim.pk
 *   WHERE fact.date < D AND dim.seg = c GROUP BY g ORDER BY g
 * price is int64 cents, disc int64 percent, so SUM is exact in cent*percent.
 * The fact rows are [row0, row0 + n_fact) of the given columns (row0 lets a
 * fragment cover a range of a larger resident table).  flagA must lie in
 * 0..2 and flagB in 0..1 (six groups); a joined row with a flag outside its
 * domain is left out of every aggregate and sets TQP_DEVERR_VALUE_RANGE. */
typedef struct {
    const int32_t* fk;
    const int32_t* date;
    const int64_t* price;
    const int64_t* disc;
    const int8_t* flagA;      /* values 0..2 */
    const int8_t* flagB;      /* values 0..1 */
    int64_t row0;
    int64_t n_fact;
    const int32_t* pk;
    const int8_t* seg;
    int64_t n_dim;
    int32_t D;
    int32_t c;
    int32_t key_bits;         /* fk and pk < 2^key_bits (0: 31) */
    int32_t reserved;
} tqp_flags_fragment;

/* Outputs of a flags fragment (device pointers): up to 6 groups. */
typedef struct {
    int32_t* key;             /* [8] */
    int64_t* sum;             /* [8] */
    int64_t* cnt;             /* [8] */
    double* avg;              /* [8] */
    int64_t* d_ngroups;       /* number of groups written */
    int64_t* d_join;          /* join cardinality (nullable) */
} tqp_flags_out;

tqp_status tqp_fragment_flags(tqp_ctx* ctx, const tqp_flags_fragment* f, const tqp_flags_out* o,
                              void* ws, size_t* ws_bytes, hipStream_t stream);

/* Custkey fragment:
 *   SELECT mid.custkey, SUM(price*(100-disc)), COUNT(*)
 *   FROM fact JOIN mid ON fact.fk = mid.pk WHERE fact.date < D
 *   GROUP BY mid.custkey, plus ORDER BY sum DESC, custkey ASC LIMIT k. */
typedef struct {
    const int32_t* fk;
    const int32_t* date;
    const int64_t* price;
    const int64_t* disc;
    int64_t n_fact;
    const int32_t* pk;
    const int32_t* custkey;
    int64_t n_mid;
    int32_t D;
    int32_t key_bits;         /* fk and pk < 2^key_bits (0: 31) */
    int32_t cust_bits;        /* custkey < 2^cust_bits (0: 31) */
    int32_t k;                /* top rows wanted, 1..1024 */
    int64_t join_cap;         /* capacity for join rows (n_fact suffices when pks are unique) */
    int32_t revenue_bits;     /* 0 or 64: revenue carried as int64.  32: the caller declares that
                               * every kept row's price*(100-disc) lies in [0, 2^32); it is carried
                               * in 4 bytes through the sorts and the join (sums stay exact int64).
                               * A row outside sets TQP_DEVERR_VALUE_RANGE (results unspecified). */
    int32_t mid_sorted;       /* non-zero: pk is already in ascending order (custkey row-aligned with it),
                               * so the mid sort is skipped, as Section 6.6's hand-optimised plans skip
                               * sorting data that is already sorted.  The caller guarantees the order
                               * and pk < 2^key_bits; neither is checked. */
} tqp_cust_fragment;

typedef struct {
    int32_t* key;             /* [gcap] all groups, custkey ascending */
    int64_t* sum;             /* [gcap] */
    int64_t* cnt;             /* [gcap] */
    int64_t gcap;
    int64_t* d_ngroups;
    int64_t* d_join;          /* join cardinality (nullable) */
    int32_t* top_key;         /* [k] */
    int64_t* top_sum;         /* [k] */
    int64_t* top_cnt;         /* [k] */
    int32_t* d_topk;          /* rows in the top arrays */
} tqp_cust_out;

tqp_status tqp_fragment_cust(tqp_ctx* ctx, const tqp_cust_fragment* f, const tqp_cust_out* o,
                             void* ws, size_t* ws_bytes, hipStream_t stream);

/* The launch plan tqp_fragment_cust uses for f with the context's digit
 * width (host only): radix passes of the fact, mid and group-key sorts, the
 * low fact-key bits the fact sort leaves to the join (its tiles then cover
 * bucket-aligned key ranges) and the low group-key bits resolved in LDS by
 * the bucket aggregation.  Any output pointer may be NULL. */
tqp_status tqp_fragment_cust_plan(tqp_ctx* ctx, const tqp_cust_fragment* f, int* fact_passes, int* fact_lowb,
                                  int* mid_passes, int* group_passes, int* group_lowb);

/* General fragment: the operators of Section 5 composed by a descriptor,
 *   SELECT pack(g_1..g_q), agg_1, ..., agg_m
 *   FROM fact [JOIN dim ON fact.col[fact_key] = dim.col[dim_key]]
 *   WHERE fact_pred(fact row) [AND dim_pred(dim row)]
 *   GROUP BY pack(g_1..g_q) ORDER BY the packed key
 *   [and ORDER BY agg_1 DESC, key ASC LIMIT topk]
 * run as one launch sequence with every data-dependent size on the device.
 * Predicates and aggregate values are postfix programs (tqp_xinstr, the
 * semantics of tqp_eval); a predicate keeps the rows where it is nonzero, and
 * an empty one (n_*_pred = 0) keeps every row.  The fact predicate numbers the
 * fact columns, the dim predicate the dim columns; group columns and aggregate
 * programs number the joined row: fact columns 0..nf-1, then dim columns
 * nf..nf+nd-1 (each program may read at most 8 different columns).  Without a
 * join (fact_key < 0) the joined rows are the kept fact rows.  Join keys are
 * int32 columns, non-negative and below 2^key_bits.  The group key packs the
 * group columns (at most 4, any integer type), column i taking bits[i] bits,
 * the first most significant, at most 31 bits in all (a value outside its
 * width sets TQP_DEVERR_KEY_RANGE and enters masked); no group column puts
 * every row in group 0.  Aggregates (at most 8): TQP_AGG_COUNT (no program),
 * TQP_AGG_SUM (int64, wrapping), TQP_AGG_MIN, TQP_AGG_MAX, TQP_AGG_AVG
 * ((double)SUM / (double)COUNT, written as a double), TQP_AGG_COUNT_DISTINCT
 * (at most one per fragment).  Each aggregate writes one value per group to
 * its out array (device, gcap entries of 8 bytes).  Groups come in ascending
 * key order; *d_ngroups receives the group count (at most gcap written,
 * TQP_DEVERR_CAPACITY beyond).  topk > 0 (1..1024, agg_1 not AVG): the first
 * topk groups by (agg_1 desc, key asc) go to top_key / top_val and their
 * number to *d_topk.  join_cap bounds the joined rows (TQP_DEVERR_CAPACITY
 * beyond; the true count goes to *d_join when given).  value_bits = 32
 * declares that the program of the one aggregate with a program lies in
 * [-2^31, 2^31) on every fact row; when that program reads fact columns
 * only (and the fragment is grouped by one int32 dim column of 16 bits or
 * more) its value is then carried in 32 bits, and a value outside sets
 * TQP_DEVERR_VALUE_RANGE; otherwise the declaration is not used.  The
 * composition is sort-based throughout: both join sides are radix-sorted with
 * their predicates fused into the sort, joined as by tqp_join, the group keys
 * (and, for COUNT(DISTINCT), the distinct values first) radix-sorted with the
 * joined-row index, and each group's run reduced; with one aggregate that has
 * a program (no COUNT(DISTINCT)) and a key of 16 bits or more, the group sort
 * covers the key bits above the last 8 to 13 and each bucket of keys is
 * reduced in LDS. */
#define TQP_AGG_COUNT 0
#define TQP_AGG_SUM 1
#define TQP_AGG_MIN 2
#define TQP_AGG_MAX 3
#define TQP_AGG_AVG 4
#define TQP_AGG_COUNT_DISTINCT 5
#define TQP_FRAGMENT_MAX_GROUP_COLS 4
#define TQP_FRAGMENT_MAX_AGGS 8
typedef struct {
    int32_t col;              /* joined column number */
    int32_t bits;             /* width of its values, >= 1 */
} tqp_group_col;
typedef struct {
    int32_t op;               /* TQP_AGG_* */
    int32_t nprog;            /* 0 for TQP_AGG_COUNT */
    const tqp_xinstr* prog;   /* host */
    void* out;                /* device, gcap values: int64, or double for TQP_AGG_AVG */
} tqp_agg;
typedef struct {
    const tqp_column* fact_cols;   /* host array of device columns, n_fact rows each */
    int32_t n_fact_cols;
    int32_t fact_key;              /* fact column of the join key, -1: no join */
    int64_t n_fact;
    const tqp_xinstr* fact_pred;
    int32_t n_fact_pred;
    int32_t key_bits;              /* join keys < 2^key_bits (0: 31) */
    const tqp_column* dim_cols;    /* n_dim rows each */
    int32_t n_dim_cols;
    int32_t dim_key;
    int64_t n_dim;
    const tqp_xinstr* dim_pred;
    int32_t n_dim_pred;
    int32_t n_group;
    const tqp_group_col* group;
    const tqp_agg* aggs;
    int32_t n_agg;
    int32_t topk;
    int64_t join_cap;
    int32_t value_bits;            /* 0 or 64; 32: see below */
    int32_t reserved;
} tqp_fragment;
typedef struct {
    int32_t* key;             /* [gcap] packed group keys, ascending */
    int64_t gcap;
    int64_t* d_ngroups;
    int64_t* d_join;          /* joined rows (nullable) */
    int32_t* top_key;         /* [topk] (when topk > 0) */
    int64_t* top_val;         /* [topk] */
    int32_t* d_topk;
} tqp_fragment_out;
tqp_status tqp_fragment_run(tqp_ctx* ctx, const tqp_fragment* f, const tqp_fragment_out* o, void* ws,
                            size_t* ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- batches
 * Many flags fragments (each with its own fact and dim columns, D and c) run
 * as one launch sequence: every stage is one persistent kernel over all
 * fragments, pulling (fragment, tile) work items from a device counter.  The
 * paper runs operators one after another (Section 4.3); batching fragments
 * into shared launches is this library's addition.
 *
 * tqp_batch_create: with ws == NULL writes the workspace size to *ws_bytes.
 * Otherwise prepares the batch over ws (device, 256-byte aligned, owned by
 * the caller, kept by the batch until tqp_batch_destroy) and copies the
 * descriptors to the device (synchronous).  Each fragment's results go to
 * its tqp_flags_out, exactly as tqp_fragment_flags would write them.
 * Configurations: 0 = 4-bit digits / 2048-row tiles, 1 = 8-bit / 2048,
 * 2 = 8-bit / 4096 (default), 3 = 11-bit / 4096.
 * tqp_batch_autotune runs every configuration `reps` times on `stream`, keeps
 * the fastest and writes the mean time of each to times_ms[4] (nullable).
 * tqp_batch_capture records the launch sequence of the chosen configuration
 * into a hipGraph (stream must not be the null stream); tqp_batch_replay
 * launches that graph.  Calls that share a batch must not overlap in time. */
typedef struct tqp_batch tqp_batch;

tqp_status tqp_batch_create(tqp_ctx* ctx, const tqp_flags_fragment* frags, const tqp_flags_out* outs, int nf,
                            void* ws, size_t* ws_bytes, tqp_batch** out);
void tqp_batch_destroy(tqp_batch* b);
tqp_status tqp_batch_run(tqp_batch* b, hipStream_t stream);
tqp_status tqp_batch_set_config(tqp_batch* b, int config);
tqp_status tqp_batch_config(const tqp_batch* b, int* config, int* digit_bits, const char** name);
tqp_status tqp_batch_autotune(tqp_batch* b, hipStream_t stream, int reps, float* times_ms);
tqp_status tqp_batch_capture(tqp_batch* b, hipStream_t stream);
tqp_status tqp_batch_replay(tqp_batch* b, hipStream_t stream);

/* ---------------------------------------------------------------- serving
 * A request loop over device-resident tables: requests are submitted from
 * any host thread, stamped on arrival, admitted first-come first-served into
 * free slots while the in-flight working set (each request's exact workspace
 * and outputs) stays within budget_bytes, and launched at once on the slot's
 * own stream, so requests that arrive while others run overlap on the device.
 * Flags requests that wait together are launched as one batch (up to
 * max_batch of them in one slot).  A background thread admits, launches and
 * collects; results are read with tqp_server_poll.  With slots = 1 and
 * max_batch = 1 the server runs one request at a time: the serial form.
 * Every slot has its own stream, side stream and device error word, so the
 * launches of different slots neither wait for each other nor mix their
 * error bits.
 *
 * Resident tables (device, owned by the caller, unchanged while the server
 * lives): the fact table carries two keys, fk_mid into the mid table and
 * fk_dim into the dim table. */
typedef struct {
    const int32_t* fk_mid;
    const int32_t* fk_dim;
    const int32_t* date;
    const int64_t* price;
    const int64_t* disc;
    const int8_t* flagA;
    const int8_t* flagB;
    int64_t n_fact;
    const int32_t* mid_pk;
    const int32_t* mid_custkey;
    int64_t n_mid;
    const int32_t* dim_pk;
    const int8_t* dim_seg;
    int64_t n_dim;
    int32_t key_bits_mid;     /* fk_mid and mid_pk < 2^key_bits_mid */
    int32_t key_bits_dim;     /* fk_dim and dim_pk < 2^key_bits_dim */
    int32_t cust_bits;        /* custkey < 2^cust_bits */
    int32_t slots;            /* requests on the device at once (1..64) */
    int32_t max_batch;        /* flags requests coalesced into one launch (1..256) */
    int32_t revenue_bits;     /* custkey requests: revenue width, as tqp_cust_fragment.revenue_bits */
    int64_t max_flags_rows;   /* largest fact row range of a flags request */
    size_t budget_bytes;      /* HBM working-set budget of in-flight requests */
    int32_t presort_mid;      /* non-zero: the mid table is sorted by pk once, when the server is
                               * created (server memory: 8 bytes per mid row), and custkey requests
                               * join against that order instead of sorting the mid table again */
    int32_t reserved;
} tqp_server_config;

#define TQP_REQ_CUST 0        /* custkey fragment over the whole fact table, top-k */
#define TQP_REQ_FLAGS 1       /* flags fragment over fact rows [row0, row0 + n_rows) */
#define TQP_TOPK_MAX 128

typedef struct {
    int32_t kind;             /* TQP_REQ_* */
    int32_t D;
    int32_t c;                /* flags: segment value */
    int32_t k;                /* custkey: top rows, 1..TQP_TOPK_MAX */
    int64_t row0;
    int64_t n_rows;
    uint64_t tag;             /* caller's value, returned with the result */
} tqp_request;

typedef struct {
    uint64_t id;
    uint64_t tag;
    int32_t kind;
    int32_t status;           /* TQP_OK, or the error of the launch */
    int64_t join_rows;
    int64_t groups;
    int32_t key[8];           /* flags: groups in key order */
    int64_t sum[8];
    int64_t cnt[8];
    double avg[8];
    int32_t top_n;            /* custkey: rows in top_* */
    int32_t top_key[TQP_TOPK_MAX];
    int64_t top_sum[TQP_TOPK_MAX];
    int64_t top_cnt[TQP_TOPK_MAX];
    double t_arrival;         /* seconds on the server clock */
    double t_admit;
    double t_done;            /* result visible on the host */
    int32_t slot;
    int32_t batch_size;       /* requests launched together with this one */
    uint32_t dev_errors;      /* TQP_DEVERR_* bits raised by this launch's kernels (every request of
                               * a batched launch gets the launch's bits); when non-zero, status is
                               * TQP_ERR_CAPACITY for a capacity overflow, else TQP_ERR_INVALID */
    int32_t reserved;
} tqp_result;

typedef struct tqp_server tqp_server;

tqp_status tqp_server_create(tqp_ctx* ctx, const tqp_server_config* cfg, tqp_server** out);
void tqp_server_destroy(tqp_server* s);
/* Seconds since the server was created (the clock of the t_* fields). */
double tqp_server_now(const tqp_server* s);
tqp_status tqp_server_submit(tqp_server* s, const tqp_request* req, uint64_t* id);
/* Moves up to cap finished results to out; *n receives how many. */
tqp_status tqp_server_poll(tqp_server* s, tqp_result* out, int cap, int* n);
/* Blocks until every submitted request has finished. */
tqp_status tqp_server_drain(tqp_server* s);
/* Counters: requests submitted, finished, launches, peak in-flight bytes. */
tqp_status tqp_server_stats(const tqp_server* s, uint64_t* submitted, uint64_t* finished, uint64_t* launches,
                            size_t* peak_bytes);

#ifdef __cplusplus
}
#endif

#endif /* TQP_H */
