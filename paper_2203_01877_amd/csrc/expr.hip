// Expression programs (Section 5.1: arithmetic, comparisons, logic and CASE
// over columns).  The paper evaluates an expression one tensor operation at a
// time, each writing its intermediate column to device memory.  Here the
// expression comes as a postfix program (a small descriptor the host checks
// once) and one kernel evaluates all of it per row, with the evaluation stack
// in registers (its top) and LDS (the rest): the intermediates never reach
// HBM, so the kernel reads the referenced columns once and writes the result
// once.
//
// Values are int64; +, -, * and unary minus wrap (two's complement); / and %
// truncate toward zero, a zero divisor gives 0 and sets
// TQP_DEVERR_VALUE_RANGE, INT64_MIN / -1 = INT64_MIN and INT64_MIN % -1 = 0;
// comparisons and logic give 0 or 1; SELECT(c, t, f) = c ? t : f.
#include "dev.hpp"
#include "host.hpp"

namespace tqp {
namespace {

constexpr int XP_MAX = 64;       // instructions
constexpr int XS_MAX = 16;       // stack depth
constexpr int XC_MAX = 8;        // columns a program reads
constexpr int XE_MAX_COLS = 64;  // columns a program may number
constexpr int XE_BLOCK = 128;
constexpr int XE_ROWS_FEW = 4;   // rows per thread when the program reads at most 4 columns

enum : int32_t {
    XO_COL = 0, XO_CONST, XO_ADD, XO_SUB, XO_MUL, XO_DIV, XO_MOD, XO_NEG,
    XO_LT, XO_LE, XO_GT, XO_GE, XO_EQ, XO_NE, XO_AND, XO_OR, XO_NOT, XO_SELECT, XO_COUNT
};

struct XProg {
    int32_t op[XP_MAX];
    int64_t arg[XP_MAX];
    const void* col[XC_MAX];
    const int32_t* idx[XC_MAX];  // null: column c is read at the row itself; else at idx[c][row]
    int32_t type[XC_MAX];
    int32_t n;
    uint32_t used;               // bit c: the program reads column c
};

__device__ __forceinline__ int64_t x_load(const XProg& p, int c, int64_t row) {
    const int64_t r = p.idx[c] ? (int64_t)p.idx[c][row] : row;
    switch (p.type[c]) {
        case TQP_I8: return static_cast<const int8_t*>(p.col[c])[r];
        case TQP_I32: return static_cast<const int32_t*>(p.col[c])[r];
        default: return static_cast<const int64_t*>(p.col[c])[r];
    }
}

// Every thread evaluates ROWS rows together, instruction by instruction:
// the top of each row's stack stays in a register, the values below it in
// LDS: level l of row slot q at st[l * ROWS * XE_BLOCK + q], as many levels
// as the program needs (its deepest stack less one).  NC (>= the columns the
// program reads) sizes the registers that hold the rows' column values, so
// programs over few columns evaluate more rows per thread.
template <int NC, int ROWS>
__global__ void __launch_bounds__(XE_BLOCK)
k_eval(XProg p, int64_t n_upper, const int64_t* d_n, int64_t* out, uint32_t* flags) {
    constexpr int XE_ROWS = ROWS;
    extern __shared__ int64_t xe_st[];
    int64_t n = n_upper;
    if (d_n) { const int64_t t = *d_n; n = t < n ? t : n; }
    const int tid = threadIdx.x;
    bool zdiv = false;
    const int64_t step = (int64_t)gridDim.x * XE_BLOCK * XE_ROWS;
    for (int64_t base = (int64_t)blockIdx.x * XE_BLOCK * XE_ROWS; base < n; base += step) {
        // the rows' referenced columns, loads issued together before the program runs
        int64_t cv[XE_ROWS][NC];
#pragma unroll
        for (int j = 0; j < XE_ROWS; ++j) {
            const int64_t row = base + (int64_t)j * XE_BLOCK + tid;
            const int64_t r = row < n ? row : n - 1;          // base < n, so n >= 1
#pragma unroll
            for (int c = 0; c < NC; ++c) cv[j][c] = (p.used >> c) & 1u ? x_load(p, c, r) : 0;
        }
        int64_t top[XE_ROWS];
#pragma unroll
        for (int j = 0; j < XE_ROWS; ++j) top[j] = 0;
        int sp = 0;                                   // values on the stack; the same in every thread
        for (int pc = 0; pc < p.n; ++pc) {
            const int32_t op = p.op[pc];
            const int64_t arg = p.arg[pc];
            if (op == XO_COL || op == XO_CONST) {
#pragma unroll
                for (int j = 0; j < XE_ROWS; ++j) {
                    if (sp > 0) xe_st[(sp - 1) * (XE_ROWS * XE_BLOCK) + j * XE_BLOCK + tid] = top[j];
                    int64_t v = arg;
                    if (op == XO_COL) {
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            if (c == arg) v = cv[j][c];
                    }
                    top[j] = v;
                }
                ++sp;
                continue;
            }
            if (op == XO_NEG || op == XO_NOT) {
#pragma unroll
                for (int j = 0; j < XE_ROWS; ++j)
                    top[j] = op == XO_NEG ? (int64_t)(0ull - (uint64_t)top[j]) : (int64_t)(top[j] == 0);
                continue;
            }
            if (op == XO_SELECT) {
#pragma unroll
                for (int j = 0; j < XE_ROWS; ++j) {
                    const int64_t c = xe_st[(sp - 3) * (XE_ROWS * XE_BLOCK) + j * XE_BLOCK + tid];
                    const int64_t t = xe_st[(sp - 2) * (XE_ROWS * XE_BLOCK) + j * XE_BLOCK + tid];
                    top[j] = c != 0 ? t : top[j];
                }
                sp -= 2;
                continue;
            }
            // binary operators: the operator is the same in every thread, so
            // the branch is taken once per instruction, outside the row loop
            auto binary = [&](auto f) {
#pragma unroll
                for (int j = 0; j < XE_ROWS; ++j)
                    top[j] = f(xe_st[(sp - 2) * (XE_ROWS * XE_BLOCK) + j * XE_BLOCK + tid], top[j]);
            };
            switch (op) {
                case XO_ADD: binary([](int64_t a, int64_t b) { return (int64_t)((uint64_t)a + (uint64_t)b); }); break;
                case XO_SUB: binary([](int64_t a, int64_t b) { return (int64_t)((uint64_t)a - (uint64_t)b); }); break;
                case XO_MUL: binary([](int64_t a, int64_t b) { return (int64_t)((uint64_t)a * (uint64_t)b); }); break;
                case XO_DIV:
                    binary([&](int64_t a, int64_t b) -> int64_t {
                        if (b == 0) { zdiv = true; return 0; }
                        if (b == -1) return (int64_t)(0ull - (uint64_t)a);
                        return a / b;
                    });
                    break;
                case XO_MOD:
                    binary([&](int64_t a, int64_t b) -> int64_t {
                        if (b == 0) { zdiv = true; return 0; }
                        if (b == -1) return 0;
                        return a % b;
                    });
                    break;
                case XO_LT: binary([](int64_t a, int64_t b) -> int64_t { return a < b; }); break;
                case XO_LE: binary([](int64_t a, int64_t b) -> int64_t { return a <= b; }); break;
                case XO_GT: binary([](int64_t a, int64_t b) -> int64_t { return a > b; }); break;
                case XO_GE: binary([](int64_t a, int64_t b) -> int64_t { return a >= b; }); break;
                case XO_EQ: binary([](int64_t a, int64_t b) -> int64_t { return a == b; }); break;
                case XO_NE: binary([](int64_t a, int64_t b) -> int64_t { return a != b; }); break;
                case XO_AND: binary([](int64_t a, int64_t b) -> int64_t { return (a != 0) && (b != 0); }); break;
                default: binary([](int64_t a, int64_t b) -> int64_t { return (a != 0) || (b != 0); }); break;
            }
            --sp;
        }
#pragma unroll
        for (int j = 0; j < XE_ROWS; ++j) {
            const int64_t row = base + (int64_t)j * XE_BLOCK + tid;
            if (row < n) out[row] = top[j];
        }
    }
    if (__any(zdiv) && lane_id() == 0) set_flag(flags, FLAG_VALUE_RANGE);
}

int x_arity(int32_t op) {
    if (op == XO_COL || op == XO_CONST) return 0;
    if (op == XO_NEG || op == XO_NOT) return 1;
    if (op == XO_SELECT) return 3;
    return 2;
}

}  // namespace

// The program checked on the host (operators, operand counts, column
// numbers, stack depth, one value left) and, when n > 0, evaluated for n (or
// *d_n) rows.  The program may number up to XE_MAX_COLS columns, of which it
// may read at most XC_MAX; columns read through idx[c] (when idx and idx[c]
// are not null) are read at idx[c][row].
tqp_status eval_program(tqp_ctx* ctx, const tqp_column* cols, const int32_t* const* idx, int ncols, int64_t n,
                        const int64_t* d_n, const tqp_xinstr* prog, int nprog, int64_t* out, hipStream_t stream,
                        const char* who, const char* label) {
    if (nprog < 1 || nprog > XP_MAX) return fail(TQP_ERR_UNSUPPORTED, "%s: 1 to %d instructions", who, XP_MAX);
    if (ncols < 0 || ncols > XE_MAX_COLS) return fail(TQP_ERR_UNSUPPORTED, "%s: %d columns", who, ncols);
    XProg p{};
    int slot[XE_MAX_COLS];
    for (int c = 0; c < ncols; ++c) slot[c] = -1;
    int used = 0;
    // the stack depth before every instruction is known here: check the program once
    int sp = 0, deepest = 1;
    for (int pc = 0; pc < nprog; ++pc) {
        const int32_t op = prog[pc].op;
        if (op < 0 || op >= XO_COUNT) return fail(TQP_ERR_INVALID, "%s: unknown operator %d at %d", who, op, pc);
        if (op == XO_COL && (prog[pc].arg < 0 || prog[pc].arg >= ncols))
            return fail(TQP_ERR_INVALID, "%s: column %lld out of range at %d", who, (long long)prog[pc].arg, pc);
        const int ar = x_arity(op);
        if (sp < ar) return fail(TQP_ERR_INVALID, "%s: operator %d at %d lacks operands", who, op, pc);
        sp = sp - ar + 1;
        if (sp > XS_MAX) return fail(TQP_ERR_UNSUPPORTED, "%s: stack deeper than %d", who, XS_MAX);
        deepest = sp > deepest ? sp : deepest;
        p.op[pc] = op;
        p.arg[pc] = prog[pc].arg;
        if (op == XO_COL) {
            // the columns the program reads get the kernel's column slots in order of first use
            const int c = (int)prog[pc].arg;
            if (slot[c] < 0) {
                if (used == XC_MAX) return fail(TQP_ERR_UNSUPPORTED, "%s: more than %d columns read", who, XC_MAX);
                const tqp_column& col = cols[c];
                if (col.type != TQP_I8 && col.type != TQP_I32 && col.type != TQP_I64)
                    return fail(TQP_ERR_INVALID, "%s: column %d has an unknown type", who, c);
                if (n > 0 && !col.data) return fail(TQP_ERR_INVALID, "%s: column %d is null", who, c);
                slot[c] = used;
                p.col[used] = col.data;
                p.type[used] = col.type;
                p.idx[used] = idx ? idx[c] : nullptr;
                p.used |= 1u << used;
                ++used;
            }
            p.arg[pc] = slot[c];
        }
    }
    if (sp != 1) return fail(TQP_ERR_INVALID, "%s: the program leaves %d values", who, sp);
    p.n = nprog;
    if (n == 0) return TQP_OK;
    auto launch = [&](auto kernel, int rows) -> tqp_status {
        const size_t lds = (size_t)(deepest > 1 ? deepest - 1 : 1) * rows * XE_BLOCK * sizeof(int64_t);
        TQP_LAUNCH(ctx, stream, label,
                   kernel<<<grid_for(n, (int64_t)XE_BLOCK * rows, (int64_t)ctx->num_cus * 16), XE_BLOCK, lds,
                            stream>>>(p, n, d_n, out, ctx->d_err));
        return TQP_OK;
    };
    // rows per thread: as many as the column registers allow
    if (used <= 2) return launch(k_eval<2, XE_ROWS_FEW>, XE_ROWS_FEW);
    if (used <= 4) return launch(k_eval<4, XE_ROWS_FEW>, XE_ROWS_FEW);
    return launch(k_eval<XC_MAX, 2>, 2);
}

}  // namespace tqp

using namespace tqp;

extern "C" {

tqp_status tqp_eval(tqp_ctx* ctx, const tqp_column* cols, int ncols, int64_t n, const int64_t* d_n,
                    const tqp_xinstr* prog, int nprog, int64_t* out, hipStream_t stream) {
    clear_error();
    if (!ctx || n < 0 || ncols < 0 || (ncols > 0 && !cols) || !prog || (n > 0 && !out))
        return fail(TQP_ERR_INVALID, "tqp_eval: null pointer or negative size");
    if (ncols > XC_MAX) return fail(TQP_ERR_UNSUPPORTED, "tqp_eval: at most %d columns", XC_MAX);
    if (n > MAX_ELEMS) return fail(TQP_ERR_UNSUPPORTED, "tqp_eval: n = %lld", (long long)n);
    for (int c = 0; c < ncols; ++c) {
        if (cols[c].type != TQP_I8 && cols[c].type != TQP_I32 && cols[c].type != TQP_I64)
            return fail(TQP_ERR_INVALID, "tqp_eval: column %d has an unknown type", c);
        if (n > 0 && !cols[c].data) return fail(TQP_ERR_INVALID, "tqp_eval: column %d is null", c);
    }
    return eval_program(ctx, cols, nullptr, ncols, n, d_n, prog, nprog, out, stream, "tqp_eval", "eval");
}

}  // extern "C"
