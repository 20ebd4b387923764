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
#include <type_traits>

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
// Word 3 of a raw buffer descriptor on gfx9-family chips: 32-bit data format,
// no swizzle, no stride; loads past the descriptor's byte range return 0.
constexpr int XE_RSRC_WORD3 = 0x00020000;
// Cache policy of the column loads: the non-temporal bit (each column byte is
// read once; with it, and non-temporal result stores, the 60M-row revenue
// program takes about 0.288 instead of 0.295 ms).
constexpr int XE_LOAD_NT = 2;
enum : int { XT_I8 = 1, XT_I32 = 2, XT_I64 = 4, XT_ALL = 7 };

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

// Every thread evaluates ROWS rows together, instruction by instruction:
// the top of each row's stack stays in a register, the values below it in
// LDS: level l of row slot q at st[l * ROWS * XE_BLOCK + q], as many levels
// as the program needs (its deepest stack less one).  NC (>= the columns the
// program reads) sizes the registers that hold the rows' column values, so
// programs over few columns evaluate more rows per thread.  GATHER: some
// column is read through a row id column.  TYPES (XT_* bits): the element
// types the direct columns may have; loads of the other types are left out.
template <int NC, int ROWS, bool GATHER, int TYPES = XT_ALL>
__global__ void __launch_bounds__(XE_BLOCK)
k_eval(XProg p, int64_t n_upper, const int64_t* d_n, void* out, int out_mode, uint32_t* flags) {
    constexpr int XE_ROWS = ROWS;
    extern __shared__ int64_t xe_st[];
    int64_t n = n_upper;
    if (d_n) { const int64_t t = *d_n; n = t < n ? t : n; }
    const int tid = threadIdx.x;
    bool zdiv = false;            // a zero divisor, or (XOUT_I32) a value outside int32: the value-range flag
    const int64_t step = (int64_t)gridDim.x * XE_BLOCK * XE_ROWS;
    for (int64_t base = (int64_t)blockIdx.x * XE_BLOCK * XE_ROWS; base < n; base += step) {
        int64_t cv[XE_ROWS][NC];
        if constexpr (!GATHER && (TYPES == XT_I64 || TYPES == XT_I32)) {
            // Direct columns of one element type: plain loads, rows past n
            // clamped to the last row; an unused slot reads slot 0's column
            // (always used here), so no branch separates the loads.
            using E = typename std::conditional<TYPES == XT_I64, int64_t, int32_t>::type;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const E* col = static_cast<const E*>(p.col[(p.used >> c) & 1u ? c : 0]);
#pragma unroll
                for (int j = 0; j < XE_ROWS; ++j) {
                    const int64_t row = base + (int64_t)j * XE_BLOCK + tid;
                    cv[j][c] = (int64_t)col[row < n ? row : n - 1];          // base < n, so n >= 1
                }
            }
        } else if constexpr (!GATHER) {
            // Direct columns: buffer loads over this tile's rows, one
            // descriptor per element type and column, whose range is zero
            // where the type is not the column's (or the column is unused):
            // a load out of its descriptor's range returns 0 without a memory
            // access, and rows at or past n are out of range too.  No branch
            // and no clamp: every load of the tile is in flight at once.
            const int64_t left = n - base;
            const uint32_t here = (uint32_t)(left < XE_ROWS * XE_BLOCK ? left : XE_ROWS * XE_BLOCK);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int t = p.type[c];
                const bool use = (p.used >> c) & 1u;
                const int w = t == TQP_I64 ? 8 : t == TQP_I32 ? 4 : 1;
                // (an unused slot's pointer may be null: its descriptors have no range)
                char* at = reinterpret_cast<char*>(reinterpret_cast<uintptr_t>(p.col[c]) + (uintptr_t)(base * w));
                const __amdgpu_buffer_rsrc_t r64 =
                    __builtin_amdgcn_make_buffer_rsrc(at, 0, use && w == 8 ? (int)(here * 8) : 0, XE_RSRC_WORD3);
                const __amdgpu_buffer_rsrc_t r32 =
                    __builtin_amdgcn_make_buffer_rsrc(at, 0, use && w == 4 ? (int)(here * 4) : 0, XE_RSRC_WORD3);
                const __amdgpu_buffer_rsrc_t r8 =
                    __builtin_amdgcn_make_buffer_rsrc(at, 0, use && w == 1 ? (int)here : 0, XE_RSRC_WORD3);
#pragma unroll
                for (int j = 0; j < XE_ROWS; ++j) {
                    const int off = j * XE_BLOCK + tid;
                    int64_t v = 0;
                    if constexpr ((TYPES & XT_I64) != 0) {
                        const auto v64 = __builtin_amdgcn_raw_buffer_load_b64(r64, off * 8, 0, XE_LOAD_NT);
                        v += (int64_t)(((uint64_t)v64[1] << 32) | v64[0]);
                    }
                    if constexpr ((TYPES & XT_I32) != 0)
                        v += (int64_t)(int32_t)__builtin_amdgcn_raw_buffer_load_b32(r32, off * 4, 0, XE_LOAD_NT);
                    if constexpr ((TYPES & XT_I8) != 0)
                        v += (int64_t)(int8_t)__builtin_amdgcn_raw_buffer_load_b8(r8, off, 0, XE_LOAD_NT);
                    cv[j][c] = v;
                }
            }
        } else {
            // Gathered columns: the row ids first (below 2^31, so 32 bits
            // hold them), then per column a branch on its type (the same in
            // every thread) that issues the tile's loads into registers of
            // that type; the values are formed after the loads.
            uint32_t rid[XE_ROWS][NC];
#pragma unroll
            for (int j = 0; j < XE_ROWS; ++j) {
                const int64_t row = base + (int64_t)j * XE_BLOCK + tid;
                const uint32_t r = (uint32_t)(row < n ? row : n - 1);     // base < n, so n >= 1
#pragma unroll
                for (int c = 0; c < NC; ++c) rid[j][c] = r;
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (((p.used >> c) & 1u) && p.idx[c]) {
#pragma unroll
                    for (int j = 0; j < XE_ROWS; ++j) rid[j][c] = (uint32_t)p.idx[c][rid[j][c]];
                }
            }
            uint64_t w64[XE_ROWS][NC];
            uint32_t w32[XE_ROWS][NC];
            int32_t w8[XE_ROWS][NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
#pragma unroll
                for (int j = 0; j < XE_ROWS; ++j) w64[j][c] = w32[j][c] = w8[j][c] = 0;
                if (!((p.used >> c) & 1u)) continue;
                const int t = p.type[c];
                if (t == TQP_I64) {
                    const uint64_t* col = static_cast<const uint64_t*>(p.col[c]);
#pragma unroll
                    for (int j = 0; j < XE_ROWS; ++j) w64[j][c] = col[rid[j][c]];
                } else if (t == TQP_I32) {
                    const uint32_t* col = static_cast<const uint32_t*>(p.col[c]);
#pragma unroll
                    for (int j = 0; j < XE_ROWS; ++j) w32[j][c] = col[rid[j][c]];
                } else {
                    const int8_t* col = static_cast<const int8_t*>(p.col[c]);
#pragma unroll
                    for (int j = 0; j < XE_ROWS; ++j) w8[j][c] = col[rid[j][c]];
                }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
#pragma unroll
                for (int j = 0; j < XE_ROWS; ++j)
                    cv[j][c] = (int64_t)w64[j][c] + (int64_t)(int32_t)w32[j][c] + (int64_t)w8[j][c];
            }
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
            // a zero divisor (the top of the stack) counts for rows below n only:
            // the rows past n in the last tile read zeros
            auto zero_divisors = [&] {
#pragma unroll
                for (int j = 0; j < XE_ROWS; ++j)
                    zdiv |= top[j] == 0 && base + (int64_t)j * XE_BLOCK + tid < n;
            };
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
                    zero_divisors();
                    binary([](int64_t a, int64_t b) -> int64_t {
                        if (b == 0) return 0;
                        if (b == -1) return (int64_t)(0ull - (uint64_t)a);
                        return a / b;
                    });
                    break;
                case XO_MOD:
                    zero_divisors();
                    binary([](int64_t a, int64_t b) -> int64_t {
                        if (b == 0) return 0;
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
            if (row < n) {
                if (out_mode == XOUT_FLAG) {
                    static_cast<uint8_t*>(out)[row] = top[j] != 0;
                } else if (out_mode == XOUT_I32) {
                    static_cast<int32_t*>(out)[row] = (int32_t)top[j];
                    zdiv |= top[j] != (int64_t)(int32_t)top[j];
                } else {
                    __builtin_nontemporal_store(top[j], &static_cast<int64_t*>(out)[row]);
                }
            }
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
                        const int64_t* d_n, const tqp_xinstr* prog, int nprog, void* out, hipStream_t stream,
                        const char* who, const char* label, int out_mode) {
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
                            stream>>>(p, n, d_n, out, out_mode, ctx->d_err));
        return TQP_OK;
    };
    // rows per thread: as many as the column registers allow
    bool gather = false;
    int types = 0;
    for (int c = 0; c < used; ++c) {
        gather |= p.idx[c] != nullptr;
        types |= p.type[c] == TQP_I64 ? XT_I64 : p.type[c] == TQP_I32 ? XT_I32 : XT_I8;
    }
    if (gather) {
        if (used <= 2) return launch(k_eval<2, XE_ROWS_FEW, true>, XE_ROWS_FEW);
        if (used <= 4) return launch(k_eval<4, XE_ROWS_FEW, true>, XE_ROWS_FEW);
        return launch(k_eval<XC_MAX, 2, true>, 2);
    }
    // columns of one element type (e.g. an int32 predicate, an int64 value
    // expression) load only that type
    if (used <= 2) {
        if (types == XT_I64) return launch(k_eval<2, XE_ROWS_FEW, false, XT_I64>, XE_ROWS_FEW);
        if (types == XT_I32) return launch(k_eval<2, XE_ROWS_FEW, false, XT_I32>, XE_ROWS_FEW);
        return launch(k_eval<2, XE_ROWS_FEW, false>, XE_ROWS_FEW);
    }
    if (used <= 4) {
        if (types == XT_I64) return launch(k_eval<4, XE_ROWS_FEW, false, XT_I64>, XE_ROWS_FEW);
        return launch(k_eval<4, XE_ROWS_FEW, false>, XE_ROWS_FEW);
    }
    return launch(k_eval<XC_MAX, 2, false>, 2);
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
