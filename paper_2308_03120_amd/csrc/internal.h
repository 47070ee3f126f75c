// Host-side internals of libcoot_mi355x.so.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "coot.h"
#include "coot_kargs.h"

namespace coot {

struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg);
void set_error(int code, const std::string& msg);

int itemsize(int dtype);
bool is_value_dtype(int dtype);  // F32, F64, F16, BF16, I32, U32
// compute precision of a tree leaf stored as dtype: FP64 for F64 and the
// 32-bit integers (exact), FP32 for F32 and the 16-bit floats
inline int dtype_prec(int dt) { return (dt == COOT_F64 || dt == COOT_I32 || dt == COOT_U32) ? 64 : 32; }
const char* dtype_name(int dtype);

// ----------------------------------------------------------------- planning
enum Kind {
    K_EW_FLAT = 0,     // element-wise, contiguous operands, linear index
    K_EW_TILED = 1,    // element-wise, 64x64 tiles (transposed reads / ld views)
    K_RED_FLAT = 2,    // reduction over all elements, contiguous
    K_RED_TILED = 3,   // reduction over all elements, tiled
    K_RED_COL = 4,     // per-column reduction, one wave per column
    K_RED_COLT = 5,    // per-column reduction, one thread per column (short columns)
    K_RED_ROW = 6,     // per-row reduction, one thread per row, column splits
};

struct Read {
    int slot;
    bool trans;       // read element (r, c) of the value as operand (c, r)
    int dtype;
    int64_t ld;       // effective leading dimension
};

// A generator leaf (memory-free operand) in a plan: op = PN_GEN, a = the
// COOT_OPERAND_GEN_* flag, conv = its element type, k / k2 = its parameters
// (fill value; linspace start and end), gn = its element count.
constexpr int PN_GEN = 1000;

struct PNode {
    int op;           // COOT_* opcode (never COOT_TRANS after planning), or PN_GEN
    int a, b;         // children (plan node indices); LEAF: a = read index
    double k;         // scalar (already rounded to the node's precision)
    int prec;         // 32 or 64
    int conv;         // COOT_CONV target dtype
    int64_t rows, cols;
    double k2 = 0.0;  // PN_GEN: second parameter
    int64_t gn = 0;   // PN_GEN: element count
};

// node classes shared by the planner, the generator and the baselines
inline bool op_is_binary(int op) { return (op >= COOT_PLUS && op <= COOT_DIV) || (op >= COOT_GT && op <= COOT_NE); }
inline bool op_is_scalar(int op)
{
    return (op >= COOT_SCAL_PLUS && op <= COOT_SCAL_POW) || (op >= COOT_SCAL_GT && op <= COOT_SCAL_NE);
}
inline bool op_is_unary(int op)
{
    return op == COOT_EXP || op == COOT_LOG || op == COOT_SQRT || op == COOT_ABS || (op >= COOT_LOG10 && op <= COOT_SIGN) ||
           (op >= COOT_COS && op <= COOT_TANH);
}
// reductions whose result is a value index (u64): indices, counts, all, any
inline bool red_has_u64_out(int r)
{
    return r == COOT_RED_INDEX_MIN || r == COOT_RED_INDEX_MAX || r == COOT_RED_COUNT || r == COOT_RED_ALL ||
           r == COOT_RED_ANY;
}
// selections: no value on an empty input
inline bool red_is_selection(int r)
{
    return r == COOT_RED_MIN || r == COOT_RED_MAX || r == COOT_RED_INDEX_MIN || r == COOT_RED_INDEX_MAX ||
           r == COOT_RED_NORMINF || r == COOT_RED_NORMNEGINF;
}
// per-record bytes of a reduction partial
inline int red_partial_bytes(int r) { return (r == COOT_RED_VAR || r == COOT_RED_STDDEV) ? 32 : 16; }

struct Plan {
    std::vector<PNode> nodes;
    std::vector<Read> reads;
    int root;                 // index of the root node
    int root_prec;
    int64_t rows, cols, n;    // shape of the tree's value
    int red_op;               // -1 for element-wise
    int dim;
    bool pairwise;
    bool product_form;        // sum over a product root: kernel splits it (TwoProduct)
    int prod_a, prod_b;
    int kind;
    int ve;                   // elements per vector access (flat kinds)
    int out_dtype;
    bool alias_out;
    bool temp_needed;         // dim reduction of a tiled tree: materialise first
    bool tile_gen = false;    // tiled kind on a thin value: shape-adaptive tiles
    int tile_lr = 6, tile_lc = 6;  // tile shape 2^lr x 2^lc of the tiled kinds
    bool tile_off32 = false;  // per-lane tile offsets fit in 32-bit byte offsets
    // tall tiles: shape-adaptive tiles over straight reads only with tile rows
    // 2^lr >= 64; the grid starts tile_sh rows above the value (a launch
    // argument, so that the output's column segments begin on 128-byte lines)
    bool tile_tall = false;
    int tile_sh = 0;
    uint32_t tile_cached = 0; // tall tiles: bit j, read j's column segments do not start on lines
                              // once shifted, so neighbouring steps share lines: load through the caches
    bool tile_v4 = false;     // tall 4096-element tiles whose operands all start their columns (less
                              // tile_sh rows) on 4-element boundaries: 4 consecutive rows per access
    // thin tiled value whose short side K = thin_k <= 16 (0: not thin): each
    // thread takes groups of thin_v positions along the long side, all K
    // elements of each, every access a whole vector (see emit_thin)
    int thin_k = 0;
    bool thin_rows = false;   // the short side is the rows (R = K), else the columns
    int thin_v = 1;           // elements per vector access
    uint32_t thin_vec = 0;    // bit j: read j moves whole vectors (bit 31: the output); else element by element
    bool gen_index = false;   // a generator needs the element's index (eye, linspace)
    std::string body_sig;     // canonical description of the element function
};

// Which transposed reads of a tiled plan are staged through LDS tiles (in
// order, while 96 KB last); the others are held in registers.
struct TileLds {
    std::vector<bool> in_lds;
    bool any_lds = false;
};
TileLds tile_lds_plan(const Plan& p);

// Rows (0..63) by which a tiled grid starts above the value: the phase, in
// elements within a 128-byte line, shared by the output's columns (else by
// most straight reads), so that their column segments begin on lines.
int64_t tile_row_shift(const Plan& p, const coot_operand* ops, const coot_operand* out);

// Validate and plan.  Throws Error.
Plan make_plan(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
               const coot_operand* out);
// make_plan memoised on everything the plan depends on (per-call entry points)
Plan make_plan_cached(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
                      const coot_operand* out);

struct LaunchCfg {
    int ept, block, split;
};

// Kernel source for a plan and configuration; `name` receives the entry point.
std::string kernel_source(const Plan& p, const LaunchCfg& cfg, std::string* name, std::string* sig);
std::string prelude_source();
std::string batch_kernel_source(const Plan& py, const Plan* pr, bool has_out, int out_dtype, int red_dtype,
                                const std::vector<int>& read_slot, std::string* name_out);
// largest unit (elements) of a batched plan: its transposed reads fit the LDS stage
int64_t batch_unit_elems(const Plan& py);

// 64-entry configuration space
LaunchCfg config_of(int index);
int config_index(const LaunchCfg& c);
LaunchCfg default_config(const Plan& p);
LaunchCfg normalise_config(const Plan& p, LaunchCfg c);

// features of a plan (cost model input)
void plan_features(const Plan& p, float* f);

// hash
uint64_t fnv1a(const std::string& s);
std::string hex64(uint64_t v);

}  // namespace coot
