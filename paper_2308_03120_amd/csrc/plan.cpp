// Validation, exact rewrites and kernel choice for one coot_eval / coot_reduce
// call.  Host only: nothing here touches the device.
//
// Semantics (Bandicoot paper, arXiv:2308.03120): column-major operands
// (Section 2, Table 1); element-wise operators (Table 2) and functions
// (Table 7); reductions (Tables 5 and 6).  Rewrites follow the paper's idea of
// restructuring an expression into an equivalent, cheaper form while it is
// built (Section 7, e.g. trans(diagmat(X)) -> diagmat(X)); only rewrites that
// leave every rounded result unchanged are applied:
//   * trans is moved down to the operands (trans(a + b) = trans(a) + trans(b),
//     trans(f(a)) = f(trans(a)), trans(trans(a)) = a), so the generated kernel
//     reads an operand transposed instead of materialising a transpose;
//   * repeated operand reads and repeated identical subtrees are merged.
// No reassociation and no constant folding is done (both change rounding).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <sstream>
#include <unordered_map>
#include <mutex>
#include <tuple>

#include "internal.h"

namespace coot {

int itemsize(int dt)
{
    switch (dt) {
    case COOT_F32: return 4;
    case COOT_F64: return 8;
    case COOT_F16: return 2;
    case COOT_BF16: return 2;
    case COOT_U64: return 8;
    case COOT_I32: return 4;
    case COOT_U32: return 4;
    }
    return 0;
}

bool is_value_dtype(int dt)
{
    return dt == COOT_F32 || dt == COOT_F64 || dt == COOT_F16 || dt == COOT_BF16 || dt == COOT_I32 || dt == COOT_U32;
}

const char* dtype_name(int dt)
{
    switch (dt) {
    case COOT_F32: return "f32";
    case COOT_F64: return "f64";
    case COOT_F16: return "f16";
    case COOT_BF16: return "bf16";
    case COOT_U64: return "u64";
    case COOT_I32: return "i32";
    case COOT_U32: return "u32";
    }
    return "?";
}

static bool is_binary(int op) { return op_is_binary(op); }
static bool is_scalar(int op) { return op_is_scalar(op); }
static bool is_unary(int op) { return op_is_unary(op); }

uint64_t fnv1a(const std::string& s)
{
    uint64_t h = 1469598103934665603ull;
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

std::string hex64(uint64_t v)
{
    char b[17];
    snprintf(b, sizeof b, "%016llx", (unsigned long long)v);
    return b;
}

static std::string shape_str(int64_t r, int64_t c)
{
    std::ostringstream o;
    o << r << "x" << c;
    return o.str();
}

static bool contiguous(const coot_operand& o) { return o.n_cols <= 1 || o.ld == o.n_rows; }

static const uint32_t kGenFlags = COOT_OPERAND_GEN_FILL | COOT_OPERAND_GEN_EYE | COOT_OPERAND_GEN_LINSPACE;
static bool is_gen(const coot_operand& o) { return (o.flags & kGenFlags) != 0; }

// byte extent [lo, hi) of an operand's storage
static void extent(const coot_operand& o, int dt, uint64_t* lo, uint64_t* hi)
{
    uint64_t base = (uint64_t)(uintptr_t)o.ptr;
    int64_t n = o.n_rows * o.n_cols;
    if (n == 0) {
        *lo = *hi = base;
        return;
    }
    uint64_t last = (uint64_t)(o.ld * (o.n_cols - 1) + o.n_rows);
    *lo = base;
    *hi = base + last * (uint64_t)itemsize(dt);
}

static void check_operand(const coot_operand& o, const char* what, bool output)
{
    if (o.n_rows < 0 || o.n_cols < 0) fail(COOT_ERR_ARG, std::string(what) + ": negative dimension");
    if (o.n_rows > 0 && o.n_cols > (int64_t)(INT64_MAX / 16) / o.n_rows)
        fail(COOT_ERR_ARG, std::string(what) + ": too many elements");
    if (o.ld < 1 || o.ld < o.n_rows) fail(COOT_ERR_ARG, std::string(what) + ": ld must be >= max(1, n_rows)");
    if (o.n_cols > 1 && o.ld > (int64_t)(INT64_MAX / 16) / o.n_cols) fail(COOT_ERR_ARG, std::string(what) + ": ld too large");
    int64_t n = o.n_rows * o.n_cols;
    if (!output && is_gen(o)) {
        // a generator: no memory, exactly one kind
        const uint32_t g = o.flags & kGenFlags;
        if ((o.flags & ~kGenFlags) || (g & (g - 1)))
            fail(COOT_ERR_ARG, std::string(what) + ": one generator flag and no other flag");
        if (o.ptr != nullptr) fail(COOT_ERR_ARG, std::string(what) + ": a generator has no memory (ptr must be NULL)");
        if (g == COOT_OPERAND_GEN_LINSPACE && o.n_rows != 1 && o.n_cols != 1)
            fail(COOT_ERR_SHAPE, std::string(what) + ": linspace is a vector (n x 1 or 1 x n)");
        return;
    }
    if (n > 0 && o.ptr == nullptr) fail(COOT_ERR_ARG, std::string(what) + ": NULL pointer with elements");
    if (!output && o.flags != 0) fail(COOT_ERR_ARG, std::string(what) + ": flags must be 0 for an input");
    if (output && (o.flags & ~COOT_OPERAND_HOST)) fail(COOT_ERR_ARG, std::string(what) + ": unknown flags");
}

static void check_config(const coot_config& c)
{
    if (c.reserved != 0) fail(COOT_ERR_ARG, "cfg.reserved must be 0");
    bool zero = c.ept == 0 && c.block == 0 && c.split == 0;
    if (zero) return;
    auto pow2in = [](int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; };
    if (!pow2in(c.ept, 1, 8) || !pow2in(c.block, 64, 512) || !pow2in(c.split, 1, 8))
        fail(COOT_ERR_ARG, "cfg: ept in {1,2,4,8}, block in {64,...,512}, split in {1,2,4,8}, or all zero");
}

struct Info {
    int64_t rows, cols;
    int prec;
};

TileLds tile_lds_plan(const Plan& p)
{
    TileLds t;
    t.in_lds.assign(p.reads.size(), false);
    int budget = 96 * 1024;
    for (size_t j = 0; j < p.reads.size(); ++j) {
        if (!p.reads[j].trans) continue;
        const int bytes = COOT_TILE_LDS * (dtype_prec(p.reads[j].dtype) == 64 ? 8 : 4);
        if (bytes <= budget) {
            t.in_lds[j] = true;
            budget -= bytes;
            t.any_lds = true;
        }
    }
    return t;
}

int64_t tile_row_shift(const Plan& p, const coot_operand* ops, const coot_operand* out)
{
    int votes[64] = {0};
    auto vote = [&](const void* ptr, int64_t ld, int sz, int w) {
        if (!ptr || sz <= 0 || (ld * sz) % 128 != 0 || (uintptr_t)ptr % (uintptr_t)sz) return;
        votes[(int)(((uintptr_t)ptr % 128) / (uintptr_t)sz)] += w;  // < 64 elements of >= 2 bytes
    };
    for (const Read& r : p.reads)
        if (!r.trans) vote(ops[r.slot].ptr, r.ld, itemsize(r.dtype), 2);
    if (p.red_op < 0) vote(out->ptr, out->ld, itemsize(out->dtype), 1 << 20);
    int best = 0;
    for (int e = 1; e < 64; ++e)
        if (votes[e] > votes[best]) best = e;
    return best;
}

Plan make_plan(int red_op_in, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
               const coot_operand* out)
{
    if (!expr) fail(COOT_ERR_ARG, "expr is NULL");
    if (!expr->nodes) fail(COOT_ERR_ARG, "expr->nodes is NULL");
    const int nn = expr->n_nodes;
    if (nn < 1 || nn > 4096) fail(COOT_ERR_BAD_TREE, "n_nodes must be in [1, 4096]");
    if (n_ops < 0 || (n_ops > 0 && !ops)) fail(COOT_ERR_ARG, "operands: bad count or NULL array");
    if (expr->flags & ~COOT_EXPR_UNFUSED) fail(COOT_ERR_ARG, "unknown expr flags");
    check_config(expr->cfg);
    if (!out) fail(COOT_ERR_ARG, "out is NULL");

    Plan P;
    P.red_op = -1;
    P.dim = -1;
    P.pairwise = false;
    if (red_op_in >= 0) {
        if (red_op_in & ~(0xff | COOT_RED_PAIRWISE)) fail(COOT_ERR_ARG, "unknown reduction flags");
        P.red_op = red_op_in & 0xff;
        P.pairwise = (red_op_in & COOT_RED_PAIRWISE) != 0;
        if (P.red_op > COOT_RED_ANY) fail(COOT_ERR_ARG, "unknown reduction");
        if (dim < -1 || dim > 1) fail(COOT_ERR_ARG, "dim must be -1, 0 or 1");
        P.dim = dim;
        bool scalar_only = P.red_op == COOT_RED_ACCU || P.red_op == COOT_RED_DOT || P.red_op == COOT_RED_NORM1 ||
                           P.red_op == COOT_RED_NORM2 || P.red_op == COOT_RED_NORMINF || P.red_op == COOT_RED_NORMNEGINF;
        if (scalar_only && dim != -1) fail(COOT_ERR_ARG, "accu, dot and norm reduce over all elements (dim = -1)");
    } else if (red_op_in != -1) {
        fail(COOT_ERR_ARG, "red_op must be -1 for element-wise evaluation");
    }

    // --- structure, operands, shapes and precisions of the user's tree
    std::vector<Info> info(nn);
    std::vector<char> slot_checked(n_ops > 0 ? n_ops : 1, 0);
    for (int i = 0; i < nn; ++i) {
        const coot_node& N = expr->nodes[i];
        // message prefix, built only when a check fails
        auto at = [i]() { return "node " + std::to_string(i); };
        if (N.reserved != 0) fail(COOT_ERR_BAD_TREE, at() + ": reserved must be 0");
        if (N.op == COOT_LEAF) {
            if (N.a < 0 || N.a >= n_ops) fail(COOT_ERR_BAD_TREE, at() + ": operand slot out of range");
            const coot_operand& o = ops[N.a];
            if (!slot_checked[N.a]) {
                std::string w = "operand " + std::to_string(N.a);
                check_operand(o, w.c_str(), false);
                if (!is_value_dtype(o.dtype)) fail(COOT_ERR_DTYPE, w + ": dtype must be f32, f64, f16, bf16, i32 or u32");
                slot_checked[N.a] = 1;
            }
            info[i] = {o.n_rows, o.n_cols, dtype_prec(o.dtype)};
            continue;
        }
        bool bin = is_binary(N.op), sc = is_scalar(N.op), un = is_unary(N.op);
        if (!bin && !sc && !un && N.op != COOT_TRANS && N.op != COOT_CONV) fail(COOT_ERR_BAD_TREE, at() + ": unknown opcode");
        if (N.a < 0 || N.a >= i) fail(COOT_ERR_BAD_TREE, at() + ": child a must be an earlier node");
        Info A = info[N.a];
        if (bin) {
            if (N.b < 0 || N.b >= i) fail(COOT_ERR_BAD_TREE, at() + ": child b must be an earlier node");
            Info B = info[N.b];
            if (A.rows != B.rows || A.cols != B.cols)
                fail(COOT_ERR_SHAPE, at() + ": operand shapes " + shape_str(A.rows, A.cols) + " and " +
                                         shape_str(B.rows, B.cols) + " differ");
            if (A.prec != B.prec) fail(COOT_ERR_DTYPE, at() + ": mixed FP32/FP64 operands need an explicit conversion");
            info[i] = A;
        } else if (N.op == COOT_CONV) {
            if (!is_value_dtype(N.b)) fail(COOT_ERR_BAD_TREE, at() + ": conversion target must be a value dtype");
            info[i] = {A.rows, A.cols, dtype_prec(N.b)};
        } else {
            if (N.b != -1) fail(COOT_ERR_BAD_TREE, at() + ": b must be -1 for a unary or scalar node");
            if (N.op == COOT_TRANS)
                info[i] = {A.cols, A.rows, A.prec};
            else
                info[i] = A;
        }
    }
    const Info R = info[nn - 1];
    P.rows = R.rows;
    P.cols = R.cols;
    P.n = R.rows * R.cols;
    P.root_prec = R.prec;

    // --- output
    check_operand(*out, "out", true);
    if (P.red_op < 0) {
        if (out->flags & COOT_OPERAND_HOST) fail(COOT_ERR_ARG, "out: element-wise results must be device memory");
        if (!is_value_dtype(out->dtype)) fail(COOT_ERR_DTYPE, "out: dtype must be f32, f64, f16, bf16, i32 or u32");
        if (out->n_rows != P.rows || out->n_cols != P.cols)
            fail(COOT_ERR_SHAPE, "out is " + shape_str(out->n_rows, out->n_cols) + ", the expression is " +
                                     shape_str(P.rows, P.cols));
        P.out_dtype = out->dtype;
    } else {
        if (red_is_selection(P.red_op) && P.n == 0) fail(COOT_ERR_EMPTY, "min/max/index of an empty object");
        if (P.red_op == COOT_RED_DOT && expr->nodes[nn - 1].op != COOT_SCHUR)
            fail(COOT_ERR_BAD_TREE, "dot: the root must be an element-wise product of the two operands");
        int64_t n_out = P.dim < 0 ? 1 : (P.dim == 0 ? P.cols : P.rows);
        if (out->n_rows * out->n_cols != n_out || (out->n_rows != 1 && out->n_cols != 1))
            fail(COOT_ERR_SHAPE, "out must be a vector of " + std::to_string(n_out) + " elements");
        if (out->n_cols > 1 && out->ld != 1) fail(COOT_ERR_ARG, "out: a row vector result must have ld = 1");
        const bool u64 = red_has_u64_out(P.red_op);
        if (u64 && out->dtype != COOT_U64) fail(COOT_ERR_DTYPE, "out: index, count, all and any results are u64");
        if (!u64 && out->dtype != COOT_F32 && out->dtype != COOT_F64) fail(COOT_ERR_DTYPE, "out: values are f32 or f64");
        P.out_dtype = out->dtype;
    }

    // --- exact rewrites: trans pushed to the operands, reads and subtrees merged
    std::map<std::pair<int, bool>, int> read_of;
    std::map<std::tuple<int, int, int, uint64_t, int, uint64_t, int64_t>, int> cse;
    std::map<std::pair<int, bool>, int> memo;
    std::function<int(int, bool)> rebuild = [&](int i, bool t) -> int {
        auto mk = memo.find({i, t});
        if (mk != memo.end()) return mk->second;
        const coot_node& N = expr->nodes[i];
        int res;
        if (N.op == COOT_TRANS) {
            res = rebuild(N.a, !t);
        } else {
            PNode pn;
            pn.op = N.op;
            pn.a = pn.b = -1;
            pn.k = 0.0;
            pn.conv = -1;
            pn.prec = info[i].prec;
            pn.rows = t ? info[i].cols : info[i].rows;
            pn.cols = t ? info[i].rows : info[i].cols;
            if (N.op == COOT_LEAF && is_gen(ops[N.a])) {
                // values from the element's index; eye and fill are their own
                // transposes (shape swapped), a linspace vector has the same
                // linear order either way
                const coot_operand& o = ops[N.a];
                pn.op = PN_GEN;
                pn.a = (int)(o.flags & kGenFlags);
                pn.conv = o.dtype;
                pn.k = o.gen[0];
                pn.k2 = o.gen[1];
                pn.gn = o.n_rows * o.n_cols;
                if (pn.a != COOT_OPERAND_GEN_FILL) P.gen_index = true;
            } else if (N.op == COOT_LEAF) {
                const coot_operand& o = ops[N.a];
                bool tt = t;
                int64_t ld = o.ld;
                bool vec = o.n_rows == 1 || o.n_cols == 1;
                if (tt && vec && contiguous(o) && (o.n_rows == 1 ? o.ld == 1 : true)) {
                    // a contiguous vector has the same linear order either way
                    tt = false;
                    ld = pn.rows > 0 ? pn.rows : 1;
                }
                auto key = std::make_pair(N.a, tt);
                auto it = read_of.find(key);
                int r;
                if (it == read_of.end()) {
                    r = (int)P.reads.size();
                    P.reads.push_back({N.a, tt, o.dtype, ld});
                    read_of[key] = r;
                } else {
                    r = it->second;
                }
                pn.a = r;
            } else {
                pn.a = rebuild(N.a, t);
                if (is_binary(N.op)) pn.b = rebuild(N.b, t);
                if (N.op == COOT_CONV) pn.conv = N.b;
                if (is_scalar(N.op)) pn.k = pn.prec == 32 ? (double)(float)N.k : N.k;
            }
            uint64_t kb, kb2;
            std::memcpy(&kb, &pn.k, 8);
            std::memcpy(&kb2, &pn.k2, 8);
            auto key = std::make_tuple(pn.op, pn.a, pn.b, kb, pn.conv, kb2, pn.gn);
            auto it = cse.find(key);
            if (it != cse.end()) {
                res = it->second;
            } else {
                res = (int)P.nodes.size();
                P.nodes.push_back(pn);
                cse[key] = res;
            }
        }
        memo[{i, t}] = res;
        return res;
    };
    P.root = rebuild(nn - 1, false);
    if ((int)P.reads.size() > COOT_MAX_READS)
        fail(COOT_ERR_UNSUPPORTED, "more than " + std::to_string(COOT_MAX_READS) + " distinct operand reads");

    // --- aliasing of the output with the operands
    {
        uint64_t olo, ohi;
        extent(*out, out->dtype, &olo, &ohi);
        P.alias_out = false;
        if (!(out->flags & COOT_OPERAND_HOST) && ohi > olo) {
            for (int s = 0; s < n_ops; ++s) {
                if (!slot_checked[s] || is_gen(ops[s])) continue;
                const coot_operand& o = ops[s];
                uint64_t lo, hi;
                extent(o, o.dtype, &lo, &hi);
                if (hi <= lo || hi <= olo || ohi <= lo) continue;
                bool same = P.red_op < 0 && o.ptr == out->ptr && o.ld == out->ld && o.dtype == out->dtype &&
                            o.n_rows == out->n_rows && o.n_cols == out->n_cols;
                for (const Read& r : P.reads)
                    if (r.slot == s && r.trans) same = false;
                if (!same) fail(COOT_ERR_ALIAS, "out overlaps operand " + std::to_string(s));
                P.alias_out = true;
            }
        }
    }

    // --- kernel kind
    bool any_trans = false, all_contig = true;
    for (const Read& r : P.reads) {
        if (r.trans) any_trans = true;
        const coot_operand& o = ops[r.slot];
        if (!r.trans && !(o.n_cols <= 1 || r.ld == P.rows || P.cols <= 1)) all_contig = false;
    }
    if (P.red_op < 0 && !(P.cols <= 1 || out->ld == P.rows)) all_contig = false;
    // the flat kinds know only an element's linear index; eye needs its row
    // and column, which the tiled kinds have
    for (const PNode& n : P.nodes)
        if (n.op == PN_GEN && n.a == COOT_OPERAND_GEN_EYE && P.rows > 1 && P.cols > 1) all_contig = false;
    P.temp_needed = false;
    P.product_form = false;
    P.prod_a = P.prod_b = -1;
    if (P.red_op < 0) {
        P.kind = (any_trans || !all_contig) ? K_EW_TILED : K_EW_FLAT;
    } else if (P.dim < 0) {
        P.kind = (any_trans || !all_contig) ? K_RED_TILED : K_RED_FLAT;
    } else {
        if (any_trans) P.temp_needed = true;
        if (P.dim == 0)
            P.kind = P.rows >= 64 ? K_RED_COL : K_RED_COLT;
        else
            P.kind = K_RED_ROW;
    }
    // Thin values, and values with no transposed read (strided views, eye),
    // take the shape-adaptive tiles.  Without a transposed operand nothing
    // needs a square tile: tall tiles (up to 4096 rows of one column) walk
    // down each column, where 64 x 64 tiles touch 64 columns per wave
    P.tile_gen = (P.kind == K_EW_TILED || P.kind == K_RED_TILED) && (P.rows < 64 || P.cols < 64 || !any_trans);
    if (P.tile_gen) {
        if (any_trans) {
            coot_tile_shape(P.rows, P.cols, &P.tile_lr, &P.tile_lc);
        } else if (P.rows >= 64) {
            // tall tiles: 8 to 16 tile rows down each column (tiles of 64 to
            // 1024 rows), so that whole tiles dominate once the grid is
            // shifted and only the first and last tile rows are partial
            const int fl = 63 - __builtin_clzll((unsigned long long)P.rows);
            P.tile_lr = std::max(6, std::min(fl - 3, 10));
            P.tile_lc = std::min(coot_lg2ceil(P.cols), 12 - P.tile_lr);
        } else {
            P.tile_lr = coot_lg2ceil(P.rows);
            P.tile_lc = std::min(coot_lg2ceil(P.cols), 12 - P.tile_lr);
        }
        // per-lane offset bounds (elements of at most 8 bytes) of the tile
        // mappings: value order k = lines per step beyond the first, a
        // transposed read either order
        const int lr = P.tile_lr, lc = P.tile_lc;
        const int64_t ky = lr <= 6 ? (64 >> lr) : 0;
        const int64_t kt = std::max<int64_t>(lc <= 6 ? (64 >> lc) : 0, lr <= 6 ? (1 << lr) : 64);
        int64_t bound = P.red_op < 0 ? 64 + ky * out->ld : 64;
        for (const Read& r : P.reads) bound = std::max(bound, 64 + (r.trans ? kt : ky) * r.ld);
        P.tile_off32 = bound < (int64_t(1) << 29);
        // tall tiles: straight reads only, tile rows of at least 64; their
        // grid shifts like the 64 x 64 one.  Whole 4096-element tall tiles
        // move 4 consecutive rows per access when every operand's columns
        // start, less the shift, on 4-element boundaries
        P.tile_tall = !any_trans && lr >= 6;
        P.tile_sh = P.tile_tall ? (int)tile_row_shift(P, ops, out) : 0;
        P.tile_v4 = false;
        if (P.tile_tall && lr + lc == 12) {
            const int64_t sh = P.tile_sh;
            auto al = [&](const void* ptr, int64_t ld, int sz) {
                const uintptr_t u = (uintptr_t)ptr;
                return u % (uintptr_t)sz == 0 && ((int64_t)((u / sz) % 4) - sh) % 4 == 0 && (P.cols == 1 || ld % 4 == 0);
            };
            bool ok = true;
            for (const Read& r : P.reads) ok = ok && al(ops[r.slot].ptr, r.ld, itemsize(r.dtype));
            if (P.red_op < 0) ok = ok && al(out->ptr, out->ld, itemsize(out->dtype));
            P.tile_v4 = ok;
        }
    }
    // thin values: a short side of at most 16 elements take the thin kernel
    // (emit_thin), unless an operand cannot follow its layout.  An operand
    // is "packed" when the K elements of each long-side position are
    // contiguous and consecutive positions follow each other (ld == K: the
    // value's layout when the rows are short, a transposed read when the
    // columns are), "strided" when it holds one run along the long side per
    // short-side index (any ld).  An operand moves whole vectors when its base
    // and (strided) its ld are whole vectors, else element by element.
    P.thin_k = 0;
    if (P.tile_gen && P.rows >= 1 && P.cols >= 1 && std::min(P.rows, P.cols) <= 16) {
        const bool sr = P.rows <= P.cols;
        const int64_t K = sr ? P.rows : P.cols;
        int maxsz = 1;
        for (const Read& r : P.reads) maxsz = std::max(maxsz, itemsize(r.dtype));
        if (P.red_op < 0) maxsz = std::max(maxsz, itemsize(out->dtype));
        const int V = 16 / maxsz;
        bool ok = true;
        uint32_t vec = 0;
        auto place = [&](const void* ptr, int64_t ld, int sz, bool packed, uint32_t bit) {
            if (packed && ld != K) ok = false;
            if ((uintptr_t)ptr % (uintptr_t)(V * sz) == 0 && (packed || ld % V == 0)) vec |= bit;
        };
        // a straight read (and the output) follows the value's layout, packed
        // when the rows are the short side; a transposed read the other way
        for (size_t j = 0; j < P.reads.size(); ++j) {
            const Read& r = P.reads[j];
            place(ops[r.slot].ptr, r.ld, itemsize(r.dtype), r.trans ? !sr : sr, 1u << j);
        }
        if (P.red_op < 0) place(out->ptr, out->ld, itemsize(out->dtype), sr, 1u << 31);
        // register budget: groups in flight x K vectors x (reads + output)
        const int64_t ug = std::max<int64_t>(1, 8 / K);
        const int64_t nvec = (int64_t)P.reads.size() + (P.red_op < 0 ? 1 : 0);
        ok = ok && ug * K * nvec <= 40;
        if (ok) {
            P.thin_k = (int)K;
            P.thin_rows = sr;
            P.thin_v = V;
            P.thin_vec = vec;
        }
    }
    // 64 x 64 and tall tiles: the grid shift, and the reads whose column
    // segments start inside a 128-byte line once shifted (a straight read) or
    // at all (a read through trans(), whose segments run along its own
    // columns): each shares its first and last line with the neighbouring
    // steps, so those loads go through the caches (a nontemporal load
    // refetches the line).  A transposed read held in registers touches a
    // line per lane for every step: always through the caches.
    P.tile_cached = 0;
    if ((P.kind == K_EW_TILED || P.kind == K_RED_TILED) && !P.thin_k && (!P.tile_gen || P.tile_tall)) {
        if (!P.tile_gen) P.tile_sh = (int)tile_row_shift(P, ops, out);
        const TileLds lds = tile_lds_plan(P);
        for (size_t j = 0; j < P.reads.size(); ++j) {
            const Read& r = P.reads[j];
            const uintptr_t u = (uintptr_t)ops[r.slot].ptr;
            const int64_t sz = itemsize(r.dtype);
            bool on_lines = u % 128 == 0 && (r.ld * sz) % 128 == 0;
            if (!r.trans)
                on_lines = u % (uintptr_t)sz == 0 && (P.cols == 1 || (r.ld * sz) % 128 == 0) &&
                           ((int64_t)(u % 128) / sz - P.tile_sh) * sz % 128 == 0;
            else if (!lds.in_lds[j])
                on_lines = false;
            if (!on_lines) P.tile_cached |= 1u << j;
        }
    }
    if (P.red_op >= 0 && (P.red_op == COOT_RED_ACCU || P.red_op == COOT_RED_SUM || P.red_op == COOT_RED_DOT) &&
        P.nodes[P.root].op == COOT_SCHUR) {
        P.product_form = true;
        P.prod_a = P.nodes[P.root].a;
        P.prod_b = P.nodes[P.root].b;
    }

    // --- vector width of the flat and per-column kinds
    P.ve = 1;
    if (P.kind == K_EW_FLAT || P.kind == K_RED_FLAT || P.kind == K_RED_COL || P.kind == K_RED_ROW) {
        int maxsz = 1;
        for (const Read& r : P.reads) maxsz = std::max(maxsz, itemsize(r.dtype));
        if (P.red_op < 0) maxsz = std::max(maxsz, itemsize(out->dtype));
        int ve = 16 / maxsz;
        bool ok = true;
        for (const Read& r : P.reads) {
            uintptr_t p = (uintptr_t)ops[r.slot].ptr;
            if (p % (uintptr_t)(ve * itemsize(r.dtype))) ok = false;
            if ((P.kind == K_RED_COL || P.kind == K_RED_ROW) && (r.ld % ve)) ok = false;
        }
        if (P.red_op < 0 && ((uintptr_t)out->ptr % (uintptr_t)(ve * itemsize(out->dtype)))) ok = false;
        P.ve = ok ? ve : 1;
    }

    // --- canonical text of the element function (part of the kernel key)
    std::string sig;
    sig.reserve(32 + 48 * P.nodes.size());
    char buf[96];
    for (const Read& r : P.reads) {
        sig += 'r';
        sig += dtype_name(r.dtype);
        sig += r.trans ? "T;" : "S;";
    }
    for (const PNode& n : P.nodes) {
        uint64_t kb, kb2;
        std::memcpy(&kb, &n.k, 8);
        std::memcpy(&kb2, &n.k2, 8);
        if (n.op == PN_GEN)
            snprintf(buf, sizeof buf, "g%d,%d,%d,%016llx,%016llx,%lld;", n.a, n.prec, n.conv, (unsigned long long)kb,
                     (unsigned long long)kb2, (long long)n.gn);
        else
            snprintf(buf, sizeof buf, "%d,%d,%d,%d,%d,%016llx;", n.op, n.a, n.b, n.prec, n.conv, (unsigned long long)kb);
        sig += buf;
    }
    sig += "root" + std::to_string(P.root);
    P.body_sig = std::move(sig);
    return P;
}

// ------------------------------------------------------------- plan cache
// make_plan for the per-call entry points, memoised.  The key holds every
// input the plan depends on: the tree, the shapes, types, leading dimensions
// and flags of the operands and the output, each pointer's 16-byte alignment
// (vector width) and whether it is NULL, and each operand's relation to the
// output's storage (overlapping, same base) that decides aliasing.  A call
// that fails its checks is never cached.
namespace {
std::mutex g_pc_mu;
std::unordered_map<std::string, Plan> g_pc;
const size_t kPlanCacheMax = 4096;

template <class T>
void put(std::string& k, const T& v)
{
    k.append(reinterpret_cast<const char*>(&v), sizeof v);
}

// a descriptor whose extent can be computed without overflow
bool sane(const coot_operand& o)
{
    const int64_t lim = int64_t(1) << 40;
    return o.n_rows >= 0 && o.n_cols >= 0 && o.ld >= 1 && o.ld >= o.n_rows && o.n_rows <= lim && o.n_cols <= lim &&
           o.ld <= lim && (is_value_dtype(o.dtype) || o.dtype == COOT_U64);
}
}  // namespace

Plan make_plan_cached(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
                      const coot_operand* out)
{
    if (!expr || !expr->nodes || expr->n_nodes <= 0 || expr->n_nodes > 4096 || n_ops < 0 || n_ops > 4096 ||
        (n_ops > 0 && !ops) || !out)
        return make_plan(red_op, dim, expr, ops, n_ops, out);  // the full checks report the error
    std::string k;
    k.reserve(64 + (size_t)expr->n_nodes * sizeof(coot_node) + (size_t)(n_ops + 1) * 48);
    put(k, red_op);
    put(k, dim);
    put(k, expr->flags);
    put(k, expr->cfg);
    put(k, n_ops);
    put(k, expr->n_nodes);
    k.append(reinterpret_cast<const char*>(expr->nodes), (size_t)expr->n_nodes * sizeof(coot_node));
    const bool out_ok = sane(*out) && !(out->flags & COOT_OPERAND_HOST);
    uint64_t olo = 0, ohi = 0;
    if (out_ok) extent(*out, out->dtype, &olo, &ohi);
    auto desc = [&](const coot_operand& o, bool rel) {
        put(k, o.n_rows);
        put(k, o.n_cols);
        put(k, o.ld);
        put(k, o.dtype);
        put(k, o.flags);
        if (is_gen(o)) {
            put(k, o.gen[0]);
            put(k, o.gen[1]);
        }
        // the pointer's place in its 128-byte line: vector widths, the tiled
        // grid's shift and the load policy of tiled reads follow from it
        put(k, (uint8_t)((uintptr_t)o.ptr & 127));
        uint8_t a = o.ptr ? 0 : 0x80;
        if (rel && out_ok && ohi > olo && sane(o)) {
            uint64_t lo, hi;
            extent(o, o.dtype, &lo, &hi);
            if (!(hi <= lo || hi <= olo || ohi <= lo)) a |= 0x20;
            if (o.ptr == out->ptr) a |= 0x40;
        } else if (rel) {
            a |= 0x10;  // relation not computed: never equal to a computed one
        }
        put(k, a);
    };
    for (int s = 0; s < n_ops; ++s) desc(ops[s], true);
    desc(*out, false);
    {
        std::lock_guard<std::mutex> lk(g_pc_mu);
        auto it = g_pc.find(k);
        if (it != g_pc.end()) return it->second;
    }
    Plan p = make_plan(red_op, dim, expr, ops, n_ops, out);
    std::lock_guard<std::mutex> lk(g_pc_mu);
    if (g_pc.size() >= kPlanCacheMax) g_pc.clear();
    g_pc.emplace(std::move(k), p);
    return p;
}

// ----------------------------------------------------------- configurations
LaunchCfg config_of(int index)
{
    LaunchCfg c;
    c.ept = 1 << ((index >> 4) & 3);
    c.block = 64 << ((index >> 2) & 3);
    c.split = 1 << (index & 3);
    return c;
}

int config_index(const LaunchCfg& c)
{
    auto lg = [](int v) {
        int l = 0;
        while ((1 << l) < v) ++l;
        return l;
    };
    return lg(c.ept) * 16 + lg(c.block / 64) * 4 + lg(c.split);
}

// Defaults from streaming measurements on MI355X: element-wise kernels (reads
// plus a write) run best as one pass of 64-thread blocks with one vector per
// thread (2^28 FP32 z 519 -> 479 us, FP64 scale 762 -> 639 us against 256
// threads with 4 vectors; the same or better from 2^20 elements on);
// read-only reductions as a persistent grid of 512-thread blocks (2 per CU)
// with two buffers of 2 vectors per thread (over 45 flat reductions of
// 2^22..2^28 FP32/FP64/FP16 elements, accu, dot and index_max: 1.016x the
// per-call best on geometric mean, worst 1.065x; 8 vectors per buffer:
// 1.065x, worst 1.216x).
// Element-wise trees bound by arithmetic rather than HBM run best with more
// elements per thread: pow (either precision), and logarithms or
// trigonometric functions computed in FP64 (2^28 elements: FP32 pow(|x|, 2.5)
// 1000 -> 757 us, FP64 1530 -> 1492 us; FP64 log(|x| + 1) 980 -> 862 us,
// FP64 sin(x) % cos(y) 1215 -> 1150 us with 256 threads x 4 vectors; FP32
// log, sin and cos and every exp stay faster with one vector per thread).
// Only large values gain: over 102 such random trees of 2^10 to 2^26
// elements, 256 x 4 took 0.71-0.82x the time of 64 x 1 from 2^23 elements
// on and 0.99-1.29x below.
static bool alu_heavy(const Plan& p)
{
    if (p.rows * p.cols < (int64_t(1) << 23)) return false;
    for (const PNode& n : p.nodes) {
        if (n.op == COOT_SCAL_POW) return true;
        const bool lg = n.op == COOT_LOG || n.op == COOT_LOG2 || n.op == COOT_LOG10;
        const bool trig = n.op >= COOT_COS && n.op <= COOT_TANH;
        if (n.prec == 64 && (lg || trig)) return true;
    }
    return false;
}

LaunchCfg default_config(const Plan& p)
{
    LaunchCfg c;
    switch (p.kind) {
    case K_EW_FLAT: c = alu_heavy(p) ? LaunchCfg{4, 256, 8} : LaunchCfg{1, 64, 8}; break;
    case K_RED_FLAT: c = {2, 512, 1}; break;
    // per-column reductions: 64-thread blocks, 4 per CU per split unit
    // (40 column sums and index_max of 7 shapes x FP32/FP64/FP16: 1.054x the
    // per-call best on geometric mean against 1.090x for 256-thread blocks)
    case K_RED_COL: c = {2, 64, 4}; break;
    // tiled element-wise: shape-adaptive (thin) tiles run best as one pass
    // (split 8: 2 x 2^26 and 2^23 x 12 FP32 adds 12% faster than split 4),
    // 64 x 64 tiles as 2 blocks per CU when every operand has 4- or 8-byte
    // elements (16384^2 FP32 and 16384 x 8192 FP64 adds 2-3% faster), as one
    // pass when one has 2-byte elements (16384^2 BF16 add: 1914 us as 2
    // blocks per CU, 706 us as one pass; over 76 random 16-bit trees 1.27x
    // the per-tree best against 1.04x); tiled reductions as 8 blocks per CU
    case K_EW_TILED: {
        bool narrow = itemsize(p.out_dtype) < 4;
        for (const Read& r : p.reads) narrow = narrow || itemsize(r.dtype) < 4;
        c = p.tile_gen || narrow ? LaunchCfg{1, 256, 8} : LaunchCfg{1, 256, 1};
        break;
    }
    case K_RED_TILED: c = {1, 256, 4}; break;
    // per-row reductions: 64-thread blocks (799 random trees: 1.04x the
    // per-tree best on geometric mean against 1.11x for 256-thread blocks);
    // per-column reductions of short columns: 64-thread blocks, 2 per CU
    // (268 trees: 1.06x against 1.11x)
    case K_RED_ROW: c = {1, 64, 8}; break;
    case K_RED_COLT: c = {1, 64, 2}; break;
    default: c = {4, 256, 8}; break;
    }
    return c;
}

// Knobs a kernel kind does not use are fixed, so that configurations that
// differ only there share one compiled kernel.
LaunchCfg normalise_config(const Plan& p, LaunchCfg c)
{
    if (p.kind == K_EW_TILED || p.kind == K_RED_TILED) {
        c.block = 256;  // fixed 64x64 tile shape
        c.ept = 1;
    }
    if (p.kind == K_RED_COLT || p.kind == K_RED_ROW) c.ept = 1;
    return c;
}

}  // namespace coot
