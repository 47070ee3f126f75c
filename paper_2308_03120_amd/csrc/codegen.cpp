// HIP source generation: one kernel per (tree signature, kind, configuration).
//
// The paper's library launches at least one kernel per node and keeps a
// temporary between nodes (Section 7: each op_type::apply calls one or more
// GPU kernels; generating code per expression is named as not yet possible).
// Here the whole tree becomes the body of a single kernel: every distinct
// operand is read once, the tree is evaluated in registers, and the result is
// either stored once or folded into a reduction accumulator.
#include <cmath>
#include <cstdio>
#include <functional>
#include <sstream>

#include "internal.h"

extern "C" const char* coot_prelude_text;

namespace coot {

std::string prelude_source() { return coot_prelude_text; }

static const char* ctype(int prec) { return prec == 64 ? "double" : "float"; }

static const char* stype(int dt)
{
    switch (dt) {
    case COOT_F32: return "float";
    case COOT_F64: return "double";
    case COOT_I32: return "int";
    case COOT_U32: return "unsigned";
    default: return "u16";
    }
}

static std::string widen(int dt, const std::string& e)
{
    if (dt == COOT_F16) return "widen_f16(" + e + ")";
    if (dt == COOT_BF16) return "widen_bf16(" + e + ")";
    if (dt == COOT_I32 || dt == COOT_U32) return "(double)(" + e + ")";
    return e;
}

// root value (compute precision prec) -> bits of the output storage type
static std::string narrow(int out_dt, int prec, const std::string& e)
{
    switch (out_dt) {
    case COOT_F32: return prec == 64 ? "(float)(" + e + ")" : e;
    case COOT_F64: return "(double)(" + e + ")";
    case COOT_F16: return (prec == 64 ? "bits_f16_d(" : "bits_f16(") + e + ")";
    case COOT_BF16: return (prec == 64 ? "bits_bf16_d(" : "bits_bf16(") + e + ")";
    case COOT_I32: return "sat_i32((double)(" + e + "))";
    case COOT_U32: return "sat_u32((double)(" + e + "))";
    }
    return e;
}

static std::string lit(double k, int prec)
{
    char b[64];
    if (prec == 32) {
        if (std::isnan(k)) return "__builtin_nanf(\"\")";
        if (std::isinf(k)) return k > 0 ? "__builtin_inff()" : "(-__builtin_inff())";
        snprintf(b, sizeof b, "(%af)", (double)(float)k);
    } else {
        if (std::isnan(k)) return "__builtin_nan(\"\")";
        if (std::isinf(k)) return k > 0 ? "__builtin_inf()" : "(-__builtin_inf())";
        snprintf(b, sizeof b, "(%a)", k);
    }
    return b;
}

// A generator's value at the element (gi_ linear index, gr_ row, gc_
// column): formed in FP64, stored in the generator's element type, widened to
// the node's precision.
static std::string gen_value(const PNode& n)
{
    std::string v;
    switch (n.a) {
    case COOT_OPERAND_GEN_FILL: v = lit(n.k, 64); break;
    case COOT_OPERAND_GEN_EYE: v = "(gr_ == gc_ ? 1.0 : 0.0)"; break;
    default: {
        // x_i = start + i*d for i < n - 1, end itself for the last element
        const double d = n.gn > 1 ? (n.k2 - n.k) / (double)(n.gn - 1) : 0.0;
        v = "(gi_ >= " + std::to_string(n.gn - 1) + " ? " + lit(n.k2, 64) + " : " + lit(n.k, 64) + " + (double)gi_ * " +
            lit(d, 64) + ")";
        break;
    }
    }
    switch (n.conv) {
    case COOT_F64: return v;
    case COOT_F32: return "(float)" + v;
    case COOT_F16: return "rnd_f16_d(" + v + ")";
    case COOT_I32: return "(double)sat_i32(" + v + ")";
    case COOT_U32: return "(double)sat_u32(" + v + ")";
    default: return "rnd_bf16_d(" + v + ")";
    }
}

// The element function: arguments are the widened values of the reads.
// pair = true emits x_pair(...) returning the two children of the root
// product instead of the product itself (exact TwoProduct in the reduction).
static std::string emit_eval(const Plan& p, bool pair, const std::string& pfx = "x")
{
    std::ostringstream s;
    std::ostringstream args;
    for (size_t j = 0; j < p.reads.size(); ++j) {
        if (j) args << ", ";
        args << ctype(dtype_prec(p.reads[j].dtype)) << " l" << j;
    }
    // generators that depend on the element take its linear index, row and column
    if (p.gen_index) args << (p.reads.empty() ? "" : ", ") << "const i64 gi_, const i64 gr_, const i64 gc_";
    const int rp = p.nodes[p.root].prec;
    if (pair)
        s << "CD void " << pfx << "_pair(" << args.str() << (args.str().empty() ? "" : ", ") << ctype(rp) << "& pa, "
          << ctype(rp) << "& pb)\n{\n";
    else
        s << "CD " << ctype(rp) << " " << pfx << "_eval(" << args.str() << ")\n{\n";
    for (size_t i = 0; i < p.nodes.size(); ++i) {
        const PNode& n = p.nodes[i];
        if (pair && (int)i == p.root) continue;
        const char* T = ctype(n.prec);
        const bool f = n.prec == 32;
        std::string a = n.a >= 0 ? "t" + std::to_string(n.a) : "";
        std::string b = n.b >= 0 ? "t" + std::to_string(n.b) : "";
        std::string k = lit(n.k, n.prec);
        // a relational node: 1 or 0 in the node's type
        auto rel = [&](const std::string& c) { return "((" + c + ") ? (" + std::string(T) + ")1 : (" + T + ")0)"; };
        std::string e;
        switch (n.op) {
        case PN_GEN: e = gen_value(n); break;
        case COOT_LEAF: e = "l" + std::to_string(n.a); break;
        case COOT_PLUS: e = a + " + " + b; break;
        case COOT_MINUS: e = a + " - " + b; break;
        case COOT_SCHUR: e = a + " * " + b; break;
        case COOT_DIV: e = a + " / " + b; break;
        case COOT_SCAL_PLUS: e = a + " + " + k; break;
        case COOT_SCAL_MINUS_POST: e = a + " - " + k; break;
        case COOT_SCAL_MINUS_PRE: e = k + " - " + a; break;
        case COOT_SCAL_TIMES: e = a + " * " + k; break;
        case COOT_SCAL_DIV_POST: e = a + " / " + k; break;
        case COOT_SCAL_DIV_PRE: e = k + " / " + a; break;
        case COOT_EXP: e = std::string(f ? "expf(" : "exp(") + a + ")"; break;
        case COOT_LOG: e = std::string(f ? "logf(" : "log(") + a + ")"; break;
        case COOT_SQRT: e = std::string(f ? "sqrtf(" : "sqrt(") + a + ")"; break;
        case COOT_ABS: e = std::string(f ? "__builtin_fabsf(" : "__builtin_fabs(") + a + ")"; break;
        case COOT_SCAL_POW: e = std::string(f ? "powf(" : "pow(") + a + ", " + k + ")"; break;
        case COOT_LOG10: e = std::string(f ? "log10f(" : "log10(") + a + ")"; break;
        case COOT_LOG2: e = std::string(f ? "log2f(" : "log2(") + a + ")"; break;
        case COOT_EXP2: e = std::string(f ? "exp2f(" : "exp2(") + a + ")"; break;
        case COOT_SQUARE: e = a + " * " + a; break;
        case COOT_FLOOR: e = std::string(f ? "floorf(" : "floor(") + a + ")"; break;
        case COOT_CEIL: e = std::string(f ? "ceilf(" : "ceil(") + a + ")"; break;
        case COOT_ROUND: e = std::string(f ? "roundf(" : "round(") + a + ")"; break;
        case COOT_TRUNC: e = std::string(f ? "truncf(" : "trunc(") + a + ")"; break;
        case COOT_SIGN:
            e = "(" + a + " > (" + T + ")0 ? (" + T + ")1 : (" + a + " < (" + T + ")0 ? (" + T + ")-1 : " + a + "))";
            break;
        case COOT_COS: e = std::string(f ? "cosf(" : "cos(") + a + ")"; break;
        case COOT_SIN: e = std::string(f ? "sinf(" : "sin(") + a + ")"; break;
        case COOT_TAN: e = std::string(f ? "tanf(" : "tan(") + a + ")"; break;
        case COOT_ACOS: e = std::string(f ? "acosf(" : "acos(") + a + ")"; break;
        case COOT_ASIN: e = std::string(f ? "asinf(" : "asin(") + a + ")"; break;
        case COOT_ATAN: e = std::string(f ? "atanf(" : "atan(") + a + ")"; break;
        case COOT_COSH: e = std::string(f ? "coshf(" : "cosh(") + a + ")"; break;
        case COOT_SINH: e = std::string(f ? "sinhf(" : "sinh(") + a + ")"; break;
        case COOT_TANH: e = std::string(f ? "tanhf(" : "tanh(") + a + ")"; break;
        case COOT_GT: e = rel(a + " > " + b); break;
        case COOT_LT: e = rel(a + " < " + b); break;
        case COOT_GE: e = rel(a + " >= " + b); break;
        case COOT_LE: e = rel(a + " <= " + b); break;
        case COOT_EQ: e = rel(a + " == " + b); break;
        case COOT_NE: e = rel(a + " != " + b); break;
        case COOT_SCAL_GT: e = rel(a + " > " + k); break;
        case COOT_SCAL_LT: e = rel(a + " < " + k); break;
        case COOT_SCAL_GE: e = rel(a + " >= " + k); break;
        case COOT_SCAL_LE: e = rel(a + " <= " + k); break;
        case COOT_SCAL_EQ: e = rel(a + " == " + k); break;
        case COOT_SCAL_NE: e = rel(a + " != " + k); break;
        case COOT_CONV: {
            const int cp = p.nodes[n.a].prec;
            switch (n.conv) {
            case COOT_F32: e = cp == 64 ? "(float)" + a : a; break;
            case COOT_F64: e = "(double)" + a; break;
            case COOT_F16: e = (cp == 64 ? "rnd_f16_d(" : "rnd_f16(") + a + ")"; break;
            case COOT_BF16: e = (cp == 64 ? "rnd_bf16_d(" : "rnd_bf16(") + a + ")"; break;
            case COOT_I32: e = "(double)sat_i32((double)" + a + ")"; break;
            case COOT_U32: e = "(double)sat_u32((double)" + a + ")"; break;
            }
            break;
        }
        }
        s << "    const " << T << " t" << i << " = " << e << ";\n";
    }
    if (pair)
        s << "    pa = t" << p.prod_a << ";\n    pb = t" << p.prod_b << ";\n}\n";
    else
        s << "    return t" << p.root << ";\n}\n";
    return s.str();
}

// --- reduction helpers ------------------------------------------------------
// Sum-like reductions share the compensated accumulators: sums and norms,
// the mean (a sum divided once at the end), and the predicate counts (count,
// all, any: a sum of 0/1 terms, exact).  The variance has its own
// accumulator; the rest are selections (value and index).
static bool red_is_sum(int r)
{
    return r == COOT_RED_ACCU || r == COOT_RED_SUM || r == COOT_RED_DOT || r == COOT_RED_NORM1 || r == COOT_RED_NORM2 ||
           r == COOT_RED_MEAN || r == COOT_RED_COUNT || r == COOT_RED_ALL || r == COOT_RED_ANY;
}

static bool red_is_var(int r) { return r == COOT_RED_VAR || r == COOT_RED_STDDEV; }

static bool red_is_max(int r) { return r == COOT_RED_MAX || r == COOT_RED_INDEX_MAX || r == COOT_RED_NORMINF; }

static std::string acc_type(const Plan& p)
{
    const int rp = p.nodes[p.root].prec;
    if (red_is_var(p.red_op)) return "AccV";
    if (red_is_sum(p.red_op)) {
        if (rp == 64) return "AccKD";
        return p.pairwise ? "AccPF" : "AccKF";
    }
    return std::string("AccI<") + ctype(rp) + (red_is_max(p.red_op) ? ", true>" : ", false>");
}

// number of elements behind one result (the mean's divisor, all's target)
static std::string red_len(const Plan& p)
{
    return p.dim < 0 ? "(double)a.n" : (p.dim == 0 ? "(double)a.rows" : "(double)a.cols");
}

static std::string accumulate_into(const Plan& p, const std::string& args, const std::string& gi);

// statement adding the tree's value at linear index `gi` to `acc`
static std::string accumulate(const Plan& p, const std::string& args, const std::string& gi,
                              const std::string& acc = "acc")
{
    std::string s = accumulate_into(p, args, gi);
    if (acc == "acc") return s;
    for (size_t pos; (pos = s.find("acc.")) != std::string::npos;) s.replace(pos, 4, acc + ".");
    return s;
}

static std::string accumulate_into(const Plan& p, const std::string& args, const std::string& gi)
{
    const int rp = p.nodes[p.root].prec;
    const std::string fab = rp == 64 ? "__builtin_fabs" : "__builtin_fabsf";
    const std::string C = ctype(rp);
    if (p.product_form)
        return "{ " + C + " pa, pb; x_pair(" + args + (args.empty() ? "" : ", ") + "pa, pb); acc.add_prod(pa, pb); }";
    switch (p.red_op) {
    case COOT_RED_ACCU:
    case COOT_RED_SUM:
    case COOT_RED_DOT:
    case COOT_RED_MEAN: return "acc.add(x_eval(" + args + "));";
    case COOT_RED_COUNT:
    case COOT_RED_ALL:
    case COOT_RED_ANY: return "acc.add(x_eval(" + args + ") != (" + C + ")0 ? (" + C + ")1 : (" + C + ")0);";
    case COOT_RED_VAR:
    case COOT_RED_STDDEV: return "acc.add((double)x_eval(" + args + "));";
    case COOT_RED_NORM1: return "acc.add(" + fab + "(x_eval(" + args + ")));";
    case COOT_RED_NORM2: return "{ const " + C + " t = x_eval(" + args + "); acc.add_prod(t, t); }";
    case COOT_RED_NORMINF:
    case COOT_RED_NORMNEGINF: return "acc.add(" + fab + "(x_eval(" + args + ")), " + gi + ");";
    default: return "acc.add(x_eval(" + args + "), " + gi + ");";
    }
}

// A compensated FP32 sum whose tree is one FP16 leaf (accu, sum, mean of the
// stored values) adds each half straight from its 32-bit storage word: the
// mixed-precision FMA w.half * 1 + s converts the half inside the add with one
// rounding, the value the add of the converted half gives, so both adds of the
// TwoSum take the half without a conversion instruction in front of them (with
// the conversion first these sums ran 4-5% slower than plain accumulation).
static bool f16_mix_sum(const Plan& p)
{
    return p.reads.size() == 1 && p.reads[0].dtype == COOT_F16 && !p.reads[0].trans &&
           p.nodes[p.root].op == COOT_LEAF && !p.product_form && !p.gen_index && acc_type(p) == "AccKF" &&
           p.ve % 2 == 0 && (p.red_op == COOT_RED_ACCU || p.red_op == COOT_RED_SUM || p.red_op == COOT_RED_MEAN);
}

// (each kernel source holds one copy: a module of many kernels wraps each in a
// namespace of its own)
static const char* const F16_MIX_SRC = R"(// w's low (HI = 0) or high (HI = 1) half as FP16, times 1, plus s: one rounding
template <int HI> CD float f16_add(u32 w, float s)
{
    float r;
    if (HI) asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w), "v"(s));
    else asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w), "v"(s));
    return r;
}
// AccKF::add of one half of w, the half read inside both adds
template <int HI> CD void acc_add_f16(AccKF& a, u32 w)
{
    const float t = f16_add<HI>(w, a.s);
    const float z = t - a.s;
    a.c += (a.s - (t - z)) + f16_add<HI>(w, -z);
    a.s = t;
}
)";

// element k (an unrolled index) of the FP16 vector `vec` added to `acc`
static std::string f16_mix_add(const std::string& vec, const std::string& acc)
{
    return "{ const u32 w = (u32)" + vec + "[k & ~1] | ((u32)" + vec + "[k | 1] << 16); if (k & 1) acc_add_f16<1>(" +
           acc + ", w); else acc_add_f16<0>(" + acc + ", w); }";
}

static std::string put_value(const Plan& p, const std::string& where, const std::string& v)
{
    return std::string(p.out_dtype == COOT_F64 ? "put_f64(" : "put_f32(") + "a.res, " + where + ", " + v + ");";
}

// statement writing result j from the combined FP64 sum v of a sum-like reduction
static std::string put_sum_result(const Plan& p, const std::string& j, const std::string& v)
{
    switch (p.red_op) {
    case COOT_RED_NORM2: return put_value(p, j, "__builtin_sqrt(" + v + ")");
    case COOT_RED_MEAN: return put_value(p, j, "(" + v + ") / " + red_len(p));
    case COOT_RED_COUNT: return "put_u64(a.res, " + j + ", (i64)(" + v + "));";
    case COOT_RED_ALL: return "put_u64(a.res, " + j + ", (" + v + ") == " + red_len(p) + " ? 1 : 0);";
    case COOT_RED_ANY: return "put_u64(a.res, " + j + ", (" + v + ") > 0.0 ? 1 : 0);";
    default: return put_value(p, j, v);
    }
}

// statement writing result j from a combined variance accumulator
static std::string put_var_result(const Plan& p, const std::string& j, const std::string& acc)
{
    return put_value(p, j, p.red_op == COOT_RED_STDDEV ? "__builtin_sqrt(" + acc + ".var())" : acc + ".var()");
}

// statements writing result `j` straight from a per-thread/wave accumulator
static std::string write_direct(const Plan& p, const std::string& j)
{
    if (red_is_var(p.red_op)) return put_var_result(p, j, "acc");
    if (red_is_sum(p.red_op)) return put_sum_result(p, j, "(acc.hi() + acc.lo())");
    if (p.red_op == COOT_RED_INDEX_MIN || p.red_op == COOT_RED_INDEX_MAX) return "put_u64(a.res, " + j + ", acc.i);";
    return put_value(p, j, "(acc.i < 0 ? __builtin_nan(\"\") : (double)acc.v)");
}

static std::string put_partial(const Plan& p, const std::string& slot)
{
    if (red_is_var(p.red_op)) return "put_var_partial((double*)a.part, " + slot + ", acc);";
    if (red_is_sum(p.red_op)) return "put_sum_partial((double*)a.part, " + slot + ", acc.hi(), acc.lo());";
    return "put_idx_partial((double*)a.part, " + slot + ", (double)acc.v, acc.i);";
}

// statements combining `count` partials (first, stride) and writing result j (thread 0)
static std::string combine_and_write(const Plan& p, const std::string& first, const std::string& count,
                                     const std::string& stride, const std::string& j)
{
    std::ostringstream s;
    if (red_is_var(p.red_op)) {
        s << "{ const AccV cv = combine_var((const double*)a.part, " << first << ", " << count << ", " << stride
          << "); if (threadIdx.x == 0) " << put_var_result(p, j, "cv") << " }";
    } else if (red_is_sum(p.red_op)) {
        s << "{ const double v = combine_sums((const double*)a.part, " << first << ", " << count << ", " << stride
          << "); if (threadIdx.x == 0) " << put_sum_result(p, j, "v") << " }";
    } else {
        s << "{ const AccI<double, " << (red_is_max(p.red_op) ? "true" : "false") << "> cr = combine_idx<"
          << (red_is_max(p.red_op) ? "true" : "false") << ">((const double*)a.part, " << first << ", " << count << ", "
          << stride << "); if (threadIdx.x == 0) { ";
        if (p.red_op == COOT_RED_INDEX_MIN || p.red_op == COOT_RED_INDEX_MAX)
            s << "put_u64(a.res, " << j << ", cr.i);";
        else
            s << put_value(p, j, "(cr.i < 0 ? __builtin_nan(\"\") : cr.v)");
        s << " } }";
    }
    return s.str();
}

// the same, done by the calling thread alone
static std::string combine_and_write_seq(const Plan& p, const std::string& first, const std::string& count,
                                         const std::string& stride, const std::string& j)
{
    std::ostringstream s;
    if (red_is_var(p.red_op)) {
        s << "{ const AccV cv = combine_var_seq((const double*)a.part, " << first << ", " << count << ", " << stride
          << "); " << put_var_result(p, j, "cv") << " }";
    } else if (red_is_sum(p.red_op)) {
        s << "{ const double v = combine_sums_seq((const double*)a.part, " << first << ", " << count << ", " << stride
          << "); " << put_sum_result(p, j, "v") << " }";
    } else {
        const char* mx = red_is_max(p.red_op) ? "true" : "false";
        s << "{ const AccI<double, " << mx << "> cr = combine_idx_seq<" << mx << ">((const double*)a.part, " << first
          << ", " << count << ", " << stride << "); ";
        if (p.red_op == COOT_RED_INDEX_MIN || p.red_op == COOT_RED_INDEX_MAX)
            s << "put_u64(a.res, " << j << ", cr.i);";
        else
            s << put_value(p, j, "(cr.i < 0 ? __builtin_nan(\"\") : cr.v)");
        s << " }";
    }
    return s.str();
}

// --- common declarations ----------------------------------------------------
static std::string decl_reads(const Plan& p, bool restrict_ok)
{
    std::ostringstream s;
    for (size_t j = 0; j < p.reads.size(); ++j) {
        const char* S = stype(p.reads[j].dtype);
        s << "    const " << S << "* " << (restrict_ok ? "__restrict__ " : "") << "L" << j << " = (const " << S
          << "*)a.leaf[" << j << "];\n";
        s << "    const i64 ld" << j << " = a.ld[" << j << "];\n";
    }
    return s.str();
}

// argument list from per-read expressions; idx = "linear index, row, column"
// of the element, passed when a generator needs them.  The flat kinds pass
// (linear, linear, 0): they run eye only on a vector, where row == column
// holds exactly at linear index 0.
template <class F>
static std::string arglist(const Plan& p, F f, const std::string& idx)
{
    std::string s;
    for (size_t j = 0; j < p.reads.size(); ++j) {
        if (j) s += ", ";
        s += widen(p.reads[j].dtype, f((int)j));
    }
    if (p.gen_index) s += (s.empty() ? "" : ", ") + idx;
    return s;
}

// --- flat kinds: linear index, VE-element vectors, grid-stride loop ----------
// Element-wise: EPT vectors per thread per step, loads first, then compute and
// store.  Reductions: a software pipeline of two register buffers, so the
// loads of the next step are in flight while the current step is folded into
// the compensated accumulators (two per thread, alternating by vector).
// A selection fed by a stream whose indices only grow needs no tie test
// against the earlier elements of that stream.
static std::string increasing(const Plan& p, std::string acc)
{
    if (acc_type(p).compare(0, 4, "AccI") != 0) return acc;
    for (size_t pos = 0; (pos = acc.find(".add(", pos)) != std::string::npos; pos += 9) acc.replace(pos, 5, ".add_inc(");
    return acc;
}

// Pass 2 of the flat and tiled reductions: one block adds the a.splits
// per-block partials of pass 1 in block order.  A kernel of its own rather
// than a last-arriving block of pass 1, whose device-scope release in every
// block writes back the L2 caches and costs tens of microseconds at the end
// of each call.
static std::string emit_partials_comb(const Plan& p, const std::string& name)
{
    std::ostringstream s;
    s << "extern \"C\" __global__ void __launch_bounds__(256) " << name << "_comb(const coot_kargs a)\n{\n    "
      << combine_and_write(p, "0", "a.splits", "1", "0") << "\n}\n";
    return s.str();
}

static std::string emit_flat(const Plan& p, const LaunchCfg& c, const std::string& name)
{
    const bool ew = p.kind == K_EW_FLAT;
    const int VE = p.ve, EPT = c.ept;
    const std::string OS = ew ? stype(p.out_dtype) : "";
    const int rp = p.nodes[p.root].prec;
    const bool mix = !ew && f16_mix_sum(p);
    std::ostringstream s;
    if (mix) s << F16_MIX_SRC;
    s << "extern \"C\" __global__ void __launch_bounds__(512) " << name << "(const coot_kargs a)\n{\n";
    s << decl_reads(p, !p.alias_out);
    if (ew) s << "    " << OS << "* " << (p.alias_out ? "" : "__restrict__ ") << "O = (" << OS << "*)a.out;\n";
    else s << "    " << acc_type(p) << " acc, acc2;\n    acc.init();\n    acc2.init();\n";
    s << "    const i64 nv = a.n / " << VE << ";\n";
    s << "    const i64 bs = blockDim.x;\n";
    s << "    const i64 step = (i64)gridDim.x * bs * " << EPT << ";\n";
    // guarded: every vector checks v < nv; unguarded: the caller knows the
    // whole step is in range (straight-line loads, so the compiler can wait
    // for exactly the loads a fold needs)
    auto load = [&](const std::string& buf, const std::string& b, bool guarded = true) {
        std::ostringstream o;
        o << "#pragma unroll\n        for (int e = 0; e < " << EPT << "; ++e) {\n";
        o << "            const i64 v = " << b << " + e * bs;\n            if (" << (guarded ? "v < nv" : "true") << ") {\n";
        for (size_t j = 0; j < p.reads.size(); ++j)
            o << "                ldv<" << stype(p.reads[j].dtype) << ", " << VE << ">(L" << j << ", v * " << VE << ", "
              << buf << j << "[e]);\n";
        o << "            }\n        }\n";
        return o.str();
    };
    auto decl = [&](const std::string& buf) {
        std::ostringstream o;
        for (size_t j = 0; j < p.reads.size(); ++j)
            o << "    " << stype(p.reads[j].dtype) << " " << buf << j << "[" << EPT << "][" << VE << "];\n";
        return o.str();
    };
    if (ew) {
        s << "    for (i64 base = (i64)blockIdx.x * bs * " << EPT << " + threadIdx.x; base < nv; base += step) {\n";
        s << decl("r");
        s << load("r", "base");
        s << "#pragma unroll\n        for (int e = 0; e < " << EPT << "; ++e) {\n";
        s << "            const i64 v = base + e * bs;\n            if (v < nv) {\n";
        std::string args = arglist(p, [](int j) { return "r" + std::to_string(j) + "[e][k]"; }, "v * " + std::to_string(VE) + " + k, v * " + std::to_string(VE) + " + k, 0");
        s << "                " << OS << " o[" << VE << "];\n";
        s << "#pragma unroll\n                for (int k = 0; k < " << VE << "; ++k) o[k] = "
          << narrow(p.out_dtype, rp, "x_eval(" + args + ")") << ";\n";
        s << "                stv<" << OS << ", " << VE << ">(O, v * " << VE << ", o);\n";
        s << "            }\n        }\n    }\n";
    } else {
        auto fold = [&](const std::string& buf, const std::string& b, bool guarded) {
            std::ostringstream o;
            std::string args = arglist(p, [&](int j) { return buf + std::to_string(j) + "[e][k]"; }, "gi, gi, 0");
            o << "#pragma unroll\n        for (int e = 0; e < " << EPT << "; ++e) {\n";
            o << "            const i64 v = " << b << " + e * bs;\n            if (" << (guarded ? "v < nv" : "true")
              << ") {\n";
            o << "#pragma unroll\n                for (int k = 0; k < " << VE << "; ++k) { const i64 gi = v * " << VE
              << " + k; (void)gi; if (e & 1) "
              << (mix ? f16_mix_add(buf + "0[e]", "acc2") : increasing(p, accumulate(p, args, "gi", "acc2"))) << " else "
              << (mix ? f16_mix_add(buf + "0[e]", "acc") : increasing(p, accumulate(p, args, "gi"))) << " }\n";
            o << "            }\n        }\n";
            return o.str();
        };
        s << decl("ra") << decl("rb");
        s << "    i64 base = (i64)blockIdx.x * bs * " << EPT << " + threadIdx.x;\n";
        s << "    {\n" << load("ra", "base") << "    }\n";
        // a step whose next step is whole in range is whole in range too
        auto stage = [&](const std::string& nxt, const std::string& cur, const std::string& b) {
            std::ostringstream o;
            o << "        if (" << b << " + " << (EPT - 1) << " * bs < nv) {\n";
            o << load(nxt, b, false) << fold(cur, "base", false);
            o << "        } else {\n";
            o << load(nxt, b, true) << fold(cur, "base", true);
            o << "        }\n";
            return o.str();
        };
        s << "    while (base < nv) {\n";
        s << "        const i64 nb = base + step;\n";
        s << stage("rb", "ra", "nb");
        s << "        base = nb;\n        if (base >= nv) break;\n";
        s << "        const i64 nb2 = base + step;\n";
        s << stage("ra", "rb", "nb2");
        s << "        base = nb2;\n    }\n";
        s << "    acc.merge(acc2);\n";
    }
    // tail elements that do not fill a vector
    std::string targs = arglist(p, [](int j) { return "ldnt(L" + std::to_string(j) + " + i)"; }, "i, i, 0");
    s << "    if (blockIdx.x == gridDim.x - 1)\n";
    s << "        for (i64 i = nv * " << VE << " + threadIdx.x; i < a.n; i += bs) ";
    if (ew) s << "stnt(O + i, (" << OS << ")(" << narrow(p.out_dtype, rp, "x_eval(" + targs + ")") << "));\n";
    else s << "{ " << accumulate(p, targs, "i") << " }\n";
    if (!ew) {
        s << "    __shared__ " << acc_type(p) << " lds_acc[8];\n";
        s << "    acc = block_reduce(acc, lds_acc);\n";
        s << "    if (threadIdx.x == 0) " << put_partial(p, "blockIdx.x") << "\n";
    }
    s << "}\n";
    if (!ew) s << emit_partials_comb(p, name);
    return s.str();
}

// --- tiled kinds: 64x64 tiles, transposed reads staged through LDS ----------
// A 256-thread block works on 64x64 tiles of the value; lane = row inside the
// tile, wave w takes columns w, w+4, ..., so every straight read and the
// output move 256-byte column segments.  A transposed read is loaded along
// its own columns (also 256-byte segments) into a padded 64x65 LDS tile and
// read back transposed (conflict-free both ways).  The tile loop is software
// pipelined: the operands of the next tile are loaded into registers while
// the current tile is computed.
typedef TileLds TilePlan;

static TilePlan tile_plan(const Plan& p) { return tile_lds_plan(p); }

static std::string tile_shared_decls(const Plan& p, const TilePlan& tp, const std::string& ind)
{
    std::ostringstream s;
    for (size_t j = 0; j < p.reads.size(); ++j)
        if (tp.in_lds[j])
            s << ind << "__shared__ " << ctype(dtype_prec(p.reads[j].dtype)) << " T" << j << "[COOT_TILE_LDS];\n";
    return s.str();
}

// A tile of 2^lr x 2^lc elements of the tree's value is handled in up to 64
// steps m = w + 4*kk (wave w, kk = 0..15) of 64 lanes.  Position
// p = 64*m + lane of the tile maps to (p mod TR, p / TR) for the value's
// layout ("Y order": straight reads, register-held transposed reads, the
// output) and to (p / TC, p mod TC) for an operand read transposed and staged
// through LDS ("A order": lanes run along the operand's own columns).  Either
// way a step touches 64 consecutive elements of a column (or whole short
// columns), so loads and stores coalesce.  The square 64 x 64 case has its
// own code: lane = row, step = column.  Register buffers: pt<j> for
// LDS-staged transposed reads, pr<j> (prefetch) and cr<j> (current) for the
// others.  Every address is a wave-uniform base plus a per-lane offset that
// is fixed for the tile; a lane outside the value reads the step's first
// element instead (same cache line, value unused).
static std::string tile_regs(const Plan& p, const TilePlan& tp, const std::string& ind)
{
    std::ostringstream s;
    for (size_t j = 0; j < p.reads.size(); ++j) {
        const std::string C = ctype(dtype_prec(p.reads[j].dtype));
        if (tp.in_lds[j]) s << ind << C << " pt" << j << "[16];\n";
        else s << ind << C << " pr" << j << "[16], cr" << j << "[16];\n";
    }
    return s.str();
}

// Names the prefetch reads through: the value's shape, its tile shape
// (log2), and the base and leading dimension of every read.
struct TileView {
    std::string R, Cn, lr, lc;
    std::function<std::string(size_t)> L, ld;
};

// --- square 64 x 64 tiles --------------------------------------------------
// shifted: the tile grid starts sh rows above the value (the per-call kernels)
static std::string tile_prefetch_sq(const Plan& p, const TilePlan& tp, const std::string& in, const std::string& ti,
                                    const std::string& tj, const TileView& v, const std::string& ldf0, bool shifted = false)
{
    std::ostringstream o;
    o << in << "{\n";
    o << in << "    const i64 pi0 = " << (shifted ? "((i64)(" + ti + ") << 6) - sh" : "(i64)(" + ti + ") << 6") << ", pj0 = (i64)("
      << tj << ") << 6;\n";
    if (shifted) o << in << "    const int plo = pi0 < 0 ? (int)-pi0 : 0;\n";
    o << in << "    const int pri = (int)(" << v.R << " - pi0 < 64 ? " << v.R << " - pi0 : 64);\n";
    o << in << "    const int prj = (int)(" << v.Cn << " - pj0 < 64 ? " << v.Cn << " - pj0 : 64);\n";
    if (shifted)
        o << in << "    const u32 lnr = lane >= plo && lane < pri ? (u32)lane : (u32)plo, lnc = lane < prj ? (u32)lane : 0u;\n";
    else
        o << in << "    const u32 lnr = lane < pri ? (u32)lane : 0u, lnc = lane < prj ? (u32)lane : 0u;\n";
    // A read whose value is converted on load (16-bit and integer storage)
    // loads unconditionally: a step outside the value reads the tile's first
    // valid step instead (a wave-uniform pointer select), and the value is
    // zeroed after the load.  With a branch around each such load the
    // compiler waited for it, to convert it, before issuing the next one
    // (16384^2 BF16 transposed add 706 -> 370 us, accu 792 -> 294 us).  FP32
    // and FP64 reads keep the branch, which costs them nothing (the
    // unconditional form measured 2-5% slower for them).
    for (size_t j = 0; j < p.reads.size(); ++j) {
        const std::string J = std::to_string(j), L = v.L(j), ld = v.ld(j), S = stype(p.reads[j].dtype);
        const bool conv = p.reads[j].dtype != COOT_F32 && p.reads[j].dtype != COOT_F64;
        if (tp.in_lds[j]) {
            o << in << "    const " << S << "* a" << J << " = " << L << " + (pj0 + (pi0 + w) * " << ld << ");\n";
            if (conv) o << in << "    const " << S << "* const z" << J << " = " << L << " + (pj0 + (pi0 + " << (shifted ? "plo" : "0")
              << ") * " << ld << ");\n";
            o << in << "    const i64 s" << J << " = 4 * " << ld << ";\n";
        } else if (p.reads[j].trans) {
            o << in << "    const " << S << "* a" << J << " = " << L << " + (pj0 + w + pi0 * " << ld << ");\n";
            if (conv) o << in << "    const " << S << "* const z" << J << " = " << L << " + (pj0 + pi0 * " << ld << ");\n";
            o << in << "    const i64 s" << J << " = 4;\n";
            o << in << "    const i64 lrs" << J << " = (i64)lnr * " << ld << ";\n";
        } else {
            o << in << "    const " << S << "* a" << J << " = " << L << " + (pi0 + (pj0 + w) * " << ld << ");\n";
            if (conv) o << in << "    const " << S << "* const z" << J << " = " << L << " + (pi0 + pj0 * " << ld << ");\n";
            o << in << "    const i64 s" << J << " = 4 * " << ld << ";\n";
        }
    }
    o << in << "#pragma unroll\n" << in << "    for (int kk = 0; kk < 16; ++kk) {\n";
    o << in << "        const int q = w + 4 * kk;\n";
    for (size_t j = 0; j < p.reads.size(); ++j) {
        const std::string J = std::to_string(j), C = ctype(dtype_prec(p.reads[j].dtype)), S = stype(p.reads[j].dtype);
        const std::string ldf = (p.tile_cached >> j) & 1u ? "ldpl" : ldf0;
        std::string ok, lane_off, dst;
        if (tp.in_lds[j]) {
            ok = std::string(shifted ? "q >= plo && " : "") + "q < pri";
            lane_off = "lnc";
            dst = "pt";
        } else {
            ok = "q < prj";
            lane_off = p.reads[j].trans ? "lrs" + J : "lnr";
            dst = "pr";
        }
        const int dt = p.reads[j].dtype;
        if (dt == COOT_F32 || dt == COOT_F64) {
            o << in << "        " << dst << J << "[kk] = " << ok << " ? " << ldf << "(a" << J << " + " << lane_off << ") : (" << C << ")0;\n";
        } else {
            o << in << "        { const bool ok = " << ok << ";\n";
            o << in << "          const " << S << " raw = " << ldf << "((ok ? a" << J << " : z" << J << ") + " << lane_off << ");\n";
            o << in << "          " << dst << J << "[kk] = ok ? " << widen(dt, "raw") << " : (" << C << ")0; }\n";
        }
        o << in << "        a" << J << " += s" << J << ";\n";
    }
    o << in << "    }\n" << in << "}\n";
    return o.str();
}

static std::string tile_stage_sq(const Plan& p, const TilePlan& tp, const std::string& in)
{
    std::ostringstream s;
    if (tp.any_lds) {
        s << in << "__syncthreads();\n";
        s << in << "#pragma unroll\n" << in << "for (int kk = 0; kk < 16; ++kk) {\n";
        for (size_t j = 0; j < p.reads.size(); ++j)
            if (tp.in_lds[j]) s << in << "    T" << j << "[(w + 4 * kk) * 65 + lane] = pt" << j << "[kk];\n";
        s << in << "}\n";
    }
    for (size_t j = 0; j < p.reads.size(); ++j)
        if (!tp.in_lds[j])
            s << in << "#pragma unroll\n" << in << "for (int kk = 0; kk < 16; ++kk) cr" << j << "[kk] = pr" << j << "[kk];\n";
    if (tp.any_lds) s << in << "__syncthreads();\n";
    return s.str();
}

// per_elem(args, indent, addr): run for every element of the tile inside the
// value; in scope: i0, j0 (tile origin), ig, jg (the element's row and
// column); addr is the element's address in the output when out is given (an
// OT* with leading dimension ldo).
template <class F>
static std::string tile_compute_sq(const Plan& p, const TilePlan& tp, const std::string& in, const std::string& ti,
                                   const std::string& tj, const std::string& R, const std::string& Cn,
                                   const std::string& out, const std::string& OT, const std::string& ldo, F per_elem,
                                   bool shifted = false)
{
    std::ostringstream s;
    s << in << "{\n";
    s << in << "    const i64 i0 = " << (shifted ? "((i64)(" + ti + ") << 6) - sh" : "(i64)(" + ti + ") << 6") << ", j0 = (i64)("
      << tj << ") << 6;\n";
    if (shifted) s << in << "    const int lo = i0 < 0 ? (int)-i0 : 0;\n";
    s << in << "    const int ri = (int)(" << R << " - i0 < 64 ? " << R << " - i0 : 64);\n";
    s << in << "    const int rj = (int)(" << Cn << " - j0 < 64 ? " << Cn << " - j0 : 64);\n";
    if (!out.empty()) s << in << "    " << OT << "* po = " << out << " + (i0 + (j0 + w) * " << ldo << ");\n";
    s << in << "    if (" << (shifted ? "lane >= lo && " : "") << "lane < ri) {\n";
    s << in << "        const i64 ig = i0 + lane;\n";
    s << in << "#pragma unroll\n" << in << "        for (int kk = 0; kk < 16; ++kk) {\n";
    s << in << "            const int jj = w + 4 * kk;\n";
    s << in << "            if (jj < rj) {\n";
    s << in << "                const i64 jg = j0 + jj;\n";
    std::string args;
    for (size_t j = 0; j < p.reads.size(); ++j) {
        if (j) args += ", ";
        args += tp.in_lds[j] ? "T" + std::to_string(j) + "[lane * 65 + jj]" : "cr" + std::to_string(j) + "[kk]";
    }
    if (p.gen_index) args += (args.empty() ? "" : ", ") + ("ig + jg * " + R + ", ig, jg");
    s << per_elem(args, in + "                ", "po + lane");
    s << in << "            }\n";
    if (!out.empty()) s << in << "            po += 4 * " << ldo << ";\n";
    s << in << "        }\n" << in << "    }\n" << in << "}\n";
    return s.str();
}

// --- shape-adaptive tiles ---------------------------------------------------
// Steps m = w + 4*kk (kk = 0..15, m < steps of the tile).  Two orders walk the
// tile: Y order (rows along lanes: the value's layout; straight reads,
// register-held transposed reads, the output) and A order (columns along
// lanes: an operand read transposed and staged through LDS).  For an order
// whose lane dimension is at most 64 long, a step covers 64/T whole lines;
// otherwise a step covers 64 elements of one line, and the step four later
// lies 256 elements further down, carrying into the next lines.  Walkers
// keep the step origin (row, column) and one running pointer per read,
// advanced by scalar arithmetic.  With off32 the per-lane part of an address
// is a 32-bit byte offset (the host checks that it fits), so loads take a
// scalar base.
static std::string tile_lanes(const std::string& in, const std::string& lr, const std::string& lc, const std::string& rr,
                              const std::string& cc)
{
    std::ostringstream o;
    o << in << "const int yi = " << lr << " <= 6 ? (lane & ((1 << " << lr << ") - 1)) : lane;\n";
    o << in << "const int yj = " << lr << " <= 6 ? (lane >> " << lr << ") : 0;\n";
    o << in << "const int aj = " << lc << " <= 6 ? (lane & ((1 << " << lc << ") - 1)) : lane;\n";
    o << in << "const int ai = " << lc << " <= 6 ? (lane >> " << lc << ") : 0;\n";
    o << in << "const int nst = " << lr << " + " << lc << " >= 6 ? 1 << (" << lr << " + " << lc << " - 6) : 1;\n";
    o << in << "const bool lin = lane < (1 << (" << lr << " + " << lc << "));\n";
    o << in << "const bool yok = lin && (" << lr << " > 6 || yi < " << rr << ");\n";
    o << in << "const bool aok = lin && (" << lc << " > 6 || aj < " << cc << ");\n";
    o << in << "int ysr = " << lr << " <= 6 ? 0 : (w & ((1 << (" << lr << " - 6)) - 1)) << 6;\n";
    o << in << "int ysc = " << lr << " <= 6 ? w << (6 - " << lr << ") : w >> (" << lr << " - 6);\n";
    o << in << "int asc = " << lc << " <= 6 ? 0 : (w & ((1 << (" << lc << " - 6)) - 1)) << 6;\n";
    o << in << "int asr = " << lc << " <= 6 ? w << (6 - " << lc << ") : w >> (" << lc << " - 6);\n";
    return o.str();
}

// Advance the Y walker by four steps.  ptrs: running pointers with their
// leading dimension and whether they are read transposed.
static std::string walk_y(const std::string& in, const std::string& lr,
                          const std::vector<std::pair<std::string, std::pair<std::string, bool>>>& ptrs)
{
    std::ostringstream o;
    o << in << "if (" << lr << " <= 6) {\n";
    o << in << "    ysc += 256 >> " << lr << ";\n";
    for (auto& p : ptrs)
        o << in << "    " << p.first << " += "
          << (p.second.second ? "(i64)(256 >> " + lr + ")" : "(i64)(256 >> " + lr + ") * " + p.second.first) << ";\n";
    o << in << "} else {\n";
    o << in << "    const int cy = (ysr + 256) >> " << lr << ";\n";
    o << in << "    ysr = (ysr + 256) & ((1 << " << lr << ") - 1);\n";
    o << in << "    ysc += cy;\n";
    for (auto& p : ptrs)
        o << in << "    " << p.first << " += "
          << (p.second.second ? "(i64)cy + (i64)(256 - (cy << " + lr + ")) * " + p.second.first
                              : "(i64)(256 - (cy << " + lr + ")) + (i64)cy * " + p.second.first)
          << ";\n";
    o << in << "}\n";
    return o.str();
}

static std::string walk_a(const std::string& in, const std::string& lc,
                          const std::vector<std::pair<std::string, std::string>>& ptrs)
{
    std::ostringstream o;
    o << in << "if (" << lc << " <= 6) {\n";
    o << in << "    asr += 256 >> " << lc << ";\n";
    for (auto& p : ptrs) o << in << "    " << p.first << " += (i64)(256 >> " << lc << ") * " << p.second << ";\n";
    o << in << "} else {\n";
    o << in << "    const int ca = (asc + 256) >> " << lc << ";\n";
    o << in << "    asc = (asc + 256) & ((1 << " << lc << ") - 1);\n";
    o << in << "    asr += ca;\n";
    for (auto& p : ptrs)
        o << in << "    " << p.first << " += (i64)(256 - (ca << " << lc << ")) + (i64)ca * " << p.second << ";\n";
    o << in << "}\n";
    return o.str();
}

// address of a running pointer plus its per-lane offset (zero when invalid)
static std::string lane_addr(const std::string& ptr, const std::string& cond, const std::string& off, bool off32)
{
    if (off32) return "at(" + ptr + ", " + cond + " ? " + off + " : 0u)";
    return ptr + " + (" + cond + " ? " + off + " : 0)";
}

// --- tall tiles ---------------------------------------------------------
// Trees with straight reads only (views, index generators) and tile rows
// 2^lr >= 64 (p.tile_tall).  The grid starts sh = a.aux rows above the value
// (0 <= sh < 64, chosen on the host so the output's column segments begin on
// 128-byte lines); tile (ti, tj) covers rows (ti << lr) - sh + [0, 2^lr) and
// columns (tj << lc) + [0, 2^lc).  Step m = w + 4*kk of a wave covers tile
// elements 64*m + [0, 64) in column order: with 64*w split off, the step's
// row and column offsets are constants of kk (no walker).  A tile wholly
// inside the value has no per-step tests; a partial one clamps each lane's
// row and the step's column into the value for its loads (so every load is
// unconditional) and tests them before it stores or accumulates.
static std::string tall_origin(const std::string& in, const Plan& p, const std::string& ti, const std::string& tj,
                               const std::string& rn, const std::string& cn)
{
    return in + "const i64 " + rn + " = ((i64)(" + ti + ") << " + std::to_string(p.tile_lr) + ") - sh, " + cn + " = (i64)(" +
           tj + ") << " + std::to_string(p.tile_lc) + ";\n";
}

static std::string gen_wave_origin(const std::string& in, int lr)
{
    const int mask = (1 << lr) - 1;
    return in + "const int wr = (64 * w) & " + std::to_string(mask) + ", wc = (64 * w) >> " + std::to_string(lr) + ";\n";
}

// step kk's row and column offsets from the wave origin (compile-time)
static std::string gen_rc(int lr) { return "((256 * kk) & " + std::to_string((1 << lr) - 1) + ")"; }
static std::string gen_cc(int lr) { return "((256 * kk) >> " + std::to_string(lr) + ")"; }

// the steps guard when the tile holds fewer than 64 steps
static std::string gen_step_guard(const Plan& p)
{
    const int nst = 1 << std::max(0, p.tile_lr + p.tile_lc - 6);
    return nst >= 64 ? "" : "if (w + 4 * kk < " + std::to_string(nst) + ") ";
}

// guarded: a partial tile (rows clamped into [lo, hi) of the tile, the step's
// column to the value's last)
static std::string tall_prefetch(const Plan& p, const std::string& in, const std::string& ti, const std::string& tj,
                                 const TileView& v, bool guarded)
{
    std::ostringstream o;
    const int lr = p.tile_lr;
    const std::string i2 = in + "    ", i3 = i2 + "    ";
    o << in << (guarded ? "{ // partial tall tile\n" : "{ // whole tall tile: steps at fixed offsets\n");
    o << tall_origin(i2, p, ti, tj, "pi0", "pj0");
    o << gen_wave_origin(i2, lr);
    if (guarded) {
        o << i2 << "const int plo = pi0 < 0 ? (int)-pi0 : 0, phi = (int)(R - pi0 < (1 << " << lr << ") ? R - pi0 : (1 << " << lr
          << "));\n";
        o << i2 << "const i64 pcl = Cn - 1 - pj0;\n";
    }
    for (size_t j = 0; j < p.reads.size(); ++j) {
        const std::string J = std::to_string(j), S = stype(p.reads[j].dtype);
        o << i2 << "const " << S << "* a" << J << " = " << v.L(j) << " + (pi0 + pj0 * " << v.ld(j) << ");\n";
    }
    o << in << "#pragma unroll\n" << i2 << "for (int kk = 0; kk < 16; ++kk) " << gen_step_guard(p) << "{\n";
    if (guarded) {
        o << i3 << "const int t = wr + " << gen_rc(lr) << " + lane;\n";
        o << i3 << "const u32 tcl = (u32)(t < plo ? plo : (t >= phi ? phi - 1 : t));\n";
        o << i3 << "const i64 jl = wc + " << gen_cc(lr) << " < pcl ? wc + " << gen_cc(lr) << " : pcl;\n";
    } else {
        o << i3 << "const u32 tcl = (u32)(wr + " << gen_rc(lr) << " + lane);\n";
        o << i3 << "const i64 jl = wc + " << gen_cc(lr) << ";\n";
    }
    for (size_t j = 0; j < p.reads.size(); ++j) {
        const std::string J = std::to_string(j), ldf = (p.tile_cached >> j) & 1u ? "ldpl" : "ldnt";
        o << i3 << "pr" << J << "[kk] = " << widen(p.reads[j].dtype, ldf + "(at(a" + J + " + jl * " + v.ld(j) + ", tcl))") << ";\n";
    }
    o << i2 << "}\n" << in << "}\n";
    return o.str();
}

template <class F>
static std::string tall_compute(const Plan& p, const std::string& in, const std::string& ti, const std::string& tj,
                                bool ew, const std::string& ldo, F per_elem, bool guarded)
{
    std::ostringstream s;
    const int lr = p.tile_lr;
    const std::string i2 = in + "    ", i3 = i2 + "    ";
    s << in << "{\n";
    s << tall_origin(i2, p, ti, tj, "i0", "j0");
    s << gen_wave_origin(i2, lr);
    if (guarded) {
        s << i2 << "const int lo = i0 < 0 ? (int)-i0 : 0, hi = (int)(R - i0 < (1 << " << lr << ") ? R - i0 : (1 << " << lr << "));\n";
        s << i2 << "const i64 ccn = Cn - j0;\n";
    }
    if (ew) s << i2 << stype(p.out_dtype) << "* po = O + (i0 + j0 * " << ldo << ");\n";
    s << in << "#pragma unroll\n" << i2 << "for (int kk = 0; kk < 16; ++kk) " << gen_step_guard(p) << "{\n";
    s << i3 << "const int t = wr + " << gen_rc(lr) << " + lane;\n";
    s << i3 << "const i64 jl = wc + " << gen_cc(lr) << ";\n";
    std::string in4 = i3;
    if (guarded) {
        s << i3 << "if (jl < ccn && t >= lo && t < hi) {\n";
        in4 = i3 + "    ";
    }
    s << in4 << "const i64 ig = i0 + t, jg = j0 + jl;\n";
    std::string args;
    for (size_t j = 0; j < p.reads.size(); ++j) args += (j ? ", cr" : "cr") + std::to_string(j) + "[kk]";
    if (p.gen_index) args += (args.empty() ? "" : ", ") + std::string("ig + jg * R, ig, jg");
    s << per_elem(args, in4, ew ? "atw(po + jl * " + ldo + ", (u32)t)" : "");
    if (guarded) s << i3 << "}\n";
    s << i2 << "}\n" << in << "}\n";
    return s.str();
}

// A whole tile with every operand's columns on 4-element boundaries
// (p.tile_v4, 4096-element tiles): a lane moves 4 consecutive rows per
// access, the wave 256 rows; its elements are 256*w + 4*lane + 1024*q
// (q = 0..3) of the tile in column order, element 4*q + e of the lane's
// registers being row e of access q.
static std::string gen_v4_lane(const std::string& in, int lr)
{
    return in + "const int el = 256 * w + 4 * lane;\n" + in + "const i64 er = el & " + std::to_string((1 << lr) - 1) +
           ", ec = el >> " + std::to_string(lr) + ";\n";
}
static std::string gen_rq(int lr) { return "((1024 * q) & " + std::to_string((1 << lr) - 1) + ")"; }
static std::string gen_cq(int lr) { return "((1024 * q) >> " + std::to_string(lr) + ")"; }

static std::string tall_prefetch_v4(const Plan& p, const std::string& in, const std::string& ti, const std::string& tj,
                                    const TileView& v)
{
    std::ostringstream o;
    const int lr = p.tile_lr;
    const std::string i2 = in + "    ";
    o << in << "{ // whole tall tile: 4 rows per access\n";
    o << tall_origin(i2, p, ti, tj, "pi0", "pj0");
    o << gen_v4_lane(i2, lr);
    for (size_t j = 0; j < p.reads.size(); ++j) {
        const std::string J = std::to_string(j), S = stype(p.reads[j].dtype);
        o << i2 << "const " << S << "* a" << J << " = " << v.L(j) << " + (pi0 + pj0 * " << v.ld(j) << ");\n";
        o << i2 << "const i64 v" << J << " = er + ec * " << v.ld(j) << ";\n";
    }
    o << in << "#pragma unroll\n" << i2 << "for (int q = 0; q < 4; ++q) {\n";
    for (size_t j = 0; j < p.reads.size(); ++j) {
        const std::string J = std::to_string(j), S = stype(p.reads[j].dtype);
        o << i2 << "    { " << S << " t[4]; ldv<" << S << ", 4>(a" << J << " + (" << gen_rq(lr) << " + (i64)" << gen_cq(lr) << " * "
          << v.ld(j) << "), v" << J << ", t);\n";
        o << i2 << "#pragma unroll\n" << i2 << "      for (int e = 0; e < 4; ++e) pr" << J << "[4 * q + e] = "
          << widen(p.reads[j].dtype, "t[e]") << "; }\n";
    }
    o << i2 << "}\n" << in << "}\n";
    return o.str();
}

static std::string tall_compute_v4(const Plan& p, const std::string& in, const std::string& ti, const std::string& tj, bool ew,
                                   const std::string& ldo)
{
    std::ostringstream s;
    const int lr = p.tile_lr, rp = p.nodes[p.root].prec;
    const std::string i2 = in + "    ", i3 = i2 + "    ";
    const std::string OS = stype(p.out_dtype);
    s << in << "{\n";
    s << tall_origin(i2, p, ti, tj, "i0", "j0");
    s << gen_v4_lane(i2, lr);
    if (ew) s << i2 << OS << "* po = O + (i0 + j0 * " << ldo << ");\n" << i2 << "const i64 vo = er + ec * " << ldo << ";\n";
    s << in << "#pragma unroll\n" << i2 << "for (int q = 0; q < 4; ++q) {\n";
    s << i3 << "const i64 ib = i0 + er + " << gen_rq(lr) << ", jg = j0 + ec + " << gen_cq(lr) << ";\n";
    if (ew) s << i3 << OS << " o[4];\n";
    s << "#pragma unroll\n" << i3 << "for (int e = 0; e < 4; ++e) {\n";
    s << i3 << "    const i64 ig = ib + e;\n";
    std::string args;
    for (size_t j = 0; j < p.reads.size(); ++j) args += (j ? ", cr" : "cr") + std::to_string(j) + "[4 * q + e]";
    if (p.gen_index) args += (args.empty() ? "" : ", ") + std::string("ig + jg * R, ig, jg");
    if (ew)
        s << i3 << "    o[e] = (" << OS << ")(" << narrow(p.out_dtype, rp, "x_eval(" + args + ")") << ");\n";
    else
        s << i3 << "    " << accumulate(p, args, "(ig + jg * R)") << "\n";
    s << i3 << "}\n";
    if (ew) s << i3 << "stv<" << OS << ", 4>(po + (" << gen_rq(lr) << " + (i64)" << gen_cq(lr) << " * " << ldo << "), vo, o);\n";
    s << i2 << "}\n" << in << "}\n";
    return s.str();
}

static std::string tile_prefetch_gen(const Plan& p, const TilePlan& tp, const std::string& in, const std::string& ti,
                                     const std::string& tj, const TileView& v, const std::string& ldf, bool off32)
{
    std::ostringstream o;
    o << in << "{\n";
    const std::string i2 = in + "    ";
    const std::string OT = off32 ? "const u32 " : "const i64 ";
    const std::string cast = off32 ? "(u32)" : "(i64)";
    o << i2 << "const i64 pi0 = (i64)(" << ti << ") << " << v.lr << ", pj0 = (i64)(" << tj << ") << " << v.lc << ";\n";
    o << i2 << "const int prr = (int)(" << v.R << " - pi0 < (1 << " << v.lr << ") ? " << v.R << " - pi0 : (1 << " << v.lr
      << "));\n";
    o << i2 << "const int pcc = (int)(" << v.Cn << " - pj0 < (1 << " << v.lc << ") ? " << v.Cn << " - pj0 : (1 << " << v.lc
      << "));\n";
    o << tile_lanes(i2, v.lr, v.lc, "prr", "pcc");
    std::vector<std::pair<std::string, std::pair<std::string, bool>>> yp;
    std::vector<std::pair<std::string, std::string>> ap;
    for (size_t j = 0; j < p.reads.size(); ++j) {
        const std::string J = std::to_string(j), L = v.L(j), ld = v.ld(j), S = stype(p.reads[j].dtype);
        // converted reads load unconditionally (see tile_prefetch_sq): a
        // step outside the value reads the tile's first element
        if (p.reads[j].dtype != COOT_F32 && p.reads[j].dtype != COOT_F64)
            o << i2 << "const " << S << "* const z" << J << " = " << L << " + "
              << (tp.in_lds[j] || p.reads[j].trans ? "(pj0 + pi0 * " : "(pi0 + pj0 * ") << ld << ");\n";
        if (tp.in_lds[j]) {
            o << i2 << "const " << S << "* a" << J << " = " << L << " + ((pj0 + asc) + (pi0 + asr) * " << ld << ");\n";
            o << i2 << OT << "v" << J << " = " << cast << "(aj + (i64)ai * " << ld << ");\n";
            ap.push_back({"a" + J, ld});
        } else if (p.reads[j].trans) {
            o << i2 << "const " << S << "* a" << J << " = " << L << " + ((pj0 + ysc) + (pi0 + ysr) * " << ld << ");\n";
            o << i2 << OT << "v" << J << " = " << cast << "(yj + (i64)yi * " << ld << ");\n";
            yp.push_back({"a" + J, {ld, true}});
        } else {
            o << i2 << "const " << S << "* a" << J << " = " << L << " + ((pi0 + ysr) + (pj0 + ysc) * " << ld << ");\n";
            o << i2 << OT << "v" << J << " = " << cast << "(yi + (i64)yj * " << ld << ");\n";
            yp.push_back({"a" + J, {ld, false}});
        }
    }
    o << in << "#pragma unroll\n" << i2 << "for (int kk = 0; kk < 16; ++kk) {\n";
    const std::string i3 = i2 + "    ";
    // (a tile of 4096 elements has a step for every kk of every wave)
    o << i3 << (p.tile_lr + p.tile_lc >= 12 ? "{\n" : "if (w + 4 * kk < nst) {\n");
    const std::string i4 = i3 + "    ";
    if (!yp.empty()) {
        o << i4 << "const bool yu = ysr < prr && ysc < pcc;\n";
        o << i4 << "const bool yv = yok && (" << v.lr << " <= 6 ? yj < pcc - ysc : yi < prr - ysr);\n";
    }
    if (!ap.empty()) {
        o << i4 << "const bool au = asr < prr && asc < pcc;\n";
        o << i4 << "const bool av = aok && (" << v.lc << " <= 6 ? ai < prr - asr : aj < pcc - asc);\n";
    }
    for (size_t j = 0; j < p.reads.size(); ++j) {
        const std::string J = std::to_string(j), C = ctype(dtype_prec(p.reads[j].dtype)), S = stype(p.reads[j].dtype);
        const std::string u = tp.in_lds[j] ? "au" : "yu", lv = tp.in_lds[j] ? "av" : "yv", dst = tp.in_lds[j] ? "pt" : "pr";
        if (p.reads[j].dtype == COOT_F32 || p.reads[j].dtype == COOT_F64)
            o << i4 << dst << J << "[kk] = " << u << " ? " << ldf + "(" + lane_addr("a" + J, lv, "v" + J, off32) + ")"
              << " : (" << C << ")0;\n";
        else
            o << i4 << "{ const " << S << " raw = " << ldf << "("
              << lane_addr("(" + u + " ? a" + J + " : z" + J + ")", "(" + u + " && " + lv + ")", "v" + J, off32) << "); " << dst << J
              << "[kk] = " << u << " ? " << widen(p.reads[j].dtype, "raw") << " : (" << C << ")0; }\n";
    }
    if (!yp.empty()) o << walk_y(i4, v.lr, yp);
    if (!ap.empty()) o << walk_a(i4, v.lc, ap);
    o << i3 << "}\n" << i2 << "}\n" << in << "}\n";
    return o.str();
}

static std::string tile_stage_gen(const Plan& p, const TilePlan& tp, const std::string& in, const std::string& R,
                                  const std::string& Cn, const std::string& ti, const std::string& tj, const std::string& lr,
                                  const std::string& lc)
{
    std::ostringstream s;
    if (tp.any_lds) {
        s << in << "__syncthreads();\n";
        s << in << "{\n";
        const std::string i2 = in + "    ";
        s << i2 << "const int prr = (int)(" << R << " - ((i64)(" << ti << ") << " << lr << ") < (1 << " << lr << ") ? " << R
          << " - ((i64)(" << ti << ") << " << lr << ") : (1 << " << lr << "));\n";
        s << i2 << "const int pcc = (int)(" << Cn << " - ((i64)(" << tj << ") << " << lc << ") < (1 << " << lc << ") ? " << Cn
          << " - ((i64)(" << tj << ") << " << lc << ") : (1 << " << lc << "));\n";
        s << tile_lanes(i2, lr, lc, "prr", "pcc");
        s << i2 << "const int sst = coot_tile_stride(" << lr << ", " << lc << ");\n";
        s << in << "#pragma unroll\n" << i2 << "for (int kk = 0; kk < 16; ++kk) {\n";
        s << i2 << "    if (w + 4 * kk < nst) {\n";
        s << i2 << "        if (lin) {\n";
        for (size_t j = 0; j < p.reads.size(); ++j)
            if (tp.in_lds[j]) s << i2 << "            T" << j << "[(asr + ai) * sst + asc + aj] = pt" << j << "[kk];\n";
        s << i2 << "        }\n";
        s << walk_a(i2 + "        ", lc, {});
        s << i2 << "    }\n" << i2 << "}\n" << in << "}\n";
    }
    for (size_t j = 0; j < p.reads.size(); ++j)
        if (!tp.in_lds[j])
            s << in << "#pragma unroll\n" << in << "for (int kk = 0; kk < 16; ++kk) cr" << j << "[kk] = pr" << j << "[kk];\n";
    if (tp.any_lds) s << in << "__syncthreads();\n";
    return s.str();
}

template <class F>
static std::string tile_compute_gen(const Plan& p, const TilePlan& tp, const std::string& in, const std::string& ti,
                                    const std::string& tj, const std::string& R, const std::string& Cn,
                                    const std::string& lr, const std::string& lc, const std::string& out,
                                    const std::string& OT, const std::string& ldo, bool off32, F per_elem)
{
    std::ostringstream s;
    s << in << "{\n";
    const std::string i2 = in + "    ";
    s << i2 << "const i64 i0 = (i64)(" << ti << ") << " << lr << ", j0 = (i64)(" << tj << ") << " << lc << ";\n";
    s << i2 << "const int rr = (int)(" << R << " - i0 < (1 << " << lr << ") ? " << R << " - i0 : (1 << " << lr << "));\n";
    s << i2 << "const int cc = (int)(" << Cn << " - j0 < (1 << " << lc << ") ? " << Cn << " - j0 : (1 << " << lc << "));\n";
    s << tile_lanes(i2, lr, lc, "rr", "cc");
    if (tp.any_lds) s << i2 << "const int sst = coot_tile_stride(" << lr << ", " << lc << ");\n";
    std::vector<std::pair<std::string, std::pair<std::string, bool>>> yp;
    if (!out.empty()) {
        s << i2 << OT << "* po = " << out << " + ((i0 + ysr) + (j0 + ysc) * " << ldo << ");\n";
        s << i2 << (off32 ? "const u32 vo = (u32)" : "const i64 vo = (i64)") << "(yi + (i64)yj * " << ldo << ");\n";
        yp.push_back({"po", {ldo, false}});
    }
    s << in << "#pragma unroll\n" << i2 << "for (int kk = 0; kk < 16; ++kk) {\n";
    s << i2 << "    if (w + 4 * kk < nst) {\n";
    const std::string i4 = i2 + "        ";
    s << i4 << "if (ysr < rr && ysc < cc && yok && (" << lr << " <= 6 ? yj < cc - ysc : yi < rr - ysr)) {\n";
    s << i4 << "    const i64 ig = i0 + ysr + yi, jg = j0 + ysc + yj;\n";
    std::string args;
    for (size_t j = 0; j < p.reads.size(); ++j) {
        if (j) args += ", ";
        args += tp.in_lds[j] ? "T" + std::to_string(j) + "[(ysr + yi) * sst + ysc + yj]" : "cr" + std::to_string(j) + "[kk]";
    }
    if (p.gen_index) args += (args.empty() ? "" : ", ") + ("ig + jg * " + R + ", ig, jg");
    s << per_elem(args, i4 + "    ", off32 ? "atw(po, vo)" : "(po + vo)");
    s << i4 << "}\n";
    s << walk_y(i4, lr, yp);
    s << i2 << "    }\n" << i2 << "}\n" << in << "}\n";
    return s.str();
}

static std::string emit_tiled(const Plan& p, const std::string& name)
{
    const bool ew = p.kind == K_EW_TILED;
    const bool gen = p.tile_gen;
    const int rp = p.nodes[p.root].prec;
    const TilePlan tp = tile_plan(p);
    std::ostringstream s;
    s << "extern \"C\" __global__ void __launch_bounds__(256) " << name << "(const coot_kargs a)\n{\n";
    s << decl_reads(p, !p.alias_out);
    s << tile_shared_decls(p, tp, "    ");
    if (ew) {
        const char* OS = stype(p.out_dtype);
        s << "    " << OS << "* " << (p.alias_out ? "" : "__restrict__ ") << "O = (" << OS << "*)a.out;\n";
        s << "    const i64 ldo = a.ld_out;\n";
    } else {
        s << "    " << acc_type(p) << " acc;\n    acc.init();\n";
    }
    s << "    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);\n";
    s << "    const i64 R = a.rows, Cn = a.cols;\n";
    // tile shape, fixed per kernel: 2^lr x 2^lc
    s << "    const int lr = " << p.tile_lr << ", lc = " << p.tile_lc << ";\n";
    // 64 x 64 and tall tiles start sh rows above the value (0 <= sh < 64),
    // so that the column segments of the reference operand begin on cache
    // lines
    const bool tall = gen && p.tile_tall;
    const bool shifted = !gen || tall;
    if (shifted) s << "    const i64 sh = a.aux;\n";
    // tile counts fit in int for every matrix that fits in device memory
    if (tall)
        s << "    const int tr = R > 0 ? (int)((R + sh + (1 << lr) - 1) >> lr) : 0;\n";
    else
        s << "    const int tr = (int)((R + " << (shifted ? "sh + " : "") << "(1 << lr) - 1) >> lr);\n";
    s << "    const int tc = tr > 0 ? (int)((Cn + (1 << lc) - 1) >> lc) : 0, trs = tr > 0 ? tr : 1;\n";
    s << "    const int gq = (int)gridDim.x / trs, gr = (int)gridDim.x % trs;\n";
    s << "    int ti = (int)blockIdx.x % trs, tj = (int)blockIdx.x / trs;\n";
    s << tile_regs(p, tp, "    ");
    TileView v{"R", "Cn", "lr", "lc", [](size_t j) { return "L" + std::to_string(j); },
               [](size_t j) { return "ld" + std::to_string(j); }};
    // a tall tile wholly inside the value
    auto tfull = [&](const std::string& a, const std::string& b) {
        return "(((i64)(" + a + ") << lr) - sh >= 0 && ((i64)(" + a + ") << lr) - sh + (1 << lr) <= R && (((i64)(" + b +
               ") + 1) << lc) <= Cn)";
    };
    auto prefetch = [&](const std::string& in, const std::string& a, const std::string& b) {
        if (tall)
            return in + "{\n" + in + "if (" + tfull(a, b) + ")\n" +
                   (p.tile_v4 ? tall_prefetch_v4(p, in + "    ", a, b, v) : tall_prefetch(p, in + "    ", a, b, v, false)) + in +
                   "else\n" + tall_prefetch(p, in + "    ", a, b, v, true) + in + "}\n";
        return gen ? tile_prefetch_gen(p, tp, in, a, b, v, "ldnt", p.tile_off32) : tile_prefetch_sq(p, tp, in, a, b, v, "ldnt", true);
    };
    auto elem = [&](const std::string& args, const std::string& in, const std::string& addr) {
        if (ew)
            return in + "stnt(" + addr + ", (" + std::string(stype(p.out_dtype)) + ")(" +
                   narrow(p.out_dtype, rp, "x_eval(" + args + ")") + "));\n";
        return in + accumulate(p, args, "(ig + jg * R)") + "\n";
    };
    s << "    if (tj < tc)\n" << prefetch("        ", "ti", "tj");
    s << "    while (tj < tc) {\n";
    s << "        int ni = ti + gr, nj = tj + gq;\n";
    s << "        if (ni >= tr) { ni -= tr; ++nj; }\n";
    s << (gen ? tile_stage_gen(p, tp, "        ", "R", "Cn", "ti", "tj", "lr", "lc") : tile_stage_sq(p, tp, "        "));
    s << "        if (nj < tc)\n" << prefetch("            ", "ni", "nj");
    if (tall)
        s << "        if (" << tfull("ti", "tj") << ")\n"
          << (p.tile_v4 ? tall_compute_v4(p, "        ", "ti", "tj", ew, "ldo") : tall_compute(p, "        ", "ti", "tj", ew, "ldo", elem, false))
          << "        else\n"
          << tall_compute(p, "        ", "ti", "tj", ew, "ldo", elem, true);
    else if (gen)
        s << tile_compute_gen(p, tp, "        ", "ti", "tj", "R", "Cn", "lr", "lc", ew ? "O" : "", stype(p.out_dtype), "ldo",
                              p.tile_off32, elem);
    else
        s << tile_compute_sq(p, tp, "        ", "ti", "tj", "R", "Cn", ew ? "O" : "", stype(p.out_dtype), "ldo", elem, true);
    s << "        ti = ni;\n        tj = nj;\n";
    s << "    }\n";
    if (!ew) {
        s << "    __shared__ " << acc_type(p) << " lds_acc[4];\n";
        s << "    acc = block_reduce(acc, lds_acc);\n";
        s << "    if (threadIdx.x == 0) " << put_partial(p, "blockIdx.x") << "\n";
    }
    s << "}\n";
    if (!ew) s << emit_partials_comb(p, name);
    return s.str();
}

// --- thin values: a short side of K <= 16 elements ---------------------------
// The value is R x Cn with K = min(R, Cn) <= 16 (thin_rows: R = K).  A thread
// takes a group of V consecutive long-side positions (one 16-byte vector
// along the long side) and all K short-side indices of them; the 64 lanes of
// a wave take 64 consecutive groups.  A strided operand (one run along the
// long side per short-side index, at k*ld + g*V) is loaded directly: K
// vectors per lane, consecutive lanes on consecutive vectors.  A packed
// operand (ld == K: the value's own layout when the rows are short, an
// operand read transposed when the columns are) holds a wave's 64 groups as
// 64*V*K contiguous elements.  With K <= 2 each lane loads its own group's V*K
// elements; otherwise the wave loads the whole run as K fully coalesced
// vectors per lane and hands every lane its own group through a region of
// LDS private to the wave (lane regions padded to an odd number of 16-byte
// units, so the lanes' vector reads do not conflict), and packed outputs go
// back the same way.  In registers element f = n*V + e of a packed group is
// short-side index f % K of position f / K; the transposition to and from
// the strided layout happens at indices fixed when the kernel is generated.
// Misaligned operands move element by element.  8/K groups per thread are in
// flight.  The positions after the last whole group (fewer than V) are done
// element by element by the last block.
static std::string emit_thin(const Plan& p, const std::string& name)
{
    const bool ew = p.kind == K_EW_TILED;
    const int K = p.thin_k, V = p.thin_v, UG = std::max(1, 8 / K);
    const bool sr = p.thin_rows;
    const int rp = p.nodes[p.root].prec;
    const std::string OS = ew ? stype(p.out_dtype) : "";
    const std::string sK = std::to_string(K), sV = std::to_string(V), sVK = std::to_string(V * K);
    auto packed = [&](int j) { return j < 0 ? sr : (p.reads[(size_t)j].trans ? !sr : sr); };
    auto vec = [&](int j) { return (p.thin_vec & (j < 0 ? (1u << 31) : (1u << j))) != 0; };
    // packed operands are exchanged through LDS from K = 2 on (2 x 2^26 FP32
    // add: 283 us loading each lane's own 32 bytes, 263 us exchanged)
    const bool stage = K >= 2;
    auto staged = [&](int j) { return stage && packed(j) && vec(j); };
    bool any_stage = ew && staged(-1);
    for (size_t j = 0; j < p.reads.size(); ++j) any_stage = any_stage || staged((int)j);
    const int maxsz = 16 / V;
    const int RS = V * K + (K % 2 == 0 ? V : 0);  // a lane's LDS region, elements
    std::ostringstream s;
    s << "// thin value: short side " << (sr ? "rows" : "columns") << ", K = " << K << ", " << V
      << "-element vectors (mask " << p.thin_vec << (any_stage ? ", packed through LDS" : "") << ")\n";
    s << "extern \"C\" __global__ void __launch_bounds__(256) " << name << "(const coot_kargs a)\n{\n";
    s << decl_reads(p, !p.alias_out);
    if (ew) {
        s << "    " << OS << "* " << (p.alias_out ? "" : "__restrict__ ") << "O = (" << OS << "*)a.out;\n";
        s << "    const i64 ldo = a.ld_out;\n";
    } else {
        s << "    " << acc_type(p) << " acc;\n    acc.init();\n";
    }
    s << "    const i64 R = a.rows, Cn = a.cols;\n";
    s << "    const i64 ln = " << (sr ? "Cn" : "R") << ", ng = ln / " << sV << ";\n";
    s << "    const i64 step = (i64)gridDim.x * 256 * " << UG << ";\n";
    s << "    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);\n";
    if (any_stage) {
        s << "    __shared__ __align__(16) unsigned char lds_thin[" << 4 * 64 * RS * maxsz << "];\n";
        s << "    unsigned char* const lw = lds_thin + w * " << 64 * RS * maxsz << ";\n";
    }
    // per-lane chunk c = n*64 + lane of a wave's packed run: its LDS slot
    auto chunk_slot = [&](const std::string& n) {
        return "((" + n + " * 64 + lane) / " + sK + ") * " + std::to_string(RS) + " + ((" + n + " * 64 + lane) % " + sK +
               ") * " + sV;
    };
    // the group a chunk belongs to
    auto chunk_group = [&](const std::string& n) { return "gw + (" + n + " * 64 + lane) / " + sK; };
    // loop over the wave's group blocks (wave-uniform: every lane runs every iteration)
    s << "    for (i64 gb = (i64)blockIdx.x * (256 * " << UG << ") + w * 64; gb < ng; gb += step) {\n";
    for (size_t j = 0; j < p.reads.size(); ++j)
        s << "        " << stype(p.reads[j].dtype) << " r" << j << "[" << UG << "][" << sK << "][" << sV << "];\n";
    // loads are unconditional (a lane past the last group reads the last
    // group again): with no branch around them the compiler keeps every load
    // of the step in flight
    s << "#pragma unroll\n        for (int u = 0; u < " << UG << "; ++u) {\n";
    s << "            const i64 gw = gb + u * 256, g = gw + lane < ng ? gw + lane : ng - 1;\n";
    s << "            const i64 gcl = (ng - gw) * " << sK << " - 1;  // last chunk of the wave inside the value\n";
    s << "            (void)gcl;\n";
    s << "#pragma unroll\n            for (int n = 0; n < " << sK << "; ++n) {\n";
    for (size_t j = 0; j < p.reads.size(); ++j) {
        const std::string J = std::to_string(j);
        const std::string S = stype(p.reads[j].dtype);
        if (staged((int)j)) {
            s << "                ldv<" << S << ", " << sV << ">(L" << J << ", gw * " << sVK << " + (n * 64 + lane < gcl ? n * 64 + lane : gcl) * "
              << sV << ", r" << J << "[u][n]);\n";
            continue;
        }
        const std::string off = packed((int)j) ? "g * " + sVK + " + n * " + sV : "n * ld" + J + " + g * " + sV;
        if (vec((int)j))
            s << "                ldv<" << S << ", " << sV << ">(L" << J << ", " << off << ", r" << J << "[u][n]);\n";
        else
            s << "#pragma unroll\n                for (int e = 0; e < " << sV << "; ++e) r" << J << "[u][n][e] = ldnt(L" << J << " + ("
              << off << " + e));\n";
    }
    s << "            }\n        }\n";
    s << "#pragma unroll\n        for (int u = 0; u < " << UG << "; ++u) {\n";
    s << "            const i64 gw = gb + u * 256, g = gw + lane;\n";
    s << "            const bool gok = g < ng;\n";
    // packed reads: chunks into the wave's LDS region, each lane's own group back
    for (size_t j = 0; j < p.reads.size(); ++j) {
        if (!staged((int)j)) continue;
        const std::string J = std::to_string(j), S = stype(p.reads[j].dtype);
        s << "            {\n                " << S << "* const T = (" << S << "*)lw;\n";
        s << "#pragma unroll\n                for (int n = 0; n < " << sK << "; ++n)\n";
        s << "                    lds_put<" << S << ", " << sV << ">(T, " << chunk_slot("n") << ", r" << J << "[u][n]);\n";
        s << "                wave_lds_sync();\n";
        s << "#pragma unroll\n                for (int n = 0; n < " << sK << "; ++n)\n";
        s << "                    lds_get<" << S << ", " << sV << ">(T, lane * " << RS << " + n * " << sV << ", r" << J << "[u][n]);\n";
        s << "                wave_lds_sync();\n            }\n";
    }
    if (ew) s << "            " << OS << " o[" << sK << "][" << sV << "];\n";
    s << "            {\n";
    // register of element (k, v) in a packed / strided operand
    auto reg = [&](bool pk, int k, int v) {
        const int f = v * K + k;
        return pk ? "[" + std::to_string(f / V) + "][" + std::to_string(f % V) + "]"
                  : "[" + std::to_string(k) + "][" + std::to_string(v) + "]";
    };
    for (int v = 0; v < V; ++v)
        for (int k = 0; k < K; ++k) {
            std::string args;
            for (size_t j = 0; j < p.reads.size(); ++j) {
                if (j) args += ", ";
                args += widen(p.reads[j].dtype, "r" + std::to_string(j) + "[u]" + reg(packed((int)j), k, v));
            }
            // row and column of the element in the value
            const std::string ig = sr ? "(i64)" + std::to_string(k) : "(g * " + sV + " + " + std::to_string(v) + ")";
            const std::string jg = sr ? "(g * " + sV + " + " + std::to_string(v) + ")" : "(i64)" + std::to_string(k);
            const std::string lin = "(" + ig + " + " + jg + " * R)";
            if (p.gen_index) args += (args.empty() ? "" : ", ") + lin + ", " + ig + ", " + jg;
            if (ew)
                s << "                o" << reg(packed(-1), k, v) << " = " << narrow(p.out_dtype, rp, "x_eval(" + args + ")")
                  << ";\n";
            else
                s << "                if (gok) " << accumulate(p, args, lin) << "\n";
        }
    if (ew && !staged(-1)) {
        const std::string off = packed(-1) ? "g * " + sVK + " + n * " + sV : "n * ldo + g * " + sV;
        if (vec(-1))
            s << "                if (gok)\n#pragma unroll\n                    for (int n = 0; n < " << sK << "; ++n) stv<" << OS << ", "
              << sV << ">(O, " << off << ", o[n]);\n";
        else
            s << "                if (gok)\n#pragma unroll\n                    for (int n = 0; n < " << sK << "; ++n)\n#pragma unroll\n"
              << "                        for (int e = 0; e < " << sV << "; ++e) stnt(O + (" << off << " + e), o[n][e]);\n";
    }
    s << "            }\n";
    if (ew && staged(-1)) {
        // each lane's group into its LDS region, the wave's run out in coalesced chunks
        s << "            {\n                " << OS << "* const T = (" << OS << "*)lw;\n";
        s << "#pragma unroll\n                for (int n = 0; n < " << sK << "; ++n)\n";
        s << "                    lds_put<" << OS << ", " << sV << ">(T, lane * " << RS << " + n * " << sV << ", o[n]);\n";
        s << "                wave_lds_sync();\n";
        s << "#pragma unroll\n                for (int n = 0; n < " << sK << "; ++n)\n";
        s << "                    if (" << chunk_group("n") << " < ng) {\n";
        s << "                        " << OS << " t[" << sV << "];\n";
        s << "                        lds_get<" << OS << ", " << sV << ">(T, " << chunk_slot("n") << ", t);\n";
        s << "                        stv<" << OS << ", " << sV << ">(O, gw * " << sVK << " + (n * 64 + lane) * " << sV << ", t);\n";
        s << "                    }\n";
        s << "                wave_lds_sync();\n            }\n";
    }
    s << "        }\n    }\n";
    // positions after the last whole group
    s << "    if (blockIdx.x == gridDim.x - 1) {\n";
    s << "        for (i64 t = threadIdx.x; t < (ln - ng * " << sV << ") * " << sK << "; t += 256) {\n";
    s << "            const i64 ps = ng * " << sV << " + t / " << sK << ", ks = t % " << sK << ";\n";
    s << "            const i64 ig = " << (sr ? "ks" : "ps") << ", jg = " << (sr ? "ps" : "ks") << ";\n";
    std::string targs;
    for (size_t j = 0; j < p.reads.size(); ++j) {
        const std::string J = std::to_string(j);
        if (j) targs += ", ";
        targs += widen(p.reads[j].dtype, p.reads[j].trans ? "ldnt(L" + J + " + (jg + ig * ld" + J + "))"
                                                          : "ldnt(L" + J + " + (ig + jg * ld" + J + "))");
    }
    if (p.gen_index) targs += (targs.empty() ? "" : ", ") + std::string("ig + jg * R, ig, jg");
    if (ew)
        s << "            stnt(O + (ig + jg * ldo), (" << OS << ")(" << narrow(p.out_dtype, rp, "x_eval(" + targs + ")")
          << "));\n";
    else
        s << "            " << accumulate(p, targs, "(ig + jg * R)") << "\n";
    s << "        }\n    }\n";
    if (!ew) {
        s << "    __shared__ " << acc_type(p) << " lds_acc[4];\n";
        s << "    acc = block_reduce(acc, lds_acc);\n";
        s << "    if (threadIdx.x == 0) " << put_partial(p, "blockIdx.x") << "\n";
    }
    s << "}\n";
    if (!ew) s << emit_partials_comb(p, name);
    return s.str();
}

// --- per-column reductions (dim 0): one wave per (column, row segment) -------
// With few columns each column is cut into a.splits segments of a.aux rows so
// that enough waves stream; segment partials are combined per column, in
// segment order, by the second entry point.
static std::string emit_col(const Plan& p, const LaunchCfg& c, const std::string& name)
{
    const int VE = p.ve, EPT = c.ept;
    const bool mix = f16_mix_sum(p);
    std::ostringstream s;
    if (mix) s << F16_MIX_SRC;
    s << "extern \"C\" __global__ void __launch_bounds__(512) " << name << "(const coot_kargs a)\n{\n";
    s << decl_reads(p, true);
    s << "    const int lane = threadIdx.x & 63;\n";
    s << "    const i64 wv = ((i64)blockIdx.x * blockDim.x + threadIdx.x) >> 6;\n";
    s << "    const i64 nw = ((i64)gridDim.x * blockDim.x) >> 6;\n";
    s << "    const i64 total = a.cols * a.splits;\n";
    s << "    for (i64 u = wv; u < total; u += nw) {\n";
    s << "        const i64 j = u % a.cols, sg = u / a.cols;\n";
    s << "        const i64 rs0 = sg * a.aux;\n";
    s << "        const i64 rs1 = rs0 + a.aux < a.rows ? rs0 + a.aux : a.rows;\n";
    s << "        const i64 nvr = (rs1 - rs0) / " << VE << ";\n";
    s << "        " << acc_type(p) << " acc;\n        acc.init();\n";
    for (size_t j = 0; j < p.reads.size(); ++j)
        s << "        const " << stype(p.reads[j].dtype) << "* C" << j << " = L" << j << " + j * ld" << j << " + rs0;\n";
    // 2- and 4-byte data: two register buffers, the next step's loads in
    // flight while the current step is folded, whole steps without per-vector
    // guards (FP32 1-3% faster, 16-bit max 20%).  8-byte data keeps one buffer
    // (the second costs FP64 columns 5%), and so do compensated sums of FP16
    // (5% slower with the second buffer at 65 VGPRs; BF16 sums break even)
    int maxsz = 1;
    bool f16 = false;
    for (const Read& r : p.reads) {
        maxsz = std::max(maxsz, itemsize(r.dtype));
        f16 = f16 || r.dtype == COOT_F16;
    }
    if (maxsz <= 4 && !(f16 && acc_type(p) == "AccKF")) {
        auto load = [&](const std::string& buf, const std::string& b, bool guarded) {
            std::ostringstream o;
            o << "#pragma unroll\n            for (int e = 0; e < " << EPT << "; ++e) {\n";
            o << "                const i64 v = " << b << " + e * 64;\n                if (" << (guarded ? "v < nvr" : "true")
              << ") {\n";
            for (size_t j = 0; j < p.reads.size(); ++j)
                o << "                    ldv<" << stype(p.reads[j].dtype) << ", " << VE << ">(C" << j << ", v * " << VE
                  << ", " << buf << j << "[e]);\n";
            o << "                }\n            }\n";
            return o.str();
        };
        auto fold = [&](const std::string& buf, bool guarded) {
            std::ostringstream o;
            std::string args = arglist(p, [&](int j) { return buf + std::to_string(j) + "[e][k]"; }, "gi + j * a.rows, gi, j");
            o << "#pragma unroll\n            for (int e = 0; e < " << EPT << "; ++e) {\n";
            o << "                const i64 v = base + e * 64;\n                if (" << (guarded ? "v < nvr" : "true") << ") {\n";
            // each lane meets its rows in increasing order
            o << "#pragma unroll\n                    for (int k = 0; k < " << VE << "; ++k) { const i64 gi = rs0 + v * " << VE
              << " + k; (void)gi; " << increasing(p, accumulate(p, args, "gi")) << " }\n";
            o << "                }\n            }\n";
            return o.str();
        };
        auto stage = [&](const std::string& nxt, const std::string& cur, const std::string& b) {
            std::ostringstream o;
            o << "            if (" << b << " + " << (EPT - 1) << " * 64 < nvr) {\n";
            o << load(nxt, b, false) << fold(cur, false);
            o << "            } else {\n";
            o << load(nxt, b, true) << fold(cur, true);
            o << "            }\n";
            return o.str();
        };
        for (size_t j = 0; j < p.reads.size(); ++j)
            s << "        " << stype(p.reads[j].dtype) << " ra" << j << "[" << EPT << "][" << VE << "], rb" << j << "[" << EPT
              << "][" << VE << "];\n";
        s << "        i64 base = lane;\n";
        s << load("ra", "base", true);
        s << "        while (base < nvr) {\n";
        s << "            const i64 nb = base + 64 * " << EPT << ";\n";
        s << stage("rb", "ra", "nb");
        s << "            base = nb;\n            if (base >= nvr) break;\n";
        s << "            const i64 nb2 = base + 64 * " << EPT << ";\n";
        s << stage("ra", "rb", "nb2");
        s << "            base = nb2;\n        }\n";
    } else {
        s << "        for (i64 base = lane; base < nvr; base += 64 * " << EPT << ") {\n";
        for (size_t j = 0; j < p.reads.size(); ++j)
            s << "            " << stype(p.reads[j].dtype) << " r" << j << "[" << EPT << "][" << VE << "];\n";
        s << "#pragma unroll\n            for (int e = 0; e < " << EPT << "; ++e) {\n";
        s << "                const i64 v = base + e * 64;\n                if (v < nvr) {\n";
        for (size_t j = 0; j < p.reads.size(); ++j)
            s << "                    ldv<" << stype(p.reads[j].dtype) << ", " << VE << ">(C" << j << ", v * " << VE << ", r"
              << j << "[e]);\n";
        s << "                }\n            }\n";
        s << "#pragma unroll\n            for (int e = 0; e < " << EPT << "; ++e) {\n";
        s << "                const i64 v = base + e * 64;\n                if (v < nvr) {\n";
        std::string args = arglist(p, [](int j) { return "r" + std::to_string(j) + "[e][k]"; }, "gi + j * a.rows, gi, j");
        s << "#pragma unroll\n                    for (int k = 0; k < " << VE << "; ++k) { const i64 gi = rs0 + v * " << VE
          << " + k; (void)gi; " << (mix ? f16_mix_add("r0[e]", "acc") : accumulate(p, args, "gi")) << " }\n";
        s << "                }\n            }\n        }\n";
    }
    std::string targs = arglist(p, [](int j) { return "ldnt(C" + std::to_string(j) + " + r)"; },
                                "(rs0 + r) + j * a.rows, rs0 + r, j");
    s << "        for (i64 r = nvr * " << VE << " + lane; r < rs1 - rs0; r += 64) { " << accumulate(p, targs, "(rs0 + r)")
      << " }\n";
    s << "        wave_reduce(acc);\n";
    s << "        if (lane == 0) { if (a.splits == 1) { " << write_direct(p, "j") << " } else { "
      << put_partial(p, "sg * a.cols + j") << " } }\n";
    s << "    }\n}\n";
    s << "extern \"C\" __global__ void __launch_bounds__(256) " << name << "_comb(const coot_kargs a)\n{\n";
    s << "    for (i64 j = blockIdx.x; j < a.cols; j += gridDim.x) {\n        "
      << combine_and_write(p, "j", "a.splits", "a.cols", "j") << "\n    }\n}\n";
    return s.str();
}

// --- per-column reductions of short columns: one thread per column -----------
static std::string emit_colt(const Plan& p, const std::string& name)
{
    std::ostringstream s;
    s << "extern \"C\" __global__ void __launch_bounds__(512) " << name << "(const coot_kargs a)\n{\n";
    s << decl_reads(p, true);
    s << "    for (i64 j = (i64)blockIdx.x * blockDim.x + threadIdx.x; j < a.cols; j += (i64)gridDim.x * blockDim.x) {\n";
    s << "        " << acc_type(p) << " acc;\n        acc.init();\n";
    std::string args = arglist(p, [](int j) { return "ldnt(L" + std::to_string(j) + " + r + j * ld" + std::to_string(j) + ")"; },
                               "r + j * a.rows, r, j");
    s << "        for (i64 r = 0; r < a.rows; ++r) { " << accumulate(p, args, "r") << " }\n";
    s << "        " << write_direct(p, "j") << "\n    }\n}\n";
    return s.str();
}

// --- per-row reductions (dim 1): thread per (VE rows, column subset) ---------
// Work unit g < RV is a group of VE consecutive rows read with one vector load
// per column; the rows % VE left over are scalar units.  With splits > 1 each
// unit folds the contiguous column range q of `splits` equal ranges (measured
// 7-20% faster than interleaved columns q, q + splits, ...), and a second
// kernel combines the ranges of every row in column order.
static std::string emit_row(const Plan& p, const std::string& name)
{
    const int VE = p.ve;
    std::ostringstream s;
    s << "extern \"C\" __global__ void __launch_bounds__(512) " << name << "(const coot_kargs a)\n{\n";
    s << decl_reads(p, true);
    s << "    const i64 RV = a.rows / " << VE << ";\n";
    s << "    const i64 groups = RV + (a.rows - RV * " << VE << ");\n";
    s << "    const i64 total = groups * a.splits;\n";
    s << "    for (i64 w = (i64)blockIdx.x * blockDim.x + threadIdx.x; w < total; w += (i64)gridDim.x * blockDim.x) {\n";
    s << "        const i64 g = w % groups, q = w / groups;\n";
    // split q folds the contiguous column range [c0, c1)
    s << "        const i64 cw = (a.cols + a.splits - 1) / a.splits, c0 = q * cw, c1 = c0 + cw < a.cols ? c0 + cw : a.cols;\n";
    if (VE > 1) {
        s << "        if (g < RV) {\n";
        s << "            " << acc_type(p) << " av[" << VE << "];\n";
        s << "#pragma unroll\n            for (int k = 0; k < " << VE << "; ++k) av[k].init();\n";
        s << "#pragma unroll 8\n            for (i64 c = c0; c < c1; ++c) {\n";
        for (size_t j = 0; j < p.reads.size(); ++j)
            s << "                " << stype(p.reads[j].dtype) << " r" << j << "[" << VE << "];\n                ldv<"
              << stype(p.reads[j].dtype) << ", " << VE << ">(L" << j << ", g * " << VE << " + c * ld" << j << ", r" << j
              << ");\n";
        std::string args = arglist(p, [](int j) { return "r" + std::to_string(j) + "[k]"; },
                                   "(g * " + std::to_string(VE) + " + k) + c * a.rows, g * " + std::to_string(VE) + " + k, c");
        s << "#pragma unroll\n                for (int k = 0; k < " << VE << "; ++k) { " << accumulate(p, args, "c", "av[k]")
          << " }\n";
        s << "            }\n";
        s << "#pragma unroll\n            for (int k = 0; k < " << VE << "; ++k) {\n";
        s << "                const i64 r = g * " << VE << " + k;\n";
        std::string wd = write_direct(p, "r"), pp = put_partial(p, "q * a.rows + r");
        for (auto* str : {&wd, &pp}) {
            for (size_t pos; (pos = str->find("acc.")) != std::string::npos;) str->replace(pos, 4, "av[k].");
            for (size_t pos; (pos = str->find(", acc)")) != std::string::npos;) str->replace(pos, 6, ", av[k])");
        }
        s << "                if (a.splits == 1) { " << wd << " } else { " << pp << " }\n";
        s << "            }\n            continue;\n        }\n";
    }
    s << "        const i64 r = RV * " << VE << " + (g - RV);\n";
    s << "        " << acc_type(p) << " acc;\n        acc.init();\n";
    std::string args = arglist(p, [](int j) { return "ldnt(L" + std::to_string(j) + " + r + c * ld" + std::to_string(j) + ")"; },
                               "r + c * a.rows, r, c");
    s << "#pragma unroll 4\n        for (i64 c = c0; c < c1; ++c) { " << accumulate(p, args, "c") << " }\n";
    s << "        if (a.splits == 1) { " << write_direct(p, "r") << " } else { " << put_partial(p, "q * a.rows + r")
      << " }\n";
    s << "    }\n}\n";
    // combine in a fixed order: a block per row from 256 splits on, four
    // waves per 64 rows from 16, a thread per row below
    s << "extern \"C\" __global__ void __launch_bounds__(256) " << name << "_comb(const coot_kargs a)\n{\n";
    s << "    if (a.splits >= 256) {\n";
    s << "        for (i64 r = blockIdx.x; r < a.rows; r += gridDim.x) {\n            "
      << combine_and_write(p, "r", "a.splits", "a.rows", "r") << "\n        }\n";
    s << "        return;\n    }\n";
    // 16 to 255 splits: four waves per 64 rows, wave k adding quarter k of
    // the splits in order (adjacent lanes read adjacent slots of one split),
    // the quarters merged in order through LDS
    std::string acc, fold, put;
    if (red_is_var(p.red_op)) {
        acc = "AccV";
        fold = "x = combine_var_seq(part, s0 * a.rows + r, s1 - s0, a.rows);";
        put = put_var_result(p, "r", "y");
    } else if (red_is_sum(p.red_op)) {
        acc = "AccKD";
        fold = "for (i64 t = s0; t < s1; t += 8) { double h[8], l[8];\n"
               "#pragma unroll\n"
               "                for (int u = 0; u < 8; ++u) { const double* pp = part + 2 * ((t + u < s1 ? t + u : t) * a.rows + r); "
               "h[u] = pp[0]; l[u] = pp[1]; }\n"
               "#pragma unroll\n"
               "                for (int u = 0; u < 8; ++u) if (t + u < s1) { x.add(h[u]); x.add(l[u]); } }";
        put = put_sum_result(p, "r", "(y.hi() + y.lo())");
    } else {
        const std::string mx = red_is_max(p.red_op) ? "true" : "false";
        acc = "AccI<double, " + mx + ">";
        fold = "x = combine_idx_seq<" + mx + ">(part, s0 * a.rows + r, s1 - s0, a.rows);";
        put = (p.red_op == COOT_RED_INDEX_MIN || p.red_op == COOT_RED_INDEX_MAX)
                  ? "put_u64(a.res, r, y.i);"
                  : put_value(p, "r", "(y.i < 0 ? __builtin_nan(\"\") : y.v)");
    }
    s << "    if (a.splits >= 16) {\n";
    s << "        const int lane = threadIdx.x & 63, k = threadIdx.x >> 6;\n";
    s << "        const i64 qs = (a.splits + 3) / 4, s0 = k * qs, s1 = s0 + qs < a.splits ? s0 + qs : a.splits;\n";
    s << "        const double* part = (const double*)a.part;\n";
    s << "        __shared__ " << acc << " lq[256];\n";
    s << "        for (i64 r0 = (i64)blockIdx.x * 64; r0 < a.rows; r0 += (i64)gridDim.x * 64) {\n";
    s << "            const i64 r = r0 + lane;\n";
    s << "            " << acc << " x;\n            x.init();\n";
    s << "            if (r < a.rows) { " << fold << " }\n";
    s << "            __syncthreads();\n            lq[threadIdx.x] = x;\n            __syncthreads();\n";
    s << "            if (k == 0 && r < a.rows) {\n";
    s << "                " << acc << " y = lq[lane];\n";
    s << "#pragma unroll\n                for (int m = 1; m < 4; ++m) y.merge(lq[m * 64 + lane]);\n";
    s << "                " << put << "\n            }\n        }\n        return;\n    }\n";
    s << "    for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < a.rows; r += (i64)gridDim.x * blockDim.x) {\n        "
      << combine_and_write_seq(p, "r", "a.splits", "a.rows", "r") << "\n    }\n}\n";
    return s.str();
}

// --- batched kernels: one pass over the units of many items ----------------
// An item's value Y_i (R x Cn, column-major) is cut into units: blocks of
// whole columns (rc = R rows, k columns) where the columns are short, or
// 64-column blocks of E/64 rows where they are long; an item of at most E/4
// elements is one unit of its own.  A unit's operands read through trans()
// are staged in LDS: read along their own columns (k consecutive elements of
// each of the unit's rc columns), stored with an odd row stride kp, and read
// back transposed without bank conflicts.  Everything else moves in the
// value's column-major order, so the output and the straight operands stream
// contiguous runs (whole units when rc = R).  A block runs one large unit
// with all its threads, or up to four small units, one per wave (each wave
// with a quarter of the LDS stage).  Each unit leaves a compensated partial of
// the item's reduction; the _comb kernel adds an item's partials in unit
// order, so r_i depends only on the item's shape and values.
int64_t batch_unit_elems(const Plan& py)
{
    int bytes = 0;
    for (const Read& r : py.reads)
        if (r.trans) bytes += itemsize(r.dtype);
    // 12288 FP32 elements: a 50 KB stage, three blocks per CU (16384: 68 KB,
    // two blocks; 10,000-matrix workload 425 -> 399 us with 16 elements in
    // flight per thread)
    int64_t e = 12288;
    while (bytes > 0 && e * bytes > COOT_BATCH_LDS_BYTES) e >>= 1;
    return e;
}

std::string batch_kernel_source(const Plan& py, const Plan* pr, bool has_out, int out_dtype, int red_dtype,
                                const std::vector<int>& read_slot, std::string* name_out)
{
    const int64_t E = batch_unit_elems(py);
    const int64_t CAP = coot_batch_stage_cap(E);  // LDS elements per staged read (block mode)
    const int rp = py.nodes[py.root].prec;
    const std::string ACC = pr ? (pr->nodes[pr->root].prec == 64 ? "AccKD" : (pr->pairwise ? "AccPF" : "AccKF")) : "";
    const std::string OS = stype(out_dtype);
    const size_t nr = py.reads.size();
    // elements per thread in flight: the pass runs a few blocks per CU (its
    // LDS stage), so each thread keeps many loads in flight (8 -> 16: 487 ->
    // 435 us with the 68 KB stage; with the 50 KB stage 16 and 24 equal,
    // 32 slower, 48 much slower)
    constexpr int U = 16;
    std::ostringstream s;
    s << "// batch tree: " << py.body_sig << "\n";
    s << emit_eval(py, false, "x");
    if (pr) {
        s << "// reduction tree over Y: " << pr->body_sig << "\n";
        s << emit_eval(*pr, pr->product_form, "r");
    }
    auto S = [&](size_t j) { return std::string(stype(py.reads[j].dtype)); };
    // the value y of one element of Y_i: store it, fold it into the reduction
    auto elem = [&](const std::string& in, const std::string& args, const std::string& yaddr) {
        std::ostringstream o;
        o << in << "const " << ctype(rp) << " y = x_eval(" << args << ");\n";
        std::string yv = "y";
        if (has_out) {
            o << in << "const " << OS << " yo = " << narrow(out_dtype, rp, "y") << ";\n";
            o << in << "O[" << yaddr << "] = yo;\n";
            if (out_dtype == COOT_F16) yv = "widen_f16(yo)";
            else if (out_dtype == COOT_BF16) yv = "widen_bf16(yo)";
            else yv = "yo";
        }
        if (pr) {
            const int pp = pr->nodes[pr->root].prec;
            if (pr->product_form)
                o << in << "{ " << ctype(pp) << " pa, pb; r_pair(" << yv << ", pa, pb); acc.add_prod(pa, pb); }\n";
            else if (pr->red_op == COOT_RED_NORM2)
                o << in << "{ const " << ctype(pp) << " u = r_eval(" << yv << "); acc.add_prod(u, u); }\n";
            else if (pr->red_op == COOT_RED_NORM1)
                o << in << "acc.add(" << (pp == 64 ? "__builtin_fabs" : "__builtin_fabsf") << "(r_eval(" << yv << ")));\n";
            else
                o << in << "acc.add(r_eval(" << yv << "));\n";
        }
        return o.str();
    };
    // One unit, run by nt threads (thread t), LDS stage at element offset sb.
    // Stage: element (pp, qq) of the unit (qq fast) of each transposed read
    // comes from T[(q0 + qq) + (p0 + pp) * Cn] and goes to lds[sb + qq + pp * kp].
    // Compute: element (pp, qq) (pp fast) of Y_i at (p0 + pp) + (q0 + qq) * R.
    // Both walks advance by nt elements per step with adds only.
    auto unit_body = [&](const std::string& in, const std::string& nt, const std::string& t, const std::string& sb,
                         bool block) {
        std::ostringstream o;
        o << in << "const coot_batch_unit_d u = b.units[ui];\n";
        o << in << "const coot_batch_item_d& it = b.items[u.item];\n";
        o << in << "const i64 R = it.rows, Cn = it.cols;\n";
        o << in << "const int rc = u.rc, k = u.k, kp = k | 1, n = rc * k;\n";
        for (size_t j = 0; j < nr; ++j)
            o << in << "const " << S(j) << "* L" << j << " = (const " << S(j) << "*)it.leaf[" << read_slot[j] << "];\n";
        // no __restrict__: an item's output may be its own straight operand (in place)
        if (has_out) o << in << OS << "* O = (" << OS << "*)it.out;\n";
        bool any_t = false;
        for (size_t j = 0; j < nr; ++j) any_t = any_t || py.reads[j].trans;
        if (any_t) {
            // stage: walk (pp, qq), qq fast
            o << in << "{\n";
            o << in << "    const int dq = " << nt << " % k, dp = " << nt << " / k;\n";
            o << in << "    int qq = " << t << " % k, pp = " << t << " / k;\n";
            o << in << "    i64 g = (i64)(u.q0 + qq) + (i64)(u.p0 + pp) * Cn;\n";
            o << in << "    int l = " << sb << " + qq + pp * kp;\n";
            o << in << "    const i64 dg = (i64)dq + (i64)dp * Cn;\n";
            o << in << "    const int dl = dq + dp * kp;\n";
            o << in << "    for (int e0 = " << t << "; e0 < n; e0 += " << U << " * " << nt << ") {\n";
            for (size_t j = 0; j < nr; ++j)
                if (py.reads[j].trans) o << in << "        " << S(j) << " v" << j << "[" << U << "];\n";
            o << in << "        int ls[" << U << "];\n";
            o << in << "#pragma unroll\n" << in << "        for (int e = 0; e < " << U << "; ++e) {\n";
            o << in << "            ls[e] = l;\n";
            o << in << "            if (e0 + e * " << nt << " < n) {\n";
            for (size_t j = 0; j < nr; ++j)
                if (py.reads[j].trans) o << in << "                v" << j << "[e] = ldpl(L" << j << " + g);\n";
            o << in << "            }\n";
            o << in << "            qq += dq; pp += dp; g += dg; l += dl;\n";
            o << in << "            if (qq >= k) { qq -= k; ++pp; g += Cn - k; l += kp - k; }\n";
            o << in << "        }\n";
            o << in << "#pragma unroll\n" << in << "        for (int e = 0; e < " << U << "; ++e)\n";
            o << in << "            if (e0 + e * " << nt << " < n) {\n";
            for (size_t j = 0; j < nr; ++j)
                if (py.reads[j].trans) o << in << "                st" << j << "[ls[e]] = v" << j << "[e];\n";
            o << in << "            }\n";
            o << in << "    }\n" << in << "}\n";
            if (block) {
                o << in << "__syncthreads();\n";
            } else {
                o << in << "__builtin_amdgcn_fence(__ATOMIC_RELEASE, \"wavefront\");\n";
                o << in << "__builtin_amdgcn_wave_barrier();\n";
                o << in << "__builtin_amdgcn_fence(__ATOMIC_ACQUIRE, \"wavefront\");\n";
            }
        }
        // compute: walk (pp, qq), pp fast
        o << in << "{\n";
        o << in << "    const int dp = " << nt << " % rc, dq = " << nt << " / rc;\n";
        o << in << "    int pp = " << t << " % rc, qq = " << t << " / rc;\n";
        o << in << "    i64 ya = (i64)(u.p0 + pp) + (i64)(u.q0 + qq) * R;\n";
        o << in << "    int l = " << sb << " + qq + pp * kp;\n";
        o << in << "    const i64 dya = (i64)dp + (i64)dq * R;\n";
        o << in << "    const int dl = dq + dp * kp;\n";
        // a straight read converted on load (16-bit, integer) loads
        // unconditionally, an element past the unit reading the unit's first:
        // behind the per-element test the compiler waited for each load to
        // convert it before issuing the next
        auto converted = [&](size_t j) {
            return !py.reads[j].trans && py.reads[j].dtype != COOT_F32 && py.reads[j].dtype != COOT_F64;
        };
        bool any_conv = false;
        for (size_t j = 0; j < nr; ++j) any_conv = any_conv || converted(j);
        if (any_conv) o << in << "    const i64 yz = (i64)u.p0 + (i64)u.q0 * R;\n";
        o << in << "    for (int e0 = " << t << "; e0 < n; e0 += " << U << " * " << nt << ") {\n";
        for (size_t j = 0; j < nr; ++j)
            o << in << "        " << ctype(dtype_prec(py.reads[j].dtype)) << " v" << j << "[" << U << "];\n";
        o << in << "        i64 ys[" << U << "];\n";
        o << in << "#pragma unroll\n" << in << "        for (int e = 0; e < " << U << "; ++e) {\n";
        o << in << "            ys[e] = ya;\n";
        for (size_t j = 0; j < nr; ++j)
            if (converted(j))
                o << in << "            v" << j << "[e] = "
                  << widen(py.reads[j].dtype, "ldpl(L" + std::to_string(j) + " + (e0 + e * " + nt + " < n ? ya : yz))") << ";\n";
        o << in << "            if (e0 + e * " << nt << " < n) {\n";
        for (size_t j = 0; j < nr; ++j) {
            if (py.reads[j].trans)
                o << in << "                v" << j << "[e] = " << widen(py.reads[j].dtype, "st" + std::to_string(j) + "[l]") << ";\n";
            else if (!converted(j))
                o << in << "                v" << j << "[e] = " << widen(py.reads[j].dtype, "ldpl(L" + std::to_string(j) + " + ya)") << ";\n";
        }
        o << in << "            }\n";
        o << in << "            pp += dp; qq += dq; ya += dya; l += dl;\n";
        o << in << "            if (pp >= rc) { pp -= rc; ++qq; ya += R - rc; l += 1 - rc * kp; }\n";
        o << in << "        }\n";
        o << in << "#pragma unroll\n" << in << "        for (int e = 0; e < " << U << "; ++e)\n";
        o << in << "            if (e0 + e * " << nt << " < n) {\n";
        std::string args;
        for (size_t j = 0; j < nr; ++j) args += (j ? ", v" : "v") + std::to_string(j) + "[e]";
        o << elem(in + "                ", args, "ys[e]");
        o << in << "            }\n";
        o << in << "    }\n" << in << "}\n";
        return o.str();
    };
    s << "extern \"C\" __global__ void __launch_bounds__(256) COOT_KERNEL_NAME(const coot_bargs b)\n{\n";
    for (size_t j = 0; j < nr; ++j)
        if (py.reads[j].trans) s << "    __shared__ " << S(j) << " st" << j << "[" << CAP << "];\n";
    if (pr) s << "    __shared__ " << ACC << " lds_acc[4];\n";
    s << "    const int first = b.blk_first[blockIdx.x], last = b.blk_first[blockIdx.x + 1];\n";
    s << "    if (last - first == 1) {\n";
    s << "        // one unit, all 256 threads\n";
    s << "        const int ui = first;\n";
    if (pr) s << "        " << ACC << " acc;\n        acc.init();\n";
    s << unit_body("        ", "256", "(int)threadIdx.x", "0", true);
    if (pr) {
        s << "        acc = block_reduce(acc, lds_acc);\n";
        s << "        if (threadIdx.x == 0) put_sum_partial(b.part, u.part, acc.hi(), acc.lo());\n";
    }
    s << "    } else {\n";
    s << "        // up to four small units, one per wave, each with a quarter of the stage\n";
    s << "        const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;\n";
    s << "        const int ui = first + w;\n";
    s << "        if (ui < last) {\n";
    if (pr) s << "            " << ACC << " acc;\n            acc.init();\n";
    s << unit_body("            ", "64", "lane", "w * " + std::to_string(CAP / 4), false);
    if (pr) {
        s << "            wave_reduce(acc);\n";
        s << "            if (lane == 0) put_sum_partial(b.part, u.part, acc.hi(), acc.lo());\n";
    }
    s << "        }\n";
    s << "    }\n}\n";
    if (pr) {
        // per item: FP64 compensated sum of its units' partials in unit order,
        // then the final transform
        s << "extern \"C\" __global__ void __launch_bounds__(256) COOT_KERNEL_NAME_comb(const coot_bargs b)\n{\n";
        s << "    const i64 i = (i64)blockIdx.x * 256 + threadIdx.x;\n";
        s << "    if (i >= b.n_items) return;\n";
        s << "    const i64 np = b.items[i].nunits, p0 = b.items[i].part0;\n";
        s << "    AccKD a;\n    a.init();\n";
        s << "    for (i64 k = 0; k < np; ++k) {\n";
        s << "        a.add(b.part[2 * (p0 + k)]);\n        a.add(b.part[2 * (p0 + k) + 1]);\n    }\n";
        std::string val = pr->red_op == COOT_RED_NORM2 ? "__builtin_sqrt(a.hi() + a.lo())" : "(a.hi() + a.lo())";
        s << "    " << (red_dtype == COOT_F64 ? "put_f64" : "put_f32") << "(b.red_out, i, " << val << ");\n";
        s << "}\n";
    }
    std::string body = s.str();
    static const uint64_t prelude_hash = fnv1a(prelude_source());
    std::string name = "coot_batch_" + hex64(fnv1a(body + (has_out ? "o" : "") + std::to_string(out_dtype) + "|" +
                                                   std::to_string(red_dtype)) ^ (prelude_hash * 0x9e3779b97f4a7c15ull));
    const std::string ph = "COOT_KERNEL_NAME";
    for (size_t pos; (pos = body.find(ph)) != std::string::npos;) body.replace(pos, ph.size(), name);
    if (name_out) *name_out = name;
    return body;
}

std::string kernel_source(const Plan& p, const LaunchCfg& cfg, std::string* name_out, std::string* sig_out)
{
    std::ostringstream body;
    const bool need_eval = !p.product_form;
    body << "// tree: " << p.body_sig << "\n";
    if (need_eval || p.red_op < 0) body << emit_eval(p, false);
    if (p.product_form) body << emit_eval(p, true);
    static const char* kname[] = {"ewf", "ewt", "redf", "redt", "col", "colt", "row"};
    std::string placeholder = "COOT_KERNEL_NAME";
    switch (p.kind) {
    case K_EW_FLAT:
    case K_RED_FLAT: body << emit_flat(p, cfg, placeholder); break;
    case K_EW_TILED:
    case K_RED_TILED: body << (p.thin_k ? emit_thin(p, placeholder) : emit_tiled(p, placeholder)); break;
    case K_RED_COL: body << emit_col(p, cfg, placeholder); break;
    case K_RED_COLT: body << emit_colt(p, placeholder); break;
    case K_RED_ROW: body << emit_row(p, placeholder); break;
    }
    std::ostringstream key;
    key << "kind" << p.kind << "|ve" << p.ve << "|ept" << cfg.ept << "|out" << p.out_dtype << "|red" << p.red_op
        << "|pw" << p.pairwise << "|" << body.str();
    std::string sig = key.str();
    // the name hashes the whole kernel text (prelude included): any change to
    // the generated code gives the kernel a new name
    static const uint64_t prelude_hash = fnv1a(prelude_source());
    std::string name = std::string("coot_") + kname[p.kind] + "_" + hex64(fnv1a(sig) ^ (prelude_hash * 0x9e3779b97f4a7c15ull));
    std::string b = body.str();
    for (size_t pos; (pos = b.find(placeholder)) != std::string::npos;) b.replace(pos, placeholder.size(), name);
    if (name_out) *name_out = name;
    if (sig_out) *sig_out = sig;
    return b;
}

}  // namespace coot
