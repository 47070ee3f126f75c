/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, unfused FP64 evaluation of element-wise expression trees and of
 * the reductions they feed.  Only the test suite, the smoke check and the CPU
 * baseline of the benchmark may load this file's library; the product path
 * never does.  It shares no code, header or table with the GPU library.
 *
 * What it follows (Bandicoot paper, arXiv:2308.03120):
 *   - storage: column by column (Section 2, Table 1, element access "(i)");
 *   - element-wise operators A+k, k-A, A*k, A+B, A-B, A%B, A/B (Table 2);
 *   - trans, exp, log, sqrt, abs (Table 7 "trans", "misc");
 *   - accu, dot, norm with p = 1, 2, "inf", "-inf", "fro" (Table 5);
 *   - sum/min/max along dim 0 (per column) and dim 1 (per row) (Table 6);
 *   - relational expressions A < x, A > B ... giving 1 or 0 per element, and
 *     all / any / the count of nonzero elements over them (Table 5; the
 *     counting example of Section 3);
 *   - mean, var and stddev over all elements or along a dim (Table 6);
 *   - the misc and trig element-wise functions (Table 7: pow, log10,
 *     square, cos, sin, tan, acos, asin, atan, ...);
 *   - delayed evaluation by post-order "apply" of each node into a temporary
 *     (Section 7: unwrap<T1> calls op_type::apply recursively);
 *   - type conversion as an explicit node (Section 7: mtOp / mtop_conv_to).
 * Readings where the paper is silent (index ties, NaN, empty input, the
 * compute precision of 16-bit storage, scalar rounding) are listed in the
 * design notes; each is repeated next to the code that implements it.
 *
 * Two evaluation modes:
 *   EXACT : every node in FP64 (the reference value);
 *   EMU   : every node computed in FP64 and then rounded to the node's compute
 *           precision (FP32 for F32/F16/BF16 data, FP64 for F64 data).  For +,
 *           -, *, / and sqrt this equals the IEEE single-precision result
 *           (double rounding is innocuous since 53 >= 2*24+2).
 *
 * Sums use Sum2 and dot products Dot2 (Ogita, Rump, Oishi, "Accurate sum and
 * dot product", SIAM J. Sci. Comput. 26(6), 2005): TwoSum (Knuth) and
 * TwoProduct through a correctly rounded fma().
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- operation codes (the oracle's own numbering) ---------------------- */
enum {
    OR_LEAF = 0,
    OR_PLUS, OR_MINUS, OR_SCHUR, OR_DIV,
    OR_SCAL_PLUS, OR_SCAL_MINUS_POST, OR_SCAL_MINUS_PRE, OR_SCAL_TIMES,
    OR_SCAL_DIV_POST, OR_SCAL_DIV_PRE,
    OR_EXP, OR_LOG, OR_SQRT, OR_ABS, OR_TRANS, OR_CONV,
    OR_GT, OR_LT, OR_GE, OR_LE, OR_EQ, OR_NE,                         /* a ? b */
    OR_SCAL_GT, OR_SCAL_LT, OR_SCAL_GE, OR_SCAL_LE, OR_SCAL_EQ, OR_SCAL_NE,  /* a ? k */
    OR_SCAL_POW,                                                        /* a^k */
    OR_LOG10, OR_LOG2, OR_EXP2, OR_SQUARE, OR_FLOOR, OR_CEIL, OR_ROUND, OR_TRUNC, OR_SIGN,
    OR_COS, OR_SIN, OR_TAN, OR_ACOS, OR_ASIN, OR_ATAN, OR_COSH, OR_SINH, OR_TANH,
    OR_NOPS
};

enum { TY_F32 = 0, TY_F64 = 1, TY_F16 = 2, TY_BF16 = 3, TY_I32 = 5, TY_U32 = 6 };

enum { MODE_EXACT = 0, MODE_EMU = 1 };

enum {
    RD_ACCU = 0, RD_SUM, RD_DOT, RD_NORM1, RD_NORM2, RD_NORMINF, RD_NORMNEGINF,
    RD_MIN, RD_MAX, RD_INDEX_MIN, RD_INDEX_MAX,
    RD_MEAN, RD_VAR, RD_STDDEV, RD_COUNT, RD_ALL, RD_ANY
};

/* error codes */
enum { OK = 0, E_TREE = -1, E_SHAPE = -2, E_EMPTY = -5, E_NOMEM = -9 };

typedef struct {
    int32_t op, a, b, pad;
    double k;
} or_node;

typedef struct {
    const void* data;
    int64_t rows, cols, ld;
    int32_t dtype, pad;
} or_leaf;

/* ---- storage widening (exact) ------------------------------------------ */
/* IEEE binary16: 1 sign, 5 exponent (bias 15), 10 fraction bits. */
static double widen_f16(uint16_t h)
{
    int s = (h >> 15) & 1, e = (h >> 10) & 31, f = h & 1023;
    double v;
    if (e == 0)
        v = ldexp((double)f, -24);                 /* zero or subnormal */
    else if (e == 31)
        v = f ? NAN : INFINITY;
    else
        v = ldexp((double)(1024 + f), e - 25);     /* (1 + f/1024) * 2^(e-15) */
    return s ? -v : v;
}

/* bfloat16: the upper 16 bits of an IEEE binary32. */
static double widen_bf16(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double leaf_at(const or_leaf* L, int64_t r, int64_t c)
{
    int64_t off = r + c * L->ld;
    switch (L->dtype) {
    case TY_F32: return (double)((const float*)L->data)[off];
    case TY_F64: return ((const double*)L->data)[off];
    case TY_F16: return widen_f16(((const uint16_t*)L->data)[off]);
    case TY_BF16: return widen_bf16(((const uint16_t*)L->data)[off]);
    case TY_I32: return (double)((const int32_t*)L->data)[off];   /* exact in FP64 */
    case TY_U32: return (double)((const uint32_t*)L->data)[off];
    }
    return NAN;
}

/* ---- conversion to a 32-bit integer type (reading of the paper's integer
 * matrices: a value is converted by dropping its fraction (toward zero), then
 * clamping to the type's range; NaN becomes 0).  lo and hi are the range
 * ends, both exact in FP64. */
static double to_integer(double x, double lo, double hi)
{
    if (isnan(x)) return 0.0;
    double t = trunc(x);
    if (t < lo) return lo;
    if (t > hi) return hi;
    return t;
}

/* ---- rounding to a storage type (round to nearest, ties to even) ------- */
/* Generic binary format with `fbits` fraction bits, minimum normal exponent
 * `emin` and maximum finite value `maxf`.  x/q is an exact power-of-two
 * scaling, nearbyint() rounds ties to even in the default rounding mode. */
static double round_format(double x, int fbits, int emin, double maxf)
{
    if (isnan(x) || isinf(x) || x == 0.0) return x;
    double ax = fabs(x);
    int e2;
    frexp(ax, &e2);          /* ax in [2^(e2-1), 2^e2) */
    int E = e2 - 1;
    if (E < emin) E = emin;  /* subnormal range keeps the minimum quantum */
    double q = ldexp(1.0, E - fbits);
    double r = nearbyint(ax / q) * q;
    if (r > maxf) r = INFINITY;
    return copysign(r, x);
}

double oracle_round_to(int dtype, double x)
{
    switch (dtype) {
    case TY_F64: return x;
    case TY_F32: return (double)(float)x;
    case TY_F16: return round_format(x, 10, -14, 65504.0);
    case TY_BF16: return round_format(x, 7, -126, ldexp(255.0, 120));  /* (2 - 2^-7) * 2^127 */
    case TY_I32: return to_integer(x, -2147483648.0, 2147483647.0);
    case TY_U32: return to_integer(x, 0.0, 4294967295.0);
    }
    return NAN;
}

double oracle_widen16(int dtype, uint16_t bits)
{
    return dtype == TY_F16 ? widen_f16(bits) : widen_bf16(bits);
}

/* ---- tree structure ---------------------------------------------------- */
static int is_binary(int op) { return (op >= OR_PLUS && op <= OR_DIV) || (op >= OR_GT && op <= OR_NE); }
static int is_scalar(int op)
{
    return (op >= OR_SCAL_PLUS && op <= OR_SCAL_DIV_PRE) || (op >= OR_SCAL_GT && op <= OR_SCAL_POW);
}
static int is_relational(int op) { return op >= OR_GT && op <= OR_SCAL_NE; }

typedef struct {
    int64_t rows, cols;
    int prec;        /* 32 or 64: compute precision of the node's value */
} node_info;

/* Shape and precision of every node.  Returns OK or an error code.
 * Precision rule (reading): F64 leaves compute in FP64; F32, F16 and BF16
 * leaves compute in FP32 (16-bit storage is widened exactly); I32 and U32
 * leaves widen exactly to FP64 and compute there.  A binary node
 * needs equal shapes and equal precision (Armadillo/Bandicoot need the same
 * element type on both sides; 16-bit and F32 data share FP32).  conv(t)
 * rounds to t and continues in FP64 if t is F64, else in FP32. */
static int infer(const or_node* nd, int nn, const or_leaf* lv, int nl, node_info* info)
{
    if (nn <= 0) return E_TREE;
    for (int i = 0; i < nn; ++i) {
        int op = nd[i].op;
        if (op == OR_LEAF) {
            if (nd[i].a < 0 || nd[i].a >= nl) return E_TREE;
            const or_leaf* L = &lv[nd[i].a];
            info[i].rows = L->rows;
            info[i].cols = L->cols;
            /* 32-bit integers widen exactly to FP64 and compute there */
            info[i].prec = (L->dtype == TY_F64 || L->dtype == TY_I32 || L->dtype == TY_U32) ? 64 : 32;
            continue;
        }
        if (op < 0 || op >= OR_NOPS) return E_TREE;
        if (nd[i].a < 0 || nd[i].a >= i) return E_TREE;
        node_info A = info[nd[i].a];
        if (is_binary(op)) {
            if (nd[i].b < 0 || nd[i].b >= i) return E_TREE;
            node_info B = info[nd[i].b];
            if (A.rows != B.rows || A.cols != B.cols) return E_SHAPE;
            if (A.prec != B.prec) return E_TREE;
            info[i] = A;
        } else if (op == OR_TRANS) {
            info[i].rows = A.cols;
            info[i].cols = A.rows;
            info[i].prec = A.prec;
        } else if (op == OR_CONV) {
            if (nd[i].b < 0 || nd[i].b > TY_U32 || nd[i].b == 4) return E_TREE;
            info[i] = A;
            info[i].prec = (nd[i].b == TY_F64 || nd[i].b == TY_I32 || nd[i].b == TY_U32) ? 64 : 32;
        } else {
            info[i] = A;
        }
    }
    return OK;
}

/* value of an element-wise node from its operand values (FP64 arithmetic) */
static double apply_op(int op, double a, double b, double k)
{
    switch (op) {
    case OR_PLUS: return a + b;
    case OR_MINUS: return a - b;
    case OR_SCHUR: return a * b;
    case OR_DIV: return a / b;
    case OR_SCAL_PLUS: return a + k;
    case OR_SCAL_MINUS_POST: return a - k;
    case OR_SCAL_MINUS_PRE: return k - a;
    case OR_SCAL_TIMES: return a * k;
    case OR_SCAL_DIV_POST: return a / k;
    case OR_SCAL_DIV_PRE: return k / a;
    case OR_EXP: return exp(a);
    case OR_LOG: return log(a);
    case OR_SQRT: return sqrt(a);
    case OR_ABS: return fabs(a);
    /* relational: 1 where the comparison holds, else 0; IEEE comparisons, so
     * a NaN operand gives 0, except for != which gives 1 */
    case OR_GT: return a > b ? 1.0 : 0.0;
    case OR_LT: return a < b ? 1.0 : 0.0;
    case OR_GE: return a >= b ? 1.0 : 0.0;
    case OR_LE: return a <= b ? 1.0 : 0.0;
    case OR_EQ: return a == b ? 1.0 : 0.0;
    case OR_NE: return a != b ? 1.0 : 0.0;
    case OR_SCAL_GT: return a > k ? 1.0 : 0.0;
    case OR_SCAL_LT: return a < k ? 1.0 : 0.0;
    case OR_SCAL_GE: return a >= k ? 1.0 : 0.0;
    case OR_SCAL_LE: return a <= k ? 1.0 : 0.0;
    case OR_SCAL_EQ: return a == k ? 1.0 : 0.0;
    case OR_SCAL_NE: return a != k ? 1.0 : 0.0;
    case OR_SCAL_POW: return pow(a, k);
    case OR_LOG10: return log10(a);
    case OR_LOG2: return log2(a);
    case OR_EXP2: return exp2(a);
    case OR_SQUARE: return a * a;
    case OR_FLOOR: return floor(a);
    case OR_CEIL: return ceil(a);
    case OR_ROUND: return round(a);   /* halfway cases away from zero */
    case OR_TRUNC: return trunc(a);
    /* sign: 1 for positive, -1 for negative; zeros and NaN are returned as they are */
    case OR_SIGN: return a > 0.0 ? 1.0 : (a < 0.0 ? -1.0 : a);
    case OR_COS: return cos(a);
    case OR_SIN: return sin(a);
    case OR_TAN: return tan(a);
    case OR_ACOS: return acos(a);
    case OR_ASIN: return asin(a);
    case OR_ATAN: return atan(a);
    case OR_COSH: return cosh(a);
    case OR_SINH: return sinh(a);
    case OR_TANH: return tanh(a);
    }
    return NAN;
}

static double to_prec(double v, int prec, int mode)
{
    return (mode == MODE_EMU && prec == 32) ? (double)(float)v : v;
}

/* The scalar k of a node is the user's literal converted once to the
 * element type of the expression (Armadillo converts the scalar to eT). */
static double scalar_of(const or_node* n, int prec)
{
    return prec == 32 ? (double)(float)n->k : n->k;
}

/* Running-error scale S of an element-wise node from its operand values a, b
 * (FP64) and their scales sa, sb: the first-order magnitude of the
 * expression evaluated on absolute values, with each unary function's
 * derivative (Higham, "Accuracy and Stability of Numerical Algorithms",
 * 2nd ed., Section 3.1).  A leaf's scale is |x|; trans and conv keep their
 * child's. */
static double scale_op(int op, double a, double b, double k, double sa, double sb)
{
    switch (op) {
    case OR_PLUS: case OR_MINUS: return sa + sb;
    case OR_SCHUR: return sa * sb;
    case OR_DIV: return (sa + fabs(a) * sb / fabs(b)) / fabs(b);
    case OR_SCAL_PLUS: case OR_SCAL_MINUS_POST: case OR_SCAL_MINUS_PRE: return sa + fabs(k);
    case OR_SCAL_TIMES: return fabs(k) * sa;
    case OR_SCAL_DIV_POST: return sa / fabs(k);
    case OR_SCAL_DIV_PRE: return fabs(k) * sa / (a * a);
    case OR_ABS: return sa;
    case OR_SQRT: return sqrt(fabs(a)) + sa / (2.0 * sqrt(fabs(a)));
    case OR_EXP: return exp(a) * (1.0 + sa);
    case OR_LOG: return fabs(log(a)) + sa / fabs(a);
    /* first-order: |f(a)| + |f'(a)| S(a); functions that jump
     * (floor ... sign) may move by a whole step */
    case OR_SCAL_POW: return fabs(pow(a, k)) * (1.0 + fabs(k) * sa / fabs(a));
    case OR_LOG10: return fabs(log10(a)) + sa / (fabs(a) * log(10.0));
    case OR_LOG2: return fabs(log2(a)) + sa / (fabs(a) * log(2.0));
    case OR_EXP2: return exp2(a) * (1.0 + sa * log(2.0));
    case OR_SQUARE: return sa * sa;
    case OR_FLOOR: case OR_CEIL: case OR_ROUND: case OR_TRUNC: return sa + 1.0;
    case OR_SIGN: return 1.0;
    case OR_COS: case OR_SIN: return 1.0 + sa;
    case OR_TAN: return fabs(tan(a)) + sa * (1.0 + tan(a) * tan(a));
    case OR_ACOS: case OR_ASIN: return fabs(apply_op(op, a, 0.0, 0.0)) + sa / sqrt(fabs(1.0 - a * a));
    case OR_ATAN: return fabs(atan(a)) + sa / (1.0 + a * a);
    case OR_COSH: case OR_SINH: return cosh(a) * (1.0 + sa);
    case OR_TANH: return fabs(tanh(a)) + sa;
    }
    /* relational: the result is exact for the operands it is given; its
     * magnitude is at most 1 */
    return is_relational(op) ? 1.0 : 0.0;
}

/* ---- unfused evaluation: one temporary per node ------------------------ */
/*
 * Evaluates the whole tree into `out` (root shape, column-major, ld = rows).
 * If `scale` is non-null it also receives the running-error magnitude S of
 * every root element (first-order error scale: evaluate the same tree on
 * absolute values with the derivative of each unary function; Higham,
 * "Accuracy and Stability of Numerical Algorithms", 2nd ed., Section 3.1).
 */
int oracle_eval(const or_node* nd, int nn, const or_leaf* lv, int nl, int mode,
                double* out, double* scale, int64_t* out_rows, int64_t* out_cols)
{
    node_info* info = (node_info*)calloc((size_t)nn, sizeof(node_info));
    if (!info) return E_NOMEM;
    int rc = infer(nd, nn, lv, nl, info);
    if (rc != OK) { free(info); return rc; }

    double** val = (double**)calloc((size_t)nn, sizeof(double*));
    double** sc = (double**)calloc((size_t)nn, sizeof(double*));
    if (!val || !sc) { free(info); free(val); free(sc); return E_NOMEM; }

    for (int i = 0; i < nn && rc == OK; ++i) {
        int64_t R = info[i].rows, C = info[i].cols, n = R * C;
        val[i] = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
        sc[i] = scale ? (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double)) : NULL;
        if (!val[i] || (scale && !sc[i])) { rc = E_NOMEM; break; }
        const or_node* N = &nd[i];
        int prec = info[i].prec;
        for (int64_t c = 0; c < C; ++c)
            for (int64_t r = 0; r < R; ++r) {
                int64_t j = r + c * R;
                double v, s = 0.0;
                if (N->op == OR_LEAF) {
                    v = leaf_at(&lv[N->a], r, c);
                    s = fabs(v);
                } else if (N->op == OR_TRANS) {
                    int64_t jc = c + r * info[N->a].rows;   /* child element (c, r) */
                    v = val[N->a][jc];
                    if (scale) s = sc[N->a][jc];
                } else if (N->op == OR_CONV) {
                    v = oracle_round_to(N->b, val[N->a][j]);
                    if (scale) s = sc[N->a][j];
                } else {
                    double a = val[N->a][j];
                    double b = is_binary(N->op) ? val[N->b][j] : 0.0;
                    double k = is_scalar(N->op) ? scalar_of(N, prec) : 0.0;
                    v = to_prec(apply_op(N->op, a, b, k), prec, mode);
                    if (scale) {
                        double sa = sc[N->a][j], sb = is_binary(N->op) ? sc[N->b][j] : 0.0;
                        s = scale_op(N->op, a, b, k, sa, sb);
                    }
                }
                val[i][j] = v;
                if (scale) sc[i][j] = s;
            }
    }
    if (rc == OK) {
        int root = nn - 1;
        int64_t n = info[root].rows * info[root].cols;
        memcpy(out, val[root], (size_t)n * sizeof(double));
        if (scale) memcpy(scale, sc[root], (size_t)n * sizeof(double));
        if (out_rows) *out_rows = info[root].rows;
        if (out_cols) *out_cols = info[root].cols;
    }
    for (int i = 0; i < nn; ++i) { free(val[i]); if (sc) free(sc[i]); }
    free(val); free(sc); free(info);
    return rc;
}

/* Shape and precision of the root without evaluating anything. */
int oracle_shape(const or_node* nd, int nn, const or_leaf* lv, int nl,
                 int64_t* rows, int64_t* cols, int32_t* prec)
{
    node_info* info = (node_info*)calloc((size_t)nn, sizeof(node_info));
    if (!info) return E_NOMEM;
    int rc = infer(nd, nn, lv, nl, info);
    if (rc == OK) {
        *rows = info[nn - 1].rows;
        *cols = info[nn - 1].cols;
        *prec = info[nn - 1].prec;
    }
    free(info);
    return rc;
}

/* ---- pointwise evaluation: recursion on one output element ------------- */
/* Independent second evaluator used to check sampled outputs of very large
 * workloads without materialising temporaries. */
static double point(const or_node* nd, const node_info* info, const or_leaf* lv, int i,
                    int64_t r, int64_t c, int mode, double* s)
{
    const or_node* N = &nd[i];
    if (N->op == OR_LEAF) {
        double v = leaf_at(&lv[N->a], r, c);
        if (s) *s = fabs(v);
        return v;
    }
    if (N->op == OR_TRANS) return point(nd, info, lv, N->a, c, r, mode, s);
    double sa = 0.0, sb = 0.0;
    double a = point(nd, info, lv, N->a, r, c, mode, s ? &sa : NULL);
    if (N->op == OR_CONV) {
        if (s) *s = sa;
        return oracle_round_to(N->b, a);
    }
    double b = is_binary(N->op) ? point(nd, info, lv, N->b, r, c, mode, s ? &sb : NULL) : 0.0;
    double k = is_scalar(N->op) ? scalar_of(N, info[i].prec) : 0.0;
    if (s) *s = scale_op(N->op, a, b, k, sa, sb);
    return to_prec(apply_op(N->op, a, b, k), info[i].prec, mode);
}

/* Values (and, if `scale` is not NULL, running-error scales) of the root at
 * the column-major linear indices lin[0..m). */
int oracle_eval_at(const or_node* nd, int nn, const or_leaf* lv, int nl, int mode,
                   const int64_t* lin, int64_t m, double* out, double* scale)
{
    node_info* info = (node_info*)calloc((size_t)nn, sizeof(node_info));
    if (!info) return E_NOMEM;
    int rc = infer(nd, nn, lv, nl, info);
    if (rc == OK) {
        int64_t R = info[nn - 1].rows;
        for (int64_t t = 0; t < m; ++t)
            out[t] = point(nd, info, lv, nn - 1, lin[t] % R, lin[t] / R, mode, scale ? &scale[t] : NULL);
    }
    free(info);
    return rc;
}

/* ---- accurate summation ------------------------------------------------ */
typedef struct { double p, s; } acc2;   /* Sum2/Dot2 state: value p, error sum s */

static void two_sum(double a, double b, double* x, double* y)
{
    *x = a + b;
    double z = *x - a;
    *y = (a - (*x - z)) + (b - z);
}

static void two_product(double a, double b, double* x, double* y)
{
    *x = a * b;
    *y = fma(a, b, -*x);
}

static void acc_add(acc2* A, double x)
{
    double q;
    two_sum(A->p, x, &A->p, &q);
    A->s += q;
}

static void acc_add_product(acc2* A, double a, double b)
{
    double h, r, q;
    two_product(a, b, &h, &r);
    two_sum(A->p, h, &A->p, &q);
    A->s += q + r;
}

static double acc_value(const acc2* A) { return A->p + A->s; }

/* Sum2 of a plain array (used to pin the summation on its own) */
double oracle_sum2(const double* x, int64_t n, double* abs_sum)
{
    acc2 A = {0.0, 0.0};
    acc2 B = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) { acc_add(&A, x[i]); acc_add(&B, fabs(x[i])); }
    if (abs_sum) *abs_sum = acc_value(&B);
    return acc_value(&A);
}

double oracle_dot2(const double* x, const double* y, int64_t n)
{
    acc2 A = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) acc_add_product(&A, x[i], y[i]);
    return acc_value(&A);
}

/* ---- reductions -------------------------------------------------------- */
/*
 * reduce(op, dim, tree):
 *   dim = -1 : over all elements (column-major linear order);
 *   dim =  0 : one result per column (output 1 x n_cols);
 *   dim =  1 : one result per row    (output n_rows x 1).
 * The tree is evaluated in `mode`: EXACT gives the reference value of the
 * expression; EMU gives the values the method itself produces per element
 * (rounded at every node), whose accurate sum isolates the error of the
 * summation from the error of the element-wise tree.  Sums (accu, sum, dot,
 * norm1, norm2/fro) use Sum2/Dot2.  For a tree whose root is an element-wise
 * product the sum is a dot product of the two children (Dot2), so no rounding
 * of the products enters the reference.  Selections (min, max, the norms
 * "inf" and "-inf", index_min, index_max) keep the lowest column-major index
 * among equal values; NaN values are skipped; if
 * every value is NaN the value is NaN and the index 0.  Empty input: sums
 * give 0, selections return E_EMPTY.
 *
 * Outputs: vals[k] (result k), idx[k] (index for selections; linear index
 * for dim = -1, row index for dim = 0, column index for dim = 1), and
 * abs_sum[k] = sum of |terms| (the scale of a sum; for dot the |products|).
 */
static int is_sum_like(int op)
{
    return op == RD_ACCU || op == RD_SUM || op == RD_DOT || op == RD_NORM1 || op == RD_NORM2;
}

/* selections have no value on an empty input */
static int is_selection(int op)
{
    return op == RD_MIN || op == RD_MAX || op == RD_INDEX_MIN || op == RD_INDEX_MAX || op == RD_NORMINF ||
           op == RD_NORMNEGINF;
}

int oracle_reduce(int rop, int dim, const or_node* nd, int nn, const or_leaf* lv, int nl,
                  int mode, double* vals, int64_t* idx, double* abs_sum)
{
    int64_t R, C;
    int32_t prec;
    int rc = oracle_shape(nd, nn, lv, nl, &R, &C, &prec);
    if (rc != OK) return rc;
    int root = nn - 1;
    int dot_form = is_sum_like(rop) && rop != RD_NORM1 && rop != RD_NORM2 && nd[root].op == OR_SCHUR;
    if (rop == RD_DOT && !dot_form) return E_TREE;
    int64_t n = R * C;
    if (n == 0 && is_selection(rop)) return E_EMPTY;

    double *va = NULL, *vb = NULL;
    if (dot_form) {
        /* children of the product, each evaluated as its own tree */
        int64_t r2, c2;
        va = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
        vb = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
        if (!va || !vb) { free(va); free(vb); return E_NOMEM; }
        rc = oracle_eval(nd, nd[root].a + 1, lv, nl, mode, va, NULL, &r2, &c2);
        /* the prefix ending at a child is a tree whose root is that child */
        if (rc == OK) rc = oracle_eval(nd, nd[root].b + 1, lv, nl, mode, vb, NULL, &r2, &c2);
    } else {
        va = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
        if (!va) return E_NOMEM;
        rc = oracle_eval(nd, nn, lv, nl, mode, va, NULL, NULL, NULL);
    }
    if (rc != OK) { free(va); free(vb); return rc; }

    int64_t n_out = dim < 0 ? 1 : (dim == 0 ? C : R);
    int64_t len = dim < 0 ? n : (dim == 0 ? R : C);
    for (int64_t o = 0; o < n_out; ++o) {
        acc2 S = {0.0, 0.0}, Sa = {0.0, 0.0};
        double best = NAN;
        int64_t besti = -1;
        for (int64_t t = 0; t < len; ++t) {
            int64_t j = dim < 0 ? t : (dim == 0 ? t + o * R : o + t * R);
            double v = va[j];
            if (rop == RD_MEAN || rop == RD_VAR || rop == RD_STDDEV) {
                acc_add(&S, v);
                acc_add(&Sa, fabs(v));
                continue;
            }
            if (rop == RD_COUNT || rop == RD_ALL || rop == RD_ANY) continue;
            if (is_sum_like(rop)) {
                if (dot_form) {
                    acc_add_product(&S, v, vb[j]);
                    acc_add(&Sa, fabs(v * vb[j]));
                } else if (rop == RD_NORM2) {
                    acc_add_product(&S, v, v);
                    acc_add(&Sa, v * v);
                } else if (rop == RD_NORM1) {
                    acc_add(&S, fabs(v));
                    acc_add(&Sa, fabs(v));
                } else {
                    acc_add(&S, v);
                    acc_add(&Sa, fabs(v));
                }
                continue;
            }
            if (rop == RD_NORMINF || rop == RD_NORMNEGINF) v = fabs(v);
            if (isnan(v)) continue;
            int take;
            if (besti < 0) take = 1;
            else if (rop == RD_MAX || rop == RD_INDEX_MAX || rop == RD_NORMINF) take = v > best;
            else take = v < best;   /* ties keep the earlier (lower) index */
            if (take) { best = v; besti = t; }
        }
        if (is_sum_like(rop)) {
            double s = acc_value(&S);
            vals[o] = rop == RD_NORM2 ? sqrt(s) : s;
            if (idx) idx[o] = 0;
            if (abs_sum) abs_sum[o] = acc_value(&Sa);
        } else if (rop == RD_MEAN || rop == RD_VAR || rop == RD_STDDEV) {
            /* two passes: the mean (compensated sum / count), then the sum of
             * squared deviations from it; var divides by count - 1 (the
             * unbiased estimate); one element gives 0, none gives NaN */
            double mean = len > 0 ? acc_value(&S) / (double)len : NAN;
            if (rop == RD_MEAN) {
                vals[o] = mean;
                if (abs_sum) abs_sum[o] = len > 0 ? acc_value(&Sa) / (double)len : 0.0;
            } else {
                acc2 M = {0.0, 0.0};
                for (int64_t t = 0; t < len; ++t) {
                    int64_t j = dim < 0 ? t : (dim == 0 ? t + o * R : o + t * R);
                    double d = va[j] - mean;
                    acc_add_product(&M, d, d);
                }
                double m2 = acc_value(&M);
                double var = len > 1 ? m2 / (double)(len - 1) : (len == 1 ? 0.0 : NAN);
                vals[o] = rop == RD_STDDEV ? sqrt(var) : var;
                if (abs_sum) abs_sum[o] = m2;
            }
            if (idx) idx[o] = 0;
        } else if (rop == RD_COUNT || rop == RD_ALL || rop == RD_ANY) {
            /* count of nonzero elements (NaN is nonzero); all: every element
             * nonzero (true for an empty input); any: at least one */
            int64_t cnt = 0;
            for (int64_t t = 0; t < len; ++t) {
                int64_t j = dim < 0 ? t : (dim == 0 ? t + o * R : o + t * R);
                if (va[j] != 0.0) ++cnt;
            }
            int64_t r = rop == RD_COUNT ? cnt : (rop == RD_ALL ? (cnt == len) : (cnt > 0));
            vals[o] = (double)r;
            if (idx) idx[o] = r;
            if (abs_sum) abs_sum[o] = 0.0;
        } else {
            vals[o] = besti < 0 ? NAN : best;
            if (idx) idx[o] = besti < 0 ? 0 : besti;
            if (abs_sum) abs_sum[o] = 0.0;
        }
    }
    free(va);
    free(vb);
    return OK;
}

/* ---- array helpers ----------------------------------------------------- */
void oracle_round_array(int dtype, const double* x, double* y, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) y[i] = oracle_round_to(dtype, x[i]);
}

void oracle_widen16_array(int dtype, const uint16_t* bits, double* y, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) y[i] = oracle_widen16(dtype, bits[i]);
}

int oracle_version(void) { return 1; }
