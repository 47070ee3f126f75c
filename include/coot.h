/*
 * coot.h -- C ABI of libcoot_mi355x.so: fused element-wise expression trees
 * and the reductions they feed, on AMD Instinct MI355X (gfx950).
 *
 * The operations are those of the Bandicoot GPU linear-algebra library
 * (Curtin, Edel, Sanderson, arXiv:2308.03120):
 *   - matrices are stored column by column (Section 2, Table 1: "(i)" accesses
 *     the i-th element "assuming a column-by-column layout");
 *   - element-wise operators A+k, k+A, A-k, k-A, A*k, A+B, A-B, A%B, A/B
 *     (Table 2), plus A/k and k/A;
 *   - trans, exp, log, sqrt (Table 7) and abs;
 *   - conversion of the element type inside an expression (Section 7, mtOp
 *     with mtop_conv_to, and the fused "two-way" conversion kernels);
 *   - accu, dot, norm (Table 5); sum, min, max along a dimension (Table 6);
 *     index_min and index_max;
 *   - delayed evaluation (Section 5 and Section 7: nothing is computed until
 *     an assignment or a scalar-valued function asks for it).  Here the whole
 *     tree is compiled into one kernel per call instead of one kernel per node
 *     with temporaries in between.
 *
 * Memory and streams: every pointer in a coot_operand is device memory owned
 * by the caller (unless COOT_OPERAND_HOST says otherwise); the library never
 * frees it.  The library owns its scratch memory, compiled kernels and plans.
 * Every call that takes a `stream` (a hipStream_t; NULL = the null stream)
 * only enqueues work and returns; results are valid once the stream has
 * reached that point (coot_synchronise).
 *
 * Errors: every int-returning call returns COOT_OK (0) or a negative code;
 * coot_last_error() gives a message for the calling thread.  No C++
 * exception crosses this interface.  Argument errors are detected on the
 * host before any device work is enqueued.
 */
#ifndef COOT_H
#define COOT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes -- */
enum {
    COOT_OK = 0,
    COOT_ERR_BAD_TREE = -1,     /* malformed tree: opcode, child index, arity, scalar */
    COOT_ERR_SHAPE = -2,        /* operand shapes do not agree */
    COOT_ERR_DTYPE = -3,        /* element types do not agree / not allowed here */
    COOT_ERR_ALIAS = -4,        /* output overlaps an operand in a forbidden way */
    COOT_ERR_EMPTY = -5,        /* min/max/index of an empty object */
    COOT_ERR_UNSUPPORTED = -6,  /* valid request the library does not implement */
    COOT_ERR_JIT = -7,          /* run-time kernel compilation failed */
    COOT_ERR_HIP = -8,          /* a HIP runtime call failed */
    COOT_ERR_NOMEM = -9,        /* host or device allocation failed */
    COOT_ERR_ARG = -10,         /* bad argument (null pointer, ld, sizes, flags) */
    COOT_ERR_NOT_INIT = -11,    /* coot_init has not been called */
    COOT_ERR_NOT_READY = -12    /* coot_reduce_noalloc: the call's kernel is not loaded yet */
};

/* -------------------------------------------------------- element types -- */
/* float, double (Section 2: Mat<eT> with eT = float, double), the 16-bit
 * storage types of the roadmap's low-precision item (Section 6), and uword
 * (an unsigned 64-bit integer, Section 2) for index results. */
typedef enum coot_dtype {
    COOT_F32 = 0,
    COOT_F64 = 1,
    COOT_F16 = 2,
    COOT_BF16 = 3,
    COOT_U64 = 4,
    COOT_I32 = 5,   /* 32-bit integers (Section 2 element types): they widen   */
    COOT_U32 = 6    /* exactly to FP64 and trees with them compute in FP64;    */
                    /* a value converted to an integer type (an output or a    */
                    /* conversion node) drops its fraction toward zero, is    */
                    /* clamped to the type's range, and NaN becomes 0          */
} coot_dtype;

/* ------------------------------------------------------------- operands -- */
/* A column-major matrix: element (r, c) lives at ptr + (r + c*ld) elements.
 * ld >= n_rows (ld > n_rows describes a submatrix view, Table 1 ".rows",
 * ".cols", ".submat").  A vector is an n x 1 (Col) or 1 x n (Row) matrix.
 * An object with n_rows*n_cols == 0 is empty; ptr may then be NULL.
 *
 * Views (Table 1 submatrix views) are operands too: .submat(p, q, r, s) is
 * ptr + (p + q*ld) with shape (r-p+1) x (s-q+1) and the parent's ld (.row,
 * .col, .rows, .cols likewise); .diag(k) is a 1 x n operand at ptr + k*ld
 * (k >= 0) or ptr - k (k < 0) whose ld is the parent's ld + 1, so element j
 * is the parent's (j - min(k,0), j + max(k,0)).  A view may be an output.
 *
 * Generators (Table 1 .fill / .ones / .zeros / .eye; Table 4 eye, ones,
 * zeros, linspace) are memory-free input operands: ptr NULL, ld =
 * max(1, n_rows), dtype = the element type the values are stored in, and
 * one COOT_OPERAND_GEN_* flag; gen[] holds the parameters.  Every value is
 * formed in FP64 and stored once (round to nearest even) in dtype, as if
 * read from memory:
 *   GEN_FILL      every element gen[0] (ones: 1, zeros: 0)
 *   GEN_EYE       1 where row == column, else 0 (any shape)
 *   GEN_LINSPACE  a vector (n x 1 or 1 x n, n = n_rows*n_cols elements):
 *                 x_i = gen[0] + i*d, d = (gen[1] - gen[0]) / (n - 1), for
 *                 i < n - 1, and x_{n-1} = gen[1] (n = 1 gives gen[1])
 * Generators are not accepted as outputs nor in batched evaluation. */
#define COOT_OPERAND_HOST 1u           /* outputs only: ptr is host memory (forces a sync) */
#define COOT_OPERAND_GEN_FILL 0x10u    /* inputs only: constant gen[0] */
#define COOT_OPERAND_GEN_EYE 0x20u     /* inputs only: identity pattern */
#define COOT_OPERAND_GEN_LINSPACE 0x40u /* inputs only: gen[0] .. gen[1] */

typedef struct coot_operand {
    void* ptr;
    int64_t n_rows;
    int64_t n_cols;
    int64_t ld;
    int32_t dtype;     /* coot_dtype */
    uint32_t flags;    /* COOT_OPERAND_* */
    double gen[2];     /* generator parameters (GEN_* flags only; else ignored) */
} coot_operand;

/* ---------------------------------------------------------- expressions -- */
/* Node kinds (Section 7: eOp = element-wise unary or scalar node, eGlue =
 * element-wise binary node, Op<.., op_htrans> = transpose, mtOp = conversion). */
enum {
    COOT_LEAF = 0,            /* a = operand slot */
    COOT_PLUS = 1,            /* a + b */
    COOT_MINUS = 2,           /* a - b */
    COOT_SCHUR = 3,           /* a % b (element-wise product) */
    COOT_DIV = 4,             /* a / b (element-wise) */
    COOT_SCAL_PLUS = 10,      /* a + k (= k + a) */
    COOT_SCAL_MINUS_POST = 11,/* a - k */
    COOT_SCAL_MINUS_PRE = 12, /* k - a */
    COOT_SCAL_TIMES = 13,     /* a * k (= k * a) */
    COOT_SCAL_DIV_POST = 14,  /* a / k */
    COOT_SCAL_DIV_PRE = 15,   /* k / a */
    COOT_SCAL_POW = 16,       /* pow(a, k) (Table 7 "misc") */
    COOT_EXP = 20,
    COOT_LOG = 21,
    COOT_SQRT = 22,
    COOT_ABS = 23,
    COOT_TRANS = 30,          /* trans(a): (r, c) -> (c, r) */
    COOT_CONV = 31,           /* conv_to<b>(a): round a to dtype b (coot_dtype) */
    /* relational expressions (Table 5: all(A < x), "other relational
     * expressions"; Section 3: A > 0.3): 1 where the comparison holds, else
     * 0, in the node's compute type.  IEEE comparisons: a NaN operand gives 0,
     * except for != which gives 1. */
    COOT_GT = 40,             /* a > b */
    COOT_LT = 41,             /* a < b */
    COOT_GE = 42,             /* a >= b */
    COOT_LE = 43,             /* a <= b */
    COOT_EQ = 44,             /* a == b */
    COOT_NE = 45,             /* a != b */
    COOT_SCAL_GT = 50,        /* a > k (k < a) */
    COOT_SCAL_LT = 51,        /* a < k (k > a) */
    COOT_SCAL_GE = 52,        /* a >= k */
    COOT_SCAL_LE = 53,        /* a <= k */
    COOT_SCAL_EQ = 54,        /* a == k */
    COOT_SCAL_NE = 55,        /* a != k */
    /* Table 7 "misc" and "trig" functions, in the node's compute type with the
     * device's single- or double-precision math library (correctly rounded:
     * square, floor, ceil, round, trunc, sign).  round: halfway cases away
     * from zero.  sign: 1 for positive, -1 for negative, zeros and NaN
     * returned unchanged. */
    COOT_LOG10 = 60,
    COOT_LOG2 = 61,
    COOT_EXP2 = 62,
    COOT_SQUARE = 63,
    COOT_FLOOR = 64,
    COOT_CEIL = 65,
    COOT_ROUND = 66,
    COOT_TRUNC = 67,
    COOT_SIGN = 68,
    COOT_COS = 70,
    COOT_SIN = 71,
    COOT_TAN = 72,
    COOT_ACOS = 73,
    COOT_ASIN = 74,
    COOT_ATAN = 75,
    COOT_COSH = 76,
    COOT_SINH = 77,
    COOT_TANH = 78
};

/* One node.  `a` and `b` are indices of EARLIER nodes of the same array
 * (post-order), except for COOT_LEAF where `a` is an operand slot.  `b` is
 * -1 for unary and scalar nodes, and the target coot_dtype for COOT_CONV.
 * `k` is the scalar of the SCAL_* nodes, converted once (round to nearest
 * even) to the expression's element type, as a scalar literal is converted
 * to eT in `fmat * 0.75`. */
typedef struct coot_node {
    int32_t op;
    int32_t a;
    int32_t b;
    int32_t reserved;   /* must be 0 */
    double k;
} coot_node;

/* Launch configuration.  ept = 16-byte vectors per thread per step
 * {1,2,4,8}; block = threads per block {64,128,256,512}; split = grid level
 * {1,2,4,8}: 1, 2, 4 give a persistent grid-stride launch of
 * split * (1024 / block) blocks per CU (for reductions: that many partial
 * results), 8 gives one pass with as many blocks as the work needs (at most
 * 16384 partial results for a reduction).  Tiled kernels (transposed reads)
 * have a fixed 256-thread 64x64 tile and use only split.  All zero = let the
 * library choose (default heuristic, tuned cache or the learned cost model,
 * see coot_set_tuning). */
typedef struct coot_config {
    int32_t ept;
    int32_t block;
    int32_t split;
    int32_t reserved;   /* must be 0 */
} coot_config;

#define COOT_EXPR_UNFUSED 1u  /* evaluate one kernel per node with temporaries
                                 (the paper's unwrap/apply evaluation; used as
                                 the baseline the fused form is measured against) */

/* A tree of n_nodes nodes; the last node is the root. */
typedef struct coot_expr {
    const coot_node* nodes;
    int32_t n_nodes;
    uint32_t flags;     /* COOT_EXPR_* */
    coot_config cfg;
} coot_expr;

/* ----------------------------------------------------------- reductions -- */
/* Reductions of the value of a tree (Table 5 accu, dot, norm; Table 6 sum,
 * min, max along dim; index_min / index_max):
 *   COOT_RED_ACCU        sum of all elements
 *   COOT_RED_SUM         sum along dim (dim 0 = per column -> 1 x n_cols,
 *                        dim 1 = per row -> n_rows x 1), or of all if dim = -1
 *   COOT_RED_DOT         the root must be a COOT_SCHUR node; sum of the
 *                        products of its two children (same as ACCU there)
 *   COOT_RED_NORM1/2     sum |x|, sqrt(sum x^2) (NORM2 of a matrix = "fro")
 *   COOT_RED_NORMINF     max |x|;  COOT_RED_NORMNEGINF  min |x|
 *   COOT_RED_MIN/MAX     smallest / largest value (all, or along dim)
 *   COOT_RED_INDEX_MIN/MAX  column-major linear index (all) or row / column
 *                        index (along dim 0 / 1) of the extremum
 * Ties in min/max/index go to the lowest index; NaN values are skipped; an
 * all-NaN input gives NaN and index 0.  Sums of an empty object are 0;
 * min/max/index of an empty object fail with COOT_ERR_EMPTY.
 *
 * Precision: F32, F16 and BF16 data are accumulated in FP32 with Kahan-style
 * compensation (TwoSum at every step, TwoProduct for products); blocks are
 * combined in FP64 in a fixed order, so the result does not depend on timing.
 * OR-ing COOT_RED_PAIRWISE selects plain FP32 accumulation (no compensation)
 * for comparison.  F64 data are accumulated in compensated FP64.
 * The output is 1 x 1 (dim -1) or the per-dim vector, of dtype F32 or F64
 * (values) or U64 (indices), contiguous. */
enum {
    COOT_RED_ACCU = 0,
    COOT_RED_SUM = 1,
    COOT_RED_DOT = 2,
    COOT_RED_NORM1 = 3,
    COOT_RED_NORM2 = 4,
    COOT_RED_NORMINF = 5,
    COOT_RED_NORMNEGINF = 6,
    COOT_RED_MIN = 7,
    COOT_RED_MAX = 8,
    COOT_RED_INDEX_MIN = 9,
    COOT_RED_INDEX_MAX = 10,
    /* statistics (Table 6): mean, and the variance with the unbiased n - 1
     * normalisation and its square root, over all elements (dim -1) or per
     * column (dim 0) / per row (dim 1).  One element gives variance 0, an
     * empty input NaN (also for the mean).  The variance is accumulated in
     * FP64 for every storage type: per thread as sums of deviations from the
     * thread's first element, merged pairwise (Chan, Golub and LeVeque) in a
     * fixed order.  Outputs F32 or F64. */
    COOT_RED_MEAN = 11,
    COOT_RED_VAR = 12,
    COOT_RED_STDDEV = 13,
    /* predicates (Table 5): the number of nonzero elements (NaN counts as
     * nonzero), 1 if all elements are nonzero (also for an empty input),
     * 1 if any is.  Outputs U64.  all(A < x) is COOT_RED_ALL of the tree
     * A < x. */
    COOT_RED_COUNT = 14,
    COOT_RED_ALL = 15,
    COOT_RED_ANY = 16
};
#define COOT_RED_PAIRWISE 0x100

/* ------------------------------------------------------------------ calls -- */
/* coot_init (Section 2, coot_init): select HIP device `device`, query it and
 * prepare the kernel cache.  flags: COOT_PRINT_INFO prints the device name,
 * CU count, clock, HBM size and cache directory to stdout.  Calling it again
 * with the same device is a no-op.  Fails with COOT_ERR_HIP if there is no
 * usable device. */
#define COOT_PRINT_INFO 1u
int coot_init(int device, unsigned flags);

/* Release scratch memory, plans and loaded kernels. */
int coot_finalize(void);

/* out = value of the tree.  `ops` holds n_ops operands (slot i = ops[i]);
 * out must have the root's shape and may be F32, F64, F16 or BF16 (the root
 * value is rounded to it, to nearest even).  out may be the same memory as an
 * operand slot (same ptr, ld, dtype) if that slot is never read transposed:
 * this is the in-place form `B += 3*A` of the paper's Task 2.  Any other
 * overlap fails with COOT_ERR_ALIAS. */
int coot_eval(const coot_expr* expr, const coot_operand* ops, int n_ops,
              const coot_operand* out, void* stream);

/* out = red_op (| COOT_RED_PAIRWISE) of the tree's value along dim
 * (-1 = all elements, 0 = per column, 1 = per row).  If out has
 * COOT_OPERAND_HOST the result is copied to host memory and the call
 * synchronises the stream (the paper's `float r = accu(f)`). */
int coot_reduce(int red_op, int dim, const coot_expr* expr, const coot_operand* ops,
                int n_ops, const coot_operand* out, void* stream);

/* coot_reduce without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments and results as coot_reduce (bit-identical
 * to it for the same call); the block partials live in one static device
 * array of COOT_NOALLOC_SCRATCH_BYTES per GPU (held until the process ends)
 * instead of per-stream memory.  It calls no hipMalloc/hipFree, compiles and
 * loads no kernel, and never synchronises.  Errors beyond coot_reduce's:
 *   COOT_ERR_NOT_INIT   coot_init has not been called on this device;
 *   COOT_ERR_NOT_READY  the kernel of this call is not loaded yet (make the
 *                       same kind of call once through coot_reduce first);
 *   COOT_ERR_ARG        out has COOT_OPERAND_HOST, the call's partials exceed
 *                       COOT_NOALLOC_SCRATCH_BYTES, or it needs a temporary
 *                       (a per-dimension reduction of a tree that reads an
 *                       operand transposed) or the unfused form.
 * The launch configuration is the caller's (expr->cfg), a tuned or an
 * already-predicted one, else the default: the learned model is not run.
 * Every call on one GPU shares the array: calls that overlap on one GPU (two
 * streams, or two host threads) race on it and must be ordered by the caller. */
#define COOT_NOALLOC_SCRATCH_BYTES (16u << 20)
int coot_reduce_noalloc(int red_op, int dim, const coot_expr* expr, const coot_operand* ops, int n_ops,
                        const coot_operand* out, void* stream);

/* Wait for all work enqueued on `stream` (Section 5: coot_synchronise). */
int coot_synchronise(void* stream);

/* Message of the last error on the calling thread ("" if none). */
const char* coot_last_error(void);

/* Host-only checks, usable without a device.  coot_validate runs exactly the
 * argument checks of coot_eval (red_op < 0) or coot_reduce (red_op >= 0).
 * coot_kernel_source writes the HIP source the library would compile for
 * this call into buf (capacity cap, NUL-terminated); it returns the source
 * length or a negative code.  Pointer values are not dereferenced. */
int coot_validate(int red_op, int dim, const coot_expr* expr, const coot_operand* ops,
                  int n_ops, const coot_operand* out);
int64_t coot_kernel_source(int red_op, int dim, const coot_expr* expr, const coot_operand* ops,
                           int n_ops, const coot_operand* out, char* buf, int64_t cap);

/* Compile (without a device) the kernels for this call into the on-disk
 * cache, so that a later run loads them instead of compiling.  Returns the
 * number of kernels compiled (0 if all were cached) or a negative code. */
int coot_precompile(int red_op, int dim, const coot_expr* expr, const coot_operand* ops,
                    int n_ops, const coot_operand* out);

/* Grouped precompilation: between coot_precompile_begin and
 * coot_precompile_end, coot_precompile only records the kernels a call needs;
 * coot_precompile_end compiles them, kernels_per_module to one code object
 * (much cheaper per kernel than one compilation each), and returns how many
 * kernels it compiled.  Host only. */
int coot_precompile_begin(void);
int coot_precompile_end(int kernels_per_module);

/* ------------------------------------------------------ batched evaluation -- */
/* Many matrices, one tree (the roadmap's "collections of matrices",
 * Section 6), evaluated by ONE persistent tile pass (plus, with a reduction,
 * one small per-item combine launch).  For item i the tree
 * reads slot s from leaf_ptrs[i*n_slots + s]; every operand and output of an
 * item is contiguous (ld = its own n_rows); item i's output is
 * shapes[2i] x shapes[2i+1] and each slot's shape follows from the tree (a
 * slot read through trans() has the transposed shape).  If out_ptrs is not
 * NULL, Y_i is stored there in out_dtype.  If red_expr is not NULL, r_i =
 * red_op of red_expr evaluated on Y_i (red_expr's slot 0 is Y_i itself; only
 * the sum-like red_ops ACCU, SUM(dim -1), DOT, NORM1, NORM2 are allowed) is
 * written to red_out[i] (red_dtype F32 or F64).  Each item's value is cut,
 * by its shape alone, into units of at most 16384 elements (fewer when the
 * operands read through trans() are wide: they are staged in 64 KiB of LDS):
 * whole columns where the columns are short, 64-column blocks where they are
 * long, and an item of at most a quarter of that one unit of its own.  One
 * pass runs every unit: a large unit per block, small ones four to a block
 * (one per wave); on the host, items are spread over the XCDs (each with its
 * own L2), largest first, so that the units of an item share one L2.  Each
 * unit leaves a compensated partial, and the combine launch adds an item's
 * partials in unit order in FP64, so r_i depends only on the item's shape and
 * values (deterministic, and the same in any batch).  expr->cfg is ignored.
 * The plan copies the tables to the device and, unless COOT_BATCH_NO_GRAPH is
 * set, captures the launches in a hipGraph that coot_batch_run replays.  The
 * caller keeps every pointer valid while the plan lives.
 *
 * Aliasing: all units of all items may run at once, so an item's output may
 * overlap only its own operand slot s, and only as the in-place form of the
 * single-matrix rule (same first byte, same size, same element type, slot s
 * never read through trans()); any other overlap of an output with an
 * operand, another output or red_out fails with COOT_ERR_ALIAS before
 * anything is allocated or launched. */
typedef struct coot_batch {
    const coot_expr* expr;
    int32_t n_slots;
    int32_t n_items;
    const int32_t* slot_dtypes;   /* n_slots coot_dtype */
    void* const* leaf_ptrs;       /* n_items * n_slots device pointers */
    void* const* out_ptrs;        /* n_items device pointers, or NULL */
    int32_t out_dtype;
    int32_t red_op;               /* used only if red_expr != NULL */
    const int64_t* shapes;        /* n_items * 2: rows, cols of Y_i */
    const coot_expr* red_expr;
    void* red_out;                /* device array of n_items values */
    int32_t red_dtype;
    uint32_t flags;               /* COOT_BATCH_* */
} coot_batch;

#define COOT_BATCH_NO_GRAPH 1u     /* launch directly instead of through a graph */
#define COOT_BATCH_PER_ITEM 2u     /* baseline: per item, the fused single-matrix calls
                                      (coot_eval of the tree, coot_reduce of red_expr) */
#define COOT_BATCH_UNFUSED 4u      /* baseline: per item, one launch per node (COOT_EXPR_UNFUSED) */

typedef struct coot_batch_plan coot_batch_plan;

int coot_batch_create(const coot_batch* batch, void* stream, coot_batch_plan** plan);
int coot_batch_run(coot_batch_plan* plan, void* stream);
/* Host only: the HIP source coot_batch_create would compile for this batch
 * (prelude included) into buf (capacity cap, NUL-terminated); returns the
 * source length or a negative code.  Pointers in the batch are not read. */
int64_t coot_batch_kernel_source(const coot_batch* batch, char* buf, int64_t cap);
int coot_batch_destroy(coot_batch_plan* plan);

/* One call for a batch (Section 6, collections of matrices; Section 3, small
 * matrices use a GPU poorly): the first call with a descriptor builds its plan
 * (coot_batch_create), later calls with a descriptor of identical contents
 * (trees, dtypes, shapes, every pointer, flags) replay the plan's graph on
 * `stream` (coot_batch_run).  The library keeps the plans of the 16 most
 * recently used descriptors and frees them in coot_finalize; the caller keeps
 * the memory a descriptor names valid while its plan may be replayed.  Errors
 * and aliasing rules are those of coot_batch_create and coot_batch_run;
 * dropping the oldest plan synchronises the device. */
int coot_eval_batched(const coot_batch* batch, void* stream);

/* ---------------------------------------------- launch-configuration choice -- */
/* The configuration space: 64 configurations, index
 * cfg = ept_i*16 + block_i*4 + split_i with ept = 1<<ept_i, block = 64<<block_i,
 * split = 1<<split_i. */
#define COOT_N_CONFIGS 64
int coot_config_of(int index, coot_config* cfg);

/* Tuning mode for calls whose expr->cfg is all zero:
 *   COOT_TUNE_DEFAULT  fixed heuristic;
 *   COOT_TUNE_CACHE    best configuration measured by coot_autotune for the
 *                      same kernel signature and size class, else default;
 *   COOT_TUNE_MODEL    the learned cost model loaded from model_path (or set
 *                      by coot_model_set), with the tuned cache taking
 *                      precedence and the default as the fallback. */
enum { COOT_TUNE_DEFAULT = 0, COOT_TUNE_CACHE = 1, COOT_TUNE_MODEL = 2 };
/* A model file (model_path) holds the 8 bytes "COOTMLP2", the feature schema
 * (uint32, COOT_FEATURE_SCHEMA), a zero uint32, the kernel stamp it was
 * trained on (uint64, coot_kernel_stamp), then COOT_MLP_N_PARAMS + 64 FP32
 * values (parameters, feature means, feature standard deviations).  A file
 * with another layout, schema or stamp is rejected with COOT_ERR_ARG and a
 * message; tuning then falls back to COOT_TUNE_CACHE (the tuned cache, then
 * the default) and no model stays installed. */
int coot_set_tuning(int mode, const char* model_path);

/* Identity of what the 64 configurations run, for cost-model files: a hash
 * over the device prelude and, for a fixed set of calls covering every kernel
 * kind, the generated source and launch geometry of each configuration.
 * Writes it to *stamp and returns COOT_FEATURE_SCHEMA, the layout version of
 * coot_features.  Host only. */
#define COOT_FEATURE_SCHEMA 1
int coot_kernel_stamp(uint64_t* stamp);

/* Index of the fixed heuristic's configuration for this call.  Host only. */
int coot_default_config(int red_op, int dim, const coot_expr* expr, const coot_operand* ops,
                        int n_ops, const coot_operand* out);

/* The 32 features of a call (op mix, depth, element types, shape), as used
 * by the cost model.  Host only. */
#define COOT_N_FEATURES 32
int coot_features(int red_op, int dim, const coot_expr* expr, const coot_operand* ops,
                  int n_ops, const coot_operand* out, float* features);

/* Exhaustive autotuner: time the call under every one of the 64
 * configurations (warm-up, then `reps` timed launches with HIP events; the
 * median is kept), write the times in milliseconds to times_ms[64] and
 * remember the best one for COOT_TUNE_CACHE.  The call's output is
 * overwritten many times.  Synchronises the stream. */
int coot_autotune(int red_op, int dim, const coot_expr* expr, const coot_operand* ops,
                  int n_ops, const coot_operand* out, int reps, float* times_ms, void* stream);

/* ------------------------------------------------------ cost-model network -- */
/* MLP 32 -> 64 (ReLU) -> 64, FP32, row-major weights; parameters packed as
 * W1[32*64] b1[64] W2[64*64] b2[64] (COOT_MLP_N_PARAMS floats).  All
 * pointers are device memory; B is the batch size.
 *   forward : Z1 = X W1 + b1, H = max(Z1, 0), Y = H W2 + b2
 *   backward: gradient of L = sum(M (Y - T)^2) / sum(M) w.r.t. the packed
 *             parameters, written to grad (same packing)
 *   adam    : one Adam step (Kingma and Ba, 2015) on params with moments m, v
 *             at 1-based step t.
 * The workspace must hold COOT_MLP_WS_FLOATS(B) floats. */
#define COOT_MLP_IN 32
#define COOT_MLP_HID 64
#define COOT_MLP_OUT 64
#define COOT_MLP_N_PARAMS (32 * 64 + 64 + 64 * 64 + 64)
#define COOT_MLP_WS_FLOATS(B) ((int64_t)(B) * (64 + 64 + 64) + 64 + 8)
int coot_mlp_forward(const float* params, const float* X, int B, float* Y, float* ws, void* stream);
int coot_mlp_backward(const float* params, const float* X, const float* T, const float* M, int B,
                      float* grad, float* loss, float* ws, void* stream);
int coot_mlp_adam(float* params, const float* grad, float* m, float* v, int n, int t,
                  float lr, float beta1, float beta2, float eps, void* stream);

/* Install cost-model weights (host array of COOT_MLP_N_PARAMS floats plus
 * the feature standardisation: mean[32], std[32]) for COOT_TUNE_MODEL. */
int coot_model_set(const float* params, const float* feat_mean, const float* feat_std);

/* Configuration index the installed model picks for this call.  Runs the
 * model's forward kernel on the device (a private stream, synchronised before
 * returning); the call itself is not launched. */
int coot_model_choose(int red_op, int dim, const coot_expr* expr, const coot_operand* ops,
                      int n_ops, const coot_operand* out);

/* --------------------------------------------------------------- counters -- */
typedef struct coot_stats {
    int64_t launches;
    int64_t jit_compiles;
    int64_t jit_disk_hits;
    int64_t jit_mem_hits;
    double jit_seconds;
} coot_stats;
int coot_get_stats(coot_stats* stats);

/* Plain device-to-device copy of `bytes` bytes with the library's streaming
 * kernel (the bandwidth ceiling the fused kernels are compared with). */
int coot_copy(void* dst, const void* src, int64_t bytes, void* stream);

/* Bandwidth probes: the simplest streaming kernels with a given mix of reads
 * and writes (one pass, nontemporal 16-byte loads and stores), so that a
 * fused call can be compared with the ceiling of its own read/write mix.
 * kind = a COOT_PROBE_* value | (shape << 8), shape the launch shape:
 * 0 = 256 threads x 4 vectors per thread (COOT_PROBE_COPY with shape 0 is
 * coot_copy), 1 = 64 x 1 (the fused element-wise default), 2 = 256 x 1,
 * 3 = 128 x 2.  `bytes` (a multiple of 16) is the length of each stream;
 * pointers are 16-byte aligned device memory:
 *   COOT_PROBE_COPY          dst = src (coot_copy): reads and writes bytes
 *   COOT_PROBE_READ          reads src; dst (16 bytes) is written only if a
 *                            thread's XOR of its data has all bits set
 *   COOT_PROBE_WRITE         writes dst (src unused)
 *   COOT_PROBE_READ2_WRITE1  dst = src[0, bytes) XOR src[bytes, 2 bytes)
 * The tiled probes move each stream as a column-major matrix of 16384 rows
 * of 4-byte elements (columns 64 KB apart) in tiles of 2^lr rows x 2^(12-lr)
 * columns, one wave access being 64 consecutive rows of one column (4 bytes
 * per lane): the access pattern of the tiled kernels, whose run down a
 * column is the tile's height.  shape selects lr = 6, 8, 10, 12 (runs of
 * 256 bytes to 16 KB); `bytes` must be a multiple of 4 MiB (64 columns):
 *   COOT_PROBE_TILED_COPY          as COOT_PROBE_COPY
 *   COOT_PROBE_TILED_READ2_WRITE1  as COOT_PROBE_READ2_WRITE1 */
enum {
    COOT_PROBE_COPY = 0,
    COOT_PROBE_READ = 1,
    COOT_PROBE_WRITE = 2,
    COOT_PROBE_READ2_WRITE1 = 3,
    COOT_PROBE_TILED_COPY = 4,
    COOT_PROBE_TILED_READ2_WRITE1 = 5
};
int coot_bandwidth_probe(int kind, void* dst, const void* src, int64_t bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* COOT_H */
