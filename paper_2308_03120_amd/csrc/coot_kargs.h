/*
 * Kernel-argument block passed by value to every generated kernel.  The same
 * text is compiled into the host library and prepended to every run-time
 * compiled kernel source, so both sides agree on the layout.
 */
#ifndef COOT_KARGS_H
#define COOT_KARGS_H

#define COOT_MAX_READS 16

#if defined(__HIPCC_RTC__) || defined(__HIP_DEVICE_COMPILE__) || defined(__HIP__)
#define COOT_HD __host__ __device__ inline
#else
#define COOT_HD static inline
#endif

/* Tile shape of an R x Cn value for the tiled kernels: TR x TC = 2^lr x 2^lc
 * with TR*TC <= 4096.  Square 64 x 64 when both sides reach 64; a thin value
 * gets whole-height (or whole-width) tiles: TR = R rounded up to a power of
 * two and TC = 4096/TR, or the mirror image capped at 2048 elements (so that
 * the padded LDS tile, TR*(TC+1) elements, stays within 4160). */
COOT_HD int coot_lg2ceil(long long v)
{
    return v <= 1 ? 0 : 64 - __builtin_clzll((unsigned long long)(v - 1));
}

COOT_HD void coot_tile_shape(long long R, long long Cn, int* lr, int* lc)
{
    const int r0 = coot_lg2ceil(R), c0 = coot_lg2ceil(Cn);
    if (r0 >= 6 && c0 >= 6) {
        *lr = 6;
        *lc = 6;
    } else if (r0 < 6) {
        *lr = r0;
        *lc = c0 < 12 - r0 ? c0 : 12 - r0;
    } else {
        const int cap = c0 == 0 ? 12 : 11 - c0;
        *lc = c0;
        *lr = r0 < cap ? r0 : cap;
    }
}

/* LDS row stride of a 2^lr x 2^lc tile.  LDS banks are resolved per 32
 * lanes: a read in the value's order puts 32/2^lr rows of 2^lr elements on
 * those lanes, so the stride is 32/2^lr modulo 32 (conflict-free); tiles of
 * 64 or more rows read one row per lane and take an odd stride. */
COOT_HD int coot_tile_stride(int lr, int lc)
{
    return lr < 6 ? (1 << lc) + (32 >> lr > 0 ? 32 >> lr : 1) : (lc == 0 ? 1 : (1 << lc) + 1);
}
#define COOT_TILE_LDS 4160

typedef struct coot_kargs {
    const void* leaf[COOT_MAX_READS];  /* distinct leaf reads (slot, transposed) */
    long long ld[COOT_MAX_READS];      /* leading dimension of each read's operand */
    void* out;                         /* element-wise output (or temp) */
    long long ld_out;
    long long rows;                    /* shape of the tree's value */
    long long cols;
    long long n;                       /* rows * cols */
    void* part;                        /* per-block (or per-split) partial accumulators */
    void* res;                         /* reduction result(s) */
    long long splits;                  /* partials per result: pass-1 blocks of a flat or tiled
                                          reduction, row segments or column splits otherwise */
    long long aux;
} coot_kargs;

/* batched evaluation: each item's value is cut into units (blocks of rc x k
 * values of Y_i starting at row p0, column q0), at most E elements each, E
 * chosen so that the operands read through trans() fit COOT_BATCH_LDS_BYTES
 * of LDS; a block runs one unit with all its threads or up to four small
 * units, one per wave */
#define COOT_BATCH_LDS_BYTES 65536
/* LDS elements of one staged operand: a unit stores its rows with an odd
 * stride kp <= k + 1, which needs at most rc more elements (rc <= E/32) */
COOT_HD long long coot_batch_stage_cap(long long E) { return E + E / 32; }

typedef struct coot_batch_item_d {
    long long rows, cols;              /* Y_i shape */
    long long nunits;                  /* units of Y_i */
    long long part0;                   /* partial slot of the item's first unit */
    void* out;
    const void* leaf[6];
} coot_batch_item_d;

typedef struct coot_batch_unit_d {
    int item;
    int p0, q0;                        /* first row and column of the unit in Y_i */
    int rc, k;                         /* rows and columns of the unit */
    int part;                          /* partial slot (an item's units are consecutive) */
} coot_batch_unit_d;

typedef struct coot_bargs {
    const coot_batch_item_d* items;
    const coot_batch_unit_d* units;    /* in block order */
    const int* blk_first;              /* block b runs units [blk_first[b], blk_first[b+1]) */
    long long n_items;
    double* part;                      /* (hi, lo) per unit when there is a reduction */
    void* red_out;
} coot_bargs;

#endif
