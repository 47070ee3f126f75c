/*
 * Kernel-argument block passed by value to every generated kernel.  The same
 * text is compiled into the host library and prepended to every run-time
 * compiled kernel source, so both sides agree on the layout.
 */
#ifndef COOT_KARGS_H
#define COOT_KARGS_H

#define COOT_MAX_READS 16

typedef struct coot_kargs {
    const void* leaf[COOT_MAX_READS];  /* distinct leaf reads (slot, transposed) */
    long long ld[COOT_MAX_READS];      /* leading dimension of each read's operand */
    void* out;                         /* element-wise output (or temp) */
    long long ld_out;
    long long rows;                    /* shape of the tree's value */
    long long cols;
    long long n;                       /* rows * cols */
    void* part;                        /* per-block partial accumulators */
    unsigned int* counter;             /* blocks-done counter (last block combines) */
    void* res;                         /* reduction result(s) */
    long long splits;                  /* column splits of a per-row reduction */
    long long aux;
} coot_kargs;

/* batched evaluation: one descriptor per item, one per 64x64 tile */
typedef struct coot_batch_item_d {
    long long rows, cols;              /* Y_i shape */
    long long tile0;                   /* first tile of the item */
    long long ntiles;
    void* out;
    const void* leaf[6];
} coot_batch_item_d;

typedef struct coot_bargs {
    const coot_batch_item_d* items;
    const int* tile_item;              /* item (index into items) of every tile */
    long long n_tiles;
    long long tile_base;               /* global index of tile 0 of this launch */
    void* part;                        /* per-tile partials */
    unsigned int* counters;            /* per-item tiles-done counters */
    void* red_out;
} coot_bargs;

#endif
