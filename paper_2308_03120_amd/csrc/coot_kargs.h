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

/* batched evaluation: one descriptor per item; the items' 64x64 tiles are cut
 * into tasks of at most COOT_BATCH_CHUNK consecutive tiles (column-major tile
 * order within the item), and every block runs a list of tasks (a static
 * longest-first schedule computed on the host) */
#define COOT_BATCH_CHUNK 4

typedef struct coot_batch_item_d {
    long long rows, cols;              /* Y_i shape */
    long long ntiles;                  /* 64x64 tiles of Y_i */
    long long part0;                   /* partial slot of the item's first task */
    void* out;
    const void* leaf[6];
} coot_batch_item_d;

typedef struct coot_batch_task_d {
    int item;
    int t0, t1;                        /* tiles [t0, t1) of the item */
    int part;                          /* partial slot (item's tasks are consecutive) */
} coot_batch_task_d;

typedef struct coot_bargs {
    const coot_batch_item_d* items;
    const coot_batch_task_d* tasks;
    const int* order;                  /* task indices, block by block */
    const int* blk_first;              /* block b runs order[blk_first[b] .. blk_first[b+1]) */
    long long n_items;
    double* part;                      /* (hi, lo) per task when there is a reduction */
    void* red_out;
} coot_bargs;

#endif
