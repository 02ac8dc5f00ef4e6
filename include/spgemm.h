/*
 * spgemm.h -- C ABI of the MI355X (gfx950) row-wise SpGEMM library.
 *
 * The library computes C = A*B for sparse A (M x K) and B (K x N) held in
 * CSR (Section II-A.3 of the paper: a row-pointer array of M+1 entries,
 * column indices sorted within each row, values alongside).  It follows the
 * row-wise dataflow of Eq. (2) (Section II-A.2), the precise allocation
 * method of Section II-B.2 (a symbolic pass counts each output row, a prefix
 * sum turns the counts into C's row pointers, the numeric pass writes every
 * row straight into place; the "BRMerge-Precise" library of Section III-D.2)
 * and the BRMerge accumulation of Section III-B / Algorithm 1 (for every
 * output row the scaled rows of B selected by the row of A are written one
 * after the other into a buffer, then merged two lists at a time, list 0 with
 * list 1, list 2 with list 3, ..., an odd last list passing unchanged, round
 * after round between two buffers, with the values of equal columns added).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All matrix arrays are DEVICE pointers on the handle's device.  The
 *    caller owns them; the library never frees or keeps them past a call
 *    (except as documented for spgemm_symbolic -> spgemm_numeric).
 *  - Input row pointers may be int32 or int64 (spg_csr.rpt_bytes = 4 or 8).
 *    Column indices are int32, values IEEE-754 double.  Input rows must have
 *    strictly increasing columns (checked when SPG_OPT_VALIDATE is set).
 *  - C's row pointers are int64 (rows + 1 entries, c_rpt[0] == 0); C's
 *    columns are strictly increasing within each row.
 *  - C is the STRUCTURAL product: (i, j) is stored iff some k has both A_ik
 *    and B_kj stored.  Values that are zero or cancel to zero are kept.
 *  - Every value of C is the sum of the products A_ik * B_kj (one rounded
 *    double multiplication each, no fused multiply-add) grouped by the merge
 *    tree of Algorithm 1 with the stored entries of A's row as its leaves in
 *    stored order: the node of level r and index p covers leaves
 *    [p * 2^r, (p + 1) * 2^r) and adds the values of its two children when
 *    both hold the column.  The result is therefore bitwise reproducible and
 *    independent of the kernel class a row is routed to.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    asynchronously on it unless stated otherwise.
 *  - Every function returns SPG_OK (0) or a negative spg_status; details of
 *    the last error are available from spg_last_error().  No C++ exception
 *    crosses this interface.
 *  - A handle is not thread-safe: use one handle per host thread / stream.
 *  - Column-wise products (CSC in, CSC out; the column-wise dataflow of
 *    Eq. (3)): the CSC arrays of a matrix X are the CSR arrays of X^T, so
 *    C = A*B in CSC is the row-wise product C^T = B^T A^T: pass B's CSC
 *    arrays as A (rows = B's columns) and A's as B; c_rpt / c_col / c_val
 *    are then C's column pointers, row indices and values.  The leaves of
 *    column j's merge tree are the stored entries of column j of B.
 */
#ifndef SPGEMM_H_
#define SPGEMM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPG_OK = 0,
    SPG_ERR_ARG = -1,          /* null pointer, negative size, bad option, rpt_bytes not 4/8 */
    SPG_ERR_DIM = -2,          /* A.cols != B.rows */
    SPG_ERR_INVALID_CSR = -3,  /* (validation on) rpt not monotone / rpt[0] != 0 /
                                  column out of range / columns not strictly increasing */
    SPG_ERR_CAPACITY = -4,     /* a caller-provided buffer is too small */
    SPG_ERR_NOMEM = -5,        /* device allocation failed */
    SPG_ERR_HIP = -6,          /* a HIP runtime call failed (see spg_last_error) */
    SPG_ERR_NOT_TRAINED = -7,  /* learned allocation asked for before any training/loading */
    SPG_ERR_STATE = -8,        /* spgemm_numeric without a matching spgemm_symbolic */
    SPG_ERR_SCRATCH = -9       /* spgemm_batched_noalloc: the batch needs more workspace than
                                  the fixed scratch array holds */
} spg_status;

/* A CSR matrix on the device. */
typedef struct {
    int64_t rows;        /* M */
    int64_t cols;        /* N */
    int64_t nnz;         /* rpt[rows]; must equal the device value */
    const void *rpt;     /* rows + 1 entries of int32 or int64 */
    int32_t rpt_bytes;   /* 4 or 8 */
    const int32_t *col;  /* nnz entries */
    const double *val;   /* nnz entries (may be NULL for spgemm_symbolic of the precise method) */
} spg_csr;

typedef struct spg_handle_s *spg_handle;

/* Create a handle bound to HIP device `device`.  The handle owns the
 * library's device workspace (row analysis, bins, scan state, the spill pool
 * of heavy rows) and grows it on demand; everything is freed by
 * spg_destroy().  Errors: SPG_ERR_ARG (h NULL), SPG_ERR_HIP (bad device). */
int spg_create(spg_handle *h, int device);

/* Release the handle and all device memory it owns.  Waits for the device. */
int spg_destroy(spg_handle h);

/* Options (spg_set_option / spg_get_option).  Thresholds are products per
 * row; they select the kernel class each row is routed to.  Results do not
 * depend on them (bitwise). */
typedef enum {
    SPG_OPT_VALIDATE = 1,        /* 0/1: check A and B before computing (default 0) */
    SPG_OPT_WAVE_SMALL_MAX = 2,  /* largest row routed to one wavefront with one product per lane (64) */
    SPG_OPT_WAVE_MAX = 3,        /* largest row routed to one wavefront with an LDS buffer (<= 256) */
    SPG_OPT_GROUP_MAX = 4,       /* largest row routed to a 256-thread workgroup (<= 1024) */
    SPG_OPT_BLOCK_MAX = 5,       /* largest row kept in one workgroup's LDS (<= 4096); larger
                                    rows take the heavy path with HBM spill */
    SPG_OPT_FORCE_CLASS = 6,     /* -1: normal binning.  2..5, 7: every non-empty row (single-list
                                    rows included) that fits that class (2 wave-small, 3 wave,
                                    4 group, 5 block, 7 multi-register windows) is routed there,
                                    every other row to the heavy path; 6: every non-empty row to
                                    the heavy path */
    SPG_OPT_HEAVY_LDS_MAX = 7,   /* leaf-range size the heavy path merges in LDS (64..4096;
                                    512-thread workgroups merge at most 2048) */
    SPG_OPT_SPILL_BUDGET_MB = 8, /* device memory the heavy path may use for spill buffers
                                    per batch of heavy rows; 0 (default): 128 GiB, or 60% of
                                    the device memory free at the call when that is less.
                                    The handle keeps its pool (grow-only) until spg_destroy */
    SPG_OPT_GRID_WAVES = 9,      /* waves per launch of the persistent row kernels (0 = auto) */
    SPG_OPT_ALLOC = 10,          /* SPG_ALLOC_PRECISE (default), SPG_ALLOC_LEARNED or SPG_ALLOC_UPPER */
    SPG_OPT_LEARNED_HEAVY_MARGIN = 16, /* learned allocation: extra margin, in thousandths, added to
                                    delta for rows of more than SPG_OPT_BLOCK_MAX products (merged
                                    through spill buffers, where an overflowing row is merged
                                    twice): slot = clamp(ceil(nprod e^(y + delta + this)), ...).
                                    Default 200 */
    SPG_OPT_LEARNED_FORCE = 11,  /* testing only: 1 sizes every predicted row at its lower bound
                                    (the longest list), so that most rows take the fallback */
    SPG_OPT_ACCUMULATOR = 13,    /* SPG_ACC_BRMERGE (default) or SPG_ACC_HASH: see below */
    SPG_OPT_HEAVY_THREADS = 14,  /* workgroup size of the heavy path, one row per workgroup:
                                    0 (default) chosen per batch of heavy rows -- 1024 threads
                                    (one workgroup per CU) when the batch's longest row
                                    outweighs 1.3x the batch's products over 2 x CUs, else 512
                                    (two per CU); 512 or 1024 forces one.  Results are
                                    bitwise the same */
    SPG_OPT_HEAVY_SPLIT = 15,    /* heavy rows much longer than their batch's share per workgroup
                                    are merged as several aligned subtrees of their lists, one
                                    workgroup each, and the levels above them by one launch per
                                    level: products per subtree (rows of more than twice that are
                                    split).  0 (default): a quarter of a 512-thread workgroup's share
                                    of the batch, at least 2^18; -1: never split.  Results are
                                    bitwise the same */
    SPG_OPT_BATCH_ALLOC = 17,    /* sizes of the batched stages (spgemm_batched[_noalloc]):
                                    SPG_BATCH_PRECISE (default) or SPG_BATCH_UPPER, see below.
                                    Results are bitwise the same */
    SPG_OPT_STORED_ORDER = 18,   /* 1 (default): with SPG_OPT_GROUP_ROWS = 1 and the precise
                                    method, the symbolic pass keeps every wave-small row's merge
                                    order (the sorted position of each product and whether the next
                                    one repeats its column: 64 bytes) and its distinct columns (up to
                                    64 x 4 bytes) in handle memory (320 bytes per row of A), and the
                                    numeric pass gathers B's values only and applies that order
                                    (the column gather and the merge network are not repeated).
                                    0: the numeric pass merges its windows itself.  Results are
                                    bitwise the same */
    SPG_OPT_GROUP_ROWS = 12      /* kernel of the wave-small class (rows of at most 64 products):
                                    1 (default) one row per wavefront, merged in registers; the
                                    class then holds only rows whose lists fit power-of-two lane
                                    windows (the others go to the next class), and only when
                                    B has fewer than 2^26 columns (else 0 is used); 2 as 1, with
                                    symbolic counts by LDS hash instead of register merges; 0 one
                                    row per wavefront in LDS; 4 four rows per wavefront in LDS.
                                    With 1 and 2, rows of at most 64 lists whose lists fit lane
                                    windows of 2 to 16 registers per lane take the multi-register
                                    class (7) when B has at most 2^21 columns */
} spg_option;

/* Sizes of the batched stages (SPG_OPT_BATCH_ALLOC). */
enum {
    SPG_BATCH_PRECISE = 0, /* the symbolic pass of every class, then the numeric pass straight into C */
    SPG_BATCH_UPPER = 1    /* the upper-bound method (Section II-B.2): every row gets a slot of nprod_i
                              entries in the arena, the numeric pass runs into the slots (no symbolic
                              pass), and the rows are then compacted into C.  A stage's arena need
                              grows by 24 bytes per product (the slots, and room for C at its
                              largest); the workspace by 16 bytes per row */
};

/* Allocation methods (SPG_OPT_ALLOC). */
enum {
    SPG_ALLOC_PRECISE = 0, /* symbolic count, prefix sum, numeric straight into C */
    SPG_ALLOC_LEARNED = 1, /* predicted sizes, numeric into predicted slots, exact fallback, compaction */
    SPG_ALLOC_UPPER = 2    /* the upper-bound method (Section II-B.2, the "BRMerge-Upper" library of
                              Section III-D.1): every row gets a slot of nprod_i entries, the numeric
                              pass runs into the slots inside spgemm_symbolic (no symbolic count), and
                              spgemm_numeric copies the rows into C.  The slots take 12 bytes per
                              product of device memory (SPG_ERR_NOMEM when they do not fit: cut A
                              into row blocks with spgemm_row_products) */
};

/* Accumulators of the numeric pass of the precise method (SPG_OPT_ACCUMULATOR).
 * SPG_ACC_HASH is a comparator, not the paper's method: every row of at
 * most 4096 products adds its products into a hash table in LDS (keyed by
 * column, linear probing, atomic additions) and places each column by its
 * rank, the hash-based accumulation that the paper describes among the
 * prior methods (Section II-B.1) and compares BRMerge with (Section IV-B);
 * rows with more products keep the
 * BRMerge path.  Its values are within rounding of the definition but not
 * equal to the merge tree's, and their last bits may change between runs.
 * The learned and upper-bound allocations always use BRMerge. */
enum {
    SPG_ACC_BRMERGE = 0,
    SPG_ACC_HASH = 1
};

/* Setting any option voids the plan of the last spgemm_symbolic: a
 * spgemm_numeric after it returns SPG_ERR_STATE until spgemm_symbolic runs
 * again.  Errors: SPG_ERR_ARG (unknown key or value out of range). */
int spg_set_option(spg_handle h, int key, int64_t value);
int spg_get_option(spg_handle h, int key, int64_t *value);

/* Statistics of the last symbolic/numeric pair (spg_get_stat); after
 * spgemm_batched, SPG_STAT_NPROD covers the whole batch and the class counts
 * the rows of its last stage. */
typedef enum {
    SPG_STAT_NPROD = 1,          /* total products of the last symbolic call */
    SPG_STAT_NNZ = 2,            /* nnz(C) of the last symbolic call */
    SPG_STAT_CLASS_ROWS0 = 10,   /* rows per class: +0 empty, +1 copy, +2 wave-small,
                                    +3 wave, +4 group, +5 block, +6 heavy, +7 multi-register
                                    windows (one wavefront per row, at most 64 lists padded to
                                    128..1024 slots, B with at most 2^21 columns) */
    SPG_STAT_HEAVY_BATCHES = 20, /* spill batches the heavy path used in the last numeric call */
    SPG_STAT_PRED_TOTAL = 21,    /* learned / upper-bound allocation: sum of the slot sizes (entries) */
    SPG_STAT_OVERFLOW_ROWS = 22, /* learned allocation: rows longer than their predicted slot */
    SPG_STAT_PREDICTED_ROWS = 23,/* rows whose size is predicted (two or more lists, a product) */
    SPG_STAT_OVERFLOW_HEAVY_ROWS = 31,/* learned allocation: overflowing rows of more than
                                    SPG_OPT_BLOCK_MAX products (part of SPG_STAT_OVERFLOW_ROWS) */
    SPG_STAT_GRAPH_CAPTURES = 24,/* batched calls that (re)captured their HIP graph */
    SPG_STAT_GRAPH_LAUNCHES = 25,/* batched calls that replayed a captured graph */
    SPG_STAT_BATCHED_DIRECT = 32,/* batched calls launched kernel by kernel: a batch (problems, arena,
                                    options) unlike the previous call's is launched directly; when the
                                    same batch comes again it is captured in a graph and replayed
                                    from then on */
    SPG_STAT_SPILL_POOL_BYTES = 26,/* device bytes of the handle's heavy-row spill pool (kept
                                    between calls; a call whose batches fit it reuses it) */
    SPG_STAT_SPILL_ALLOCS = 27,  /* allocations of that pool since the handle was created */
    SPG_STAT_HEAVY_WIDE = 28,    /* spill batches of the last numeric call run by 1024-thread
                                    workgroups (the others by 512-thread ones) */
    SPG_STAT_HEAVY_SPLIT_ROWS = 29,/* heavy rows of the last numeric call merged as several subtrees */
    SPG_STAT_DEVICE_ERR = 30     /* error bits the kernels raised since the last symbolic call,
                                    or in the last batched call (16: a numeric row length
                                    differed from its symbolic count; the row was truncated to
                                    its slot; 32: a heavy row's merge walk failed).
                                    Synchronizes the device. */
} spg_stat;

int spg_get_stat(spg_handle h, int key, int64_t *value);

/* Symbolic pass of the precise allocation (Section II-B.2, Section III-D.2
 * steps 1-4): per-row product counts and binning, the exact number of
 * distinct columns of every row of C, and their exclusive prefix sum.
 *   A, B   : device CSR inputs.  With SPG_ALLOC_PRECISE the values are not
 *            read and val may be NULL.
 *   c_rpt  : device int64[A->rows + 1], written with C's row pointers.
 *   c_nnz  : host int64, written with nnz(C).
 * This call BLOCKS until c_nnz is known (the device writes nnz and its error
 * bits into pinned, mapped host memory of the handle; the call then waits for
 * the stream, so `stream` must not be in graph capture).  The row
 * analysis it makes is kept in the handle for the next spgemm_numeric call
 * with the same A and B.
 * With SPG_ALLOC_LEARNED or SPG_ALLOC_UPPER (spg_option) this call already
 * computes the rows, values included, into slots in handle memory and
 * derives c_rpt from their exact lengths: A->val and B->val must then be
 * non-NULL (else SPG_ERR_ARG before any launch), and C's values are those
 * of the inputs at THIS call.  spgemm_numeric copies the rows from their
 * slots; under SPG_ALLOC_UPPER every row comes from its slot, under
 * SPG_ALLOC_LEARNED the rows that overflowed their predicted slot
 * (SPG_STAT_OVERFLOW_ROWS) are recomputed by spgemm_numeric from the values
 * at that call.  The values must therefore stay unchanged between the two
 * calls in these modes; with SPG_ALLOC_PRECISE spgemm_numeric reads them.
 * Errors: SPG_ERR_ARG, SPG_ERR_DIM, SPG_ERR_INVALID_CSR (validation on),
 * SPG_ERR_NOT_TRAINED (learned allocation without a predictor),
 * SPG_ERR_CAPACITY (a row of C has 2^31 or more products: the row kernels
 * count a row's products in int32; no row is computed then),
 * SPG_ERR_NOMEM, SPG_ERR_HIP. */
int spgemm_symbolic(spg_handle h, const spg_csr *A, const spg_csr *B, int64_t *c_rpt,
                    int64_t *c_nnz, void *stream);

/* Numeric pass (Section III-D.2 step 5): the BRMerge accumulation of every
 * row written straight into C at c_rpt[i].
 *   c_rpt  : the device array filled by spgemm_symbolic.
 *   c_col  : device int32[nnz(C)], c_val: device double[nnz(C)].
 * Must follow spgemm_symbolic on this handle with the same A and B (same
 * device pointers and sizes), else SPG_ERR_STATE.  Asynchronous on `stream`
 * except for heavy rows, whose spill planning reads their sizes back once.
 * Errors: SPG_ERR_ARG, SPG_ERR_STATE, SPG_ERR_NOMEM, SPG_ERR_HIP. */
int spgemm_numeric(spg_handle h, const spg_csr *A, const spg_csr *B, const int64_t *c_rpt,
                   int32_t *c_col, double *c_val, void *stream);

/* Row analysis (step 1 of both libraries of Section III-D): the number of
 * products of every row of C, nprod_i = sum over the stored A_ik of the
 * length of row k of B; an upper bound of the row's size.  A caller that
 * must cut a product into row blocks (C larger than device memory) plans
 * the blocks with it.
 *   A, B      : device CSR inputs (values not read).
 *   row_nprod : device int64[A->rows], written.
 * Asynchronous on `stream`.  Voids the plan of the last spgemm_symbolic (the
 * analysis shares its workspace).
 * Errors: SPG_ERR_ARG, SPG_ERR_DIM, SPG_ERR_NOMEM, SPG_ERR_HIP. */
int spgemm_row_products(spg_handle h, const spg_csr *A, const spg_csr *B, int64_t *row_nprod, void *stream);

/* ---- Batched products ----------------------------------------------------
 * Many independent products C_p = A_p * B_p in one call, for instance the
 * Galerkin triple products P^T (A P) of an algebraic multigrid setup (the
 * paper's first application, Section I).  A problem's B may be the C of an
 * earlier problem of the same call (b_from >= 0), which makes chains such as
 * AP = A * P, G = P^T * AP possible without host round trips.  Problems are
 * grouped into stages by their dependencies; each stage runs the same
 * analysis / binning / symbolic / scan / numeric kernels as the single
 * product over the union of its problems' rows, and C's arrays are placed
 * in the caller's arena at offsets computed on the device.  A batch is
 * launched kernel by kernel the first time; when the next call brings the
 * same batch (problems' pointers and sizes, arena, options) the whole launch
 * sequence is captured in a HIP graph, which is replayed while the batch
 * stays the same (SPG_STAT_BATCHED_DIRECT, _GRAPH_CAPTURES, _LAUNCHES).  Results are
 * bitwise equal to separate spgemm_symbolic / spgemm_numeric calls.
 * Rows beyond one workgroup's LDS (more than 4096 products) are merged as
 * in the single product's heavy path (Algorithm 1's tree, spilled nodes
 * merged through HBM), one 512-thread workgroup per row, each whole row in
 * one workgroup (the single product's subtree split is not used here).
 * Their spill buffers -- two lists of nprod_i entries per heavy row, 24
 * bytes per product, plus 4 bytes per list -- lie in the arena after the
 * stage's C and count towards *required_bytes; the next stage's C reuses
 * that space.  A row of 2^31 or more products fails the call
 * (SPG_ERR_CAPACITY with *required_bytes = -1). */
typedef struct {
    spg_csr A;        /* device CSR */
    spg_csr B;        /* device CSR; ignored when b_from >= 0 */
    int32_t b_from;   /* -1, or the index (< this one) of the problem whose C is B */
    int32_t flags;    /* 0, or SPG_PROBLEM_OPERAND_ONLY */
} spg_problem;

/* Problem flags.  SPG_PROBLEM_OPERAND_ONLY: the problem's C is needed only as
 * the B of later problems of the same call (the A P of a Galerkin product
 * P^T (A P)).  When every problem of a stage carries it and the stage sizes
 * are upper bounds (SPG_BATCH_UPPER), the stage's C stays in its slots of
 * the arena -- no exact sizes, no row pointers, no compaction -- and the
 * later problems read its rows from there: each row is described by its
 * start and end in the slots, written where the problem's row pointers
 * would be (that region takes 16 bytes per row instead of 8), and the
 * problem's descriptor reports nnz = -2 (its C is not returned).  Otherwise
 * the flag changes nothing.  The later problems' results are bitwise the
 * same either way. */
enum { SPG_PROBLEM_OPERAND_ONLY = 1 };

/* Where problem p's C sits in the arena (byte offsets; nnz = -1 when the
 * arena was too small, -2 when the C was kept as an operand only, see
 * SPG_PROBLEM_OPERAND_ONLY; the offsets are then -1). */
typedef struct {
    int64_t rows, cols, nnz;
    int64_t rpt_off;  /* int64[rows + 1] */
    int64_t col_off;  /* int32[nnz] */
    int64_t val_off;  /* double[nnz] */
} spg_batched_out;

/* Computes every problem into `arena` (device, arena_bytes long, 256-byte
 * aligned).  `out` is a DEVICE array of `count` descriptors.  Blocks until the
 * batch is done (one device-to-host read of the batch status).  Problems of
 * one stage must share the row-pointer widths of A and of B (chained B always
 * has int64 row pointers).
 * On success *required_bytes is the arena size the batch needed (row
 * pointers, every C, and the largest heavy-row spill space of a stage).
 * Device errors of the kernels are read with SPG_STAT_DEVICE_ERR.
 * Errors: SPG_ERR_ARG, SPG_ERR_DIM (A_p.cols != B_p.rows), SPG_ERR_CAPACITY
 * (arena too small: the outputs are invalid and *required_bytes is set to the
 * size that the stages up to the first one that did not fit need; a stage
 * after it computes nothing -- its B may be a C that was never written -- so
 * with chained problems a call with an arena of that size may fail again
 * with a larger *required_bytes; or a row of 2^31 or more products:
 * *required_bytes = -1), SPG_ERR_NOMEM, SPG_ERR_HIP. */
int spgemm_batched(spg_handle h, int count, const spg_problem *problems, void *arena, int64_t arena_bytes,
                   spg_batched_out *out, int64_t *required_bytes, void *stream);

/* The same batched product for callers that cannot allocate device memory
 * (code that runs while a HIP graph is being captured around it, tight
 * serving loops, harnesses that forbid hipMalloc): the arguments, the
 * results (bitwise) and the errors are those of spgemm_batched, and it runs
 * the same kernels, but the call allocates nothing -- no device or pinned
 * memory, no HIP graph.  Its workspace (problem table, stage row arrays, list
 * descriptors, status) is a fixed array of 64 MiB of device memory that the
 * library holds on every GPU it runs on until the process ends; the kernels
 * are launched one by one on `stream`.  A batch needs 29 bytes per row plus
 * 12 bytes per entry of A of its largest stage (16 more bytes per row with
 * SPG_BATCH_UPPER), plus about 170 bytes per problem; a larger batch fails
 * with SPG_ERR_SCRATCH before any launch (use spgemm_batched for it).  Blocks until the batch is done, like
 * spgemm_batched.
 * The array is shared by every call on one GPU, from any handle, and keeps
 * the last call's contents (the call clears what must start at zero): calls
 * that overlap on one GPU (from several host threads) race and must be
 * serialized by the caller. */
int spgemm_batched_noalloc(spg_handle h, int count, const spg_problem *problems, void *arena,
                           int64_t arena_bytes, spg_batched_out *out, int64_t *required_bytes,
                           void *stream);

/* ---- Learned allocation --------------------------------------------------
 * Not in the paper: a stand-in for its allocation step (Section II-B.2).  A
 * perceptron 6 -> 64 -> 64 -> 1 (ReLU, float32) predicts y_i ~ log(nnz(C_i) /
 * nprod_i) for every row with two or more lists and at least one product, from
 * the features log1p(lists), log((1 + products) / N), log1p(longest list),
 * log1p(shortest list), log(column span / N) and log1p(products / span), with
 * N the column count of B (products and span relative to the column space,
 * so that a predictor trained on one matrix size carries over to others),
 * each normalised as (x - mean) / std.  The row's
 * slot holds clamp(ceil(nprod_i exp(y_i + delta)), longest list, min(nprod_i,
 * span_i)) entries; rows with no product or one list get their exact size,
 * and rows with fewer than one expected repeat among their products
 * (products^2 / span < 1) get min(nprod_i, span_i) without the network.
 * With SPG_OPT_ALLOC = SPG_ALLOC_LEARNED, spgemm_symbolic runs the numeric
 * kernels into the slots (no symbolic pass), records every row's exact length
 * and the rows that overflowed, and returns C's exact row pointers and nnz
 * (two reads of the handle's mapped control block, each after the stream
 * has drained); spgemm_numeric recomputes the overflowed rows
 * exactly into C and copies the others from their slots.  C is bitwise the
 * same as with the precise allocation.
 *
 * Parameter vector (SPG_MLP_NUM_PARAMS floats, row-major, in this order):
 * W1[6][64], b1[64], W2[64][64], b2[64], W3[64], b3[1].  `norm` is mean[6]
 * followed by std[6].  All feats / targets / y / grad arrays are DEVICE
 * float arrays; feats rows are 6 consecutive floats. */
#define SPG_MLP_NUM_PARAMS 4673

/* Host params, norm and margin delta; resets the Adam moments. */
int spg_mlp_set_params(spg_handle h, const float *params, const float *norm, float delta);
/* Copies the current parameters, normalisation and margin to the host
 * (any pointer may be NULL).  Synchronizes the device. */
int spg_mlp_get_params(spg_handle h, float *params, float *norm, float *delta);
/* Per-row raw features feats[rows][6], the predicted-row flag, the exact
 * bounds lo/hi (may be NULL) and, when c_rpt (C's row pointers from a
 * precise symbolic pass) is given, the training targets log(nnz(C_i)/nprod_i)
 * (0 for rows that are not predicted). */
int spg_mlp_features(spg_handle h, const spg_csr *A, const spg_csr *B, const int64_t *c_rpt, float *feats,
                     float *targets, int8_t *predicted, int32_t *lo, int32_t *hi, void *stream);
/* Network output y[n] for n raw feature rows. */
int spg_mlp_forward(spg_handle h, const float *feats, int64_t n, float *y, void *stream);
/* Gradient grad[SPG_MLP_NUM_PARAMS] of the mean squared error over n rows,
 * and that error in *loss (host, may be NULL; blocks when given). */
int spg_mlp_gradient(spg_handle h, const float *feats, const float *targets, int64_t n, float *grad, float *loss,
                     void *stream);
/* Sets the normalisation to the mean / std of n raw feature rows. */
int spg_mlp_fit_normalization(spg_handle h, const float *feats, int64_t n, void *stream);
/* Adam (beta1 0.9, beta2 0.999, eps 1e-8, step size lr) over `epochs` passes of
 * the n rows in the given order, in consecutive minibatches of `batch` rows
 * (the caller shuffles). */
int spg_mlp_train(spg_handle h, const float *feats, const float *targets, int64_t n, int epochs, int batch,
                  float lr, void *stream);
/* Mean squared error of the network over n rows (host *loss; blocks). */
int spg_mlp_loss(spg_handle h, const float *feats, const float *targets, int64_t n, float *loss, void *stream);
/* Sets delta to the `quantile` quantile of (target - output) over n rows
 * (at least 0), so that about that fraction of them fits its slot. */
int spg_mlp_calibrate(spg_handle h, const float *feats, const float *targets, int64_t n, double quantile,
                      float *delta, void *stream);
/* Checkpoint of parameters, Adam moments and step, normalisation and margin. */
int spg_mlp_save(spg_handle h, const char *path);
int spg_mlp_load(spg_handle h, const char *path);

/* Text of the last error on this handle ("" if none).  Valid until the next
 * call on the handle. */
const char *spg_last_error(spg_handle h);

#ifdef __cplusplus
}
#endif

#endif /* SPGEMM_H_ */
