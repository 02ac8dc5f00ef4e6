// Internal interface between the host orchestration (brm_api.cpp) and the
// kernel launchers (brm_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spgemm.h"

namespace brm {

// Kernel classes a row of C is routed to (by its product count).
enum RowClass : int {
    kClassEmpty = 0,   // no product: empty row
    kClassCopy = 1,    // one list: the scaled B row is the result
    kClassWaveSmall = 2,  // one wavefront, one product per lane
    kClassWave = 3,    // one wavefront, LDS buffer
    kClassGroup = 4,   // 256-thread workgroup, LDS buffer
    kClassBlock = 5,   // 1024-thread workgroup, LDS buffer
    kClassHeavy = 6,   // beyond one workgroup's LDS: HBM spill
    kClassMulti = 7,   // one wavefront, lane windows of 2 to 16 registers per lane
    kNumClasses = 8
};

// The classes whose rows one kernel launch per class merges in LDS or in
// registers (every class but empty, heavy), in launch order.
constexpr int kLightClasses[] = {kClassCopy, kClassWaveSmall, kClassMulti, kClassWave, kClassGroup, kClassBlock};

// Compile-time capacities (products per row) of the LDS classes.
constexpr int kCapWaveSmall = 64;
constexpr int kCapWave = 256;
constexpr int kCapGroup = 1024;
constexpr int kCapBlock = 4096;
constexpr int kGroupRows = 4;  // rows of the wave-small class merged together by one wavefront
// Heavy rows: one workgroup per row, of 512 threads (two per compute unit)
// or 1024 (one per compute unit), chosen per batch; tree nodes of at most
// 4 x threads products (and lists) in LDS.
constexpr int kHeavyLdsCapMax = 4096;

struct Thresholds {
    int64_t wave_small_max;
    int64_t wave_max;
    int64_t group_max;
    int64_t block_max;
    int32_t force;  // -1: none
    int32_t windows;  // 1: the wave-small class holds only rows whose lists fit lane windows
    int32_t multi;    // 1: rows whose lists fit windows of 2 to 16 registers per lane take kClassMulti
};

// row_class byte: the class in the low bits; for rows under lane windows
// (wave-small, multi), log2 of the window width above them
constexpr int kClassBits = 3;
constexpr uint8_t kClassMask = (1u << kClassBits) - 1;

// Device control block (one per handle).
struct Ctl {
    int64_t count[8];   // rows per class
    int64_t cursor[8];  // scatter cursors
    int64_t nnz;        // nnz(C)
    int64_t nprod;      // total products
    int64_t err;        // error bits set by kernels
    int64_t ovf_light;  // learned allocation: rows that did not fit their slot (light / heavy)
    int64_t ovf_heavy;
    int64_t pred_total; // learned allocation: sum of the predicted row sizes
    int64_t pad[2];
};

enum CtlErr : int64_t {
    kErrRptA = 1, kErrColA = 2, kErrRptB = 4, kErrColB = 8,
    kErrSizeMismatch = 16,  // numeric row length differs from the symbolic count
    kErrHeavyCapacity = 32,
    kErrRowProducts = 64    // a row has 2^31 or more products (routed to no kernel)
};

// Row-pointer types are dispatched at run time: 4 or 8 bytes.
struct CsrView {
    int64_t rows, cols, nnz;
    const void *rpt;
    int rpt_bytes;
    const int32_t *col;
    const double *val;
};

struct Workspace {
    int64_t *row_nprod;   // [M]
    uint8_t *row_class;   // [M]
    int32_t *row_size;    // [M]
    int32_t *class_rows;  // [M], grouped by class
    int64_t *tile_sum;    // [ntiles]
    Ctl *ctl;
    void *ent_bs;         // [nnz(A)] start of each A entry's B row (B's row-pointer type)
    int32_t *ent_len;     // [nnz(A)] length of each A entry's B row
    int32_t *row_prob;    // batched stages: [M] the problem of every row
    // the precise method's wave-small rows with register windows: each row's
    // merge order and distinct columns, kept by the symbolic pass for the
    // numeric pass ([64 M] bytes and [64 M] columns), or nullptr
    uint8_t *order = nullptr;
    int32_t *ucol = nullptr;
};

constexpr int kScanTile = 1024;  // rows per scan tile (256 threads x 4)

// ---- launchers (brm_kernels.hip) -----------------------------------------
hipError_t launch_zero_ctl(Ctl *ctl, hipStream_t s);
hipError_t launch_zero_words(unsigned long long *p, int64_t n, hipStream_t s);
hipError_t launch_validate(const CsrView &X, int64_t ncols_limit, int64_t err_rpt, int64_t err_col,
                           Ctl *ctl, hipStream_t s);
// the size predictor's inputs per row, written by the analysis when asked
struct RowFeatures {
    const int32_t *b_ends;  // per row of B: first and last column, length, start (launch_row_ends)
    float *feats;       // [M * 6]
    int32_t *lo, *hi;   // bounds of the row size
    int8_t *predicted;  // 1: the row's size is predicted (products, two lists or more)
    int64_t ncols;      // columns of B (the features relative to the column space)
};
// ends[4k .. 4k+3]: first and last column of B's row k (-1, -1 when empty),
// its length and its start (the low 32 bits)
hipError_t launch_row_ends(const CsrView &B, int32_t *ends, hipStream_t s);
hipError_t launch_analysis(const CsrView &A, const CsrView &B, const Thresholds &th,
                           const Workspace &ws, int grid, hipStream_t s, const RowFeatures *rf = nullptr);
hipError_t launch_bin(int64_t M, const Workspace &ws, int grid, hipStream_t s);
// slot sizes of the upper-bound allocation: the product count of every row
hipError_t launch_upper_sizes(int64_t M, const int64_t *row_nprod, int32_t *size, hipStream_t s);
// counts then bins the rows of a list by their class (ctl zeroed beforehand)
hipError_t launch_bin_list(int64_t n, const int32_t *rows, const uint8_t *row_class, int32_t *class_rows,
                           Ctl *ctl, hipStream_t s);
// the symbolic pass of the wave-small class (cls = kClassWaveSmall), in the
// kernel group_rows selects; the other classes' passes share the two
// launches below
hipError_t launch_symbolic(const CsrView &A, const CsrView &B, const Workspace &ws, int cls,
                           int grid, hipStream_t s, int group_rows);
// the symbolic passes of the multi-register, wave and group classes in one
// launch of g_mw + g_wave + g_group workgroups of 256 threads
hipError_t launch_symbolic_mid(const CsrView &A, const CsrView &B, const Workspace &ws, int g_mw, int g_wave,
                               int g_group, hipStream_t s);
// the block class and the heavy rows in one launch of 1024-thread workgroups
hipError_t launch_symbolic_big(const CsrView &A, const CsrView &B, const Workspace &ws, int g_block, int g_heavy,
                               hipStream_t s);
// row sizes -> row pointers and their total (*total, a word of ctl_src when
// ctl_dst is given); with ctl_dst (the device address of a mapped host copy
// of the control block) the scan also writes ctl_src, total in place, there
hipError_t launch_scan(int64_t M, const int32_t *sizes, int64_t *tile_sum, int64_t *out_rpt,
                       int64_t *total, hipStream_t s, const Ctl *ctl_src = nullptr, Ctl *ctl_dst = nullptr);

// Output mode of the numeric kernels.
struct NumOut {
    int bound;          // 0: C slots are exact (symbolic counts); 1: slots are upper bounds
    int32_t *row_size;  // bound mode: exact length of every row
    int32_t *ovf_rows;  // bound mode: rows longer than their slot; 2*M entries, light rows
                        // from index M-1 downwards, heavy rows from index M upwards
    int64_t M;
};
hipError_t launch_numeric(const CsrView &A, const CsrView &B, const Workspace &ws, int cls,
                          int grid, const int64_t *c_rpt, int32_t *c_col, double *c_val,
                          const NumOut &no, hipStream_t s, int group_rows);
// the hash-accumulator comparator for one light class (exact slots)
hipError_t launch_numeric_hash(const CsrView &A, const CsrView &B, const Workspace &ws, int cls, int num_cu,
                               const int64_t *c_rpt, int32_t *c_col, double *c_val, hipStream_t s);

// Heavy rows: one workgroup of 512 or 1024 threads per work item, spill
// buffers in HBM.  A work item is a whole row, or an aligned subtree of a long
// row's lists (lists [q 2^H, (q+1) 2^H) of the merge tree) whose result stays
// in the row's spill buffers; the levels above a split row's subtrees are
// merged by later launches, one per level (HeavyTop items).
struct HeavyItem {
    int32_t bi;     // the row's index in the batch (rows, spill_off, leaf_off)
    int32_t res;    // -1: the whole row (its root goes to C); else the subtree's result slot
    int64_t l0, l1; // list range [l0, l1)
    int64_t nprod;  // the row's products
};
struct HeavyTop {
    int32_t bi;
    int32_t res_x;  // result slot of the left node (the merged node's slot)
    int32_t res_y;  // result slot of the right node; -1: the left node alone is the root
    int32_t root;   // 1: the merged node is the row (written to C)
    int64_t lx, ly; // first lists of the two nodes
    int64_t nprod;
};
struct HeavyArgs {
    unsigned long long *ticket;  // zeroed counter handing out the work items
    const int32_t *rows;       // heavy row ids of this batch
    const int64_t *spill_off;  // element offset of each row's two spill buffers (2 * nprod)
    const int64_t *leaf_off;   // offset of each row's list-offset array (lists + 1 entries)
    const HeavyItem *items;    // work items of this launch, largest first
    int64_t nitems;
    int64_t *res;              // subtree results: (buffer 0 / 1, length) per slot
    int32_t *spill_col;
    double *spill_val;
    int32_t *leaf;
    int lds_cap;               // largest list range merged in LDS (products and lists)
    int threads;               // 512 or 1024 threads per workgroup
};
hipError_t launch_heavy_info(const CsrView &A, const Workspace &ws, const int32_t *rows, int64_t n,
                             int64_t *info, hipStream_t s);
hipError_t launch_numeric_heavy(const CsrView &A, const CsrView &B, const Workspace &ws, const HeavyArgs &h,
                                int grid, const int64_t *c_rpt, int32_t *c_col, double *c_val, Ctl *ctl,
                                const NumOut &no, hipStream_t s);
// one level of merges above the subtrees of split rows (1024-thread workgroups)
hipError_t launch_heavy_top(const HeavyArgs &h, const HeavyTop *tops, int64_t ntops, int grid, const int64_t *c_rpt,
                            int32_t *c_col, double *c_val, Ctl *ctl, const NumOut &no, hipStream_t s);

// ---- batched products ------------------------------------------------------
struct BatchProb {
    int64_t row_off;   // first row in the stage's row space
    int64_t rows, ncols_b;
    const void *a_rpt;
    const int32_t *a_col;
    const double *a_val;
    const void *b_rpt;
    const int64_t *b_end;  // end of every row of B when B is a C kept in slots, else nullptr
    const int32_t *b_col;
    const double *b_val;
    int64_t *c_rpt;    // in the arena (offset chosen on the host)
    int64_t *c_end;    // a C kept in slots: end of every row (c_rpt holds the starts), else nullptr
    int32_t *c_col;    // in the arena (offset chosen on the device)
    double *c_val;
    int64_t nnz;
    int64_t rpt_off, col_off, val_off;  // byte offsets in the arena
    int32_t b_from;    // -1, or the problem whose C is this problem's B
    int32_t pad;
    int64_t ent_off;   // first entry of this problem's A in the stage's list descriptors
};

enum BatchFlags : int { kBatchOverflow = 1, kBatchRowProducts = 2 };  // arena too small / a row of 2^31+ products

struct BatchStatus {
    int flags;
    int skip;            // the flags were set when the current stage began: the stage reads no operand
                         // (a chained B may be an unwritten C) and routes every row to the empty class
    int64_t required;    // arena bytes the batch needs
    int64_t arena_used;  // running arena fill (row pointers, then each stage's C)
    int64_t nprod;
    int64_t err;         // device errors (Ctl::err) of the stages before the current one
    // the current stage's heavy-row spill space in the arena (set when it fits)
    int64_t *h_tab;      // (spill offset, list-offset offset) per heavy row, in class order
    int32_t *h_col;
    double *h_val;
    int32_t *h_leaf;
    int64_t spill_base;  // arena offset where the current stage's heavy spill space may start
    // the current stage's upper-bound slots (set when they fit)
    int32_t *s_col;
    double *s_val;
    int64_t slots_end;   // arena offset where they end
};

constexpr int kBatchHeavyThreads = 512;  // workgroup of the batched heavy-row merge
constexpr int kBatchChunkRows = 64;  // rows per wavefront pass of the batched analysis (one wavefront)
// device bytes of the allocation-free batched call's static workspace
constexpr int64_t kNoAllocScratchBytes = (int64_t)64 << 20;

struct BatchStage {
    BatchProb *all;      // every problem of the call
    BatchProb *tab;      // this stage's problems (all + first)
    int first, nprob;
    int64_t *row_off;    // nprob + 1 entries
    int64_t *chunk_off;  // nprob + 1 entries: first chunk of 64 rows of every problem
    int64_t chunks;      // chunks of the stage
    int64_t rows;        // rows of the stage
    int a_rpt_bytes, b_rpt_bytes;
    int link;            // B operands come from earlier problems
    int64_t *S;          // rows + 1 prefix sums
    char *arena;
    int64_t arena_bytes, data_off;
    BatchStatus *status;
    int heavy_lds_cap;   // largest list range of a heavy row merged in LDS
    int upper;           // upper-bound slots instead of the symbolic pass
    int64_t *S2;         // rows + 1: prefix sums of the slot sizes (upper)
    int32_t *ovf;        // 2 * rows: overflow list of the bound-mode bookkeeping (upper; never filled,
                         // a slot holds all of its row's products)
    int keep;            // upper: every problem of the stage is an operand only; its slots are kept
};

hipError_t launch_batched_begin(BatchStatus *st, Ctl *ctl, hipStream_t s);
hipError_t launch_batched_stage(const BatchStage &bs, const Workspace &ws, const Thresholds &th, int num_cu,
                                int64_t grid_waves, hipStream_t s);
hipError_t launch_batched_describe(const BatchProb *all, int n, spg_batched_out *out, const BatchStatus *st,
                                   hipStream_t s);

// ---- learned allocation (brm_learned.hip) ---------------------------------
constexpr int kMlpParams = 4673;
constexpr int kMlpActStride = 6 + 4 * 64 + 1;
constexpr int kMlpGradChunks = 64;
hipError_t launch_features(const CsrView &A, const CsrView &B, float *feats, int32_t *lo, int32_t *hi,
                           int8_t *predicted, const int64_t *c_rpt, float *targets, hipStream_t s);
hipError_t launch_mlp_sizes(int64_t M, const float *feats, const int8_t *predicted, const int32_t *lo,
                            const int32_t *hi, const int64_t *row_nprod, const float *params,
                            const float *norm, float delta, int force, int64_t heavy_min, float heavy_margin,
                            int32_t *pred_size, hipStream_t s);
hipError_t launch_mlp_forward(int64_t n, const float *feats, const float *params, const float *norm,
                              float *y, hipStream_t s);
hipError_t launch_mlp_gradient(int64_t n, const float *feats, const float *targets, const float *params,
                               const float *norm, float *act, float *partial, float *grad, float *loss,
                               hipStream_t s);
hipError_t launch_adam(float *params, const float *grad, float *m, float *v, int64_t t, float lr,
                       hipStream_t s);
hipError_t launch_feature_stats(int64_t n, const float *feats, float *norm, hipStream_t s);
hipError_t launch_mse(int64_t n, const float *y, const float *t, float *out, hipStream_t s);
hipError_t launch_compact(int64_t M, const int64_t *slot_off, const int32_t *row_size, const int64_t *c_rpt,
                          const int32_t *s_col, const double *s_val, int32_t *c_col, double *c_val,
                          int grid, hipStream_t s);
hipError_t launch_fallback_ctl(const Ctl *src, Ctl *dst, int64_t M, hipStream_t s);

}  // namespace brm
