/*
 * CPU oracle for C = A*B on CSR.  TEST INFRASTRUCTURE ONLY: it is built and
 * called by the test-suite, by the smoke check and by the benchmark's CPU
 * baseline leg.  The GPU library never links, loads or calls it, and it
 * shares no code, header or table with the GPU library.
 *
 * Two independent functions are provided.
 *
 * 1. oracle_spa_* -- the plain definition.  The row-wise formulation of the
 *    product (Eq. (2), Section II-A.2) sums A_ik * B_k* over the stored
 *    entries k of row i of A.  The structure of C is the structural product:
 *    (i, j) is stored iff some k has A_ik and B_kj both stored (no value is
 *    ever dropped, also when it is zero).  Columns are emitted in ascending
 *    order (the CSR convention of Section II-A.3).  Values are accumulated in a
 *    dense per-thread accumulator with Neumaier's compensated summation
 *    (A. Neumaier, ZAMM 54, 1974), so that the oracle's own rounding error is
 *    about 2u|C_ij| and a tolerance relative to sum_k |A_ik B_kj| measures the
 *    method under test only.  The sum of absolute products is returned too.
 *
 * 2. oracle_brmerge_rows -- the accumulation method of Section III-B
 *    (Algorithm 1), one row at a time: a multiplying phase that appends the
 *    scaled rows B_k* for the entries of A_i* in stored order into one buffer
 *    while recording where each list starts, then the accumulating phase.
 *    The method's rounds merge the lists two by two in order (lists 0 and 1,
 *    lists 2 and 3, ...; an odd last list passes unchanged) between two
 *    buffers, adding the values of equal columns; after r rounds list p is
 *    the merge of the original lists [p 2^r, (p+1) 2^r).  This file
 *    evaluates that binary tree depth first (tree_node), each level in the
 *    buffer its round would write.  Its floating-point additions are
 *    therefore grouped exactly as the method groups them, which makes its
 *    values the bitwise expectation for any implementation that keeps that
 *    grouping.
 *
 * All products are single IEEE-754 double multiplications; the file must be
 * compiled without floating-point contraction (-ffp-contract=off) and without
 * fast-math.
 *
 * Row pointers are int64 here (the Python wrapper widens int32 inputs).
 * Return value of every entry point: 0 on success, -1 on allocation failure,
 * -2 on an argument error.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int cmp_i32(const void *x, const void *y) {
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

static int clamp_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    return nthreads < 1 ? 1 : nthreads;
}

/* Number of products of each row: nprod_i = sum over stored A_ik of |B_k*|
 * (the per-row work measure of Sections II-A.4 and III-D). */
int oracle_row_nprod(int64_t row_begin, int64_t row_end, const int64_t *a_rpt,
                     const int32_t *a_col, const int64_t *b_rpt, int64_t *nprod) {
    for (int64_t i = row_begin; i < row_end; ++i) {
        int64_t s = 0;
        for (int64_t p = a_rpt[i]; p < a_rpt[i + 1]; ++p) {
            int32_t k = a_col[p];
            s += b_rpt[k + 1] - b_rpt[k];
        }
        nprod[i - row_begin] = s;
    }
    return 0;
}

/* Pass 1 of the definition: the number of distinct columns of each row of C,
 * found with a marker array over the N columns of B. */
int oracle_spa_counts(int64_t N, int64_t row_begin, int64_t row_end, const int64_t *a_rpt,
                      const int32_t *a_col, const int64_t *b_rpt, const int32_t *b_col,
                      int64_t *counts, int nthreads) {
    if (N < 0 || row_end < row_begin) return -2;
    int err = 0;
    nthreads = clamp_threads(nthreads);
#pragma omp parallel num_threads(nthreads)
    {
        int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
        if (!mark) {
#pragma omp atomic write
            err = -1;
        } else {
            for (int64_t j = 0; j < N; ++j) mark[j] = -1;
#pragma omp for schedule(dynamic, 256)
            for (int64_t i = row_begin; i < row_end; ++i) {
                int64_t cnt = 0;
                for (int64_t p = a_rpt[i]; p < a_rpt[i + 1]; ++p) {
                    int32_t k = a_col[p];
                    for (int64_t q = b_rpt[k]; q < b_rpt[k + 1]; ++q) {
                        int32_t j = b_col[q];
                        if (mark[j] != i) {
                            mark[j] = i;
                            ++cnt;
                        }
                    }
                }
                counts[i - row_begin] = cnt;
            }
            free(mark);
        }
    }
    return err;
}

/* The structure of C alone, for products too large to hold on the host:
 * per row the number of distinct columns (as oracle_spa_counts) and their
 * sum, from the same marker-array walk. */
int oracle_spa_pattern_sums(int64_t N, int64_t row_begin, int64_t row_end, const int64_t *a_rpt,
                            const int32_t *a_col, const int64_t *b_rpt, const int32_t *b_col,
                            int64_t *counts, int64_t *colsums, int nthreads) {
    if (N < 0 || row_end < row_begin) return -2;
    int err = 0;
    nthreads = clamp_threads(nthreads);
#pragma omp parallel num_threads(nthreads)
    {
        int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
        if (!mark) {
#pragma omp atomic write
            err = -1;
        } else {
            for (int64_t j = 0; j < N; ++j) mark[j] = -1;
#pragma omp for schedule(dynamic, 256)
            for (int64_t i = row_begin; i < row_end; ++i) {
                int64_t cnt = 0, sum = 0;
                for (int64_t p = a_rpt[i]; p < a_rpt[i + 1]; ++p) {
                    int32_t k = a_col[p];
                    for (int64_t q = b_rpt[k]; q < b_rpt[k + 1]; ++q) {
                        int32_t j = b_col[q];
                        if (mark[j] != i) {
                            mark[j] = i;
                            ++cnt;
                            sum += j;
                        }
                    }
                }
                counts[i - row_begin] = cnt;
                colsums[i - row_begin] = sum;
            }
            free(mark);
        }
    }
    return err;
}

/* Pass 2 of the definition.  c_off[i - row_begin] is where row i starts in
 * c_col / c_val / c_abs (so the caller can compute any subset of rows). */
int oracle_spa_fill(int64_t N, int64_t row_begin, int64_t row_end, const int64_t *a_rpt,
                    const int32_t *a_col, const double *a_val, const int64_t *b_rpt,
                    const int32_t *b_col, const double *b_val, const int64_t *c_off,
                    int32_t *c_col, double *c_val, double *c_abs, int nthreads) {
    if (N < 0 || row_end < row_begin) return -2;
    int err = 0;
    nthreads = clamp_threads(nthreads);
#pragma omp parallel num_threads(nthreads)
    {
        size_t n = (size_t)(N > 0 ? N : 1);
        int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * n);
        double *sum = (double *)malloc(sizeof(double) * n);
        double *comp = (double *)malloc(sizeof(double) * n);
        double *absum = (double *)malloc(sizeof(double) * n);
        if (!mark || !sum || !comp || !absum) {
#pragma omp atomic write
            err = -1;
        } else {
            for (int64_t j = 0; j < N; ++j) mark[j] = -1;
#pragma omp for schedule(dynamic, 64)
            for (int64_t i = row_begin; i < row_end; ++i) {
                int32_t *touched = c_col + c_off[i - row_begin];
                int64_t cnt = 0;
                for (int64_t p = a_rpt[i]; p < a_rpt[i + 1]; ++p) {
                    int32_t k = a_col[p];
                    double a = a_val[p];
                    for (int64_t q = b_rpt[k]; q < b_rpt[k + 1]; ++q) {
                        int32_t j = b_col[q];
                        double prod = a * b_val[q];
                        if (mark[j] != i) {
                            mark[j] = i;
                            touched[cnt++] = j;
                            sum[j] = 0.0;
                            comp[j] = 0.0;
                            absum[j] = 0.0;
                        }
                        /* Neumaier's compensated update of sum[j] by prod */
                        double s = sum[j], t = s + prod;
                        if (fabs(s) >= fabs(prod))
                            comp[j] += (s - t) + prod;
                        else
                            comp[j] += (prod - t) + s;
                        sum[j] = t;
                        absum[j] += fabs(prod);
                    }
                }
                qsort(touched, (size_t)cnt, sizeof(int32_t), cmp_i32);
                double *v = c_val + c_off[i - row_begin];
                double *av = c_abs + c_off[i - row_begin];
                for (int64_t e = 0; e < cnt; ++e) {
                    int32_t j = touched[e];
                    v[e] = sum[j] + comp[j];
                    av[e] = absum[j];
                }
            }
        }
        free(mark);
        free(sum);
        free(comp);
        free(absum);
    }
    return err;
}

/* Merge two ascending (col, val) lists; equal columns are combined by one
 * addition of the left list's value and the right list's value.  Returns the
 * length of the merged list. */
static int64_t merge_two(const int32_t *xc, const double *xv, int64_t nx, const int32_t *yc,
                         const double *yv, int64_t ny, int32_t *oc, double *ov) {
    int64_t i = 0, j = 0, o = 0;
    while (i < nx && j < ny) {
        if (xc[i] < yc[j]) {
            oc[o] = xc[i];
            ov[o++] = xv[i++];
        } else if (yc[j] < xc[i]) {
            oc[o] = yc[j];
            ov[o++] = yv[j++];
        } else {
            oc[o] = xc[i];
            ov[o++] = xv[i++] + yv[j++];
        }
    }
    while (i < nx) {
        oc[o] = xc[i];
        ov[o++] = xv[i++];
    }
    while (j < ny) {
        oc[o] = yc[j];
        ov[o++] = yv[j++];
    }
    return o;
}

/* One row's lists after the multiplying phase: list l occupies positions
 * [start[l], start[l+1]) of buf[0]; buf[1] is scratch of the same size. */
typedef struct {
    int64_t nlists;
    const int64_t *start;
    int32_t *col[2];
    double *val[2];
} row_lists;

/* The node of the merge tree at level h with index p: the merged list of the
 * lists [p 2^h, (p+1) 2^h) (clipped to the row's list count).  Section III-B
 * pairs the lists of a round two by two in order -- list 2p with list 2p+1 --
 * and lets an odd last list through unchanged, round after round, so after h
 * rounds the p-th list is exactly the merge of these leaves, and the left
 * half is always added before the right half.  A node's result is placed at
 * the position of its first leaf in buffer h mod 2: the children of a level-h
 * node sit in buffer (h-1) mod 2 inside the node's own range of positions,
 * so the two buffers alternate between levels as the ping-pong buffers of
 * the method alternate between rounds.  Returns the node's length. */
static int64_t tree_node(const row_lists *r, int h, int64_t p) {
    const int64_t first = p << h;
    if (h == 0) return r->start[first + 1] - r->start[first];
    const int64_t half = (int64_t)1 << (h - 1);
    const int64_t pos = r->start[first];
    const int src = (h - 1) & 1, dst = h & 1;
    const int64_t nl = tree_node(r, h - 1, 2 * p);
    if (first + half >= r->nlists) {
        /* no right half: the left child moves up a level as it is */
        memcpy(r->col[dst] + pos, r->col[src] + pos, 4 * (size_t)nl);
        memcpy(r->val[dst] + pos, r->val[src] + pos, 8 * (size_t)nl);
        return nl;
    }
    const int64_t nr = tree_node(r, h - 1, 2 * p + 1);
    const int64_t rpos = r->start[first + half];
    return merge_two(r->col[src] + pos, r->val[src] + pos, nl, r->col[src] + rpos, r->val[src] + rpos, nr,
                     r->col[dst] + pos, r->val[dst] + pos);
}

/* The accumulation method of Section III-B, one row at a time (see the file
 * header).  c_off as in oracle_spa_fill; row_len receives each row's length
 * and rounds (may be NULL) the number of merge rounds each row took,
 * ceil(log2(lists)).  Rows whose list count is 0 produce an empty row; a
 * single list is the result as it is.  Empty B rows still count as lists. */
int oracle_brmerge_rows(int64_t row_begin, int64_t row_end, const int64_t *a_rpt,
                        const int32_t *a_col, const double *a_val, const int64_t *b_rpt,
                        const int32_t *b_col, const double *b_val, const int64_t *c_off,
                        int32_t *c_col, double *c_val, int64_t *row_len, int32_t *rounds,
                        int nthreads) {
    if (row_end < row_begin) return -2;
    /* scratch sizes: the largest product count and list count of a row */
    int64_t max_nprod = 0, max_lists = 0;
    for (int64_t i = row_begin; i < row_end; ++i) {
        int64_t np = 0;
        for (int64_t p = a_rpt[i]; p < a_rpt[i + 1]; ++p) np += b_rpt[a_col[p] + 1] - b_rpt[a_col[p]];
        if (np > max_nprod) max_nprod = np;
        if (a_rpt[i + 1] - a_rpt[i] > max_lists) max_lists = a_rpt[i + 1] - a_rpt[i];
    }
    int err = 0;
    nthreads = clamp_threads(nthreads);
#pragma omp parallel num_threads(nthreads)
    {
        size_t cap = (size_t)(max_nprod > 0 ? max_nprod : 1);
        int64_t *start = (int64_t *)malloc(8 * ((size_t)max_lists + 1));
        row_lists r;
        r.start = start;
        r.col[0] = (int32_t *)malloc(4 * cap);
        r.col[1] = (int32_t *)malloc(4 * cap);
        r.val[0] = (double *)malloc(8 * cap);
        r.val[1] = (double *)malloc(8 * cap);
        if (!start || !r.col[0] || !r.col[1] || !r.val[0] || !r.val[1]) {
#pragma omp atomic write
            err = -1;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (int64_t i = row_begin; i < row_end; ++i) {
                /* multiplying phase: the scaled row B_k* of every stored A_ik,
                 * in stored order, one list each, appended to buffer 0 */
                int64_t L = a_rpt[i + 1] - a_rpt[i], fill = 0;
                for (int64_t l = 0; l < L; ++l) {
                    const int64_t p = a_rpt[i] + l;
                    const int32_t k = a_col[p];
                    start[l] = fill;
                    for (int64_t q = b_rpt[k]; q < b_rpt[k + 1]; ++q, ++fill) {
                        r.col[0][fill] = b_col[q];
                        r.val[0][fill] = a_val[p] * b_val[q];
                    }
                }
                start[L] = fill;
                /* accumulating phase: the root of the tree of ceil(log2 L)
                 * levels holds the row */
                int H = 0;
                while (((int64_t)1 << H) < L) ++H;
                int64_t len = 0;
                if (L > 0) {
                    r.nlists = L;
                    len = tree_node(&r, H, 0);
                }
                memcpy(c_col + c_off[i - row_begin], r.col[H & 1], 4 * (size_t)len);
                memcpy(c_val + c_off[i - row_begin], r.val[H & 1], 8 * (size_t)len);
                row_len[i - row_begin] = len;
                if (rounds) rounds[i - row_begin] = H;
            }
        }
        free(start);
        free(r.col[0]);
        free(r.col[1]);
        free(r.val[0]);
        free(r.val[1]);
    }
    return err;
}

/* Threads the OpenMP runtime would use by default (1 without OpenMP). */
int oracle_max_threads(void) { return clamp_threads(0); }
