// Kernels of the row-wise SpGEMM C = A*B with the BRMerge accumulation
// (Section III-B, Algorithm 1) and the precise allocation (Section II-B.2,
// Section III-D.2), written for CDNA4 (gfx950, 64-lane wavefronts, 160 KB of
// LDS per workgroup).
//
//   analysis  : per row the number of stored A entries (= lists) and of
//               products (Section III-D.2 step 1); the row's kernel class.
//   bin       : counting-sort of row ids by class (replaces the static split
//               of rows into equal-product groups, Section III-D).
//   symbolic  : exact distinct-column count per row (step 3), by hashing in
//               LDS (the paper's symbolic method) or, for heavy rows, by an
//               LDS bitmap over column slabs.
//   scan      : exclusive prefix sum of the counts into C's int64 row
//               pointers and nnz(C) (step 4).
//   numeric   : multiplying phase (scaled B rows appended in the order of
//               A's entries, coalesced) and accumulating phase (rounds of
//               pairwise merges, ping-pong between two LDS buffers), written
//               straight into C (step 5 and Algorithm 1's final store).
//
// The merge of two sorted lists inside a round is parallel: every element
// finds its place in the merged list by a binary search in its sibling list
// (a merge-path rank), duplicates are detected in the same search and
// removed with a team-wide prefix count built from wavefront ballots.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "brm_device.h"
#include "brm_internal.h"

namespace brm {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
template <typename I>
__device__ __forceinline__ int64_t ld_rpt(const void *p, int64_t i) {
    return (int64_t)gload(reinterpret_cast<const I *>(p) + i);
}

__host__ __device__ __forceinline__ int ceil_log2(int64_t x) {
    int r = 0;
    while (((int64_t)1 << r) < x) ++r;
    return r;
}

// Lane windows of a row (register merging of rows with at most 64 products):
// its lists padded to the next power of two of the longest, their count to
// the next power of two, all in one wavefront.  Returns log2 of the window
// width, or -1 when the row does not fit.
__device__ __forceinline__ int window_shift(int64_t nlists, int64_t maxlen) {
    if (nlists > kWave || maxlen > kWave) return -1;
    const int sw = ceil_log2(maxlen > 0 ? maxlen : 1);
    const int sl = ceil_log2(nlists > 0 ? nlists : 1);
    return sw + sl <= 6 ? sw : -1;
}

// Lane windows of 2 to 16 registers per lane (kClassMulti): at most 64
// lists, padded total between 128 and 1024 slots, and at most 8 slots per
// product (more padding than that is cheaper in the LDS classes).  Returns
// log2 of the window width, or -1 when the row does not fit.
constexpr int kMwSlots = 1024;
__device__ __forceinline__ int multi_shift(int64_t nlists, int64_t maxlen, int64_t nprod) {
    if (nlists > kWave || maxlen > kMwSlots) return -1;
    const int sw = ceil_log2(maxlen > 0 ? maxlen : 1);
    const int t = sw + ceil_log2(nlists > 0 ? nlists : 1);
    if (t <= 6 || t > 10 || ((int64_t)1 << t) > 8 * nprod) return -1;
    return sw;
}

__device__ __forceinline__ int classify(int64_t nlists, int64_t nprod, int64_t maxlen, const Thresholds &th) {
    if (nprod == 0) return kClassEmpty;
    const int64_t w = nprod > nlists ? nprod : nlists;  // LDS holds both products and lists
    // under lane windows, the wave-small class takes only rows that fit them
    const bool small_ok = !th.windows || window_shift(nlists, maxlen) >= 0;
    if (th.force >= kClassWaveSmall) {
        // debug routing: every non-empty row that fits the forced class goes
        // there (single-list rows included), every other row to the heavy path
        const int64_t cap = th.force == kClassWaveSmall ? kCapWaveSmall
                            : th.force == kClassWave    ? kCapWave
                            : th.force == kClassGroup   ? kCapGroup
                            : th.force == kClassBlock   ? kCapBlock
                                                        : 0;
        if (th.force == kClassWaveSmall && !small_ok) return kClassHeavy;
        if (th.force == kClassMulti) return th.multi && multi_shift(nlists, maxlen, nprod) >= 0 ? kClassMulti : kClassHeavy;
        return w <= cap ? th.force : kClassHeavy;
    }
    if (nlists == 1) return kClassCopy;
    if (w <= th.wave_small_max && small_ok) return kClassWaveSmall;
    if (th.multi && multi_shift(nlists, maxlen, nprod) >= 0) return kClassMulti;
    if (w <= th.wave_max) return kClassWave;
    if (w <= th.group_max) return kClassGroup;
    if (w <= th.block_max) return kClassBlock;
    return kClassHeavy;
}

// Where the list (B row) of A's entry p comes from: B's row pointers through
// A's column index, or the per-entry (start, length) arrays that the analysis
// pass fills (one coalesced read instead of a dependent gather).
template <typename IB>
struct Lists {
    const int32_t *a_col;
    const void *b_rpt;
    const int64_t *b_end;    // end of every B row (B kept in slots), or nullptr: the next row's start
    const void *ent_bs;      // IB per entry of A, or nullptr
    const int32_t *ent_len;  // per entry of A, or nullptr
    __device__ __forceinline__ void get(int64_t p, int64_t &bs, int &ln) const {
        if (ent_len) {
            bs = ld_rpt<IB>(ent_bs, p);
            ln = gload(ent_len + p);
        } else {
            const int32_t k = gload(a_col + p);
            bs = ld_rpt<IB>(b_rpt, k);
            ln = (int)((b_end ? gload(b_end + k) : (int64_t)ld_rpt<IB>(b_rpt, k + 1)) - bs);
        }
    }
    // the per-entry arrays only (they must be present)
    __device__ __forceinline__ void get_ent(int64_t p, int64_t &bs, int &ln) const {
        bs = ld_rpt<IB>(ent_bs, p);
        ln = gload(ent_len + p);
    }
};

template <typename IB>
__host__ __device__ __forceinline__ Lists<IB> direct_lists(const int32_t *a_col, const void *b_rpt,
                                                           const int64_t *b_end = nullptr) {
    Lists<IB> l;
    l.a_col = a_col;
    l.b_rpt = b_rpt;
    l.b_end = b_end;
    l.ent_bs = nullptr;
    l.ent_len = nullptr;
    return l;
}

template <typename IB>
__host__ __forceinline__ Lists<IB> ws_lists(const CsrView &A, const CsrView &B, const Workspace &ws) {
    Lists<IB> l;
    l.a_col = A.col;
    l.b_rpt = B.rpt;
    l.b_end = nullptr;
    l.ent_bs = ws.ent_bs;
    l.ent_len = ws.ent_len;
    return l;
}

// ---------------------------------------------------------------------------
// control block reset
// ---------------------------------------------------------------------------
__global__ void k_zero_ctl(Ctl *ctl) {
    int64_t *p = reinterpret_cast<int64_t *>(ctl);
    const int n = (int)(sizeof(Ctl) / sizeof(int64_t));
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

hipError_t launch_zero_ctl(Ctl *ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_ctl, dim3(1), dim3(64), 0, s, ctl);
    return hipGetLastError();
}

__global__ void k_zero_words(unsigned long long *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

hipError_t launch_zero_words(unsigned long long *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned g = (unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    hipLaunchKernelGGL(k_zero_words, dim3(g), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// validation (optional): rpt[0] == 0, monotone, rpt[rows] == nnz, columns in
// range and strictly increasing within rows
// ---------------------------------------------------------------------------
template <typename I>
__global__ void k_validate(int64_t rows, int64_t nnz, const void *rpt, const int32_t *col,
                           int64_t ncols, int64_t err_rpt, int64_t err_col, Ctl *ctl) {
    int64_t bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += stride) {
        const int64_t a = ld_rpt<I>(rpt, i), b = ld_rpt<I>(rpt, i + 1);
        if ((i == 0 && a != 0) || b < a || (i == rows - 1 && b != nnz) || a < 0 || b > nnz) {
            bad |= err_rpt;
            continue;
        }
        int32_t prev = -1;
        for (int64_t p = a; p < b; ++p) {
            const int32_t c = col[p];
            if (c < 0 || (int64_t)c >= ncols || c <= prev) {
                bad |= err_col;
                break;
            }
            prev = c;
        }
    }
    if (rows == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        if (ld_rpt<I>(rpt, 0) != 0 || nnz != 0) bad |= err_rpt;
    }
    if (bad) atomicOr(reinterpret_cast<unsigned long long *>(&ctl->err), (unsigned long long)bad);
}

hipError_t launch_validate(const CsrView &X, int64_t ncols_limit, int64_t err_rpt, int64_t err_col,
                           Ctl *ctl, hipStream_t s) {
    int64_t blocks = (X.rows + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    if (X.rpt_bytes == 4)
        hipLaunchKernelGGL(k_validate<int32_t>, dim3((unsigned)blocks), dim3(256), 0, s, X.rows,
                           X.nnz, X.rpt, X.col, ncols_limit, err_rpt, err_col, ctl);
    else
        hipLaunchKernelGGL(k_validate<int64_t>, dim3((unsigned)blocks), dim3(256), 0, s, X.rows,
                           X.nnz, X.rpt, X.col, ncols_limit, err_rpt, err_col, ctl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// analysis: lists, products and class of every row
// ---------------------------------------------------------------------------
constexpr int kAnalysisThreads = 256;

// Per-row sums and maxima over one 64-entry window of a wavefront's chunk of
// consecutive rows (whose entries are one contiguous range, row after row):
// the window's lanes form segments that start at lane 0 and at every row
// whose first entry lies in the window (flags in LDS, then a ballot); a
// segmented inclusive scan leaves each lane its segment's sum and maximum so
// far, and every row's lane adds the values of the lane that holds the row's
// last entry in the window.  No atomics: rows of many entries in one window
// (27 for a 27-point stencil) do not serialize on one LDS address.
// The segment structure of one window: lane `seg0` is the first lane of the
// calling lane's segment; `src` is the lane holding the calling row's last
// entry in the window (or the calling lane), `mine` whether the row has
// entries in it.
struct WindowSegs {
    int seg0, src;
    bool mine;
};
__device__ __forceinline__ WindowSegs window_segs(int64_t eb, bool in, int64_t a0, int64_t a1, int32_t *flag,
                                                  int lane) {
    flag[lane] = 0;
    wave_sync();
    if (in && a0 < a1 && a0 >= eb && a0 < eb + kWave) flag[a0 - eb] = 1;
    wave_sync();
    const uint64_t heads = wave_ballot(lane == 0 || flag[lane] != 0);
    const uint64_t upto = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull);
    WindowSegs w;
    w.seg0 = 63 - __builtin_clzll(heads & upto);
    const int64_t lo = a0 > eb ? a0 : eb;
    const int64_t hi = a1 < eb + kWave ? a1 : eb + kWave;
    w.mine = in && lo < hi;
    w.src = w.mine ? (int)(hi - 1 - eb) : lane;
    wave_sync();  // the flags are cleared again by the next window
    return w;
}

// Segmented inclusive scan of one quantity over the window (op: 0 sum, 1
// max, 2 min), then the value at the row's last entry.
template <int OP, typename V>
__device__ __forceinline__ V segmented_at_row_end(V v, const WindowSegs &w, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const V y = __shfl_up(v, d, kWave);
        if (lane - d >= w.seg0) {
            if constexpr (OP == 0) v += y;
            else if constexpr (OP == 1) v = v > y ? v : y;
            else v = v < y ? v : y;
        }
    }
    return __shfl(v, w.src, kWave);
}

// Per-row sums and maxima over one 64-entry window of a wavefront's chunk of
// consecutive rows (whose entries are one contiguous range, row after row):
// the window's lanes form segments that start at lane 0 and at every row
// whose first entry lies in the window (flags in LDS, then a ballot); a
// segmented inclusive scan leaves each lane its segment's sum and maximum so
// far, and every row's lane adds the values of the lane that holds the row's
// last entry in the window.  No atomics: rows of many entries in one window
// (27 for a 27-point stencil) do not serialize on one LDS address.
__device__ __forceinline__ void window_row_reduce(int64_t eb, bool in, int64_t a0, int64_t a1, int64_t n,
                                                  int32_t *flag, int lane, int64_t &np_r, int &mx_r) {
    const WindowSegs w = window_segs(eb, in, a0, a1, flag, lane);
    const int64_t gs = segmented_at_row_end<0>(n, w, lane);
    const int gm = segmented_at_row_end<1>((int)n, w, lane);
    if (w.mine) {
        np_r += gs;
        mx_r = mx_r > gm ? mx_r : gm;
    }
}

// The windows of one wavefront's chunk of entries [e0, e1) (consecutive
// rows), kAnaUnroll windows at a time: their columns, then B's row pointers
// of all of them gathered together (the loads in flight at once) while the
// next block's columns load, then each window's list descriptors stored and
// its rows reduced in window order.
constexpr int kAnaUnroll = 4;
template <typename IB>
__device__ __forceinline__ void analysis_windows(int64_t e0, int64_t e1, const int32_t *a_col, const IB *brp,
                                                 const int64_t *bend, IB *ent_bs, int32_t *ent_len, bool in,
                                                 int64_t a0, int64_t a1,
                                                 int32_t *flag, int lane, int64_t &np_r, int &mx_r) {
    constexpr int U = kAnaUnroll;
    int32_t k[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t e = e0 + u * kWave + lane;
        k[u] = e < e1 ? gload(a_col + e) : 0;
    }
    for (int64_t eb = e0; eb < e1; eb += U * kWave) {
        IB bs[U], be[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = eb + u * kWave + lane;
            bs[u] = 0;
            be[u] = 0;
            if (e < e1) {
                bs[u] = gload(brp + k[u]);
                be[u] = bend ? (IB)gload(bend + k[u]) : gload(brp + k[u] + 1);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = eb + (U + u) * kWave + lane;
            k[u] = e < e1 ? gload(a_col + e) : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t wb = eb + u * kWave;
            if (wb >= e1) break;  // uniform over the wavefront
            const int64_t e = wb + lane;
            const bool valid = e < e1;
            const int64_t n = valid ? (int64_t)be[u] - (int64_t)bs[u] : 0;
            if (valid) {
                gstore(ent_bs + e, bs[u]);
                gstore(ent_len + e, (int32_t)n);
            }
            window_row_reduce(wb, in, a0, a1, n, flag, lane, np_r, mx_r);
        }
    }
}

// first and last column of every row of B
template <typename IB>
__global__ __launch_bounds__(256) void k_row_ends(int64_t K, const IB *rpt, const int32_t *col, int4 *ends) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b0 = rpt[k], b1 = rpt[k + 1];
        // first and last column, length, start (low 32 bits; the whole start
        // with 32-bit row pointers): one 16-byte gather per A entry gives the
        // analysis of the features everything it needs of a B row
        ends[k] = b1 > b0 ? make_int4(col[b0], col[b1 - 1], (int)(b1 - b0), (int)b0)
                          : make_int4(-1, -1, 0, (int)b0);
    }
}

hipError_t launch_row_ends(const CsrView &B, int32_t *ends, hipStream_t s) {
    if (B.rows == 0) return hipSuccess;
    const int g = (int)std::min<int64_t>((B.rows + 255) / 256, 4096);
    if (B.rpt_bytes == 4)
        hipLaunchKernelGGL((k_row_ends<int32_t>), dim3(g), dim3(256), 0, s, B.rows,
                           static_cast<const int32_t *>(B.rpt), B.col, reinterpret_cast<int4 *>(ends));
    else
        hipLaunchKernelGGL((k_row_ends<int64_t>), dim3(g), dim3(256), 0, s, B.rows,
                           static_cast<const int64_t *>(B.rpt), B.col, reinterpret_cast<int4 *>(ends));
    return hipGetLastError();
}

// FEAT: also the size predictor's features of every row (the learned
// allocation), from the same pass over A's entries
template <typename IA, typename IB, bool FEAT>
__global__ __launch_bounds__(kAnalysisThreads) void k_analysis(
    int64_t M, const void *a_rpt, const int32_t *a_col, const void *b_rpt, Thresholds th,
    int64_t *row_nprod, uint8_t *row_class, int32_t *row_size, Ctl *ctl, IB *ent_bs, int32_t *ent_len,
    RowFeatures rf) {
    constexpr int kW = kAnalysisThreads / kWave;
    __shared__ int64_t s_count[kNumClasses];
    __shared__ int64_t s_nprod;
    __shared__ int64_t s_start[kW][kWave + 1];  // entry offset of every row of the wave's chunk
    __shared__ int32_t s_flag[kW][kWave];  // row heads of a window
    if (threadIdx.x < kNumClasses) s_count[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_nprod = 0;
    __syncthreads();

    // rows per class, counted per chunk by ballots (wavefront totals: scalar registers)
    int64_t my_count[kNumClasses];
#pragma unroll
    for (int c = 0; c < kNumClasses; ++c) my_count[c] = 0;
    int64_t my_nprod = 0;

    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // a wavefront takes 64 consecutive rows; their entries are one contiguous
    // range of A, walked entry by entry so that every access is coalesced
    const int64_t base0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1));
    for (int64_t base = base0; base < M; base += stride) {
        const int64_t i = base + lane;
        const bool in = i < M;
        const int nrows = (M - base) < kWave ? (int)(M - base) : kWave;
        int64_t a0 = 0, a1 = 0;
        if (in) {
            a0 = ld_rpt<IA>(a_rpt, i);
            a1 = ld_rpt<IA>(a_rpt, i + 1);
            s_start[w][lane] = a0;
        }
        if (lane == nrows - 1) s_start[w][nrows] = a1;
        wave_sync();
        const int64_t e0 = s_start[w][0], e1 = s_start[w][nrows];
        int64_t np_r = 0;
        int mx_r = 0;
        int mn_r = INT32_MAX, first_r = INT32_MAX, last_r = -1;
        if constexpr (FEAT) {
            // the predictor's features need the shortest list and the column
            // span as well: three more segmented reductions per window
            const IB *brp = reinterpret_cast<const IB *>(b_rpt);
            for (int64_t eb = e0; eb < e1; eb += kWave) {
                const int64_t e = eb + lane;
                int64_t n = 0;
                int f = INT32_MAX, l = -1;
                int mnv = INT32_MAX;
                if (e < e1) {
                    const int32_t k = a_col[e];
                    // the row's 16-byte record, as two 64-bit words of one line
                    const int64_t *rp = reinterpret_cast<const int64_t *>(rf.b_ends) + 2 * (int64_t)k;
                    const int64_t w0 = gload(rp), w1 = gload(rp + 1);
                    const int4 re = make_int4((int)w0, (int)(w0 >> 32), (int)w1, (int)(w1 >> 32));
                    IB bs;
                    if constexpr (sizeof(IB) == 4) {
                        bs = (IB)re.w;  // the row's start: no gather of B's row pointers
                        n = re.z;
                    } else {
                        bs = brp[k];
                        n = (int64_t)brp[k + 1] - (int64_t)bs;
                    }
                    ent_bs[e] = bs;
                    ent_len[e] = (int32_t)n;
                    mnv = (int)n;
                    if (n > 0) {
                        f = re.x;
                        l = re.y;
                    }
                }
                const WindowSegs ws = window_segs(eb, in, a0, a1, s_flag[w], lane);
                const int64_t gs = segmented_at_row_end<0>(n, ws, lane);
                const int gm = segmented_at_row_end<1>((int)n, ws, lane);
                const int gn = segmented_at_row_end<2>(mnv, ws, lane);
                const int gf = segmented_at_row_end<2>(f, ws, lane);
                const int gl = segmented_at_row_end<1>(l, ws, lane);
                if (ws.mine) {
                    np_r += gs;
                    mx_r = mx_r > gm ? mx_r : gm;
                    mn_r = mn_r < gn ? mn_r : gn;
                    first_r = first_r < gf ? first_r : gf;
                    last_r = last_r > gl ? last_r : gl;
                }
            }
        } else {
            analysis_windows<IB>(e0, e1, a_col, reinterpret_cast<const IB *>(b_rpt), nullptr, ent_bs, ent_len, in,
                                 a0, a1,
                                 s_flag[w], lane, np_r, mx_r);
        }
        int cls_l = -1;  // the lane's row's class
        if (in) {
            const int64_t np = np_r;
            const int mx = mx_r;
            // the row kernels count a row's products in int32: a longer row
            // goes to no kernel and fails the call
            const bool too_long = np > (int64_t)INT32_MAX;
            if (too_long)
                atomicOr(reinterpret_cast<unsigned long long *>(&ctl->err), (unsigned long long)kErrRowProducts);
            const int cls = too_long ? (int)kClassEmpty : classify(a1 - a0, np, mx, th);
            row_nprod[i] = np;
            const int sw = (cls == kClassWaveSmall && th.windows) ? window_shift(a1 - a0, mx)
                           : cls == kClassMulti                   ? multi_shift(a1 - a0, mx, np)
                                                                  : 0;
            row_class[i] = (uint8_t)(cls | (sw << kClassBits));
            cls_l = cls;
            if constexpr (FEAT) {
                // the predictor's features (lists, products and column span
                // the last two relative to B's column count, longest and
                // shortest list, products per spanned column); bounds of
                // the row size
                const int64_t L = a1 - a0;
                const int64_t mn = L == 0 ? 0 : mn_r;
                const int64_t first = first_r, last = last_r;
                const int64_t span = last >= first ? last - first + 1 : 0;
                row_features6(rf.feats + 6 * i, L, np, mx, mn, span, rf.ncols);
                rf.predicted[i] = (np > 0 && L >= 2) ? 1 : 0;
                rf.lo[i] = (int32_t)(np == 0 ? 0 : (L == 1 ? np : mx));
                rf.hi[i] = (int32_t)(np == 0 ? 0 : (L == 1 ? np : (np < span ? np : span)));
            }
            if (cls == kClassEmpty) row_size[i] = 0;
            if (cls == kClassCopy) row_size[i] = (int32_t)np;
            my_nprod += np;
        }
#pragma unroll
        for (int c = 0; c < kNumClasses; ++c) my_count[c] += __popcll(wave_ballot(cls_l == c));
        wave_sync();
    }
#pragma unroll
    for (int c = 0; c < kNumClasses; ++c) {
        const int64_t t = my_count[c];
        if (lane == 0 && t) atomicAdd(reinterpret_cast<unsigned long long *>(&s_count[c]),
                                      (unsigned long long)t);
    }
    {
        const int64_t t = wave_sum(my_nprod);
        if (lane == 0 && t) atomicAdd(reinterpret_cast<unsigned long long *>(&s_nprod),
                                      (unsigned long long)t);
    }
    __syncthreads();
    if (threadIdx.x < kNumClasses && s_count[threadIdx.x])
        atomicAdd(reinterpret_cast<unsigned long long *>(&ctl->count[threadIdx.x]),
                  (unsigned long long)s_count[threadIdx.x]);
    if (threadIdx.x == 0 && s_nprod)
        atomicAdd(reinterpret_cast<unsigned long long *>(&ctl->nprod), (unsigned long long)s_nprod);
}

hipError_t launch_analysis(const CsrView &A, const CsrView &B, const Thresholds &th,
                           const Workspace &ws, int grid, hipStream_t s, const RowFeatures *rf) {
    const dim3 g(grid), b(kAnalysisThreads);
    RowFeatures none{};
#define BRM_ANALYSIS(IA, IB)                                                                         \
    do {                                                                                             \
        if (rf)                                                                                      \
            hipLaunchKernelGGL((k_analysis<IA, IB, true>), g, b, 0, s, A.rows, A.rpt, A.col, B.rpt, th, \
                               ws.row_nprod, ws.row_class, ws.row_size, ws.ctl,                      \
                               reinterpret_cast<IB *>(ws.ent_bs), ws.ent_len, *rf);                  \
        else                                                                                         \
            hipLaunchKernelGGL((k_analysis<IA, IB, false>), g, b, 0, s, A.rows, A.rpt, A.col, B.rpt,    \
                               th, ws.row_nprod, ws.row_class, ws.row_size, ws.ctl,                  \
                               reinterpret_cast<IB *>(ws.ent_bs), ws.ent_len, none);                 \
    } while (0)
    if (A.rpt_bytes == 4 && B.rpt_bytes == 4) BRM_ANALYSIS(int32_t, int32_t);
    else if (A.rpt_bytes == 4) BRM_ANALYSIS(int32_t, int64_t);
    else if (B.rpt_bytes == 4) BRM_ANALYSIS(int64_t, int32_t);
    else BRM_ANALYSIS(int64_t, int64_t);
#undef BRM_ANALYSIS
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// binning: row ids grouped by class (order inside a class is unspecified)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t class_start(const Ctl *ctl, int cls) {
    int64_t s = 0;
    for (int c = 0; c < cls; ++c) s += ctl->count[c];
    return s;
}

// Counting sort of rows by class: class_rows[class_start(c) + k] is the k-th
// row of class c.  The rows are 0 .. M-1, or rows[0 .. M-1] when a list is
// given; ctl->count must hold the totals per class, ctl->cursor zero.
__global__ __launch_bounds__(256) void k_bin(int64_t M, const int32_t *rows, const uint8_t *row_class,
                                             int32_t *class_rows, Ctl *ctl) {
    __shared__ int64_t s_base[kNumClasses];
    __shared__ int s_wave_cnt[kNumClasses];
    const int lane = lane_id();
    if (rows == nullptr) {
        // every row in one class (the counts hold exactly these M rows):
        // the class list is the identity, written as one coalesced stream
        int64_t tot = 0;
        bool one = false;
#pragma unroll
        for (int c = 0; c < kNumClasses; ++c) {
            const int64_t k = ctl->count[c];
            tot += k;
            one = one || k == M;
        }
        if (tot == M && one) {
            for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x)
                class_rows[i] = (int32_t)i;
            return;
        }
    }
    // every workgroup bins one contiguous range of rows, so the rows of a
    // class sit in row order inside each workgroup's reservation
    const int64_t per = ((M + gridDim.x - 1) / gridDim.x + blockDim.x - 1) / blockDim.x * blockDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < M ? lo + per : M;
    const int64_t stride = blockDim.x;
    // pass 1: this block's rows per class, one global reservation per class
    int64_t my_count[kNumClasses];
#pragma unroll
    for (int c = 0; c < kNumClasses; ++c) my_count[c] = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += stride) {
        const int cls = row_class[rows ? (int64_t)rows[i] : i] & kClassMask;
#pragma unroll
        for (int c = 0; c < kNumClasses; ++c) my_count[c] += (cls == c);
    }
    if (threadIdx.x < kNumClasses) s_wave_cnt[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kNumClasses; ++c) {
        const int64_t t = wave_sum(my_count[c]);
        if (lane == 0 && t) atomicAdd(&s_wave_cnt[c], (int)t);
    }
    __syncthreads();
    if (threadIdx.x < kNumClasses) {
        const int c = threadIdx.x;
        const int n = s_wave_cnt[c];
        s_base[c] = class_start(ctl, c) +
                    (n ? (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(&ctl->cursor[c]),
                                            (unsigned long long)n)
                       : 0);
        s_wave_cnt[c] = 0;
    }
    __syncthreads();
    // pass 2: scatter; wavefront-aggregated LDS cursors
    const int64_t base0 = lo + (threadIdx.x & ~(kWave - 1));
    for (int64_t base = base0; base < hi; base += stride) {
        const int64_t i = base + lane;
        const int64_t r = i < hi ? (rows ? (int64_t)rows[i] : i) : 0;
        const int cls = i < hi ? (int)(row_class[r] & kClassMask) : -1;
#pragma unroll
        for (int c = 0; c < kNumClasses; ++c) {
            const uint64_t m = wave_ballot(cls == c);
            if (!m) continue;
            int wbase = 0;
            if (lane == __builtin_ctzll(m)) wbase = atomicAdd(&s_wave_cnt[c], __popcll(m));
            wbase = __shfl(wbase, __builtin_ctzll(m), kWave);
            if (cls == c) class_rows[s_base[c] + wbase + lanes_below(m)] = (int32_t)r;
        }
    }
}

hipError_t launch_bin(int64_t M, const Workspace &ws, int grid, hipStream_t s) {
    // every workgroup reserves its class ranges with one atomic per class on
    // the same counters: a grid of one workgroup per compute unit keeps
    // that contention low (each thread bins M / 65536 rows)
    grid = grid < 256 ? grid : 256;
    hipLaunchKernelGGL(k_bin, dim3(grid), dim3(256), 0, s, M, nullptr, ws.row_class, ws.class_rows, ws.ctl);
    return hipGetLastError();
}

// the upper bound of Section II-B.2: a row of C has at most as many entries
// as it has products
__global__ __launch_bounds__(256) void k_upper_sizes(int64_t M, const int64_t *row_nprod, int32_t *size) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x)
        size[i] = (int32_t)row_nprod[i];
}

hipError_t launch_upper_sizes(int64_t M, const int64_t *row_nprod, int32_t *size, hipStream_t s) {
    if (M == 0) return hipSuccess;
    const unsigned g = (unsigned)((M + 255) / 256 < 4096 ? (M + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_upper_sizes, dim3(g), dim3(256), 0, s, M, row_nprod, size);
    return hipGetLastError();
}

// per-class counts of a row list (wavefront-aggregated atomics)
__global__ __launch_bounds__(256) void k_count_list(int64_t n, const int32_t *rows, const uint8_t *row_class,
                                                    Ctl *ctl) {
    __shared__ int s_cnt[kNumClasses];
    const int lane = lane_id();
    if (threadIdx.x < kNumClasses) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    int my[kNumClasses];
#pragma unroll
    for (int c = 0; c < kNumClasses; ++c) my[c] = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int cls = (int)(row_class[rows[i]] & kClassMask);
#pragma unroll
        for (int c = 0; c < kNumClasses; ++c) my[c] += cls == c;
    }
#pragma unroll
    for (int c = 0; c < kNumClasses; ++c) {
        const int t = wave_sum(my[c]);
        if (lane == 0 && t) atomicAdd(&s_cnt[c], t);
    }
    __syncthreads();
    if (threadIdx.x < kNumClasses && s_cnt[threadIdx.x])
        atomicAdd(reinterpret_cast<unsigned long long *>(&ctl->count[threadIdx.x]),
                  (unsigned long long)s_cnt[threadIdx.x]);
}

hipError_t launch_bin_list(int64_t n, const int32_t *rows, const uint8_t *row_class, int32_t *class_rows,
                           Ctl *ctl, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_count_list, dim3(grid), dim3(256), 0, s, n, rows, row_class, ctl);
    hipLaunchKernelGGL(k_bin, dim3(grid), dim3(256), 0, s, n, rows, row_class, class_rows, ctl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gathering the products of one row, chunk of T lists at a time.  For every
// product the callback receives (position in the row, B entry index, list).
// ---------------------------------------------------------------------------
template <int T>
struct ListStage {
    int64_t bs[T];    // B row start of each list of the chunk
    int32_t off[T];   // offset of each list inside the chunk
    int32_t scan[Team<T>::kWaves + 1];
};

template <int T, typename IB, typename F>
__device__ __forceinline__ int64_t for_each_product(ListStage<T> &st, int tid, int64_t a0,
                                                    int64_t L, const Lists<IB> &lists, F &&f) {
    int64_t carry = 0;
    for (int64_t lb = 0; lb < L; lb += T) {
        const int64_t l = lb + tid;
        int ln = 0;
        int64_t bs = 0;
        if (l < L) lists.get(a0 + l, bs, ln);
        int tot;
        const int ex = Team<T>::excl_scan(ln, &tot, st.scan, tid);
        st.bs[tid] = bs;
        st.off[tid] = ex;
        const int nl = (int)((L - lb) < T ? (L - lb) : T);
        Team<T>::sync();
        for (int q = tid; q < tot; q += T) {
            const int t = upper_bound(st.off, nl, q) - 1;
            f(carry + q, st.bs[t] + (q - st.off[t]), (int)(lb + t));
        }
        carry += tot;
        Team<T>::sync();
    }
    return carry;
}

// ---------------------------------------------------------------------------
// symbolic, LDS hash table (open addressing, linear probing, load <= 1/2)
// ---------------------------------------------------------------------------
template <int TS>
__device__ __forceinline__ int hash_insert(int32_t *tab, int32_t c) {
    constexpr int kBits = __builtin_ctz(TS);
    uint32_t h = ((uint32_t)c * 2654435761u) >> (32 - kBits);
    while (true) {
        const int32_t old = atomicCAS(&tab[h], -1, c);
        if (old == -1) return 1;
        if (old == c) return 0;
        h = (h + 1) & (TS - 1);
    }
}

template <int T, int TS>
struct SymLds {
    int32_t tab[TS];
    ListStage<T> st;
    int32_t red[Team<T>::kWaves + 1];
};

// distinct columns of one row: every product's column is inserted once
template <int T, int TS, typename IA, typename IB>
__device__ __forceinline__ int sym_hash_row(SymLds<T, TS> &s, int tid, int64_t row, const void *a_rpt,
                                            const Lists<IB> &lists, const int32_t *b_col) {
    for (int t = tid; t < TS; t += T) s.tab[t] = -1;
    Team<T>::sync();
    const int64_t a0 = ld_rpt<IA>(a_rpt, row);
    const int64_t L = ld_rpt<IA>(a_rpt, row + 1) - a0;
    int added = 0;
    for_each_product<T, IB>(s.st, tid, a0, L, lists,
                            [&](int64_t, int64_t q, int) { added += hash_insert<TS>(s.tab, gload(b_col + (q))); });
    const int total = Team<T>::sum(added, s.red, tid);
    Team<T>::sync();
    return total;
}

// the rows of one class counted by LDS hash, TEAMS rows at a time per
// workgroup; `block` of `grid` workgroups take part
template <int T, int TEAMS, int TS, typename IA, typename IB>
__device__ __forceinline__ void sym_hash_rows(SymLds<T, TS> *lds, int cls, int64_t block, int64_t grid,
                                              const void *a_rpt, const Lists<IB> &lists, const int32_t *b_col,
                                              const int32_t *class_rows, int32_t *row_size, const Ctl *ctl) {
    const int team = threadIdx.x / T, tid = threadIdx.x % T;
    SymLds<T, TS> &s = lds[team];
    const int64_t count = ctl->count[cls];
    const int64_t start = class_start(ctl, cls);
    for (int64_t idx = block * TEAMS + team; idx < count; idx += grid * TEAMS) {
        const int64_t row = class_rows[start + idx];
        const int total = sym_hash_row<T, TS, IA, IB>(s, tid, row, a_rpt, lists, b_col);
        if (tid == 0) row_size[row] = total;
    }
}

template <int T, int TEAMS, int TS, typename IA, typename IB>
__global__ __launch_bounds__(T *TEAMS) void k_sym_hash(
    int cls, const void *a_rpt, Lists<IB> lists, const int32_t *b_col,
    const int32_t *class_rows, int32_t *row_size, const Ctl *ctl) {
    __shared__ SymLds<T, TS> lds[TEAMS];
    sym_hash_rows<T, TEAMS, TS, IA, IB>(lds, cls, blockIdx.x, gridDim.x, a_rpt, lists, b_col, class_rows,
                                        row_size, ctl);
}

// symbolic for heavy rows: LDS bitmap over column slabs of kBitmapBits
constexpr int kBitmapUnroll = 8;  // products per thread whose column gathers are in flight together
constexpr int kBitmapWords = 32768;  // 128 KB
constexpr int64_t kBitmapBits = (int64_t)kBitmapWords * 32;
constexpr int kHeavyThreads = 1024;

struct BitmapLds {
    uint32_t bm[kBitmapWords];
    ListStage<kHeavyThreads> st;
    int64_t red[Team<kHeavyThreads>::kWaves + 1];
};

// distinct columns of one row (columns below ncols) by the bitmap count
template <typename IA, typename IB>
__device__ __forceinline__ int64_t sym_bitmap_row(BitmapLds &s, int tid, int64_t row, int64_t ncols,
                                                  const void *a_rpt, const Lists<IB> &lists,
                                                  const int32_t *b_col) {
    const int64_t a0 = ld_rpt<IA>(a_rpt, row);
    const int64_t L = ld_rpt<IA>(a_rpt, row + 1) - a0;
    int64_t total = 0;
    for (int64_t lo = 0; lo < ncols; lo += kBitmapBits) {
        for (int w = tid; w < kBitmapWords; w += kHeavyThreads) s.bm[w] = 0u;
        __syncthreads();
        // the lists in chunks of kHeavyThreads; every thread takes
        // kBitmapUnroll products of a chunk at a time and gathers their
        // columns before setting any bit, so the gathers are in flight
        // together
        for (int64_t lb = 0; lb < L; lb += kHeavyThreads) {
            const int64_t l = lb + tid;
            int ln = 0;
            int64_t bs = 0;
            if (l < L) lists.get(a0 + l, bs, ln);
            int tot;
            const int ex = Team<kHeavyThreads>::excl_scan(ln, &tot, s.st.scan, tid);
            s.st.bs[tid] = bs;
            s.st.off[tid] = ex;
            const int nl = (int)((L - lb) < kHeavyThreads ? (L - lb) : kHeavyThreads);
            __syncthreads();
            for (int qb = 0; qb < tot; qb += kBitmapUnroll * kHeavyThreads) {
                int32_t col[kBitmapUnroll];
#pragma unroll
                for (int u = 0; u < kBitmapUnroll; ++u) {
                    const int q = qb + u * kHeavyThreads + tid;
                    col[u] = -1;
                    if (q < tot) {
                        const int t = upper_bound(s.st.off, nl, q) - 1;
                        col[u] = gload(b_col + (s.st.bs[t] + (q - s.st.off[t])));
                    }
                }
#pragma unroll
                for (int u = 0; u < kBitmapUnroll; ++u) {
                    const int64_t c = (int64_t)col[u] - lo;
                    if (col[u] >= 0 && c >= 0 && c < kBitmapBits) atomicOr(&s.bm[c >> 5], 1u << (c & 31));
                }
            }
            __syncthreads();
        }
        int64_t cnt = 0;
        for (int w = tid; w < kBitmapWords; w += kHeavyThreads) cnt += __popc(s.bm[w]);
        total += Team<kHeavyThreads>::sum(cnt, s.red, tid);
    }
    return total;
}

// the rows of one class counted by the bitmap, one row per workgroup at a
// time; `block` of `grid` workgroups take part
template <typename IA, typename IB>
__device__ __forceinline__ void sym_bitmap_rows(BitmapLds &s, int cls, int64_t block, int64_t grid, int64_t ncols,
                                                const void *a_rpt, const Lists<IB> &lists, const int32_t *b_col,
                                                const int32_t *class_rows, int32_t *row_size, const Ctl *ctl) {
    const int tid = threadIdx.x;
    const int64_t count = ctl->count[cls];
    const int64_t start = class_start(ctl, cls);
    for (int64_t idx = block; idx < count; idx += grid) {
        const int64_t row = class_rows[start + idx];
        const int64_t total = sym_bitmap_row<IA, IB>(s, tid, row, ncols, a_rpt, lists, b_col);
        if (tid == 0) row_size[row] = (int32_t)total;
        __syncthreads();
    }
}

// The symbolic passes of the block class (LDS hash, one row per workgroup)
// and of the heavy rows (LDS bitmap) in one launch of 1024-thread
// workgroups: workgroups [0, g_block) count the block class, the rest the
// heavy rows, each in the same LDS.  A class without rows then costs no
// launch of its own, and the heavy rows start on the CUs the block class
// has left.
template <typename IA, typename IB>
__global__ __launch_bounds__(kHeavyThreads) void k_sym_big(int64_t ncols, const void *a_rpt, Lists<IB> lists,
                                                           const int32_t *b_col, const int32_t *class_rows,
                                                           int32_t *row_size, const Ctl *ctl, int g_block) {
    using BlockLds = SymLds<kHeavyThreads, 2 * kCapBlock>;
    constexpr size_t kBlockBytes = sizeof(BlockLds), kHeavyBytes = sizeof(BitmapLds);
    __shared__ __align__(16) unsigned char raw[kBlockBytes > kHeavyBytes ? kBlockBytes : kHeavyBytes];
    const int b = blockIdx.x;  // uniform: every workgroup takes one branch whole
    if (b < g_block)
        sym_hash_rows<kHeavyThreads, 1, 2 * kCapBlock, IA, IB>(reinterpret_cast<BlockLds *>(raw), kClassBlock, b,
                                                               g_block, a_rpt, lists, b_col, class_rows, row_size,
                                                               ctl);
    else
        sym_bitmap_rows<IA, IB>(*reinterpret_cast<BitmapLds *>(raw), kClassHeavy, b - g_block,
                                (int64_t)gridDim.x - g_block, ncols, a_rpt, lists, b_col, class_rows, row_size,
                                ctl);
}

hipError_t launch_symbolic_big(const CsrView &A, const CsrView &B, const Workspace &ws, int g_block, int g_heavy,
                               hipStream_t s) {
    const int grid = g_block + g_heavy;
#define BRM_SYM_BIG(IA, IB)                                                                                \
    hipLaunchKernelGGL((k_sym_big<IA, IB>), dim3(grid), dim3(kHeavyThreads), 0, s, B.cols, A.rpt,             \
                       ws_lists<IB>(A, B, ws), B.col, ws.class_rows, ws.row_size, ws.ctl, g_block)
    if (A.rpt_bytes == 4 && B.rpt_bytes == 4) BRM_SYM_BIG(int32_t, int32_t);
    else if (A.rpt_bytes == 4) BRM_SYM_BIG(int32_t, int64_t);
    else if (B.rpt_bytes == 4) BRM_SYM_BIG(int64_t, int32_t);
    else BRM_SYM_BIG(int64_t, int64_t);
#undef BRM_SYM_BIG
    return hipGetLastError();
}

// symbolic for several short rows per team: one hash table of TS slots per row
template <int T, int G, int TS>
struct SymGroupLds {
    int32_t tab[G][TS];
    int32_t cnt[G];
    int32_t fl[G + 1];
    int64_t a0[G];
    int32_t L[G];
    int64_t row[G];
    int64_t bs[T];
    int32_t off[T + 1];
    int32_t lseg[T];
    int32_t scan[Team<T>::kWaves + 1];
};

template <int T, int TEAMS, int G, int TS, typename IA, typename IB>
__global__ __launch_bounds__(T *TEAMS) void k_sym_group(int cls, const void *a_rpt, Lists<IB> lists,
                                                        const int32_t *b_col, const int32_t *class_rows,
                                                        int32_t *row_size, const Ctl *ctl) {
    __shared__ SymGroupLds<T, G, TS> lds[TEAMS];
    const int team = threadIdx.x / T, tid = threadIdx.x % T;
    SymGroupLds<T, G, TS> &s = lds[team];
    const int64_t count = ctl->count[cls];
    const int64_t start = class_start(ctl, cls);
    for (int64_t base = ((int64_t)blockIdx.x * TEAMS + team) * G; base < count;
         base += (int64_t)gridDim.x * TEAMS * G) {
        const int n = (count - base) < G ? (int)(count - base) : G;
        for (int t = tid; t < G * TS; t += T) (&s.tab[0][0])[t] = -1;
        if (tid < kWave) {
            int Lj = 0;
            if (tid < n) {
                const int64_t row = class_rows[start + base + tid];
                const int64_t a0 = ld_rpt<IA>(a_rpt, row);
                Lj = (int)(ld_rpt<IA>(a_rpt, row + 1) - a0);
                s.row[tid] = row;
                s.a0[tid] = a0;
                s.L[tid] = Lj;
                s.cnt[tid] = 0;
            }
            const int incl = wave_incl_scan(Lj);
            if (tid < n) s.fl[tid + 1] = incl;
            if (tid == 0) s.fl[0] = 0;
        }
        Team<T>::sync();
        const int LT = s.fl[n];
        for (int lb = 0; lb < LT; lb += T) {
            const int gl = lb + tid;
            int ln = 0, j = 0;
            int64_t bs = 0;
            if (gl < LT) {
                j = upper_bound(s.fl, n, gl) - 1;
                lists.get(s.a0[j] + (gl - s.fl[j]), bs, ln);
            }
            int tot;
            const int ex = Team<T>::excl_scan(ln, &tot, s.scan, tid);
            s.bs[tid] = bs;
            s.off[tid] = ex;
            s.lseg[tid] = j;
            const int nl = (LT - lb) < T ? (LT - lb) : T;
            Team<T>::sync();
            for (int q = tid; q < tot; q += T) {
                const int t = upper_bound(s.off, nl, q) - 1;
                const int jj = s.lseg[t];
                if (hash_insert<TS>(s.tab[jj], gload(b_col + (s.bs[t] + (q - s.off[t]))))) atomicAdd(&s.cnt[jj], 1);
            }
            Team<T>::sync();
        }
        if (tid < n) row_size[s.row[tid]] = s.cnt[tid];
        Team<T>::sync();
    }
}

// pipelined counting of short rows (defined with the numeric kernels)
// The order of the register windows of the wave-small class, kept by the
// symbolic pass for the numeric pass of the precise method: for the class
// row of index j, perm[64 j + t] is the source lane of position t of the
// row's sorted window (bits 0-5) and whether the next position holds the
// same column (bit 6), 0xFF for an empty position; ucol[64 j + i] is the
// row's i-th distinct column.  The numeric pass then gathers B's values
// only and takes the tree's additions on the stored order (the bits of the
// merge are those of the round-by-round merges).
struct WinOrder {
    uint8_t *perm;
    int32_t *ucol;
};

template <bool HASH, typename IA, typename IB, bool ORD>
__global__ __launch_bounds__(256) void k_sym_win(int cls, const void *a_rpt, Lists<IB> lists,
                                                 const int32_t *b_col, const uint8_t *row_class,
                                                 const int32_t *class_rows, int32_t *row_size, Ctl *ctl,
                                                 WinOrder ord);
hipError_t launch_symbolic(const CsrView &A, const CsrView &B, const Workspace &ws, int cls,
                           int grid, hipStream_t s, int group_rows) {
#define BRM_SYM(KERNEL, BLOCK, IA, IB)                                                        \
    hipLaunchKernelGGL((KERNEL), dim3(grid), dim3(BLOCK), 0, s, cls, A.rpt, ws_lists<IB>(A, B, ws), \
                       B.col, ws.class_rows, ws.row_size, ws.ctl)
#define BRM_SYM_ALL(T, TEAMS, TS)                                                             \
    do {                                                                                      \
        if (A.rpt_bytes == 4 && B.rpt_bytes == 4)                                             \
            BRM_SYM((k_sym_hash<T, TEAMS, TS, int32_t, int32_t>), T *TEAMS, int32_t, int32_t); \
        else if (A.rpt_bytes == 4)                                                            \
            BRM_SYM((k_sym_hash<T, TEAMS, TS, int32_t, int64_t>), T *TEAMS, int32_t, int64_t); \
        else if (B.rpt_bytes == 4)                                                            \
            BRM_SYM((k_sym_hash<T, TEAMS, TS, int64_t, int32_t>), T *TEAMS, int64_t, int32_t); \
        else                                                                                  \
            BRM_SYM((k_sym_hash<T, TEAMS, TS, int64_t, int64_t>), T *TEAMS, int64_t, int64_t); \
    } while (0)
    switch (cls) {
        case kClassWaveSmall:
            if (group_rows == 0) {
                BRM_SYM_ALL(64, 4, 2 * kCapWaveSmall);
                break;
            }
            if (group_rows == 1 || group_rows == 2) {
                // 1: window-merge counts, 2: LDS hash counts
#define BRM_SYM_WIN(H, IA, IB)                                                                              \
    do {                                                                                                    \
        const WinOrder ord{ws.order, ws.ucol};                                                              \
        if (!H && ws.order)                                                                                 \
            hipLaunchKernelGGL((k_sym_win<H, IA, IB, true>), dim3(grid), dim3(256), 0, s, cls, A.rpt,        \
                               ws_lists<IB>(A, B, ws), B.col, ws.row_class, ws.class_rows, ws.row_size,     \
                               ws.ctl, ord);                                                                \
        else                                                                                                \
            hipLaunchKernelGGL((k_sym_win<H, IA, IB, false>), dim3(grid), dim3(256), 0, s, cls, A.rpt,       \
                               ws_lists<IB>(A, B, ws), B.col, ws.row_class, ws.class_rows, ws.row_size,     \
                               ws.ctl, ord);                                                                \
    } while (0)
#define BRM_SYM_WIN_ALL(H)                                                        \
    if (A.rpt_bytes == 4 && B.rpt_bytes == 4) BRM_SYM_WIN(H, int32_t, int32_t);  \
    else if (A.rpt_bytes == 4) BRM_SYM_WIN(H, int32_t, int64_t);                 \
    else if (B.rpt_bytes == 4) BRM_SYM_WIN(H, int64_t, int32_t);                 \
    else BRM_SYM_WIN(H, int64_t, int64_t)
                if (group_rows == 2) {
                    BRM_SYM_WIN_ALL(true);
                } else {
                    BRM_SYM_WIN_ALL(false);
                }
#undef BRM_SYM_WIN_ALL
#undef BRM_SYM_WIN
                break;
            }
            if (A.rpt_bytes == 4 && B.rpt_bytes == 4)
                BRM_SYM((k_sym_group<64, 4, kGroupRows, 2 * kCapWaveSmall, int32_t, int32_t>), 256, int32_t, int32_t);
            else if (A.rpt_bytes == 4)
                BRM_SYM((k_sym_group<64, 4, kGroupRows, 2 * kCapWaveSmall, int32_t, int64_t>), 256, int32_t, int64_t);
            else if (B.rpt_bytes == 4)
                BRM_SYM((k_sym_group<64, 4, kGroupRows, 2 * kCapWaveSmall, int64_t, int32_t>), 256, int64_t, int32_t);
            else
                BRM_SYM((k_sym_group<64, 4, kGroupRows, 2 * kCapWaveSmall, int64_t, int64_t>), 256, int64_t, int64_t);
            break;
        default: return hipErrorInvalidValue;
    }
#undef BRM_SYM_ALL
#undef BRM_SYM
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// scan: row sizes (int32) -> C's row pointers (int64) and nnz(C)
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanPer = kScanTile / kScanThreads;  // 4 rows per thread

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(int64_t M, const int32_t *row_size,
                                                              int64_t *tile_sum) {
    __shared__ int64_t red[Team<kScanThreads>::kWaves + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j)
        if (base + j < M) s += row_size[base + j];
    s = Team<kScanThreads>::sum(s, red, threadIdx.x);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = s;
}

// The control block into its host copy (pinned, mapped, coherent) with the
// scan's total in place: the host reads it once the stream has drained,
// without a copy of its own.  Called by every thread of the one workgroup
// that holds the total.
__device__ __forceinline__ void publish_ctl(const Ctl *src, Ctl *dst, const int64_t *total, int64_t value) {
    if (!dst) return;
    constexpr int kWords = (int)(sizeof(Ctl) / sizeof(int64_t));
    static_assert(sizeof(Ctl) % sizeof(int64_t) == 0, "control block in 64-bit words");
    const int t = threadIdx.x;
    if (t < kWords) {
        const int64_t *w = reinterpret_cast<const int64_t *>(src);
        reinterpret_cast<int64_t *>(dst)[t] = (w + t == total) ? value : w[t];
        __threadfence_system();
    }
}

__global__ __launch_bounds__(1024) void k_scan_top(int64_t ntiles, int64_t *tile_sum, int64_t M,
                                                   int64_t *c_rpt, int64_t *total, const Ctl *ctl_src,
                                                   Ctl *ctl_dst) {
    __shared__ int64_t scr[Team<1024>::kWaves + 1];
    int64_t carry = 0;
    for (int64_t b = 0; b < ntiles; b += 1024) {
        const int64_t i = b + threadIdx.x;
        const int64_t v = i < ntiles ? tile_sum[i] : 0;
        int64_t tot;
        const int64_t ex = Team<1024>::excl_scan(v, &tot, scr, threadIdx.x);
        if (i < ntiles) tile_sum[i] = carry + ex;  // in place: exclusive tile offsets
        carry += tot;
    }
    if (threadIdx.x == 0) {
        *total = carry;
        c_rpt[M] = carry;
    }
    publish_ctl(ctl_src, ctl_dst, total, carry);
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(int64_t M, const int32_t *row_size,
                                                             const int64_t *tile_off,
                                                             int64_t *c_rpt) {
    __shared__ int64_t scr[Team<kScanThreads>::kWaves + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int32_t v[kScanPer];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        v[j] = base + j < M ? row_size[base + j] : 0;
        s += v[j];
    }
    int64_t tot;
    int64_t run = tile_off[blockIdx.x] + Team<kScanThreads>::excl_scan(s, &tot, scr, threadIdx.x);
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        if (base + j < M) c_rpt[base + j] = run;
        run += v[j];
    }
}

// The top-level scan folded into the apply pass, for at most kScanFusedTiles
// tiles: every block adds up the sums of the tiles before its own (one
// strided pass and a block reduction), the last one also writes the total.
constexpr int64_t kScanFusedTiles = 4096;

__global__ __launch_bounds__(kScanThreads) void k_scan_apply_fused(int64_t M, int64_t ntiles,
                                                                   const int32_t *row_size,
                                                                   const int64_t *tile_sum, int64_t *c_rpt,
                                                                   int64_t *total, const Ctl *ctl_src,
                                                                   Ctl *ctl_dst) {
    __shared__ int64_t scr[Team<kScanThreads>::kWaves + 1];
    int64_t before = 0;
    for (int64_t i = threadIdx.x; i < (int64_t)blockIdx.x; i += kScanThreads) before += tile_sum[i];
    before = Team<kScanThreads>::sum(before, scr, threadIdx.x);
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int32_t v[kScanPer];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        v[j] = base + j < M ? row_size[base + j] : 0;
        s += v[j];
    }
    int64_t tot;
    int64_t run = before + Team<kScanThreads>::excl_scan(s, &tot, scr, threadIdx.x);
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        if (base + j < M) c_rpt[base + j] = run;
        run += v[j];
    }
    if ((int64_t)blockIdx.x == ntiles - 1) {
        if (threadIdx.x == 0) {
            *total = before + tot;
            c_rpt[M] = before + tot;
        }
        publish_ctl(ctl_src, ctl_dst, total, before + tot);
    }
}

hipError_t launch_scan(int64_t M, const int32_t *sizes, int64_t *tile_sum, int64_t *out_rpt,
                       int64_t *total, hipStream_t s, const Ctl *ctl_src, Ctl *ctl_dst) {
    const int64_t ntiles = (M + kScanTile - 1) / kScanTile;
    if (ntiles > 0 && ntiles <= kScanFusedTiles) {
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, M, sizes,
                           tile_sum);
        hipLaunchKernelGGL(k_scan_apply_fused, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, M, ntiles,
                           sizes, tile_sum, out_rpt, total, ctl_src, ctl_dst);
        return hipGetLastError();
    }
    if (ntiles > 0)
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, M, sizes,
                           tile_sum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, ntiles, tile_sum, M, out_rpt, total, ctl_src,
                       ctl_dst);
    if (ntiles > 0)
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, M, sizes,
                           tile_sum, out_rpt);
    return hipGetLastError();
}

// End of a row of the numeric pass.  Exact mode: the slot came from the
// symbolic count and must match.  Bound mode (learned allocation): the slot
// is a predicted upper bound; the exact length is recorded and a row that did
// not fit is queued for the exact fallback.
__device__ __forceinline__ void finish_row(const NumOut &no, Ctl *ctl, int64_t row, int64_t len,
                                           int64_t cap, bool heavy) {
    if (!no.bound) {
        if (len != cap)
            atomicOr(reinterpret_cast<unsigned long long *>(&ctl->err), (unsigned long long)kErrSizeMismatch);
        return;
    }
    no.row_size[row] = (int32_t)len;
    if (len > cap) {
        if (heavy) {
            const unsigned long long i = atomicAdd(reinterpret_cast<unsigned long long *>(&ctl->ovf_heavy), 1ull);
            no.ovf_rows[no.M + (int64_t)i] = (int32_t)row;
        } else {
            const unsigned long long i = atomicAdd(reinterpret_cast<unsigned long long *>(&ctl->ovf_light), 1ull);
            no.ovf_rows[no.M - 1 - (int64_t)i] = (int32_t)row;
        }
    }
}

// ---------------------------------------------------------------------------
// numeric, single list: the result row is the scaled B row (wave per row)
// ---------------------------------------------------------------------------
// `row` indexes A and C; `id` is the row's id for the bound-mode bookkeeping
template <typename IA, typename IB>
__device__ __forceinline__ void copy_row(int lane, int64_t row, int64_t id, const void *a_rpt,
                                         const Lists<IB> &lists, const double *a_val,
                                         const int32_t *b_col, const double *b_val, const int64_t *c_rpt,
                                         int32_t *c_col, double *c_val, Ctl *ctl, const NumOut &no) {
    const int64_t p = ld_rpt<IA>(a_rpt, row);
    const double a = gload(a_val + (p));
    int64_t bs;
    int ln;
    lists.get(p, bs, ln);
    const int64_t n = ln;
    const int64_t cs = gload(c_rpt + (row));
    const int64_t cap = gload(c_rpt + (row + 1)) - cs;
    if (lane == 0) finish_row(no, ctl, id, n, cap, false);
    const int64_t m = n < cap ? n : cap;
    for (int64_t j = lane; j < m; j += kWave) {
        gstore(c_col + (cs + j), gload(b_col + (bs + j)));
        gstore(c_val + (cs + j), a * gload(b_val + (bs + j)));
    }
}

template <typename IA, typename IB>
__global__ __launch_bounds__(256) void k_num_copy(int cls, const void *a_rpt, Lists<IB> lists,
                                                  const double *a_val,
                                                  const int32_t *b_col, const double *b_val,
                                                  const int32_t *class_rows, const int64_t *c_rpt,
                                                  int32_t *c_col, double *c_val, Ctl *ctl, NumOut no) {
    const int lane = lane_id();
    const int64_t count = ctl->count[cls];
    const int64_t start = class_start(ctl, cls);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t idx = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; idx < count;
         idx += waves) {
        const int64_t row = class_rows[start + idx];
        copy_row<IA, IB>(lane, row, row, a_rpt, lists, a_val, b_col, b_val, c_rpt, c_col, c_val, ctl, no);
    }
}

// ---------------------------------------------------------------------------
// numeric, one row in LDS (a team of T threads, CAP products at most)
// ---------------------------------------------------------------------------
// One output list to build: the lists [a0, a0 + L) of A's entries (a whole
// row, or an aligned range of a heavy row's lists), merged into out_col /
// out_val (at most out_cap entries are written).
struct Seg {
    int64_t a0;
    int32_t *out_col;
    double *out_val;
    int64_t out_cap;
    int32_t L;
    int32_t pad;
};

template <int T, int CAP, int G = 1>
struct NumLds {
    static constexpr int kE = CAP / T;                     // positions per thread
    static constexpr int kSlots = kE * Team<T>::kWaves;    // (slice, wave) counters
    int32_t col[2][CAP + 1];
    double val[2][CAP + 1];
    int32_t off[CAP + 1];  // start of every list (leaf) of the group; off[leaves] = products
    int32_t len[CAP];      // current length of a node, stored at its first leaf
    int32_t scan[(kSlots > Team<T>::kWaves ? kSlots : Team<T>::kWaves) + 1];
    int32_t fl[G + 1];     // first leaf of every segment
    int32_t seg_len[G];    // merged length of every segment
    int64_t row[G];
    Seg seg[G];
    // merge-path rounds with one position per thread: every thread's first
    // entry and last column (with more positions per thread they sit in the
    // round's destination buffers, free at that point)
    int32_t bnd_c[kE == 1 ? T : 1];
    double bnd_v[kE == 1 ? T : 1];
    int32_t bnd_last[kE == 1 ? T : 1];
};

// Merge path: how many entries of X are among the first d entries of the
// merge of sorted X and Y (X first on equal columns).
__device__ __forceinline__ int mp_split_lds(const int32_t *X, int nx, const int32_t *Y, int ny, int d) {
    int lo = d > ny ? d - ny : 0, hi = d < nx ? d : nx;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (X[mid] <= Y[d - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Exclusive count of `flag` over the positions p = tid + e*T in increasing p.
// Writes the count before every position p < n into x[p] and the total into x[n].
template <int T, int CAP, int G>
__device__ __forceinline__ void team_flag_scan(NumLds<T, CAP, G> &s, int tid, const bool (&flag)[CAP / T],
                                               int n, int32_t *x) {
    constexpr int E = CAP / T;
    constexpr int W = Team<T>::kWaves;
    uint64_t m[E];
#pragma unroll
    for (int e = 0; e < E; ++e) m[e] = wave_ballot(flag[e]);
    if constexpr (T == kWave) {
        int run = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = tid + e * T;
            if (p < n) x[p] = run + lanes_below(m[e]);
            run += __popcll(m[e]);
        }
        if (tid == 0) x[n] = run;
    } else {
        const int w = tid / kWave;
        if (lane_id() == 0) {
#pragma unroll
            for (int e = 0; e < E; ++e) s.scan[e * W + w] = __popcll(m[e]);
        }
        __syncthreads();
        if (tid < kWave) {
            // E*W <= 64 slots: one wavefront scans them
            const int v = tid < E * W ? s.scan[tid] : 0;
            const int incl = wave_incl_scan(v);
            if (tid < E * W) s.scan[tid] = incl - v;
            if (tid == kWave - 1) s.scan[E * W] = incl;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = tid + e * T;
            if (p < n) x[p] = s.scan[e * W + w] + lanes_below(m[e]);
        }
        if (tid == 0) x[n] = s.scan[E * W];
    }
}

// BRMerge of n segments (s.seg[0..n), set and visible to the team) in the
// team's LDS: the lists of all segments share the two buffers, each
// segment's merge tree stays its own (a node never pairs with another
// segment's lists).  Requires the segments' lists and products to total at
// most CAP each.  On return s.seg_len[j] holds segment j's merged length.
template <int T, int CAP, int G, typename IB>
__device__ __forceinline__ void brmerge_segs_lds(NumLds<T, CAP, G> &s, int tid, int n, const Lists<IB> &lists,
                                                 const double *a_val, const int32_t *b_col,
                                                 const double *b_val) {
    constexpr int E = CAP / T;
    static_assert(E * Team<T>::kWaves <= 64, "flag scan assumes at most 64 (slice, wave) slots");
    static_assert(G <= kWave, "at most one wavefront of segments");
    // first list of every segment
    if (tid < kWave) {
        const int Lj = tid < n ? s.seg[tid].L : 0;
        const int incl = wave_incl_scan(Lj);
        if (tid < n) s.fl[tid + 1] = incl;
        if (tid == 0) s.fl[0] = 0;
    }
    Team<T>::sync();
    const int LT = s.fl[n];
    int maxL = 0;
    for (int j = 0; j < n; ++j) maxL = s.seg[j].L > maxL ? s.seg[j].L : maxL;

    // list offsets; B row start and A value of every list staged in the
    // second buffer (free until the first round)
    int carry = 0;
    for (int lb = 0; lb < LT; lb += T) {
        const int gl = lb + tid;
        int ln = 0;
        int64_t bs = 0;
        double av = 0.0;
        if (gl < LT) {
            const int j = upper_bound(s.fl, n, gl) - 1;
            const int64_t p = s.seg[j].a0 + (gl - s.fl[j]);
            av = gload(a_val + (p));
            lists.get(p, bs, ln);
        }
        int tot;
        const int ex = Team<T>::excl_scan(ln, &tot, s.scan, tid);
        if (gl < LT) {
            s.off[gl] = carry + ex;
            s.col[1][gl] = (int32_t)(uint32_t)(uint64_t)bs;
            s.len[gl] = (int32_t)(bs >> 32);
            s.val[1][gl] = av;
        }
        carry += tot;
    }
    const int nprod = carry;
    if (tid == 0) s.off[LT] = nprod;
    Team<T>::sync();

    // multiplying phase: position p holds A_ik * B_kj of list leaf[e] of
    // segment sg[e]; consecutive positions read consecutive B entries
    int leaf[E], sg[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = tid + e * T;
        leaf[e] = 0;
        sg[e] = 0;
        if (p < nprod) {
            const int gl = upper_bound(s.off, LT + 1, p) - 1;
            leaf[e] = gl;
            sg[e] = upper_bound(s.fl, n, gl) - 1;
            const int64_t bs = ((int64_t)s.len[gl] << 32) | (int64_t)(uint32_t)s.col[1][gl];
            const int64_t q = bs + (p - s.off[gl]);
            s.col[0][p] = gload(b_col + (q));
            s.val[0][p] = s.val[1][gl] * gload(b_val + (q));
        }
    }
    Team<T>::sync();
    for (int gl = tid; gl < LT; gl += T) s.len[gl] = s.off[gl + 1] - s.off[gl];
    Team<T>::sync();

    // accumulating phase: round sh merges the nodes of level sh pairwise
    int cur = 0;
    for (int sh = 0; (1 << sh) < maxL; ++sh) {
        const int nxt = cur ^ 1;
        const int32_t *sc = s.col[cur];
        const double *sv = s.val[cur];
        int32_t *dc = s.col[nxt];
        double *dv = s.val[nxt];
        int32_t c[E];
        double v[E];
        int k[E], i[E], st[E], sst[E], ln[E], sln[E], node[E], rfl[E];
        bool valid[E], dup[E], sib[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = tid + e * T;
            valid[e] = false;
            dup[e] = false;
            sib[e] = false;
            k[e] = 0;
            c[e] = 0;
            v[e] = 0.0;
            rfl[e] = s.fl[sg[e]];
            const int rL = s.fl[sg[e] + 1] - rfl[e];
            node[e] = (leaf[e] - rfl[e]) >> sh;
            const int fl = rfl[e] + (node[e] << sh);
            st[e] = s.off[fl];
            ln[e] = s.len[fl];
            i[e] = p - st[e];
            sst[e] = 0;
            sln[e] = 0;
            if (p < nprod && i[e] < ln[e]) {
                valid[e] = true;
                c[e] = sc[p];
                v[e] = sv[p];
                const int sl = (node[e] ^ 1) << sh;
                if (sl < rL) {
                    sib[e] = true;
                    sst[e] = s.off[rfl[e] + sl];
                    sln[e] = s.len[rfl[e] + sl];
                    if ((node[e] & 1) == 0) {
                        k[e] = lower_bound(sc + sst[e], sln[e], c[e]);
                        if (k[e] < sln[e] && sc[sst[e] + k[e]] == c[e]) v[e] = v[e] + sv[sst[e] + k[e]];
                    } else {
                        k[e] = upper_bound(sc + sst[e], sln[e], c[e]);
                        dup[e] = k[e] > 0 && sc[sst[e] + k[e] - 1] == c[e];
                    }
                }
            }
        }
        // dup counts over positions, kept in the destination column buffer
        team_flag_scan<T, CAP, G>(s, tid, dup, nprod, dc);
        Team<T>::sync();
        int dest[E], newlen[E], newlen_at[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            dest[e] = -1;
            newlen[e] = -1;
            newlen_at[e] = 0;
            if (valid[e] && !dup[e]) {
                int pos;
                if (!sib[e]) {
                    pos = i[e];
                } else if ((node[e] & 1) == 0) {
                    pos = i[e] + k[e] - (dc[sst[e] + k[e]] - dc[sst[e]]);
                } else {
                    const int p = tid + e * T;
                    pos = i[e] + k[e] - (dc[p] - dc[st[e]]);
                }
                dest[e] = s.off[rfl[e] + ((node[e] >> 1) << (sh + 1))] + pos;
            }
            if (valid[e] && sib[e] && (node[e] & 1) && i[e] == 0) {
                // first element of a right list: the parent's length
                newlen[e] = sln[e] + ln[e] - (dc[st[e] + ln[e]] - dc[st[e]]);
                newlen_at[e] = rfl[e] + ((node[e] ^ 1) << sh);
            }
        }
        Team<T>::sync();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (dest[e] >= 0) {
                dc[dest[e]] = c[e];
                dv[dest[e]] = v[e];
            }
            if (newlen[e] >= 0) s.len[newlen_at[e]] = newlen[e];
        }
        Team<T>::sync();
        cur = nxt;
    }

    // Algorithm 1's final store: every segment's single list goes out
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = tid + e * T;
        if (p < nprod) {
            const int j = sg[e];
            const int f = s.fl[j];
            const int o = p - s.off[f];
            if (o < s.len[f] && (int64_t)o < s.seg[j].out_cap) {
                gstore(s.seg[j].out_col + (o), s.col[cur][p]);
                gstore(s.seg[j].out_val + (o), s.val[cur][p]);
            }
        }
    }
    if (tid < n) s.seg_len[tid] = s.len[s.fl[tid]];
    Team<T>::sync();
}

// BRMerge of one segment, the lists [a0, a0 + L) of A's entries (a whole row,
// or an aligned range of a heavy row's lists), in the team's LDS.  The merged list
// is written to out_col / out_val (at most out_cap entries); its length is
// returned to every thread of the team.
template <int T, int CAP, int G, typename IB>
__device__ __forceinline__ int brmerge_range_lds(NumLds<T, CAP, G> &s, int tid, int64_t a0, int L,
                                                 const Lists<IB> &lists, const double *a_val,
                                                 const int32_t *b_col, const double *b_val,
                                                 int32_t *out_col, double *out_val, int64_t out_cap) {
    constexpr int E = CAP / T;
    static_assert(E * Team<T>::kWaves <= 64, "flag scan assumes at most 64 (slice, wave) slots");

    // list offsets; B row start and A value of every list staged in the
    // second buffer (free until the first round)
    int carry = 0;
    for (int lb = 0; lb < L; lb += T) {
        const int l = lb + tid;
        int ln = 0;
        int64_t bs = 0;
        double av = 0.0;
        if (l < L) {
            av = gload(a_val + (a0 + l));
            lists.get(a0 + l, bs, ln);
        }
        int tot;
        const int ex = Team<T>::excl_scan(ln, &tot, s.scan, tid);
        if (l < L) {
            s.off[l] = carry + ex;
            s.col[1][l] = (int32_t)(uint32_t)(uint64_t)bs;
            s.len[l] = (int32_t)(bs >> 32);
            s.val[1][l] = av;
        }
        carry += tot;
    }
    const int nprod = carry;
    if (tid == 0) s.off[L] = nprod;
    Team<T>::sync();

    // multiplying phase: position p of the row holds A_ik * B_kj of list
    // (leaf) leaf[e]; consecutive positions read consecutive B entries
    int leaf[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = tid + e * T;
        leaf[e] = 0;
        if (p < nprod) {
            const int lf = upper_bound(s.off, L + 1, p) - 1;
            leaf[e] = lf;
            const int64_t bs = ((int64_t)s.len[lf] << 32) | (int64_t)(uint32_t)s.col[1][lf];
            const int64_t q = bs + (p - s.off[lf]);
            s.col[0][p] = gload(b_col + (q));
            s.val[0][p] = s.val[1][lf] * gload(b_val + (q));
        }
    }
    Team<T>::sync();
    for (int l = tid; l < L; l += T) s.len[l] = s.off[l + 1] - s.off[l];
    Team<T>::sync();

    // accumulating phase: round sh merges the nodes of level sh pairwise.
    // Thread tid owns the E consecutive positions tid*E .. tid*E+E-1 of the
    // merge-path order of whichever sibling pair covers them (a pair's merged
    // sequence, duplicates included, starts at its left node's offset); one
    // merge-path search per pair a thread meets, then sequential steps.
    int leafc[E];
    {
        const int p0 = tid * E;
        int lf = p0 < nprod ? upper_bound(s.off, L + 1, p0) - 1 : 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = p0 + e;
            if (p < nprod)
                while (s.off[lf + 1] <= p) ++lf;  // lists may be empty: skip leaves that end before p
            leafc[e] = lf;
        }
    }
    int cur = 0;
    for (int sh = 0; (1 << sh) < L; ++sh) {
        const int nxt = cur ^ 1;
        const int32_t *sc = s.col[cur];
        const double *sv = s.val[cur];
        int32_t *dc = s.col[nxt];
        double *dv = s.val[nxt];
        int32_t c[E];
        double v[E];
        int base[E], span[E], d[E];
        bool valid[E], left[E], dup[E];
        {
            int run_pfl = -1, x = 0, y = 0, rb = 0, lnL = 0, lnR = 0;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int p = tid * E + e;
                const int pfl = (leafc[e] >> (sh + 1)) << (sh + 1);
                valid[e] = false;
                left[e] = true;
                c[e] = 0;
                v[e] = 0.0;
                base[e] = 0;
                span[e] = 0;
                d[e] = 0;
                if (p < nprod) {
                    if (pfl != run_pfl) {
                        // a new pair: its merged sequence and this position's split
                        run_pfl = pfl;
                        const int sfl = pfl + (1 << sh);
                        lnL = s.len[pfl];
                        lnR = sfl < L ? s.len[sfl] : 0;
                        rb = sfl < L ? s.off[sfl] : 0;
                        const int dd = p - s.off[pfl];
                        if (dd < lnL + lnR) {
                            x = mp_split_lds(sc + s.off[pfl], lnL, sc + rb, lnR, dd);
                            y = dd - x;
                        }
                    }
                    base[e] = s.off[pfl];
                    span[e] = lnL + lnR;
                    d[e] = p - base[e];
                    if (d[e] < span[e]) {
                        valid[e] = true;
                        if (x < lnL && (y >= lnR || sc[base[e] + x] <= sc[rb + y])) {
                            c[e] = sc[base[e] + x];
                            v[e] = sv[base[e] + x];
                            ++x;
                        } else {
                            c[e] = sc[rb + y];
                            v[e] = sv[rb + y];
                            left[e] = false;
                            ++y;
                        }
                    }
                }
            }
        }
        // neighbours across threads: the merged entries just before and
        // after this thread's positions
        int32_t *bnd_c = E == 1 ? s.bnd_c : dc;
        int32_t *bnd_last = E == 1 ? s.bnd_last : dc + T;
        double *bnd_v = E == 1 ? s.bnd_v : dv;
        bnd_c[tid] = c[0];
        bnd_v[tid] = v[0];
        bnd_last[tid] = c[E - 1];
        Team<T>::sync();
        int ndup = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            dup[e] = false;
            if (!valid[e]) continue;
            // a right entry equal to the entry before it: the pair's column
            // already held by the left list (inputs have no repeats)
            if (!left[e] && d[e] > 0) {
                const int32_t pc = e > 0 ? c[e - 1] : bnd_last[tid - 1];
                dup[e] = pc == c[e];
            }
            // a left entry whose next entry repeats its column takes left + right
            if (left[e] && d[e] + 1 < span[e]) {
                const int32_t nc = e + 1 < E ? c[e + 1] : bnd_c[tid + 1];
                const double nv = e + 1 < E ? v[e + 1] : bnd_v[tid + 1];
                if (nc == c[e]) v[e] = v[e] + nv;
            }
            ndup += dup[e];
        }
        // exclusive count of duplicates over positions, kept in the
        // destination column buffer (and its total at nprod); the scan's
        // barriers come after every read of the neighbours above
        int tot;
        const int before = Team<T>::excl_scan(ndup, &tot, s.scan, tid);
        {
            int run = before;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int p = tid * E + e;
                if (p < nprod) dc[p] = run;
                run += dup[e];
            }
            if (tid == 0) dc[nprod] = tot;
        }
        Team<T>::sync();
        // (a thread may hold the first position of several pairs)
        int dest[E], newlen[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            dest[e] = -1;
            newlen[e] = -1;
            if (valid[e] && !dup[e]) dest[e] = base[e] + d[e] - (dc[tid * E + e] - dc[base[e]]);
            // the pair's first position: the parent's length
            if (valid[e] && d[e] == 0) newlen[e] = span[e] - (dc[base[e] + span[e]] - dc[base[e]]);
        }
        Team<T>::sync();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (dest[e] >= 0) {
                dc[dest[e]] = c[e];
                dv[dest[e]] = v[e];
            }
            if (newlen[e] >= 0) s.len[(leafc[e] >> (sh + 1)) << (sh + 1)] = newlen[e];
        }
        Team<T>::sync();
        cur = nxt;
    }

    // Algorithm 1's final store: the single list left goes to the output
    const int rl = s.len[0];
    const int m = (int64_t)rl < out_cap ? rl : (int)out_cap;
    for (int p = tid; p < m; p += T) {
        gstore(out_col + (p), s.col[cur][p]);
        gstore(out_val + (p), s.val[cur][p]);
    }
    Team<T>::sync();
    return rl;
}

template <int T, int CAP, typename IA, typename IB>
__device__ __forceinline__ void brmerge_row_lds(NumLds<T, CAP> &s, int tid, int64_t row,
                                                const void *a_rpt, const Lists<IB> &lists,
                                                const double *a_val,
                                                const int32_t *b_col, const double *b_val,
                                                const int64_t *c_rpt, int32_t *c_col,
                                                double *c_val, Ctl *ctl, const NumOut &no, int64_t id) {
    const int64_t a0 = ld_rpt<IA>(a_rpt, row);
    const int L = (int)(ld_rpt<IA>(a_rpt, row + 1) - a0);
    const int64_t cs = gload(c_rpt + (row));
    const int64_t cap = gload(c_rpt + (row + 1)) - cs;
    const int rl = brmerge_range_lds<T, CAP, 1, IB>(s, tid, a0, L, lists, a_val, b_col, b_val,
                                                 c_col + cs, c_val + cs, cap);
    // Algorithm 1's final store went straight to C's row (truncated to the slot)
    if (tid == 0) finish_row(no, ctl, id, rl, cap, false);
}

template <int T, int TEAMS, int CAP, typename IA, typename IB>
__global__ __launch_bounds__(T *TEAMS) void k_num_lds(int cls, const void *a_rpt,
                                                      Lists<IB> lists, const double *a_val,
                                                      const int32_t *b_col, const double *b_val,
                                                      const int32_t *class_rows,
                                                      const int64_t *c_rpt, int32_t *c_col,
                                                      double *c_val, Ctl *ctl, NumOut no) {
    __shared__ NumLds<T, CAP> lds[TEAMS];
    const int team = threadIdx.x / T, tid = threadIdx.x % T;
    const int64_t count = ctl->count[cls];
    const int64_t start = class_start(ctl, cls);
    for (int64_t idx = (int64_t)blockIdx.x * TEAMS + team; idx < count;
         idx += (int64_t)gridDim.x * TEAMS) {
        const int64_t row = class_rows[start + idx];
        brmerge_row_lds<T, CAP, IA, IB>(lds[team], tid, row, a_rpt, lists, a_val, b_col,
                                        b_val, c_rpt, c_col, c_val, ctl, no, row);
    }
}

// ---------------------------------------------------------------------------
// rows of at most 64 products whose lists fit power-of-two lane windows
// (lists padded to W0 = the next power of two of the longest list, their
// count to the next power of two, W0 * lists <= 64): the whole BRMerge runs
// in registers.  Every lane holds one entry; list p occupies lanes
// [p W0, (p+1) W0) in ascending column order, padded with empty slots.
// Round r merges windows 2q and 2q+1 of width W0 2^r with a bitonic merge
// (a mirror compare-exchange, then half-cleaners at distances W/2 .. 1), so
// the two lists of a pair are merged, never mixed with another pair.
//
// What the network sorts is a 32-bit key: the column above kKeyLaneBits bits
// that name the lane holding the entry's value; an empty slot has all column
// bits set (it sorts after every column) and its own lane below them.  The
// fp64 values stay where the multiplying phase formed them, so a
// compare-exchange moves one register.  Lanes of the left list of a pair
// always have lower numbers than those of the right list (entries never
// leave their window pair), so of two equal columns the left one comes
// first.  When a round leaves equal columns (one from each list) side by
// side, the first takes the sum left + right, the second is dropped and
// every window is compacted through LDS, values moving into key order
// (skipped when the wavefront has no such pair).  Columns must be below
// 2^(32 - kKeyLaneBits) - 1.
// ---------------------------------------------------------------------------
constexpr int32_t kEmptyCol = 0x7fffffff;
constexpr int kKeyLaneBits = 6;
constexpr uint32_t kKeyEmpty = ~0u << kKeyLaneBits;
constexpr uint32_t kKeyLaneMask = (1u << kKeyLaneBits) - 1;

// value of lane (lane ^ D) for a distance known at compile time: DPP inside
// a row of 16 lanes where one pattern serves, ds_swizzle inside 32 lanes,
// ds_bpermute across the halves of the wavefront.  Every lane must be active.
template <int D>
__device__ __forceinline__ uint32_t xor_lane(uint32_t x, int lane) {
    static_assert(D > 0 && D < kWave, "lane distance");
    const int xi = (int)x;
    if constexpr (D == 1)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, xi, 0xB1, 0xF, 0xF, false);  // quad_perm 1,0,3,2
    else if constexpr (D == 2)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, xi, 0x4E, 0xF, 0xF, false);  // quad_perm 2,3,0,1
    else if constexpr (D == 3)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, xi, 0x1B, 0xF, 0xF, false);  // quad_perm 3,2,1,0
    else if constexpr (D == 7)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, xi, 0x141, 0xF, 0xF, false);  // row_half_mirror
    else if constexpr (D == 15)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, xi, 0x140, 0xF, 0xF, false);  // row_mirror
    else if constexpr (D < 32)
        return (uint32_t)__builtin_amdgcn_ds_swizzle(xi, 0x1F | (D << 10));  // bit mode: and 31, xor D
    else
        return (uint32_t)__builtin_amdgcn_ds_bpermute((lane ^ D) << 2, xi);
}

// value of lane - 1 / lane + 1 (DPP shifts across the wavefront; the lane
// at the edge gets 0)
__device__ __forceinline__ uint32_t lane_prev(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x138, 0xF, 0xF, false);  // wave_shr:1
}
__device__ __forceinline__ uint32_t lane_next(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x130, 0xF, 0xF, false);  // wave_shl:1
}

// compare-exchange at distance D: the lower lane of a pair keeps the smaller
// key (keys of a wavefront are distinct, or equal keys are interchangeable)
template <int D>
__device__ __forceinline__ void key_cmpx(uint32_t &k, int lane, bool lower) {
    const uint32_t p = xor_lane<D>(k, lane);
    const uint32_t lo = p < k ? p : k;
    const uint32_t hi = p < k ? k : p;
    k = lower ? lo : hi;
}

template <int D>
__device__ __forceinline__ void key_half_cleaners(uint32_t &k, int lane) {
    if constexpr (D >= 1) {
        key_cmpx<D>(k, lane, (lane & D) == 0);
        key_half_cleaners<D / 2>(k, lane);
    }
}

// bitonic merge of every pair of sorted windows of width W into one sorted
// window of width 2W (the mirror stage turns the pair into a bitonic
// sequence, the half-cleaners sort it)
template <int W>
__device__ __forceinline__ void key_merge(uint32_t &k, int lane) {
    key_cmpx<2 * W - 1>(k, lane, (lane & W) == 0);
    key_half_cleaners<W / 2>(k, lane);
}

// One round of the accumulating phase (see above).  v: the values, held by
// the lanes the keys name.  Returns whether the round compacted (values are
// then in key order: every key names its own lane).
template <int W>
__device__ __forceinline__ bool key_round(uint32_t &k, double &v, int lane, uint32_t *xk, double *xv) {
    key_merge<W>(k, lane);
    constexpr int W2 = 2 * W;
    const int wpos = lane & (W2 - 1);
    const uint32_t pk = lane_prev(k);
    const bool dead = wpos > 0 && k < kKeyEmpty && (k & kKeyEmpty) == (pk & kKeyEmpty);
    if (!wave_ballot(dead)) return false;
    const uint32_t nk = lane_next(k);
    const bool head_dup = wpos + 1 < W2 && k < kKeyEmpty && (k & kKeyEmpty) == (nk & kKeyEmpty);
    double mv = __shfl(v, (int)(k & kKeyLaneMask), kWave);
    const double nv = __shfl(v, (int)(nk & kKeyLaneMask), kWave);
    if (head_dup) mv = mv + nv;  // left + right
    const bool live = !dead && k < kKeyEmpty;
    const uint64_t lm = wave_ballot(live);
    const int wbase = lane & ~(W2 - 1);
    const uint64_t wmask = (W2 == 64) ? ~0ull : (((1ull << W2) - 1) << wbase);
    const int rank = __popcll(lm & wmask & ((1ull << lane) - 1));
    xk[lane] = kKeyEmpty | (uint32_t)lane;
    wave_sync();
    if (live) {
        xk[wbase + rank] = (k & kKeyEmpty) | (uint32_t)(wbase + rank);
        xv[wbase + rank] = mv;
    }
    wave_sync();
    k = xk[lane];
    v = xv[lane];
    wave_sync();
    return true;
}

// rounds from list width W0 up to the padded total T (both powers of two,
// wavefront-uniform); returns whether values are in key order at the end
__device__ __forceinline__ bool key_rounds(uint32_t &k, double &v, int W0, int T, int lane, uint32_t *xk,
                                           double *xv) {
    bool placed = true;
    for (int W = W0; W < T; W <<= 1) {
        switch (W) {
            case 1: placed = key_round<1>(k, v, lane, xk, xv); break;
            case 2: placed = key_round<2>(k, v, lane, xk, xv); break;
            case 4: placed = key_round<4>(k, v, lane, xk, xv); break;
            case 8: placed = key_round<8>(k, v, lane, xk, xv); break;
            case 16: placed = key_round<16>(k, v, lane, xk, xv); break;
            default: placed = key_round<32>(k, v, lane, xk, xv); break;
        }
    }
    return placed;
}

// The rounds' merge network on the keys alone, from sorted windows of width
// W0 up to the padded total T: every row's window ends sorted by (column,
// lane), and a row's lanes are in list order.
__device__ __forceinline__ void key_sort(uint32_t &k, int W0, int T, int lane) {
    for (int W = W0; W < T; W <<= 1) {
        switch (W) {
            case 1: key_merge<1>(k, lane); break;
            case 2: key_merge<2>(k, lane); break;
            case 4: key_merge<4>(k, lane); break;
            case 8: key_merge<8>(k, lane); break;
            case 16: key_merge<16>(k, lane); break;
            default: key_merge<32>(k, lane); break;
        }
    }
}

// Algorithm 1's accumulating phase on a sorted key window, without moving
// entries between rounds.  k: the lane's key (column, source lane), v: the
// value of that key.  Two products of one column from lists a < b meet in
// the merge tree at the level of the lowest common ancestor of a and b, the
// position of the highest bit of a ^ b (list p of a row is the tree's leaf
// p; node (r, q) covers lists [q 2^r, (q+1) 2^r)).  In a column's run of
// lanes (ascending lists), the lanes joined by levels below r hold the
// column's entries of one node of level r-1; level by level, each such run's
// first lane adds the first lane of the next run when the two meet at level
// r exactly (left + right).  So every column's sum has the tree's grouping,
// as in the round-by-round merges.  lsw: log2 of the lane's row's list width;
// rows are windows of T lanes.  Returns the lanes holding a column's sum
// (its first lane in the row).
__device__ __forceinline__ uint64_t tree_adds(uint32_t k, double &v, int lsw, int T, int lane, int levels) {
    const bool live = k < kKeyEmpty;
    const uint32_t col = k >> kKeyLaneBits;
    const int li = (int)((k & kKeyLaneMask) & (uint32_t)(T - 1)) >> lsw;
    const uint32_t nk = lane_next(k), pk = lane_prev(k);
    const bool first = (lane & (T - 1)) == 0, last = ((lane + 1) & (T - 1)) == 0;
    const bool same_next = live && !last && nk < kKeyEmpty && (nk >> kKeyLaneBits) == col;
    const bool head = live && (first || pk >= kKeyEmpty || (pk >> kKeyLaneBits) != col);
    const uint64_t heads = wave_ballot(head);
    if (wave_ballot(same_next) == 0ull) return heads;  // no column repeats: nothing to add
    const int li_next = (int)((nk & kKeyLaneMask) & (uint32_t)(T - 1)) >> lsw;
    // the level at which this lane's entry meets the next lane's (64: never)
    const int lvl = same_next ? 32 - __clz(li ^ li_next) : 64;
    // the previous lane's level (64 at a row's first lane).  The shift is
    // taken in every lane and then masked: a shift under a condition would
    // run with the first lanes disabled, and their neighbours would read the
    // shift's fallback instead of their level
    const int plvl = (int)lane_prev((uint32_t)lvl) | (first ? 64 : 0);
    for (int r = 1; r <= levels; ++r) {
        const uint64_t ends = wave_ballot(lvl >= r);  // the last lane of every run
        const uint64_t meet = wave_ballot(lvl == r);
        const int e = lane + __builtin_ctzll(ends >> lane);  // this lane's run ends at lane e
        const double w = __shfl(v, e + 1 < kWave ? e + 1 : e, kWave);
        const bool rep = head || plvl >= r;  // the first lane of its run
        if (live && rep && ((meet >> e) & 1ull)) v = v + w;  // left + right
    }
    return heads;
}

// tree_adds on a window whose order was stored by the symbolic pass: the
// lane's entry came from lane src, is live or not, and holds the same column
// as the next lane's (same_next).  The same grouping of additions.
__device__ __forceinline__ uint64_t tree_adds_stored(bool live, bool same_next, int src, double &v, int lsw, int T,
                                                     int lane, int levels) {
    const bool first = (lane & (T - 1)) == 0;
    // a run's first lane: the previous lane (shifted in every lane) holds another column
    const uint32_t psame = lane_prev(same_next ? 1u : 0u);
    const bool head = live && (first || psame == 0u);
    const uint64_t heads = wave_ballot(head);
    if (wave_ballot(same_next) == 0ull) return heads;  // no column repeats: nothing to add
    const int li = (src & (T - 1)) >> lsw;
    const int li_next = (int)lane_next((uint32_t)li);
    const int lvl = same_next ? 32 - __clz(li ^ li_next) : 64;
    const int plvl = (int)lane_prev((uint32_t)lvl) | (first ? 64 : 0);
    for (int r = 1; r <= levels; ++r) {
        const uint64_t ends = wave_ballot(lvl >= r);
        const uint64_t meet = wave_ballot(lvl == r);
        const int e = lane + __builtin_ctzll(ends >> lane);
        const double w = __shfl(v, e + 1 < kWave ? e + 1 : e, kWave);
        const bool rep = head || plvl >= r;
        if (live && rep && ((meet >> e) & 1ull)) v = v + w;  // left + right
    }
    return heads;
}

// Symbolic use: the same merges on bare columns (empty = all ones), equal
// columns left in place; the lanes holding the first entry of a distinct
// column are returned as a mask.  A second row may start at lane `seg`
// (kWave: one row).
__device__ __forceinline__ uint64_t distinct_merged(uint32_t k, int W0, int T, int lane, int seg) {
    for (int W = W0; W < T; W <<= 1) {
        switch (W) {
            case 1: key_merge<1>(k, lane); break;
            case 2: key_merge<2>(k, lane); break;
            case 4: key_merge<4>(k, lane); break;
            case 8: key_merge<8>(k, lane); break;
            case 16: key_merge<16>(k, lane); break;
            default: key_merge<32>(k, lane); break;
        }
    }
    const uint32_t pk = lane_prev(k);
    return wave_ballot(k != ~0u && (lane == 0 || lane == seg || pk != k));
}

// 64-bit value of lane j (j wavefront-uniform)
__device__ __forceinline__ int64_t lane_value(int64_t x, int j) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(x >> 32), j);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int lane_value(int x, int j) { return __builtin_amdgcn_readlane(x, j); }


// Where the window kernels of a batched stage find a row's problem: the
// stage's problem table and the problem of every row (from the analysis).
struct BatchRows {
    const BatchProb *tab = nullptr;
    const int32_t *row_prob = nullptr;
};

// What masked lanes of the pipelined short-row kernels read instead of A's
// and B's arrays: an empty column and zeros, so that no value needs masking
// after its load.  Never written; not const, so that the compiler keeps them
// as global loads instead of folding their contents into branches.
__device__ int32_t g_empty_col[1] = {kEmptyCol};
__device__ int64_t g_zeros[1] = {0};

// Global load through an address the optimiser may not look into: a select
// between a real and a sentinel address stays one load, instead of becoming
// a branch per case (which would make the count of loads in flight depend on
// the path).  The asm statement only pins the address register; it emits no
// instruction.
template <typename T>
__device__ __forceinline__ T load_opaque(const T *p) {
    using GP = const __attribute__((address_space(1))) T *;
    GP g = (GP)p;
    asm volatile("" : "+v"(g));
    return *g;
}

// The rows of the wave-small class under lane windows (every one fits them:
// the analysis put the others in the next class), streamed by one wavefront
// in chunks of kWave rows.  A chunk's row ids, A row pointers, window widths
// and C row pointers are loaded at once (lane j holds row j's), so the
// per-row chain of dependent loads is list descriptors -> B entries only, and
// that chain is software-pipelined: while row j merges, the B entries of row
// j+D-1 and the list descriptors of row j+D are in flight (D = kWinNumDepth
// for the numeric pass, 2 for counts).  Every lane issues
// every load of a stage on every iteration (masked lanes read the sentinels
// above), so the number of memory operations in flight does not depend on
// the path and the waits stay partial.  Rows 2i and 2i+1 of a chunk whose
// windows both fit 32 lanes are merged together, one in each half of the
// wavefront.  VALUES = false counts row sizes; HASH then selects counting by
// LDS hash instead of window merges (one row at a time).
// items in flight behind the one being merged in the numeric window pipeline,
// and in the numeric pipeline that applies a stored order (fewer registers per
// item: B's values, the order byte and a column; ER-8 numeric 445 -> 428 us
// from 3 to 6 items, 103 VGPRs and 4 waves per SIMD; 8 gave the same, 10 less)
constexpr int kWinNumDepth = 3;
constexpr int kWinOrdDepth = 6;

template <bool VALUES, bool HASH, typename IA, typename IB, bool BATCH = false, bool ORD = false>
__device__ __forceinline__ void win_chunks(int cls, const void *a_rpt, const Lists<IB> &lists, const double *a_val,
                                           const int32_t *b_col, const double *b_val, const uint8_t *row_class,
                                           const int32_t *class_rows, const int64_t *c_rpt, int32_t *c_col,
                                           double *c_val, int32_t *row_size, Ctl *ctl, const NumOut &no,
                                           int32_t *tab, uint32_t *xk, double *xv, int64_t first, int64_t stride,
                                           BatchRows br = BatchRows{}, WinOrder ord = WinOrder{nullptr, nullptr}) {
    const int lane = lane_id();
    const int64_t count = ctl->count[cls];
    const int64_t start = class_start(ctl, cls);
    const int64_t nchunks = (count + kWave - 1) / kWave;
    const IB *ent_bs = static_cast<const IB *>(lists.ent_bs);
    const int32_t *ent_len = lists.ent_len;
    constexpr int kHalf = kWave / 2;
    for (int64_t ch = first; ch < nchunks; ch += stride) {
        const int64_t base = ch * kWave;
        const int n = (int)(count - base < kWave ? count - base : kWave);
        // chunk meta data, one row per lane: row (row ids fit 31 bits), first
        // entry of A, lists, window width (log2) and padded total (0 beyond
        // the chunk)
        int32_t m_row = 0;
        int64_t m_a0 = 0, m_cs = 0;
        int m_L = 0, m_sw = 0, m_T = 0, m_cap = 0;
        // batched: the row's problem (its arrays are read through the scalar
        // cache when an item needs them: one register per lane instead of
        // twelve)
        int m_prob = 0;
        if (lane < n) {
            m_row = class_rows[start + base + lane];
            const void *rpt = a_rpt;
            const int64_t *crpt = c_rpt;
            int64_t r = m_row;
            if constexpr (BATCH) {
                m_prob = br.row_prob[m_row];
                const BatchProb &pr = br.tab[m_prob];
                rpt = pr.a_rpt;
                crpt = pr.c_rpt;
                r = m_row - pr.row_off;
            }
            m_a0 = ld_rpt<IA>(rpt, r);
            m_L = (int)(ld_rpt<IA>(rpt, r + 1) - m_a0);
            m_sw = row_class[m_row] >> kClassBits;
            m_T = 1 << (m_sw + ceil_log2(m_L > 0 ? m_L : 1));
            if constexpr (VALUES) {
                m_cs = gload(crpt + r);
                m_cap = (int)(gload(crpt + r + 1) - m_cs);  // a row's size fits 31 bits
            }
        }
        // When every row of the chunk fits 32 lanes, rows 2i and 2i+1 share
        // one wavefront (the first in lanes 0..31, the second in lanes
        // 32..63): the pipeline below runs over pairs (P) instead of rows.
        // The two versions of the pipeline are separate code, so that the
        // one-row version keeps its uniform per-row values and partial waits.
        struct ListStageRegs {  // list descriptors of one item
            IB bs;
            int ln;
            double av;
        };
        struct GatherRegs {  // B entries of one item in the lane windows
            int32_t c;
            double bv, av;
            uint32_t q;  // stored order: the lane's byte of it
            int32_t u;   // stored order: the lane's distinct column of its row
        };
        uint64_t ovf_mask = 0;  // rows of the chunk that overflowed their slot (slot mode)
        // the length of chunk row j is known: slot bookkeeping or the check
        auto done = [&](int j, int len) {
            const int64_t row = lane_value(m_row, j);
            if constexpr (VALUES) {
                const int cap = lane_value(m_cap, j);
                if (no.bound) {
                    // slot mode: exact length kept; an overflowing row is
                    // listed for the fallback once per chunk (below)
                    if (lane == 0) no.row_size[row] = len;
                    // (batched slots are upper bounds: no row outgrows its slot)
                    if (!BATCH && len > cap) ovf_mask |= 1ull << j;
                } else if (lane == 0 && len != cap) {
                    atomicOr(reinterpret_cast<unsigned long long *>(&ctl->err), (unsigned long long)kErrSizeMismatch);
                }
            } else {
                if (lane == 0) row_size[row] = len;
            }
        };
        const bool all_small = !HASH && wave_ballot(lane < n && m_T > kHalf) == 0ull;
        auto run = [&](auto pt) {
            constexpr bool P = decltype(pt)::value;
            const int nv = P ? (n + 1) / 2 : n;
            // item v: row a (lanes 0..31 of a pair, all lanes of a single
            // row) and row b (lanes 32..63 of a pair; -1 when missing)
            auto item = [&](int v, int &a, int &b) {
                const int vv = v < nv ? v : 0;
                if constexpr (P) {
                    a = 2 * vv;
                    b = 2 * vv + 1 < n ? 2 * vv + 1 : -1;
                } else {
                    a = vv;
                    b = -1;
                }
            };
            // a per-row value for the lane's row; rows missing from a pair
            // read row a's (every use of them is masked by their list count)
            // batched: a field of the problem of row a (of row b in the upper
            // half of a pair), by scalar loads (the problem indices are
            // uniform; the table does not change during the launch)
            auto pick = [&](int a, int b, auto get) -> int64_t {
                using CP = const __attribute__((address_space(4))) BatchProb *;
                const CP ctab = (CP)br.tab;
                const int pa = lane_value(m_prob, a);
                const int64_t xa = get(ctab[pa]);
                if constexpr (!P) {
                    return xa;
                } else {
                    const int pb = lane_value(m_prob, b >= 0 ? b : a);
                    if (pb == pa) return xa;
                    const int64_t xb = get(ctab[pb]);
                    return lane >= kHalf ? xb : xa;
                }
            };
            auto sel64 = [&](int64_t m, int a, int b) -> int64_t {
                if constexpr (!P) {
                    return lane_value(m, a);
                } else {
                    const int64_t xa = lane_value(m, a), xb = lane_value(m, b >= 0 ? b : a);
                    return lane >= kHalf ? xb : xa;
                }
            };
            auto sel32 = [&](int m, int a, int b) -> int {
                if constexpr (!P) {
                    return lane_value(m, a);
                } else {
                    const int xa = lane_value(m, a), xb = lane_value(m, b >= 0 ? b : a);
                    return lane >= kHalf ? xb : xa;
                }
            };
            auto lists_of = [&](int v, int a, int b) -> int {  // list count of the lane's row
                if (v >= nv) return 0;
                if constexpr (P) {
                    if (b < 0 && lane >= kHalf) return 0;
                }
                return sel32(m_L, a, b);
            };
            // list descriptors of item v: lane t < L holds list t of its row
            // (the lanes of each half for a pair)
            auto load_lists = [&](int v, IB &bs, int &ln, double &av) {
                int a, b;
                item(v, a, b);
                const int t = P ? (lane & (kHalf - 1)) : lane;
                const int64_t p = sel64(m_a0, a, b) + t;
                const int64_t pe = BATCH ? pick(a, b, [](const auto &q) { return q.ent_off; }) + p : p;
                const bool ok = t < lists_of(v, a, b);
                bs = load_opaque(ok ? ent_bs + pe : reinterpret_cast<const IB *>(&g_zeros[0]));
                ln = load_opaque(ok ? ent_len + pe : reinterpret_cast<const int32_t *>(&g_zeros[0]));
                if constexpr (VALUES) {
                    const double *av_p =
                        BATCH ? reinterpret_cast<const double *>(
                                    pick(a, b, [](const auto &q) { return reinterpret_cast<int64_t>(q.a_val); }))
                              : a_val;
                    av = load_opaque(ok ? av_p + p : reinterpret_cast<const double *>(&g_zeros[0]));
                }
            };
            // multiplying phase of item v into the lane windows (the products
            // are formed where the row is consumed): lane t of a row's lanes
            // holds entry t mod W0 of its list t / W0
            auto gather = [&](int v, IB bs, int ln, double av, int32_t &c, double &bv, double &lav, uint32_t &q,
                              int32_t &u) {
                int a, b;
                item(v, a, b);
                const int L = lists_of(v, a, b);
                const int sw = sel32(m_sw, a, b);
                const int t = P ? (lane & (kHalf - 1)) : lane;
                const int li = t >> sw, o = t & ((1 << sw) - 1);
                const int src = (P && lane >= kHalf ? kHalf : 0) + (li & (kWave - 1));
                // every shuffle with all lanes active
                const int64_t lbs = __shfl((int64_t)bs, src, kWave);
                const int lln = __shfl(ln, src, kWave);
                lav = 0.0;
                if constexpr (VALUES) lav = __shfl(av, src, kWave);
                const bool ok = li < L && o < lln;
                const int32_t *bc =
                    BATCH ? reinterpret_cast<const int32_t *>(
                                pick(a, b, [](const auto &q) { return reinterpret_cast<int64_t>(q.b_col); }))
                          : b_col;
                if constexpr (ORD && VALUES) {
                    // the columns come with the stored order
                    c = 0;
                    const int rr = (P && lane >= kHalf) ? b : a;
                    const int T = P ? kHalf : lane_value(m_T, a);
                    const bool inrow = v < nv && rr >= 0 && t < T;
                    const int64_t at = (base + (inrow ? rr : 0)) * kWave + t;
                    q = inrow ? (uint32_t)load_opaque(ord.perm + at) : 0xFFu;
                    u = load_opaque(inrow ? ord.ucol + at : &g_empty_col[0]);
                } else {
                    c = load_opaque(ok ? bc + (lbs + o) : &g_empty_col[0]);
                    q = 0xFFu;
                    u = 0;
                }
                bv = 0.0;
                if constexpr (VALUES) {
                    const double *bvp =
                        BATCH ? reinterpret_cast<const double *>(
                                    pick(a, b, [](const auto &q) { return reinterpret_cast<int64_t>(q.b_val); }))
                              : b_val;
                    bv = load_opaque(ok ? bvp + (lbs + o) : reinterpret_cast<const double *>(&g_zeros[0]));
                }
            };
            // pipeline depth: the numeric pass keeps D = kWinNumDepth items in
            // flight behind the one being merged (kWinOrdDepth with a stored
            // order), the symbolic pass (column gathers only, slower with
            // more in flight) D = 2
            constexpr int D = VALUES ? (ORD ? kWinOrdDepth : kWinNumDepth) : 2;
            // one pipeline step: lists of item v+D -> lo, B entries of item
            // v+D-1 (from li) -> go, accumulating phase and write-out of item v
            auto step = [&](int v, const ListStageRegs &li, ListStageRegs &lo, const GatherRegs &gi, GatherRegs &go) {
                load_lists(v + D, lo.bs, lo.ln, lo.av);
                gather(v + D - 1, li.bs, li.ln, li.av, go.c, go.bv, go.av, go.q, go.u);
                int a, b;
                item(v, a, b);
                // a pair runs the rounds of both rows: from the narrower list
                // window to 32 lanes (a round below a row's own list width
                // merges halves of its sorted lists, one above its total
                // merges it with empty lanes: neither changes the row)
                int sw = lane_value(m_sw, a);
                if (P && b >= 0) {
                    const int swb = lane_value(m_sw, b);
                    sw = swb < sw ? swb : sw;
                }
                const int T = P ? kHalf : lane_value(m_T, a);
                if constexpr (!VALUES && HASH) {
                    tab[lane] = -1;
                    tab[lane + kWave] = -1;
                    wave_sync();
                    const int added = gi.c != kEmptyCol ? hash_insert<2 * kWave>(tab, gi.c) : 0;
                    const int len = __popcll(wave_ballot(added != 0));
                    wave_sync();
                    done(a, len);
                } else if constexpr (!VALUES && ORD) {
                    // sorted (column, lane) keys: the row's size, and its order kept for the numeric pass
                    uint32_t k = gi.c == kEmptyCol ? (kKeyEmpty | (uint32_t)lane)
                                                   : (((uint32_t)gi.c << kKeyLaneBits) | (uint32_t)lane);
                    key_sort(k, 1 << sw, T, lane);
                    const bool live = k < kKeyEmpty;
                    const uint32_t col = k >> kKeyLaneBits;
                    const uint32_t nk = lane_next(k), pk = lane_prev(k);
                    const bool first = (lane & (T - 1)) == 0, last = ((lane + 1) & (T - 1)) == 0;
                    const bool same = live && !last && nk < kKeyEmpty && (nk >> kKeyLaneBits) == col;
                    const bool head = live && (first || pk >= kKeyEmpty || (pk >> kKeyLaneBits) != col);
                    const uint64_t hm = wave_ballot(head);
                    const int rr = (P && lane >= kHalf) ? b : a;
                    const int t = P ? (lane & (kHalf - 1)) : lane;
                    if (rr >= 0 && t < T) {
                        const int64_t at = (base + rr) * kWave;
                        gstore(ord.perm + at + t,
                               (uint8_t)(live ? ((k & kKeyLaneMask) | (same ? 64u : 0u)) : 0xFFu));
                        const uint64_t rowm = !P ? ~0ull : lane >= kHalf ? ~0ull << kHalf : ~0ull >> kHalf;
                        if (head) gstore(ord.ucol + at + __popcll(hm & rowm & ((1ull << lane) - 1ull)), (int32_t)col);
                    }
                    if constexpr (P) {
                        done(a, __popcll(hm & 0xffffffffull));
                        if (b >= 0) done(b, __popcll(hm >> kHalf));
                    } else {
                        done(a, __popcll(hm));
                    }
                } else if constexpr (!VALUES) {
                    const uint64_t m = distinct_merged(gi.c == kEmptyCol ? ~0u : (uint32_t)gi.c, 1 << sw, T, lane,
                                                       P ? kHalf : kWave);
                    if constexpr (P) {
                        done(a, __popcll(m & 0xffffffffull));
                        if (b >= 0) done(b, __popcll(m >> kHalf));
                    } else {
                        done(a, __popcll(m));
                    }
                } else {
                    uint32_t k = gi.c == kEmptyCol ? (kKeyEmpty | (uint32_t)lane)
                                                   : (((uint32_t)gi.c << kKeyLaneBits) | (uint32_t)lane);
                    double v = gi.av * gi.bv;  // one rounded product
                    uint64_t lm;
                    bool live;
                    int pos;
                    if constexpr (ORD && !BATCH) {
                        // the order the symbolic pass kept: the values in it, then the tree's additions
                        (void)k;
                        live = gi.q != 0xFFu;
                        const int src = (int)(gi.q & kKeyLaneMask);
                        const bool same = live && ((gi.q >> 6) & 1u);
                        v = __shfl(v, src, kWave);
                        const int lsw = P ? sel32(m_sw, a, b) : sw;  // the lane's own row's list width
                        lm = tree_adds_stored(live, same, src, v, lsw, T, lane, ceil_log2(T) - sw);
                        live = (lm >> lane) & 1ull;
                        const uint64_t rowm = !P ? ~0ull : lane >= kHalf ? ~0ull << kHalf : ~0ull >> kHalf;
                        pos = __popcll(lm & rowm & ((1ull << lane) - 1ull));
                        // the column: the row's pos-th distinct column (held by lane pos of the row's lanes)
                        const int ul = (P && lane >= kHalf ? kHalf : 0) + (pos & (kWave - 1));
                        k = (uint32_t)__shfl(gi.u, ul < kWave ? ul : 0, kWave) << kKeyLaneBits;
                    } else if constexpr (BATCH) {
                        // one sort, then the tree's additions level by level
                        // (rows of single-entry lists with many repeated
                        // columns: no compaction between rounds)
                        key_sort(k, 1 << sw, T, lane);
                        v = __shfl(v, (int)(k & kKeyLaneMask), kWave);  // the values in key order
                        // the lane's own row's list width (the rows of a pair may differ)
                        const int lsw = P ? sel32(m_sw, a, b) : sw;
                        lm = tree_adds(k, v, lsw, T, lane, ceil_log2(T) - sw);
                        live = (lm >> lane) & 1ull;
                        // a column's position in its row: the sums before it in the row's lanes
                        const uint64_t rowm = !P ? ~0ull : lane >= kHalf ? ~0ull << kHalf : ~0ull >> kHalf;
                        pos = __popcll(lm & rowm & ((1ull << lane) - 1ull));
                    } else {
                        // round by round, compacting after every round that
                        // added (few repeats: most rounds only check)
                        if (!key_rounds(k, v, 1 << sw, T, lane, xk, xv)) v = __shfl(v, (int)(k & kKeyLaneMask), kWave);
                        live = k < kKeyEmpty;
                        lm = wave_ballot(live);
                        // live entries sit at the front of their row's lanes
                        pos = P ? (lane & (kHalf - 1)) : lane;
                    }
                    const int64_t cs = sel64(m_cs, a, b);
                    const int cap = sel32(m_cap, a, b);
                    int32_t *cc = c_col;
                    double *cv = c_val;
                    if constexpr (BATCH) {
                        cc = reinterpret_cast<int32_t *>(
                            pick(a, b, [](const auto &q) { return reinterpret_cast<int64_t>(q.c_col); }));
                        cv = reinterpret_cast<double *>(
                            pick(a, b, [](const auto &q) { return reinterpret_cast<int64_t>(q.c_val); }));
                    }
                    if (live && pos < cap) {
                        gstore(cc + cs + pos, (int32_t)(k >> kKeyLaneBits));
                        gstore(cv + cs + pos, v);
                    }
                    if constexpr (P) {
                        done(a, __popcll(lm & 0xffffffffull));
                        if (b >= 0) done(b, __popcll(lm >> kHalf));
                    } else {
                        done(a, __popcll(lm));
                    }
                }
            };
            // D register sets of each kind: item v's lists sit in set v mod D
            // until its B entries are gathered into gather set v mod D (the
            // arrays are indexed by unrolled constants: registers)
            ListStageRegs l[D];
            GatherRegs g[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                l[i].av = 0.0;
                load_lists(i, l[i].bs, l[i].ln, l[i].av);
            }
#pragma unroll
            for (int i = 0; i + 1 < D; ++i)
                gather(i, l[i].bs, l[i].ln, l[i].av, g[i].c, g[i].bv, g[i].av, g[i].q, g[i].u);
            // unrolled by D: the register sets rotate roles, so no register
            // with a load in flight is copied at the loop latch
            for (int v = 0; v < nv; v += D) {
#pragma unroll
                for (int i = 0; i < D; ++i)
                    if (v + i < nv) step(v + i, l[(i + D - 1) % D], l[i], g[i], g[(i + D - 1) % D]);
            }
            // the stages loaded past the chunk's end are drained here, once
#pragma unroll
            for (int i = 0; i < D; ++i) {
                asm volatile("" ::"v"(g[i].c), "v"(l[i].ln), "v"(l[i].bs));
                if constexpr (VALUES) asm volatile("" ::"v"(g[i].bv), "v"(l[i].av));
                if constexpr (ORD && VALUES) asm volatile("" ::"v"(g[i].q), "v"(g[i].u));
            }
        };
        if (all_small) run(std::true_type{});
        else run(std::false_type{});
        if constexpr (VALUES && !BATCH) {
            if (ovf_mask) {
                // one reservation for the chunk's overflowing rows (light rows
                // fill the list from its end)
                unsigned long long at = 0;
                if (lane == 0)
                    at = atomicAdd(reinterpret_cast<unsigned long long *>(&ctl->ovf_light),
                                   (unsigned long long)__popcll(ovf_mask));
                at = (unsigned long long)wave_uniform((int64_t)__shfl((int64_t)at, 0, kWave));
                if ((ovf_mask >> lane) & 1) {
                    const int rank = __popcll(ovf_mask & ((1ull << lane) - 1));
                    no.ovf_rows[no.M - 1 - (int64_t)(at + rank)] = (int32_t)m_row;
                }
            }
        }
    }
}

// ORD: the numeric pass of the precise method with the order the symbolic
// pass kept (ord), else the merges of the windows themselves
template <typename IA, typename IB, bool ORD>
__global__ __launch_bounds__(256) void k_num_win(int cls, const void *a_rpt, Lists<IB> lists,
                                                 const double *a_val, const int32_t *b_col,
                                                 const double *b_val, const uint8_t *row_class,
                                                 const int32_t *class_rows, const int64_t *c_rpt, int32_t *c_col,
                                                 double *c_val, Ctl *ctl, NumOut no, WinOrder ord) {
    __shared__ uint32_t xk[4][kWave];
    __shared__ double xv[4][kWave];
    const int team = wave_uniform((int)(threadIdx.x / kWave));
    win_chunks<true, false, IA, IB, false, ORD>(cls, a_rpt, lists, a_val, b_col, b_val, row_class, class_rows,
                                                c_rpt, c_col, c_val, nullptr, ctl, no, nullptr, xk[team], xv[team],
                                                (int64_t)blockIdx.x * 4 + team, (int64_t)gridDim.x * 4, BatchRows{},
                                                ord);
}

// ORD: the symbolic pass also keeps each row's window order for the numeric pass
template <bool HASH, typename IA, typename IB, bool ORD>
__global__ __launch_bounds__(256) void k_sym_win(int cls, const void *a_rpt, Lists<IB> lists,
                                                 const int32_t *b_col, const uint8_t *row_class,
                                                 const int32_t *class_rows, int32_t *row_size, Ctl *ctl,
                                                 WinOrder ord) {
    __shared__ int32_t tab[4][2 * kWave];
    const int team = wave_uniform((int)(threadIdx.x / kWave));
    NumOut no;
    no.bound = 0;
    win_chunks<false, HASH, IA, IB, false, ORD>(cls, a_rpt, lists, nullptr, b_col, nullptr, row_class, class_rows,
                                                nullptr, nullptr, nullptr, row_size, ctl, no, tab[team], nullptr,
                                                nullptr, (int64_t)blockIdx.x * 4 + team, (int64_t)gridDim.x * 4,
                                                BatchRows{}, ord);
}

// ---------------------------------------------------------------------------
// Rows whose lists fit lane windows of NR = 2..16 registers per lane
// (kClassMulti, see multi_shift): the register merge above with NR keys per
// lane.  Element x of the row's window lives in lane x / NR, register
// x % NR, so list p occupies elements [p W0, (p+1) W0), and since there are
// at most 64 lists, W0 >= NR: the NR elements of a lane are consecutive
// entries of one list.  A merge stage at distance d >= NR exchanges between
// lanes (lane xor d / NR), one at d < NR between two registers of a lane.
//
// The key is the column above kMwShift = 11 bits.  Its low 10 bits name the
// LDS slot of the entry's value (register e of lane l stores at e * 64 + l,
// so that the multiplying phase writes without bank conflicts); bit 10 marks
// an entry that was added into its neighbour.  A dropped entry has all 11
// low bits set: the dropped entries of a column are equal keys behind its
// live one, so every window stays sorted without compaction.  After each
// round, of two live entries with equal columns (one from each list of a
// pair, next to each other) the first takes the sum and the second is
// dropped.  Columns must be below 2^21 (a dropped entry of column 2^21 - 1
// then equals the empty key; neither is live).
// ---------------------------------------------------------------------------
constexpr int kMwShift = 11;
constexpr uint32_t kMwDrop = 1u << 10;
constexpr uint32_t kMwLow = (1u << kMwShift) - 1;
constexpr uint32_t kMwSlotMask = kMwDrop - 1;
constexpr uint32_t kMwEmpty = ~0u;

// compare-exchange of every register with the same register of lane ^ LD
template <int NR, int LD>
__device__ __forceinline__ void mw_cmpx_lanes(uint32_t (&k)[NR], int lane) {
    const bool lower = (lane & LD) == 0;
#pragma unroll
    for (int e = 0; e < NR; ++e) {
        const uint32_t p = xor_lane<LD>(k[e], lane);
        const uint32_t lo = p < k[e] ? p : k[e], hi = p < k[e] ? k[e] : p;
        k[e] = lower ? lo : hi;
    }
}

// half-cleaners at element distances D, D/2, ..., 1
template <int NR, int D>
__device__ __forceinline__ void mw_half_cleaners(uint32_t (&k)[NR], int lane) {
    if constexpr (D >= 1) {
        if constexpr (D >= NR) {
            mw_cmpx_lanes<NR, D / NR>(k, lane);
        } else {
#pragma unroll
            for (int e = 0; e < NR; ++e) {
                if ((e & D) == 0) {
                    const uint32_t a = k[e], b = k[e + D];
                    k[e] = a < b ? a : b;
                    k[e + D] = a < b ? b : a;
                }
            }
        }
        mw_half_cleaners<NR, D / 2>(k, lane);
    }
}

// bitonic merge of every pair of sorted windows of width W: the mirror
// stage (element x against x ^ (2W - 1)), then the half-cleaners
template <int NR, int W>
__device__ __forceinline__ void mw_merge(uint32_t (&k)[NR], int lane) {
    if constexpr (2 * W <= NR) {
#pragma unroll
        for (int e = 0; e < NR; ++e) {
            if ((e & W) == 0) {
                const int f = e ^ (2 * W - 1);
                const uint32_t a = k[e], b = k[f];
                k[e] = a < b ? a : b;
                k[f] = a < b ? b : a;
            }
        }
    } else {
        // the mirror of lane l, register e is lane l ^ (2W/NR - 1), register NR-1-e
        const bool lower = (lane & (W / NR)) == 0;
        uint32_t p[NR];
#pragma unroll
        for (int e = 0; e < NR; ++e) p[e] = xor_lane<2 * W / NR - 1>(k[NR - 1 - e], lane);
#pragma unroll
        for (int e = 0; e < NR; ++e) {
            const uint32_t lo = p[e] < k[e] ? p[e] : k[e], hi = p[e] < k[e] ? k[e] : p[e];
            k[e] = lower ? lo : hi;
        }
    }
    mw_half_cleaners<NR, W / 2>(k, lane);
}

template <int NR>
__device__ __forceinline__ void mw_merge_w(uint32_t (&k)[NR], int lane, int W) {
#define BRM_MW_CASE(X)                                     \
    case X:                                                \
        if constexpr (X <= 32 * NR) mw_merge<NR, X>(k, lane); \
        break;
    switch (W) {
        BRM_MW_CASE(1)
        BRM_MW_CASE(2)
        BRM_MW_CASE(4)
        BRM_MW_CASE(8)
        BRM_MW_CASE(16)
        BRM_MW_CASE(32)
        BRM_MW_CASE(64)
        BRM_MW_CASE(128)
        BRM_MW_CASE(256)
        BRM_MW_CASE(512)
        default: break;
    }
#undef BRM_MW_CASE
}

// after a merge into windows of W2: a live entry whose predecessor in its
// window is live with the same column is added into it and dropped
template <int NR>
__device__ __forceinline__ void mw_dedup(uint32_t (&k)[NR], int lane, int W2, double *vals) {
    uint32_t prev[NR];
    prev[0] = lane_prev(k[NR - 1]);
#pragma unroll
    for (int e = 1; e < NR; ++e) prev[e] = k[e - 1];
    bool dup[NR];
    bool any = false;
#pragma unroll
    for (int e = 0; e < NR; ++e) {
        const int x = lane * NR + e;
        dup[e] = (x & (W2 - 1)) != 0 && ((k[e] | prev[e]) & kMwDrop) == 0 &&
                 (k[e] >> kMwShift) == (prev[e] >> kMwShift);
        any = any || dup[e];
    }
    if (!wave_ballot(any)) return;
#pragma unroll
    for (int e = 0; e < NR; ++e) {
        if (dup[e]) {
            const uint32_t a = prev[e] & kMwSlotMask, b = k[e] & kMwSlotMask;
            vals[a] = vals[a] + vals[b];  // the two children of one node
            k[e] |= kMwLow;
        }
    }
}

// One row under windows of NR registers: multiplying phase from the list
// descriptors (lane t < L holds list t: B row start, length, A value),
// accumulating rounds, write-out (VALUES) or count of distinct columns.
// Returns the row's length to every lane.
template <int NR, bool VALUES, typename IB>
__device__ __forceinline__ int mw_row(int lane, int sw, IB bs, int ln, double av, const int32_t *b_col,
                                      const double *b_val, double *vals, int32_t *out_col, double *out_val,
                                      int cap) {
    constexpr int T = kWave * NR;
    const int W0 = 1 << sw;
    // the lane's elements are entries o0 .. o0 + NR - 1 of list li
    const int li = (lane * NR) >> sw;
    const int o0 = (lane * NR) & (W0 - 1);
    const int64_t lbs = __shfl((int64_t)bs, li, kWave);
    const int lln = __shfl(ln, li, kWave);
    double lav = 0.0;
    if constexpr (VALUES) lav = __shfl(av, li, kWave);
    uint32_t k[NR];
    int32_t c[NR];
    double bv[NR];
#pragma unroll
    for (int e = 0; e < NR; ++e) {
        c[e] = kEmptyCol;
        bv[e] = 0.0;
        if (o0 + e < lln) {
            c[e] = gload(b_col + lbs + o0 + e);
            if constexpr (VALUES) bv[e] = gload(b_val + lbs + o0 + e);
        }
    }
#pragma unroll
    for (int e = 0; e < NR; ++e) {
        if constexpr (VALUES) {
            const int slot = e * kWave + lane;
            vals[slot] = lav * bv[e];  // one rounded product
            k[e] = c[e] == kEmptyCol ? kMwEmpty : (((uint32_t)c[e] << kMwShift) | (uint32_t)slot);
        } else {
            k[e] = c[e] == kEmptyCol ? kMwEmpty : (uint32_t)c[e];
        }
    }
    for (int W = W0; W < T; W <<= 1) {
        mw_merge_w<NR>(k, lane, W);
        if constexpr (VALUES) mw_dedup<NR>(k, lane, 2 * W, vals);
    }
    if constexpr (VALUES) {
        int cnt = 0;
#pragma unroll
        for (int e = 0; e < NR; ++e) cnt += (k[e] & kMwDrop) == 0;
        const int incl = wave_incl_scan(cnt);
        int pos = incl - cnt;
#pragma unroll
        for (int e = 0; e < NR; ++e) {
            if ((k[e] & kMwDrop) == 0) {
                if (pos < cap) {
                    gstore(out_col + pos, (int32_t)(k[e] >> kMwShift));
                    gstore(out_val + pos, vals[k[e] & kMwSlotMask]);
                }
                ++pos;
            }
        }
        return __builtin_amdgcn_readlane(incl, kWave - 1);
    } else {
        const uint32_t p0 = lane_prev(k[NR - 1]);
        int cnt = 0;
#pragma unroll
        for (int e = 0; e < NR; ++e) {
            const uint32_t prev = e == 0 ? p0 : k[e - 1];
            cnt += k[e] != kMwEmpty && ((lane == 0 && e == 0) || k[e] != prev);
        }
        return __builtin_amdgcn_readlane(wave_incl_scan(cnt), kWave - 1);
    }
}

// The rows of kClassMulti, one wavefront per row, in chunks of kWave rows
// whose row ids, A row pointers, window widths and C row pointers are
// loaded at once (lane j holds row j's).
template <bool VALUES, typename IA, typename IB, bool BATCH = false>
__device__ __forceinline__ void mw_rows(int cls, const void *a_rpt, const Lists<IB> &lists, const double *a_val,
                                        const int32_t *b_col, const double *b_val, const uint8_t *row_class,
                                        const int32_t *class_rows, const int64_t *c_rpt, int32_t *c_col,
                                        double *c_val, int32_t *row_size, Ctl *ctl, const NumOut &no, double *vals,
                                        int64_t first, int64_t stride, BatchRows br = BatchRows{}) {
    const int lane = lane_id();
    const int64_t count = ctl->count[cls];
    const int64_t start = class_start(ctl, cls);
    const int64_t nchunks = (count + kWave - 1) / kWave;
    const IB *ent_bs = static_cast<const IB *>(lists.ent_bs);
    const int32_t *ent_len = lists.ent_len;
    for (int64_t ch = first; ch < nchunks; ch += stride) {
        const int64_t base = ch * kWave;
        const int n = (int)(count - base < kWave ? count - base : kWave);
        int64_t m_row = 0, m_a0 = 0, m_cs = 0;
        int m_L = 0, m_sw = 0, m_cap = 0;
        // batched: the row's problem (first descriptor, operand and output arrays)
        int64_t m_eo = 0, m_aval = 0, m_bcol = 0, m_bval = 0, m_ccol = 0, m_cval = 0;
        if (lane < n) {
            m_row = class_rows[start + base + lane];
            const void *rpt = a_rpt;
            const int64_t *crpt = c_rpt;
            int64_t r = m_row;
            if constexpr (BATCH) {
                const BatchProb &pr = br.tab[br.row_prob[m_row]];
                rpt = pr.a_rpt;
                crpt = pr.c_rpt;
                r = m_row - pr.row_off;
                m_eo = pr.ent_off;
                m_aval = reinterpret_cast<int64_t>(pr.a_val);
                m_bcol = reinterpret_cast<int64_t>(pr.b_col);
                m_bval = reinterpret_cast<int64_t>(pr.b_val);
                m_ccol = reinterpret_cast<int64_t>(pr.c_col);
                m_cval = reinterpret_cast<int64_t>(pr.c_val);
            }
            m_a0 = ld_rpt<IA>(rpt, r);
            m_L = (int)(ld_rpt<IA>(rpt, r + 1) - m_a0);
            m_sw = row_class[m_row] >> kClassBits;
            if constexpr (VALUES) {
                m_cs = gload(crpt + r);
                m_cap = (int)(gload(crpt + r + 1) - m_cs);  // a row's size fits 31 bits
            }
        }
        for (int j = 0; j < n; ++j) {
            const int64_t row = lane_value(m_row, j);
            const int64_t a0 = lane_value(m_a0, j);
            const int L = lane_value(m_L, j);
            const int sw = lane_value(m_sw, j);
            const double *av_p = a_val;
            const int32_t *bc_p = b_col;
            const double *bv_p = b_val;
            int32_t *cc_p = c_col;
            double *cv_p = c_val;
            int64_t e0 = a0;
            if constexpr (BATCH) {
                e0 = lane_value(m_eo, j) + a0;
                av_p = reinterpret_cast<const double *>(lane_value(m_aval, j));
                bc_p = reinterpret_cast<const int32_t *>(lane_value(m_bcol, j));
                bv_p = reinterpret_cast<const double *>(lane_value(m_bval, j));
                cc_p = reinterpret_cast<int32_t *>(lane_value(m_ccol, j));
                cv_p = reinterpret_cast<double *>(lane_value(m_cval, j));
            }
            IB bs = 0;
            int ln = 0;
            double av = 0.0;
            if (lane < L) {
                bs = gload(ent_bs + e0 + lane);
                ln = gload(ent_len + e0 + lane);
                if constexpr (VALUES) av = gload(av_p + a0 + lane);
            }
            int64_t cs = 0;
            int cap = 0;
            if constexpr (VALUES) {
                cs = lane_value(m_cs, j);
                cap = lane_value(m_cap, j);
            }
            int32_t *oc = VALUES ? cc_p + cs : nullptr;
            double *ov = VALUES ? cv_p + cs : nullptr;
            const int t = sw + ceil_log2(L);  // log2 of the padded total, 7..10
            int len;
            switch (t) {
                case 7: len = mw_row<2, VALUES, IB>(lane, sw, bs, ln, av, bc_p, bv_p, vals, oc, ov, cap); break;
                case 8: len = mw_row<4, VALUES, IB>(lane, sw, bs, ln, av, bc_p, bv_p, vals, oc, ov, cap); break;
                case 9: len = mw_row<8, VALUES, IB>(lane, sw, bs, ln, av, bc_p, bv_p, vals, oc, ov, cap); break;
                default: len = mw_row<16, VALUES, IB>(lane, sw, bs, ln, av, bc_p, bv_p, vals, oc, ov, cap); break;
            }
            if constexpr (VALUES) {
                if (no.bound) {
                    // slot mode: exact length kept, an overflowing row listed
                    // for the fallback (light rows fill the list from its end)
                    if (lane == 0) {
                        no.row_size[row] = len;
                        if (len > cap) {
                            const unsigned long long at =
                                atomicAdd(reinterpret_cast<unsigned long long *>(&ctl->ovf_light), 1ull);
                            no.ovf_rows[no.M - 1 - (int64_t)at] = (int32_t)row;
                        }
                    }
                } else if (lane == 0 && len != cap) {
                    atomicOr(reinterpret_cast<unsigned long long *>(&ctl->err), (unsigned long long)kErrSizeMismatch);
                }
            } else {
                if (lane == 0) row_size[row] = len;
            }
        }
    }
}

template <typename IA, typename IB>
__global__ __launch_bounds__(256) void k_num_mw(int cls, const void *a_rpt, Lists<IB> lists, const double *a_val,
                                                const int32_t *b_col, const double *b_val, const uint8_t *row_class,
                                                const int32_t *class_rows, const int64_t *c_rpt, int32_t *c_col,
                                                double *c_val, Ctl *ctl, NumOut no) {
    __shared__ double vals[4][kMwSlots];
    const int team = wave_uniform((int)(threadIdx.x / kWave));
    mw_rows<true, IA, IB>(cls, a_rpt, lists, a_val, b_col, b_val, row_class, class_rows, c_rpt, c_col, c_val,
                          nullptr, ctl, no, vals[team], (int64_t)blockIdx.x * 4 + team, (int64_t)gridDim.x * 4);
}

// The symbolic passes of the multi-register window, wave and group classes
// (all 256-thread workgroups) in one launch: workgroups [0, g_mw) count the
// multi-register rows, the next g_wave the wave class by LDS hash (four rows
// per workgroup), the last g_group the group class (one row per workgroup).
// A class without rows then costs no launch of its own.
template <typename IA, typename IB>
__global__ __launch_bounds__(256) void k_sym_mid(const void *a_rpt, Lists<IB> lists, const int32_t *b_col,
                                                 const uint8_t *row_class, const int32_t *class_rows,
                                                 int32_t *row_size, Ctl *ctl, int g_mw, int g_wave, int g_group) {
    using WaveLds = SymLds<64, 2 * kCapWave>;
    using GroupLds = SymLds<256, 2 * kCapGroup>;
    constexpr size_t kWaveBytes = 4 * sizeof(WaveLds), kGroupBytes = sizeof(GroupLds);
    __shared__ __align__(16) unsigned char raw[kWaveBytes > kGroupBytes ? kWaveBytes : kGroupBytes];
    const int b = blockIdx.x;  // uniform: every workgroup takes one branch whole
    if (b < g_mw) {
        const int team = wave_uniform((int)(threadIdx.x / kWave));
        NumOut no;
        no.bound = 0;
        mw_rows<false, IA, IB>(kClassMulti, a_rpt, lists, nullptr, b_col, nullptr, row_class, class_rows, nullptr,
                               nullptr, nullptr, row_size, ctl, no, nullptr, (int64_t)b * 4 + team,
                               (int64_t)g_mw * 4);
    } else if (b < g_mw + g_wave) {
        sym_hash_rows<64, 4, 2 * kCapWave, IA, IB>(reinterpret_cast<WaveLds *>(raw), kClassWave, b - g_mw, g_wave,
                                                   a_rpt, lists, b_col, class_rows, row_size, ctl);
    } else {
        sym_hash_rows<256, 1, 2 * kCapGroup, IA, IB>(reinterpret_cast<GroupLds *>(raw), kClassGroup,
                                                     b - g_mw - g_wave, g_group, a_rpt, lists, b_col, class_rows,
                                                     row_size, ctl);
    }
}

hipError_t launch_symbolic_mid(const CsrView &A, const CsrView &B, const Workspace &ws, int g_mw, int g_wave,
                               int g_group, hipStream_t s) {
    const int grid = g_mw + g_wave + g_group;
#define BRM_SYM_MID(IA, IB)                                                                                  \
    hipLaunchKernelGGL((k_sym_mid<IA, IB>), dim3(grid), dim3(256), 0, s, A.rpt, ws_lists<IB>(A, B, ws), B.col, \
                       ws.row_class, ws.class_rows, ws.row_size, ws.ctl, g_mw, g_wave, g_group)
    if (A.rpt_bytes == 4 && B.rpt_bytes == 4) BRM_SYM_MID(int32_t, int32_t);
    else if (A.rpt_bytes == 4) BRM_SYM_MID(int32_t, int64_t);
    else if (B.rpt_bytes == 4) BRM_SYM_MID(int64_t, int32_t);
    else BRM_SYM_MID(int64_t, int64_t);
#undef BRM_SYM_MID
    return hipGetLastError();
}

// Several short rows per team: the rows of a class whose lists and products
// each stay within CAP / G are merged G at a time, so that one wavefront
// keeps G rows' loads in flight.
template <int T, int TEAMS, int CAP, int G, typename IA, typename IB>
__global__ __launch_bounds__(T *TEAMS) void k_num_group(int cls, const void *a_rpt, Lists<IB> lists,
                                                        const double *a_val, const int32_t *b_col,
                                                        const double *b_val, const int32_t *class_rows,
                                                        const int64_t *c_rpt, int32_t *c_col, double *c_val,
                                                        Ctl *ctl, NumOut no) {
    __shared__ NumLds<T, CAP, G> lds[TEAMS];
    const int team = threadIdx.x / T, tid = threadIdx.x % T;
    NumLds<T, CAP, G> &s = lds[team];
    const int64_t count = ctl->count[cls];
    const int64_t start = class_start(ctl, cls);
    for (int64_t base = ((int64_t)blockIdx.x * TEAMS + team) * G; base < count;
         base += (int64_t)gridDim.x * TEAMS * G) {
        const int n = (count - base) < G ? (int)(count - base) : G;
        if (tid < n) {
            const int64_t row = class_rows[start + base + tid];
            const int64_t a0 = ld_rpt<IA>(a_rpt, row);
            const int64_t cs = gload(c_rpt + (row));
            s.row[tid] = row;
            s.seg[tid].a0 = a0;
            s.seg[tid].L = (int32_t)(ld_rpt<IA>(a_rpt, row + 1) - a0);
            s.seg[tid].out_col = c_col + cs;
            s.seg[tid].out_val = c_val + cs;
            s.seg[tid].out_cap = gload(c_rpt + (row + 1)) - cs;
        }
        Team<T>::sync();
        brmerge_segs_lds<T, CAP, G, IB>(s, tid, n, lists, a_val, b_col, b_val);
        if (tid < n) finish_row(no, ctl, s.row[tid], s.seg_len[tid], s.seg[tid].out_cap, false);
        Team<T>::sync();
    }
}

// ---------------------------------------------------------------------------
// Hash accumulator (a comparator for the BRMerge kernels, not the paper's
// method): a row's products are added into an LDS hash table keyed by
// column (open addressing, linear probing, atomic compare-and-swap of the
// key and atomic addition of the value), the occupied slots are packed and
// each entry's place in the row is its rank among the row's columns.  Sums
// are formed in whatever order the atomics land: within rounding of the
// definition, not equal to the merge tree's bits, and not reproducible
// between runs.  Rows must hold at most TS / 2 products (the table then
// stays at most half full) and their exact sizes come from the symbolic
// pass.
// ---------------------------------------------------------------------------
template <int T, int TS>
struct HashLds {
    int32_t key[TS];
    double val[TS];
    int32_t off[TS / 2 + 1];  // list offsets of the row's products
    int32_t n;                // packed entries
};

template <int T, int TEAMS, int TS, typename IA, typename IB>
__global__ __launch_bounds__(T *TEAMS) void k_num_hash(int cls, const void *a_rpt, Lists<IB> lists,
                                                       const double *a_val, const int32_t *b_col,
                                                       const double *b_val, const int32_t *class_rows,
                                                       const int64_t *c_rpt, int32_t *c_col, double *c_val, Ctl *ctl) {
    __shared__ HashLds<T, TS> lds[TEAMS];
    __shared__ int32_t scan[TEAMS][Team<T>::kWaves + 1];
    const int team = threadIdx.x / T, tid = threadIdx.x % T;
    HashLds<T, TS> &s = lds[team];
    const int64_t count = ctl->count[cls];
    const int64_t start = class_start(ctl, cls);
    for (int64_t idx = (int64_t)blockIdx.x * TEAMS + team; idx < count; idx += (int64_t)gridDim.x * TEAMS) {
        const int64_t row = class_rows[start + idx];
        const int64_t a0 = ld_rpt<IA>(a_rpt, row);
        const int L = (int)(ld_rpt<IA>(a_rpt, row + 1) - a0);
        const int64_t cs = gload(c_rpt + (row));
        const int cap = (int)(gload(c_rpt + (row + 1)) - cs);
        if (2 * (int64_t)cap > TS) {  // row pointers that are not the symbolic pass's
            if (tid == 0)
                atomicOr(reinterpret_cast<unsigned long long *>(&ctl->err), (unsigned long long)kErrSizeMismatch);
            continue;
        }
        // a table of at least twice the row's size, a power of two
        int lg = 1;
        while ((1 << lg) < 2 * cap) ++lg;
        const int tsz = 1 << lg;
        for (int i = tid; i < tsz; i += T) {
            s.key[i] = -1;
            s.val[i] = 0.0;
        }
        // list offsets
        int carry = 0;
        for (int lb = 0; lb < L; lb += T) {
            const int t = lb + tid;
            int64_t bs = 0;
            int ln = 0;
            if (t < L) lists.get(a0 + t, bs, ln);
            int tot;
            const int ex = Team<T>::excl_scan(ln, &tot, scan[team], tid);
            if (t < L) s.off[t] = carry + ex;
            carry += tot;
        }
        const int nprod = carry;
        if (tid == 0) s.off[L] = nprod;
        Team<T>::sync();
        // multiplying phase straight into the table
        bool lost = false;
        for (int p = tid; p < nprod; p += T) {
            const int t = upper_bound(s.off, L + 1, p) - 1;
            int64_t bs;
            int ln;
            lists.get(a0 + t, bs, ln);
            const int64_t q = bs + (p - s.off[t]);
            const int32_t c = gload(b_col + (q));
            const double v = gload(a_val + (a0 + t)) * gload(b_val + (q));  // one rounded product
            uint32_t h = ((uint32_t)c * 2654435761u) >> (32 - lg);
            int probes = 0;
            for (;;) {
                const int k = atomicCAS(&s.key[h], -1, c);
                if (k == -1 || k == c) {
                    atomicAdd(&s.val[h], v);
                    break;
                }
                h = (h + 1) & (uint32_t)(tsz - 1);
                if (++probes == tsz) {  // only when the symbolic size is wrong
                    lost = true;
                    break;
                }
            }
        }
        if (lost) atomicOr(reinterpret_cast<unsigned long long *>(&ctl->err), (unsigned long long)kErrSizeMismatch);
        Team<T>::sync();
        // pack the occupied slots to the front (slots -> registers -> front)
        constexpr int PER = TS / T;
        int32_t kc[PER];
        double kv[PER];
        int mine = 0;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int i = tid * PER + e;
            kc[e] = i < tsz ? s.key[i] : -1;
            kv[e] = i < tsz ? s.val[i] : 0.0;
            mine += kc[e] >= 0;
        }
        int n;
        const int at = Team<T>::excl_scan(mine, &n, scan[team], tid);
        Team<T>::sync();
        int w = at;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            if (kc[e] >= 0) {
                s.key[w] = kc[e];
                s.val[w] = kv[e];
                ++w;
            }
        }
        Team<T>::sync();
        // place = rank among the row's columns
        for (int i = tid; i < n; i += T) {
            const int32_t c = s.key[i];
            int r = 0;
            for (int j = 0; j < n; ++j) r += s.key[j] < c;
            if (r < cap) {
                gstore(c_col + (cs + r), c);
                gstore(c_val + (cs + r), s.val[i]);
            }
        }
        if (tid == 0 && n != cap)
            atomicOr(reinterpret_cast<unsigned long long *>(&ctl->err), (unsigned long long)kErrSizeMismatch);
        Team<T>::sync();
    }
}

hipError_t launch_numeric_hash(const CsrView &A, const CsrView &B, const Workspace &ws, int cls, int num_cu,
                               const int64_t *c_rpt, int32_t *c_col, double *c_val, hipStream_t s) {
#define BRM_HASH(T, TEAMS, TS, PER_CU, IA, IB)                                                                   \
    hipLaunchKernelGGL((k_num_hash<T, TEAMS, TS, IA, IB>), dim3(num_cu * PER_CU), dim3(T * TEAMS), 0, s, cls,   \
                       A.rpt, ws_lists<IB>(A, B, ws), A.val, B.col, B.val, ws.class_rows, c_rpt, c_col, c_val, \
                       ws.ctl)
#define BRM_HASH_ALL(T, TEAMS, TS, PER_CU)                                                     \
    do {                                                                                       \
        if (A.rpt_bytes == 4 && B.rpt_bytes == 4) BRM_HASH(T, TEAMS, TS, PER_CU, int32_t, int32_t); \
        else if (A.rpt_bytes == 4) BRM_HASH(T, TEAMS, TS, PER_CU, int32_t, int64_t);           \
        else if (B.rpt_bytes == 4) BRM_HASH(T, TEAMS, TS, PER_CU, int64_t, int32_t);           \
        else BRM_HASH(T, TEAMS, TS, PER_CU, int64_t, int64_t);                                 \
    } while (0)
    switch (cls) {
        case kClassWaveSmall: BRM_HASH_ALL(64, 4, 2 * kCapWaveSmall, 8); break;
        case kClassWave: BRM_HASH_ALL(64, 4, 2 * kCapWave, 4); break;
        case kClassMulti:  // at most 1024 products
        case kClassGroup: BRM_HASH_ALL(256, 1, 2 * kCapGroup, 4); break;
        case kClassBlock: BRM_HASH_ALL(1024, 1, 2 * kCapBlock, 1); break;
        default: return hipErrorInvalidValue;
    }
#undef BRM_HASH_ALL
#undef BRM_HASH
    return hipGetLastError();
}

hipError_t launch_numeric(const CsrView &A, const CsrView &B, const Workspace &ws, int cls,
                          int grid, const int64_t *c_rpt, int32_t *c_col, double *c_val,
                          const NumOut &no, hipStream_t s, int group_rows) {
#define BRM_NUM(KERNEL, BLOCK, IB)                                                               \
    hipLaunchKernelGGL((KERNEL), dim3(grid), dim3(BLOCK), 0, s, cls, A.rpt, ws_lists<IB>(A, B, ws), \
                       A.val, B.col, B.val, ws.class_rows, c_rpt, c_col, c_val, ws.ctl, no)
#define BRM_NUM_ALL(T, TEAMS, CAP)                                                               \
    do {                                                                                         \
        if (A.rpt_bytes == 4 && B.rpt_bytes == 4)                                                \
            BRM_NUM((k_num_lds<T, TEAMS, CAP, int32_t, int32_t>), T *TEAMS, int32_t);            \
        else if (A.rpt_bytes == 4)                                                               \
            BRM_NUM((k_num_lds<T, TEAMS, CAP, int32_t, int64_t>), T *TEAMS, int64_t);            \
        else if (B.rpt_bytes == 4)                                                               \
            BRM_NUM((k_num_lds<T, TEAMS, CAP, int64_t, int32_t>), T *TEAMS, int32_t);            \
        else                                                                                     \
            BRM_NUM((k_num_lds<T, TEAMS, CAP, int64_t, int64_t>), T *TEAMS, int64_t);            \
    } while (0)
    switch (cls) {
        case kClassCopy:
            if (A.rpt_bytes == 4 && B.rpt_bytes == 4) BRM_NUM((k_num_copy<int32_t, int32_t>), 256, int32_t);
            else if (A.rpt_bytes == 4) BRM_NUM((k_num_copy<int32_t, int64_t>), 256, int64_t);
            else if (B.rpt_bytes == 4) BRM_NUM((k_num_copy<int64_t, int32_t>), 256, int32_t);
            else BRM_NUM((k_num_copy<int64_t, int64_t>), 256, int64_t);
            break;
        case kClassWaveSmall:
            if (group_rows == 0) {
                BRM_NUM_ALL(64, 4, kCapWaveSmall);
                break;
            }
            if (group_rows == 1 || group_rows == 2) {
#define BRM_NUM_WIN(IA, IB)                                                                                      \
    do {                                                                                                         \
        const WinOrder ord{ws.order, ws.ucol};                                                                   \
        if (ws.order && !no.bound)                                                                               \
            hipLaunchKernelGGL((k_num_win<IA, IB, true>), dim3(grid), dim3(256), 0, s, cls, A.rpt,                \
                               ws_lists<IB>(A, B, ws), A.val, B.col, B.val, ws.row_class, ws.class_rows, c_rpt,  \
                               c_col, c_val, ws.ctl, no, ord);                                                   \
        else                                                                                                     \
            hipLaunchKernelGGL((k_num_win<IA, IB, false>), dim3(grid), dim3(256), 0, s, cls, A.rpt,               \
                               ws_lists<IB>(A, B, ws), A.val, B.col, B.val, ws.row_class, ws.class_rows, c_rpt,  \
                               c_col, c_val, ws.ctl, no, ord);                                                   \
    } while (0)
                if (A.rpt_bytes == 4 && B.rpt_bytes == 4) BRM_NUM_WIN(int32_t, int32_t);
                else if (A.rpt_bytes == 4) BRM_NUM_WIN(int32_t, int64_t);
                else if (B.rpt_bytes == 4) BRM_NUM_WIN(int64_t, int32_t);
                else BRM_NUM_WIN(int64_t, int64_t);
#undef BRM_NUM_WIN
                break;
            }
            if (A.rpt_bytes == 4 && B.rpt_bytes == 4)
                BRM_NUM((k_num_group<64, 4, kGroupRows * kCapWaveSmall, kGroupRows, int32_t, int32_t>), 256, int32_t);
            else if (A.rpt_bytes == 4)
                BRM_NUM((k_num_group<64, 4, kGroupRows * kCapWaveSmall, kGroupRows, int32_t, int64_t>), 256, int64_t);
            else if (B.rpt_bytes == 4)
                BRM_NUM((k_num_group<64, 4, kGroupRows * kCapWaveSmall, kGroupRows, int64_t, int32_t>), 256, int32_t);
            else
                BRM_NUM((k_num_group<64, 4, kGroupRows * kCapWaveSmall, kGroupRows, int64_t, int64_t>), 256, int64_t);
            break;
        case kClassMulti:
#define BRM_NUM_MW(IA, IB)                                                                                      \
    hipLaunchKernelGGL((k_num_mw<IA, IB>), dim3(grid), dim3(256), 0, s, cls, A.rpt, ws_lists<IB>(A, B, ws), A.val, \
                       B.col, B.val, ws.row_class, ws.class_rows, c_rpt, c_col, c_val, ws.ctl, no)
            if (A.rpt_bytes == 4 && B.rpt_bytes == 4) BRM_NUM_MW(int32_t, int32_t);
            else if (A.rpt_bytes == 4) BRM_NUM_MW(int32_t, int64_t);
            else if (B.rpt_bytes == 4) BRM_NUM_MW(int64_t, int32_t);
            else BRM_NUM_MW(int64_t, int64_t);
#undef BRM_NUM_MW
            break;
        case kClassWave: BRM_NUM_ALL(64, 4, kCapWave); break;
        case kClassGroup: BRM_NUM_ALL(256, 1, kCapGroup); break;
        case kClassBlock: BRM_NUM_ALL(1024, 1, kCapBlock); break;
        default: return hipErrorInvalidValue;
    }
#undef BRM_NUM_ALL
#undef BRM_NUM
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// heavy rows: more products than one workgroup's LDS holds
//
// One workgroup of T threads per row: T = 512 (two per compute unit, each
// merging its own row, so one waits at a barrier while the other works; LDS
// nodes of 2048 products) or T = 1024 (one per compute unit, nodes of 4096:
// faster on one very long row).  The row's lists are consumed left to
// right as aligned ranges [p 2^h, (p+1) 2^h) -- nodes of the merge tree --
// each the largest one whose products fit in LDS; such a node is merged in
// LDS exactly like a light row, a single list too long for LDS is scaled
// into place.  Finished nodes go to one of two HBM buffers (ping-pong, every
// node at the offset of its first list's products, so a parent always fits
// where its children were) and a stack of finished nodes combines two
// siblings as soon as both exist (a binary counter over the lists).  When
// the lists run out, a left child without a right sibling is promoted
// unchanged (Algorithm 1's odd last list) and right children merge with the
// node below them.  The grouping of additions is therefore the tree of
// Algorithm 1; two HBM nodes are merged with a merge-path split per tile of
// 4096 output steps staged through LDS, equal columns being added across
// tile boundaries through a carried element.  The root is written straight
// into C.
// ---------------------------------------------------------------------------
// entries of each input staged per tile, and merge steps per thread (a tile
// merges up to 2 kMergeWin entries, kMergeSteps per thread)
// (the heavy kernel exists for T = 512 and T = 1024 threads per workgroup;
// its LDS nodes hold at most 4 T products)
constexpr int kMergeSteps = 4;
constexpr int kWinPer = 2;  // staged entries per thread and input: windows of kWinPer T entries
static_assert(kMergeSteps >= 2 * kWinPer, "a tile's merge steps must cover both windows");

template <int T>
struct MergeLds {
    // two window sets: a tile merges from one while the next tile's windows
    // are staged into the other
    int32_t xc[2][kWinPer * T];
    double xv[2][kWinPer * T];
    int32_t yc[2][kWinPer * T];
    double yv[2][kWinPer * T];
    int32_t first_c[T];
    double first_v[T];
    int32_t last_c[T];
};

struct HeavyNode {
    int64_t p;    // index of the node at its level
    int64_t len;  // length of its merged list
    int h;        // level (the node covers lists [p 2^h, (p+1) 2^h))
    int buf;      // 0 / 1: spill buffer, 2: C
};

template <int T>
struct HeavyState {
    HeavyNode stack[64];
    int sp;
    int64_t next_list;  // first list not consumed yet
    int action;
    int64_t l0, l1;     // list range of a new node
    int h;
    int root;
    int64_t carry_c;
    double carry_v;
    int has_carry;
    int64_t out;
    int64_t scr[Team<T>::kWaves + 1];
};

enum HeavyAction { kActNode = 0, kActMerge = 1, kActPromote = 2, kActToC = 3, kActDone = 4, kActFail = 5 };

// Merge sorted, duplicate-free lists X (left child) and Y (right child) into
// Z, adding the values of equal columns (left + right).  Tiles: the next
// kMergeWin entries of X and of Y sit in LDS; when a window stops short of
// its list's end, every later entry of that list has a larger column than its
// last one, so all entries up to the smaller such last column are present in
// both windows.  The tile merges exactly those (a tile ends on a column
// boundary: the two entries of a column are never split between tiles), and
// the next windows are loaded into registers while it merges.  Z may alias
// the region that Y occupies as long as Z starts at or before X's region
// start and X's region is at least |X| long: output written so far never
// passes the first Y entry not yet consumed, and the next windows are read
// before the tile writes.  Writes at most zcap entries; returns the merged
// length (uniform).
template <int T>
__device__ int64_t merge_hbm(MergeLds<T> &m, HeavyState<T> &st, int tid, const int32_t *Xc,
                             const double *Xv, int64_t nx, const int32_t *Yc, const double *Yv,
                             int64_t ny, int32_t *Zc, double *Zv, int64_t zcap) {
    constexpr int kMergeWin = kWinPer * T;
    int32_t pxc[kWinPer], pyc[kWinPer];
    double pxv[kWinPer], pyv[kWinPer];
    auto win = [](int64_t n, int64_t at) -> int {
        return (int)((n - at) < (int64_t)kMergeWin ? (n - at) : (int64_t)kMergeWin);
    };
    auto fetch = [&](int64_t xs, int64_t ys) {
        const int wx = win(nx, xs), wy = win(ny, ys);
#pragma unroll
        for (int e = 0; e < kWinPer; ++e) {
            const int i = tid + e * T;
            if (i < wx) {
                pxc[e] = gload(Xc + xs + i);
                pxv[e] = gload(Xv + xs + i);
            }
            if (i < wy) {
                pyc[e] = gload(Yc + ys + i);
                pyv[e] = gload(Yv + ys + i);
            }
        }
    };
    auto stage = [&](int64_t xs, int64_t ys, int buf) {
        const int wx = win(nx, xs), wy = win(ny, ys);
#pragma unroll
        for (int e = 0; e < kWinPer; ++e) {
            const int i = tid + e * T;
            if (i < wx) {
                m.xc[buf][i] = pxc[e];
                m.xv[buf][i] = pxv[e];
            }
            if (i < wy) {
                m.yc[buf][i] = pyc[e];
                m.yv[buf][i] = pyv[e];
            }
        }
    };
    int64_t x0 = 0, y0 = 0, out = 0;  // uniform
    int cur = 0;  // window set of the current tile
    fetch(0, 0);
    stage(0, 0, 0);
    __syncthreads();
    while (x0 < nx || y0 < ny) {
        const int32_t *xc = m.xc[cur], *yc = m.yc[cur];
        const double *xv = m.xv[cur], *yv = m.yv[cur];
        const int wx = win(nx, x0), wy = win(ny, y0);
        // the tile: every entry of both windows up to the column `lim`
        // (uniform values are moved to scalar registers)
        int cx = wx, cy = wy;
        {
            const bool tx = x0 + wx < nx, ty = y0 + wy < ny;
            if (tx || ty) {
                int32_t lim = INT32_MAX;
                if (tx) lim = xc[wx - 1];
                if (ty && yc[wy - 1] < lim) lim = yc[wy - 1];
                lim = wave_uniform(lim);
                // a window whose last column is the limit is taken whole
                // (sorted): only the other one is searched
                if (!(tx && wave_uniform(xc[wx - 1]) == lim)) cx = wave_uniform(upper_bound(xc, wx, lim));
                if (!(ty && wave_uniform(yc[wy - 1]) == lim)) cy = wave_uniform(upper_bound(yc, wy, lim));
            }
        }
        const int64_t nx0 = x0 + cx, ny0 = y0 + cy;
        fetch(nx0, ny0);
        // kMergeSteps merge steps per thread; every register array is
        // indexed by unrolled constants only
        const int D = cx + cy;
        const int s0 = tid * kMergeSteps;
        const int cnt = s0 < D ? (D - s0 < kMergeSteps ? D - s0 : kMergeSteps) : 0;
        int32_t c[kMergeSteps];
        double v[kMergeSteps];
        if (cnt > 0) {
            const int x = mp_split_lds(xc, cx, yc, cy, s0);
            const int y = s0 - x;
            // the next kMergeSteps columns of each side, read together; the
            // steps are then decided in registers and their values read
            // together (two LDS round trips instead of one per step)
            int32_t xs[kMergeSteps], ys[kMergeSteps];
#pragma unroll
            for (int j = 0; j < kMergeSteps; ++j) {
                xs[j] = x + j < cx ? xc[x + j] : 0;
                ys[j] = y + j < cy ? yc[y + j] : 0;
            }
            int ix = 0, iy = 0;
            int src[kMergeSteps];  // entry of the step: x index, or ~y index
            int32_t last = 0;
#pragma unroll
            for (int j = 0; j < kMergeSteps; ++j) {
                c[j] = 0;
                src[j] = 0;
                if (j < cnt) {
                    int32_t xcur = xs[0], ycur = ys[0];
#pragma unroll
                    for (int q = 1; q <= j; ++q) {
                        if (ix == q) xcur = xs[q];
                        if (iy == q) ycur = ys[q];
                    }
                    if (x + ix < cx && (y + iy >= cy || xcur <= ycur)) {
                        c[j] = xcur;
                        src[j] = x + ix;
                        ++ix;
                    } else {
                        c[j] = ycur;
                        src[j] = ~(y + iy);
                        ++iy;
                    }
                    last = c[j];
                }
            }
#pragma unroll
            for (int j = 0; j < kMergeSteps; ++j) v[j] = j < cnt ? (src[j] >= 0 ? xv[src[j]] : yv[~src[j]]) : 0.0;
            m.first_c[tid] = c[0];
            m.first_v[tid] = v[0];
            m.last_c[tid] = last;
        }
        const int nthr = (D + kMergeSteps - 1) / kMergeSteps;
        __syncthreads();
        // every thread is done with this tile's windows; the next tile's
        // windows go to the other set, made visible by the scan's barriers
        stage(nx0, ny0, cur ^ 1);
        // heads (first entry of a column) and their values: the two entries
        // of a column are adjacent, the left one first
        bool nb = false;  // the next thread's first entry follows this thread's last
        int32_t nbc = 0;
        double nbv = 0.0;
        bool head0 = true;
        if (cnt > 0) {
            if (tid + 1 < nthr) {
                nb = true;
                nbc = m.first_c[tid + 1];
                nbv = m.first_v[tid + 1];
            }
            if (tid > 0) head0 = c[0] != m.last_c[tid - 1];
        }
        bool hd[kMergeSteps];
        int items = 0;
#pragma unroll
        for (int j = 0; j < kMergeSteps; ++j) {
            hd[j] = j < cnt && (j == 0 ? head0 : c[j] != c[j - 1]);
            bool has_next = j + 1 < cnt;
            int32_t nc = j + 1 < kMergeSteps ? c[j + 1 < kMergeSteps ? j + 1 : j] : 0;
            double nv = j + 1 < kMergeSteps ? v[j + 1 < kMergeSteps ? j + 1 : j] : 0.0;
            if (j == cnt - 1 && nb) {
                has_next = true;
                nc = nbc;
                nv = nbv;
            }
            if (hd[j] && has_next && nc == c[j]) v[j] = v[j] + nv;  // left + right
            items += hd[j] ? 1 : 0;
        }
        int tot;
        const int rank = Team<T>::excl_scan(items, &tot, reinterpret_cast<int *>(st.scr), tid);
        tot = wave_uniform(tot);
        int64_t o = out + rank;
#pragma unroll
        for (int j = 0; j < kMergeSteps; ++j) {
            if (hd[j]) {
                if (o < zcap) {
                    gstore(Zc + o, c[j]);
                    gstore(Zv + o, v[j]);
                }
                ++o;
            }
        }
        out += tot;
        x0 = nx0;
        y0 = ny0;
        cur ^= 1;
        // the boundary arrays were read before the scan's barriers: the next
        // tile may overwrite them
    }
    return out;
}

struct HeavyBatch {
    unsigned long long *ticket;  // next work item of the launch (zeroed before the launch)
    const int32_t *rows;
    const int64_t *spill_off;  // element offset of each row's two spill buffers
    const int64_t *leaf_off;   // offset of each row's list-offset array
    const HeavyItem *items;
    int64_t nitems;
    int64_t *res;              // (buffer, length) of every subtree result
    int32_t *spill_col;
    double *spill_val;
    int32_t *leaf;
    int lds_cap;
};

// The merge tree of lists [lb0, lb1) of one row, walked by one workgroup
// (Algorithm 1's accumulating phase, §III-B): LDS nodes of up to lds_cap
// products and lists, merges of two spilled nodes through HBM.  A whole row
// (res_slot < 0) ends in C; a subtree leaves its merged list in the row's
// spill buffers (spill_col / spill_val: two buffers of nprod entries) and
// its (buffer, length) in res[2 * res_slot].  leaf receives the row's list
// offsets inside its product space.  `id` is the row's id for the
// bound-mode bookkeeping.
template <typename IA, typename IB, int T>
__device__ __forceinline__ void heavy_walk(NumLds<T, 4 * T> &node_lds, MergeLds<T> &mrg, HeavyState<T> &st,
                                           int tid, int64_t row, int64_t lb0, int64_t lb1, int res_slot,
                                           int64_t nprod, int32_t *leaf, int32_t *spill_col, double *spill_val,
                                           int lds_cap, int64_t *res, const void *a_rpt, const Lists<IB> &lists,
                                           const double *a_val, const int32_t *b_col, const double *b_val,
                                           const int64_t *c_rpt, int32_t *c_col, double *c_val, Ctl *ctl,
                                           const NumOut &no, int64_t id) {
    constexpr int kCap = 4 * T;  // products (and lists) of an LDS node
    const bool whole = res_slot < 0;
    const int64_t a0 = ld_rpt<IA>(a_rpt, row);
    const int64_t L = ld_rpt<IA>(a_rpt, row + 1) - a0;
    // list offsets inside the row's product space, for lists [lb0, lb1]:
    // the products of the lists before lb0 first (a reduction only)
    int64_t carry = 0;
    for (int64_t lb = 0; lb < lb0; lb += T) {
        const int64_t l = lb + tid;
        int64_t ln = 0;
        if (l < lb0) {
            int64_t bs;
            int n;
            lists.get(a0 + l, bs, n);
            ln = n;
        }
        int64_t tot;
        (void)Team<T>::excl_scan(ln, &tot, st.scr, tid);
        carry += wave_uniform(tot);
    }
    for (int64_t lb = lb0; lb < lb1; lb += T) {
        const int64_t l = lb + tid;
        int64_t ln = 0;
        if (l < lb1) {
            int64_t bs;
            int n;
            lists.get(a0 + l, bs, n);
            ln = n;
        }
        int64_t tot;
        const int64_t ex = Team<T>::excl_scan(ln, &tot, st.scr, tid);
        if (l < lb1) leaf[l] = (int32_t)(carry + ex);
        carry += wave_uniform(tot);
    }
    // the end offset (also the next item's first offset: the same value)
    if (tid == 0) leaf[lb1] = (int32_t)carry;
    int32_t *bcol[2] = {spill_col, spill_col + nprod};
    double *bval[2] = {spill_val, spill_val + nprod};
    const int64_t cs = c_rpt[row];
    const int64_t ccap = c_rpt[row + 1] - cs;
    if (tid == 0) {
        st.sp = 0;
        st.next_list = lb0;
    }
    // global stores of this workgroup become visible to it at the barrier (workgroup scope)
    __syncthreads();
    int64_t guard = 0;
    while (true) {
        if (tid == 0) {
            int act = kActFail;
            const int sp = st.sp;
            if (++guard > 4 * (lb1 - lb0 + 64)) {
                act = kActFail;
            } else if (sp >= 2 && st.stack[sp - 2].h == st.stack[sp - 1].h &&
                       (st.stack[sp - 1].p & 1) && st.stack[sp - 2].p == st.stack[sp - 1].p - 1) {
                act = kActMerge;
                const HeavyNode &y = st.stack[sp - 1];
                st.root = whole && (y.p >> 1) == 0 && ((int64_t)1 << (y.h + 1)) >= L;
            } else if (st.next_list < lb1) {
                const int64_t l = st.next_list;
                int h = 0;
                while (h < 40 && ((l >> h) & 1) == 0 && l + ((int64_t)1 << h) < lb1) {
                    const int64_t e = (l + ((int64_t)1 << (h + 1))) < lb1 ? l + ((int64_t)1 << (h + 1)) : lb1;
                    if ((int64_t)leaf[e] - leaf[l] <= lds_cap && e - l <= lds_cap) ++h;
                    else break;
                }
                st.h = h;
                st.l0 = l;
                st.l1 = (l + ((int64_t)1 << h)) < lb1 ? l + ((int64_t)1 << h) : lb1;
                st.root = whole && l == 0 && st.l1 == L;
                act = kActNode;
            } else if (sp == 1) {
                act = (!whole || st.stack[0].buf == 2) ? kActDone : kActToC;
            } else if (sp >= 2 && (st.stack[sp - 1].p & 1) == 0) {
                act = kActPromote;
            }
            st.action = act;
        }
        __syncthreads();
        const int act = wave_uniform(st.action);
        if (act == kActDone) break;
        if (act == kActFail) {
            if (tid == 0) {
                atomicOr(reinterpret_cast<unsigned long long *>(&ctl->err),
                         (unsigned long long)kErrHeavyCapacity);
                st.sp = 0;
            }
            break;
        }
        if (act == kActNode) {
            const int64_t l0 = wave_uniform(st.l0), l1 = wave_uniform(st.l1);
            const int root = wave_uniform(st.root);
            const int64_t r0 = leaf[l0];
            const int64_t np = (int64_t)leaf[l1] - r0;
            int32_t *oc = root ? c_col + cs : bcol[0] + r0;
            double *ov = root ? c_val + cs : bval[0] + r0;
            const int64_t cap = root ? ccap : np;
            int64_t len;
            if (np <= lds_cap && (l1 - l0) <= lds_cap) {
                len = brmerge_range_lds<T, kCap, 1, IB>(
                    node_lds, tid, a0 + l0, (int)(l1 - l0), lists, a_val, b_col, b_val, oc, ov, cap);
            } else {
                // one list longer than LDS: the scaled B row is the node
                const double a = a_val[a0 + l0];
                int64_t bs;
                int nb;
                lists.get(a0 + l0, bs, nb);
                for (int64_t j = tid; j < np && j < cap; j += T) {
                    gstore(oc + j, gload(b_col + bs + j));
                    gstore(ov + j, a * gload(b_val + bs + j));
                }
                len = np;
            }
            __syncthreads();
            if (tid == 0) {
                if (st.sp < 64) {
                    HeavyNode &nd = st.stack[st.sp++];
                    nd.p = l0 >> st.h;
                    nd.h = st.h;
                    nd.len = len;
                    nd.buf = root ? 2 : 0;
                }
                st.next_list = l1;
            }
        } else if (act == kActMerge) {
            const int sp = wave_uniform(st.sp);
            HeavyNode x = st.stack[sp - 2];
            HeavyNode y = st.stack[sp - 1];
            x.p = wave_uniform(x.p);
            x.len = wave_uniform(x.len);
            x.h = wave_uniform(x.h);
            x.buf = wave_uniform(x.buf);
            y.p = wave_uniform(y.p);
            y.len = wave_uniform(y.len);
            y.h = wave_uniform(y.h);
            y.buf = wave_uniform(y.buf);
            const int root = wave_uniform(st.root);
            const int64_t rx = leaf[x.p << x.h];
            const int64_t ry = leaf[y.p << y.h];
            const int ob = root ? 2 : (x.buf == y.buf ? 1 - x.buf : y.buf);
            int32_t *oc = root ? c_col + cs : bcol[ob] + rx;
            double *ov = root ? c_val + cs : bval[ob] + rx;
            const int64_t cap = root ? ccap : (nprod - rx);
            const int64_t len = merge_hbm<T>(mrg, st, tid, bcol[x.buf] + rx, bval[x.buf] + rx, x.len,
                                          bcol[y.buf] + ry, bval[y.buf] + ry, y.len, oc, ov, cap);
            if (tid == 0) {
                st.sp -= 2;
                HeavyNode &nd = st.stack[st.sp++];
                nd.p = x.p >> 1;
                nd.h = x.h + 1;
                nd.len = len;
                nd.buf = ob;
            }
        } else if (act == kActPromote) {
            if (tid == 0) {
                HeavyNode &nd = st.stack[st.sp - 1];
                nd.p >>= 1;
                nd.h += 1;
            }
        } else if (act == kActToC) {
            const HeavyNode x = st.stack[0];
            const int64_t n = x.len < ccap ? x.len : ccap;
            for (int64_t j = tid; j < n; j += T) {
                gstore(c_col + cs + j, gload(bcol[x.buf] + j));
                gstore(c_val + cs + j, gload(bval[x.buf] + j));
            }
            if (tid == 0) st.stack[0].buf = 2;
        }
        // global stores of this workgroup become visible to it at the barrier (workgroup scope)
        __syncthreads();
    }
    if (tid == 0) {
        if (whole) {
            if (st.sp == 1) finish_row(no, ctl, id, st.stack[0].len, ccap, true);
        } else {
            // a failed walk leaves an empty list in buffer 0 (the error bit is set)
            const bool ok = st.sp == 1;
            res[2 * res_slot] = ok ? st.stack[0].buf : 0;
            res[2 * res_slot + 1] = ok ? st.stack[0].len : 0;
        }
    }
    // the workgroup's LDS state is free again only after thread 0 has read it
    __syncthreads();
}

// One work item per workgroup: a whole row (its root written to C), or the
// aligned subtree [l0, l1) of a long row's lists, whose merged list is left in
// the row's spill buffers (at the offset of its first list's products) and
// described in its result slot for the merges above it.
template <typename IA, typename IB, int T>
__global__ __launch_bounds__(T, 4) void k_num_heavy(
    HeavyBatch hb, const void *a_rpt, Lists<IB> lists, const double *a_val,
    const int32_t *b_col, const double *b_val, const int64_t *c_rpt, int32_t *c_col, double *c_val,
    Ctl *ctl, NumOut no) {
    constexpr int kCap = 4 * T;  // products (and lists) of an LDS node
    constexpr size_t kUnion = sizeof(NumLds<T, kCap>) > sizeof(MergeLds<T>) ? sizeof(NumLds<T, kCap>)
                                                                            : sizeof(MergeLds<T>);
    __shared__ __align__(16) unsigned char raw[kUnion];
    __shared__ HeavyState<T> st;
    auto &node_lds = *reinterpret_cast<NumLds<T, kCap> *>(raw);
    auto &mrg = *reinterpret_cast<MergeLds<T> *>(raw);
    const int tid = threadIdx.x;
    __shared__ int64_t s_bi;
    while (true) {
        // items arrive largest first; a ticket hands the next one to a free workgroup
        if (tid == 0) s_bi = (int64_t)atomicAdd(hb.ticket, 1ull);
        __syncthreads();
        const int64_t ii = wave_uniform(s_bi);
        __syncthreads();
        if (ii >= hb.nitems) break;
        const HeavyItem &it = hb.items[ii];
        const int64_t bi = wave_uniform((int64_t)it.bi);
        const int res_slot = wave_uniform(it.res);
        const int64_t lb0 = wave_uniform(it.l0), lb1 = wave_uniform(it.l1);
        const int64_t nprod = wave_uniform(it.nprod);
        heavy_walk<IA, IB, T>(node_lds, mrg, st, tid, hb.rows[bi], lb0, lb1, res_slot, nprod,
                              hb.leaf + hb.leaf_off[bi], hb.spill_col + hb.spill_off[bi],
                              hb.spill_val + hb.spill_off[bi], hb.lds_cap, hb.res, a_rpt, lists, a_val, b_col,
                              b_val, c_rpt, c_col, c_val, ctl, no, hb.rows[bi]);
    }
}

// The merges above the subtrees of split rows, one level per launch: the
// two nodes (siblings of the merge tree, every level below already merged)
// are merged into the other spill buffer or into the right node's region
// (merge_hbm's overlap rule), or into C at the row's root; a root whose
// right sibling does not exist is copied into C.  One workgroup per merge.
template <int T>
__global__ __launch_bounds__(T) void k_heavy_top(HeavyBatch hb, const HeavyTop *tops, int64_t ntops,
                                                 const int64_t *c_rpt, int32_t *c_col, double *c_val, Ctl *ctl,
                                                 NumOut no) {
    __shared__ MergeLds<T> mrg;
    __shared__ HeavyState<T> st;
    __shared__ int64_t s_i;
    const int tid = threadIdx.x;
    while (true) {
        if (tid == 0) s_i = (int64_t)atomicAdd(hb.ticket, 1ull);
        __syncthreads();
        const int64_t ti = wave_uniform(s_i);
        __syncthreads();
        if (ti >= ntops) break;
        const HeavyTop &t = tops[ti];
        const int64_t bi = wave_uniform((int64_t)t.bi);
        const int rxs = wave_uniform(t.res_x), rys = wave_uniform(t.res_y);
        const bool root = wave_uniform(t.root) != 0;
        const int64_t nprod = wave_uniform(t.nprod);
        const int64_t row = hb.rows[bi];
        const int32_t *leaf = hb.leaf + hb.leaf_off[bi];
        int32_t *bcol[2] = {hb.spill_col + hb.spill_off[bi], hb.spill_col + hb.spill_off[bi] + nprod};
        double *bval[2] = {hb.spill_val + hb.spill_off[bi], hb.spill_val + hb.spill_off[bi] + nprod};
        const int64_t cs = c_rpt[row];
        const int64_t ccap = c_rpt[row + 1] - cs;
        const int64_t rx = wave_uniform((int64_t)leaf[wave_uniform(t.lx)]);
        const int xb = (int)wave_uniform(hb.res[2 * rxs]);
        const int64_t xl = wave_uniform(hb.res[2 * rxs + 1]);
        int yb = 0;
        int64_t yl = 0, ry = nprod;
        if (rys >= 0) {
            ry = wave_uniform((int64_t)leaf[wave_uniform(t.ly)]);
            yb = (int)wave_uniform(hb.res[2 * rys]);
            yl = wave_uniform(hb.res[2 * rys + 1]);
        }
        // every node lies inside its products: a result out of these bounds
        // (a failed walk below) is reported, not read
        const bool ok = (xb == 0 || xb == 1) && (yb == 0 || yb == 1) && rx >= 0 && xl >= 0 && rx + xl <= ry &&
                        yl >= 0 && ry + yl <= nprod;
        if (!ok) {
            if (tid == 0)
                atomicOr(reinterpret_cast<unsigned long long *>(&ctl->err), (unsigned long long)kErrHeavyCapacity);
            __syncthreads();
            continue;
        }
        if (rys < 0) {
            // the root is the left node alone
            const int64_t n = xl < ccap ? xl : ccap;
            for (int64_t j = tid; j < n; j += T) {
                gstore(c_col + cs + j, gload(bcol[xb] + rx + j));
                gstore(c_val + cs + j, gload(bval[xb] + rx + j));
            }
            if (tid == 0) finish_row(no, ctl, row, xl, ccap, true);
        } else {
            const int ob = root ? 2 : (xb == yb ? 1 - xb : yb);
            int32_t *oc = root ? c_col + cs : bcol[ob] + rx;
            double *ov = root ? c_val + cs : bval[ob] + rx;
            const int64_t cap = root ? ccap : (nprod - rx);
            const int64_t len = merge_hbm<T>(mrg, st, tid, bcol[xb] + rx, bval[xb] + rx, xl, bcol[yb] + ry,
                                          bval[yb] + ry, yl, oc, ov, cap);
            if (tid == 0) {
                if (root) {
                    finish_row(no, ctl, row, len, ccap, true);
                } else {
                    hb.res[2 * rxs] = ob;
                    hb.res[2 * rxs + 1] = len;
                }
            }
        }
        __syncthreads();
    }
}

static HeavyBatch heavy_batch(const HeavyArgs &h) {
    HeavyBatch hb;
    hb.ticket = h.ticket;
    hb.rows = h.rows;
    hb.spill_off = h.spill_off;
    hb.leaf_off = h.leaf_off;
    hb.items = h.items;
    hb.nitems = h.nitems;
    hb.res = h.res;
    hb.spill_col = h.spill_col;
    hb.spill_val = h.spill_val;
    hb.leaf = h.leaf;
    hb.lds_cap = h.lds_cap;
    return hb;
}

hipError_t launch_numeric_heavy(const CsrView &A, const CsrView &B, const Workspace &ws, const HeavyArgs &h,
                                int grid, const int64_t *c_rpt, int32_t *c_col, double *c_val, Ctl *ctl,
                                const NumOut &no, hipStream_t s) {
    const HeavyBatch hb = heavy_batch(h);
#define BRM_HEAVY(IA, IB)                                                                              \
    do {                                                                                               \
        if (h.threads == 1024)                                                                         \
            hipLaunchKernelGGL((k_num_heavy<IA, IB, 1024>), dim3(grid), dim3(1024), 0, s, hb, A.rpt,  \
                               ws_lists<IB>(A, B, ws), A.val, B.col, B.val, c_rpt, c_col, c_val, ctl, no); \
        else                                                                                           \
            hipLaunchKernelGGL((k_num_heavy<IA, IB, 512>), dim3(grid), dim3(512), 0, s, hb, A.rpt,    \
                               ws_lists<IB>(A, B, ws), A.val, B.col, B.val, c_rpt, c_col, c_val, ctl, no); \
    } while (0)
    if (A.rpt_bytes == 4 && B.rpt_bytes == 4) BRM_HEAVY(int32_t, int32_t);
    else if (A.rpt_bytes == 4) BRM_HEAVY(int32_t, int64_t);
    else if (B.rpt_bytes == 4) BRM_HEAVY(int64_t, int32_t);
    else BRM_HEAVY(int64_t, int64_t);
#undef BRM_HEAVY
    return hipGetLastError();
}

hipError_t launch_heavy_top(const HeavyArgs &h, const HeavyTop *tops, int64_t ntops, int grid, const int64_t *c_rpt,
                            int32_t *c_col, double *c_val, Ctl *ctl, const NumOut &no, hipStream_t s) {
    if (ntops == 0) return hipSuccess;
    const HeavyBatch hb = heavy_batch(h);
    hipLaunchKernelGGL((k_heavy_top<1024>), dim3(grid), dim3(1024), 0, s, hb, tops, ntops, c_rpt, c_col, c_val,
                       ctl, no);
    return hipGetLastError();
}

// compact (row, nprod, lists) of the heavy rows, in class order
template <typename IA>
__global__ void k_heavy_info(int64_t n, const int32_t *rows, const void *a_rpt,
                             const int64_t *row_nprod, int64_t *info) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = rows[i];
        info[3 * i] = r;
        info[3 * i + 1] = row_nprod[r];
        info[3 * i + 2] = ld_rpt<IA>(a_rpt, r + 1) - ld_rpt<IA>(a_rpt, r);
    }
}

hipError_t launch_heavy_info(const CsrView &A, const Workspace &ws, const int32_t *rows, int64_t n,
                             int64_t *info, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned g = (unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    if (A.rpt_bytes == 4)
        hipLaunchKernelGGL(k_heavy_info<int32_t>, dim3(g), dim3(256), 0, s, n, rows, A.rpt, ws.row_nprod,
                           info);
    else
        hipLaunchKernelGGL(k_heavy_info<int64_t>, dim3(g), dim3(256), 0, s, n, rows, A.rpt, ws.row_nprod,
                           info);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched products: many independent C_p = A_p * B_p share each launch.  The
// rows of all problems of a stage form one row space; a row finds its
// problem by a binary search over the problems' first rows (kept in LDS).
// Outputs live in a caller-provided arena at offsets computed on the device,
// so the whole sequence of both stages of a Galerkin product can be captured
// in one graph without any host round trip.
// ---------------------------------------------------------------------------
constexpr int kMaxLdsProbs = 2048;

struct ProbLookup {
    int64_t off[kMaxLdsProbs + 1];
};

__device__ __forceinline__ void load_lookup(ProbLookup &lk, const int64_t *row_off, int np) {
    const int n = np + 1 < kMaxLdsProbs + 1 ? np + 1 : kMaxLdsProbs + 1;
    for (int i = threadIdx.x; i < n; i += blockDim.x) lk.off[i] = row_off[i];
    __syncthreads();
}

__device__ __forceinline__ int find_prob(const ProbLookup &lk, const int64_t *row_off, int np, int64_t g) {
    // last problem whose first row is <= g (problems are ordered by first row)
    const int64_t *o = np < kMaxLdsProbs ? lk.off : row_off;
    return upper_bound(o, np, g) - 1;
}

// Row analysis of a batched stage, as in the single product: a wavefront
// takes 64 consecutive rows of one problem (chunk c of the stage; the
// problems' chunk ranges are consecutive) and walks their entries, one
// contiguous range of that problem's A, coalesced.  Besides the per-row
// products, class and list descriptors it records every row's problem.
template <typename IA, typename IB>
__global__ __launch_bounds__(256) void k_b_analysis(const BatchProb *tab, const int64_t *chunk_off, int np,
                                                    int64_t nchunks, Thresholds th, int64_t *row_nprod,
                                                    uint8_t *row_class, int32_t *row_size, Ctl *ctl,
                                                    BatchStatus *st, int32_t *row_prob, IB *ent_bs,
                                                    int32_t *ent_len, int upper) {
    constexpr int kW = 256 / kWave;
    __shared__ ProbLookup lk;
    __shared__ int64_t s_count[kNumClasses];
    __shared__ int64_t s_nprod;
    __shared__ int64_t s_start[kW][kWave + 1];
    __shared__ int32_t s_flag[kW][kWave];  // row heads of a window
    __shared__ int s_long;                  // a row of 2^31 or more products
    load_lookup(lk, chunk_off, np);
    if (threadIdx.x < kNumClasses) s_count[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        s_nprod = 0;
        s_long = 0;
    }
    __syncthreads();
    // rows per class, counted per chunk by ballots (wavefront totals: scalar registers)
    int64_t my_count[kNumClasses];
#pragma unroll
    for (int c = 0; c < kNumClasses; ++c) my_count[c] = 0;
    int64_t my_nprod = 0;
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    const bool skip = st->skip != 0;  // one value for the whole stage (set before this launch)
    // A chunk's problem (its fields in registers: the stores below could
    // otherwise alias the table and force reloads), first row, row count and
    // the lanes' row pointers.  The next chunk's are loaded while this one is
    // walked, which takes the head of the chunk's chain of dependent loads
    // off its critical path.
    struct Meta {
        int p, nrows;
        int64_t rows, row_off, ent_off, r0, a0, a1;
        const void *a_rpt, *b_rpt;
        const int64_t *b_end;
        const int32_t *a_col;
    };
    static_assert(kBatchChunkRows == kWave, "a chunk is one wavefront's rows");
    auto meta = [&](int64_t c, Meta &m) {
        m.p = find_prob(lk, chunk_off, np, c);
        const BatchProb &tp = tab[m.p];
        m.rows = wave_uniform(tp.rows);
        m.row_off = wave_uniform(tp.row_off);
        m.ent_off = wave_uniform(tp.ent_off);
        m.a_rpt = tp.a_rpt;
        m.b_rpt = tp.b_rpt;
        m.b_end = tp.b_end;
        m.a_col = tp.a_col;
        m.r0 = (c - (np < kMaxLdsProbs ? lk.off[m.p] : gload(chunk_off + m.p))) * kWave;
        m.nrows = m.rows - m.r0 < kWave ? (int)(m.rows - m.r0) : kWave;
        m.a0 = 0;
        m.a1 = 0;
        if (!skip && lane < m.nrows) {
            m.a0 = ld_rpt<IA>(m.a_rpt, m.r0 + lane);
            m.a1 = ld_rpt<IA>(m.a_rpt, m.r0 + lane + 1);
        }
    };
    const int64_t cstride = (int64_t)gridDim.x * kW;
    int64_t c = (int64_t)blockIdx.x * kW + w;
    Meta cur, nxt;
    if (c < nchunks) meta(c, cur);
    for (; c < nchunks; c += cstride) {
        if (c + cstride < nchunks) meta(c + cstride, nxt);
        const int p = cur.p;
        struct {
            int64_t rows, row_off, ent_off;
            const void *a_rpt, *b_rpt;
            const int64_t *b_end;
            const int32_t *a_col;
        } pr = {cur.rows, cur.row_off, cur.ent_off, cur.a_rpt, cur.b_rpt, cur.b_end, cur.a_col};
        const int64_t r0 = cur.r0;
        const int nrows = cur.nrows;
        const int64_t i = r0 + lane;
        const bool in = lane < nrows;
        if (skip) {
            // an earlier stage failed: this stage's B may be an unwritten C
            if (in) {
                const int64_t g = pr.row_off + i;
                row_nprod[g] = 0;
                row_class[g] = (uint8_t)kClassEmpty;
                row_prob[g] = p;
                row_size[g] = 0;
            }
            my_count[kClassEmpty] += __popcll(wave_ballot(in));
            cur = nxt;
            continue;
        }
        const int64_t a0 = cur.a0, a1 = cur.a1;
        if (in) s_start[w][lane] = a0;
        if (lane == nrows - 1) s_start[w][nrows] = a1;
        wave_sync();
        const int64_t e0 = s_start[w][0], e1 = s_start[w][nrows];
        int64_t np_r = 0;
        int mx_r = 0;
        analysis_windows<IB>(e0, e1, pr.a_col, reinterpret_cast<const IB *>(pr.b_rpt), pr.b_end, ent_bs + pr.ent_off,
                             ent_len + pr.ent_off, in, a0, a1, s_flag[w], lane, np_r, mx_r);
        int cls_l = -1;  // the lane's row's class
        if (in) {
            const int64_t g = pr.row_off + i;
            const int64_t nprod = np_r;
            const int mx = mx_r;
            // rows of 2^31 or more products go to no kernel and fail the batch
            const bool too_long = nprod > (int64_t)INT32_MAX;
            if (too_long) s_long = 1;
            const int cls = too_long ? (int)kClassEmpty : classify(a1 - a0, nprod, mx, th);
            const int sw = (cls == kClassWaveSmall && th.windows) ? window_shift(a1 - a0, mx)
                           : cls == kClassMulti                   ? multi_shift(a1 - a0, mx, nprod)
                                                                  : 0;
            row_nprod[g] = nprod;
            row_class[g] = (uint8_t)(cls | (sw << kClassBits));
            row_prob[g] = p;
            cls_l = cls;
            // upper-bound slots: every row's slot holds its products
            if (cls == kClassEmpty) row_size[g] = 0;
            else if (cls == kClassCopy || upper) row_size[g] = (int32_t)nprod;
            my_nprod += nprod;
        }
#pragma unroll
        for (int q = 0; q < kNumClasses; ++q) my_count[q] += __popcll(wave_ballot(cls_l == q));
        wave_sync();
        cur = nxt;
    }
#pragma unroll
    for (int c = 0; c < kNumClasses; ++c) {
        const int64_t t = my_count[c];
        if (lane == 0 && t) atomicAdd(reinterpret_cast<unsigned long long *>(&s_count[c]), (unsigned long long)t);
    }
    {
        const int64_t t = wave_sum(my_nprod);
        if (lane == 0 && t) atomicAdd(reinterpret_cast<unsigned long long *>(&s_nprod), (unsigned long long)t);
    }
    __syncthreads();
    if (threadIdx.x < kNumClasses && s_count[threadIdx.x])
        atomicAdd(reinterpret_cast<unsigned long long *>(&ctl->count[threadIdx.x]),
                  (unsigned long long)s_count[threadIdx.x]);
    if (threadIdx.x == 0 && s_nprod) {
        atomicAdd(reinterpret_cast<unsigned long long *>(&ctl->nprod), (unsigned long long)s_nprod);
        atomicAdd(reinterpret_cast<unsigned long long *>(&st->nprod), (unsigned long long)s_nprod);
    }
    if (threadIdx.x == kNumClasses && s_long) atomicOr(&st->flags, (int)kBatchRowProducts);
}

template <int T, int TEAMS, int TS, typename IA, typename IB>
__global__ __launch_bounds__(T *TEAMS) void k_b_sym_hash(int cls, const BatchProb *tab, const int64_t *row_off,
                                                         int np, const int32_t *class_rows, int32_t *row_size,
                                                         const Ctl *ctl) {
    if (ctl->count[cls] == 0) return;  // an empty class: nothing to load or do
    __shared__ ProbLookup lk;
    __shared__ SymLds<T, TS> lds[TEAMS];
    load_lookup(lk, row_off, np);
    const int team = threadIdx.x / T, tid = threadIdx.x % T;
    const int64_t count = ctl->count[cls];
    const int64_t start = class_start(ctl, cls);
    for (int64_t idx = (int64_t)blockIdx.x * TEAMS + team; idx < count; idx += (int64_t)gridDim.x * TEAMS) {
        const int64_t g = class_rows[start + idx];
        const BatchProb &pr = tab[find_prob(lk, row_off, np, g)];
        const int total = sym_hash_row<T, TS, IA, IB>(lds[team], tid, g - pr.row_off, pr.a_rpt,
                                                      direct_lists<IB>(pr.a_col, pr.b_rpt, pr.b_end), pr.b_col);
        if (tid == 0) row_size[g] = total;
    }
}

// per-problem nnz, arena offsets of every C (columns then values, 256-byte
// aligned, after the row-pointer region) and the capacity check
__global__ __launch_bounds__(1024) void k_b_distribute(BatchProb *tab, int np, const int64_t *S, char *arena,
                                                       int64_t arena_bytes, int64_t data_off, BatchStatus *st) {
    __shared__ int64_t scr[Team<1024>::kWaves + 1];
    __shared__ int64_t s_base;
    if (threadIdx.x == 0) s_base = st->arena_used > data_off ? st->arena_used : data_off;
    __syncthreads();
    int64_t carry = s_base;
    for (int b = 0; b < np; b += 1024) {
        const int p = b + threadIdx.x;
        int64_t nnz = 0, bytes = 0;
        if (p < np) {
            nnz = S[tab[p].row_off + tab[p].rows] - S[tab[p].row_off];
            bytes = ((4 * nnz + 255) / 256) * 256 + ((8 * nnz + 255) / 256) * 256;
        }
        int64_t tot;
        const int64_t ex = Team<1024>::excl_scan(bytes, &tot, scr, threadIdx.x);
        if (p < np) {
            const int64_t o = carry + ex;
            tab[p].nnz = nnz;
            tab[p].col_off = o;
            tab[p].val_off = o + ((4 * nnz + 255) / 256) * 256;
            tab[p].c_col = reinterpret_cast<int32_t *>(arena + o);
            tab[p].c_val = reinterpret_cast<double *>(arena + tab[p].val_off);
            tab[p].c_rpt = reinterpret_cast<int64_t *>(arena + tab[p].rpt_off);  // (slots before, under upper bounds)
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        st->arena_used = carry;
        st->spill_base = carry;
        if (carry > arena_bytes) st->flags |= kBatchOverflow;
        if (carry > st->required) st->required = carry;
    }
}

// C's row pointers of every problem from the stage-wide prefix sum
__global__ __launch_bounds__(256) void k_b_rpt(BatchProb *tab, const int64_t *row_off, int np, int64_t R,
                                               const int64_t *S, const BatchStatus *st) {
    __shared__ ProbLookup lk;
    load_lookup(lk, row_off, np);
    if (st->flags & (kBatchOverflow | kBatchRowProducts)) return;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < R; g += (int64_t)gridDim.x * blockDim.x) {
        const int p = find_prob(lk, row_off, np, g);
        const BatchProb &pr = tab[p];
        const int64_t r = g - pr.row_off;
        gstore(pr.c_rpt + (r), S[g] - S[pr.row_off]);
        if (r == pr.rows - 1) gstore(pr.c_rpt + (pr.rows), S[g + 1] - S[pr.row_off]);
    }
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x)
        if (tab[p].rows == 0) gstore(tab[p].c_rpt + (0), (int64_t)0);
}

// the B operand of a chained problem is the C of an earlier one
__global__ void k_b_link(BatchProb *all, int first, int np) {
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        BatchProb &q = all[first + i];
        if (q.b_from >= 0) {
            const BatchProb &src = all[q.b_from];
            q.b_rpt = src.c_rpt;
            q.b_end = src.c_end;
            q.b_col = src.c_col;
            q.b_val = src.c_val;
        }
    }
}

// SLOT (every batched numeric kernel): C's rows are upper-bound slots whose
// exact lengths are recorded (a compile-time choice: the bookkeeping of the
// other mode costs the kernel nothing)
template <typename IA, typename IB, bool SLOT>
__global__ __launch_bounds__(256) void k_b_num_copy(int cls, const BatchProb *tab, const int64_t *row_off, int np,
                                                    const int32_t *class_rows, Ctl *ctl, const BatchStatus *st,
                                                    NumOut no_in) {
    if (ctl->count[cls] == 0) return;  // an empty class: nothing to load or do
    NumOut no = no_in;
    no.bound = SLOT ? 1 : 0;
    __shared__ ProbLookup lk;
    load_lookup(lk, row_off, np);
    if (st->flags & (kBatchOverflow | kBatchRowProducts)) return;
    const int lane = lane_id();
    const int64_t count = ctl->count[cls];
    const int64_t start = class_start(ctl, cls);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t idx = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; idx < count;
         idx += waves) {
        const int64_t g = class_rows[start + idx];
        const BatchProb &pr = tab[find_prob(lk, row_off, np, g)];
        copy_row<IA, IB>(lane, g - pr.row_off, g, pr.a_rpt, direct_lists<IB>(pr.a_col, pr.b_rpt, pr.b_end), pr.a_val,
                         pr.b_col, pr.b_val, pr.c_rpt, pr.c_col, pr.c_val, ctl, no);
    }
}

template <int T, int TEAMS, int CAP, typename IA, typename IB, bool SLOT>
__global__ __launch_bounds__(T *TEAMS) void k_b_num_lds(int cls, const BatchProb *tab, const int64_t *row_off,
                                                        int np, const int32_t *class_rows, Ctl *ctl,
                                                        const BatchStatus *st, NumOut no_in) {
    if (ctl->count[cls] == 0) return;  // an empty class: nothing to load or do
    NumOut no = no_in;
    no.bound = SLOT ? 1 : 0;
    __shared__ ProbLookup lk;
    __shared__ NumLds<T, CAP> lds[TEAMS];
    load_lookup(lk, row_off, np);
    if (st->flags & (kBatchOverflow | kBatchRowProducts)) return;
    const int team = threadIdx.x / T, tid = threadIdx.x % T;
    const int64_t count = ctl->count[cls];
    const int64_t start = class_start(ctl, cls);
    for (int64_t idx = (int64_t)blockIdx.x * TEAMS + team; idx < count; idx += (int64_t)gridDim.x * TEAMS) {
        const int64_t g = class_rows[start + idx];
        const BatchProb &pr = tab[find_prob(lk, row_off, np, g)];
        brmerge_row_lds<T, CAP, IA, IB>(lds[team], tid, g - pr.row_off, pr.a_rpt,
                                        direct_lists<IB>(pr.a_col, pr.b_rpt, pr.b_end), pr.a_val, pr.b_col, pr.b_val,
                                        pr.c_rpt, pr.c_col, pr.c_val, ctl, no, g);
    }
}

// the window kernels over a batched stage's rows (lists from the analysis's
// descriptors, every row's arrays from its problem)
template <typename IA, typename IB, bool SLOT>
__global__ __launch_bounds__(256) void k_b_num_win(int cls, const BatchProb *tab, const int32_t *row_prob,
                                                   const IB *ent_bs, const int32_t *ent_len, const uint8_t *row_class,
                                                   const int32_t *class_rows, Ctl *ctl, const BatchStatus *st,
                                                   NumOut no_in) {
    if (ctl->count[cls] == 0) return;  // an empty class: nothing to load or do
    NumOut no = no_in;
    no.bound = SLOT ? 1 : 0;
    __shared__ uint32_t xk[4][kWave];
    __shared__ double xv[4][kWave];
    if (st->flags & (kBatchOverflow | kBatchRowProducts)) return;
    const int team = wave_uniform((int)(threadIdx.x / kWave));
    Lists<IB> lists = direct_lists<IB>(nullptr, nullptr);
    lists.ent_bs = ent_bs;
    lists.ent_len = ent_len;
    BatchRows br;
    br.tab = tab;
    br.row_prob = row_prob;
    win_chunks<true, false, IA, IB, true>(cls, nullptr, lists, nullptr, nullptr, nullptr, row_class, class_rows,
                                          nullptr, nullptr, nullptr, nullptr, ctl, no, nullptr, xk[team], xv[team],
                                          (int64_t)blockIdx.x * 4 + team, (int64_t)gridDim.x * 4, br);
}

template <typename IA, typename IB>
__global__ __launch_bounds__(256) void k_b_sym_win(int cls, const BatchProb *tab, const int32_t *row_prob,
                                                   const IB *ent_bs, const int32_t *ent_len, const uint8_t *row_class,
                                                   const int32_t *class_rows, int32_t *row_size, Ctl *ctl) {
    if (ctl->count[cls] == 0) return;  // an empty class: nothing to load or do
    const int team = wave_uniform((int)(threadIdx.x / kWave));
    Lists<IB> lists = direct_lists<IB>(nullptr, nullptr);
    lists.ent_bs = ent_bs;
    lists.ent_len = ent_len;
    NumOut no;
    no.bound = 0;
    BatchRows br;
    br.tab = tab;
    br.row_prob = row_prob;
    win_chunks<false, false, IA, IB, true>(cls, nullptr, lists, nullptr, nullptr, nullptr, row_class, class_rows,
                                           nullptr, nullptr, nullptr, row_size, ctl, no, nullptr, nullptr, nullptr,
                                           (int64_t)blockIdx.x * 4 + team, (int64_t)gridDim.x * 4, br);
}

template <typename IA, typename IB, bool SLOT>
__global__ __launch_bounds__(256) void k_b_num_mw(int cls, const BatchProb *tab, const int32_t *row_prob,
                                                  const IB *ent_bs, const int32_t *ent_len, const uint8_t *row_class,
                                                  const int32_t *class_rows, Ctl *ctl, const BatchStatus *st,
                                                  NumOut no_in) {
    if (ctl->count[cls] == 0) return;  // an empty class: nothing to load or do
    NumOut no = no_in;
    no.bound = SLOT ? 1 : 0;
    __shared__ double vals[4][kMwSlots];
    if (st->flags & (kBatchOverflow | kBatchRowProducts)) return;
    const int team = wave_uniform((int)(threadIdx.x / kWave));
    Lists<IB> lists = direct_lists<IB>(nullptr, nullptr);
    lists.ent_bs = ent_bs;
    lists.ent_len = ent_len;
    BatchRows br;
    br.tab = tab;
    br.row_prob = row_prob;
    mw_rows<true, IA, IB, true>(cls, nullptr, lists, nullptr, nullptr, nullptr, row_class, class_rows, nullptr,
                                nullptr, nullptr, nullptr, ctl, no, vals[team], (int64_t)blockIdx.x * 4 + team,
                                (int64_t)gridDim.x * 4, br);
}

template <typename IA, typename IB>
__global__ __launch_bounds__(256) void k_b_sym_mw(int cls, const BatchProb *tab, const int32_t *row_prob,
                                                  const IB *ent_bs, const int32_t *ent_len, const uint8_t *row_class,
                                                  const int32_t *class_rows, int32_t *row_size, Ctl *ctl) {
    if (ctl->count[cls] == 0) return;  // an empty class: nothing to load or do
    const int team = wave_uniform((int)(threadIdx.x / kWave));
    Lists<IB> lists = direct_lists<IB>(nullptr, nullptr);
    lists.ent_bs = ent_bs;
    lists.ent_len = ent_len;
    NumOut no;
    no.bound = 0;
    BatchRows br;
    br.tab = tab;
    br.row_prob = row_prob;
    mw_rows<false, IA, IB, true>(cls, nullptr, lists, nullptr, nullptr, nullptr, row_class, class_rows, nullptr,
                                 nullptr, nullptr, row_size, ctl, no, nullptr, (int64_t)blockIdx.x * 4 + team,
                                 (int64_t)gridDim.x * 4, br);
}

// Heavy rows of a batched stage (more products than a 1024-thread LDS
// row): the bitmap count for the symbolic pass, one 1024-thread workgroup
// per row
template <typename IA, typename IB>
__global__ __launch_bounds__(kHeavyThreads) void k_b_sym_bitmap(const BatchProb *tab, const int32_t *row_prob,
                                                                const int32_t *class_rows, int32_t *row_size,
                                                                const Ctl *ctl) {
    if (ctl->count[kClassHeavy] == 0) return;  // no heavy row in this stage
    __shared__ BitmapLds s;
    const int tid = threadIdx.x;
    const int64_t count = ctl->count[kClassHeavy];
    const int64_t start = class_start(ctl, kClassHeavy);
    for (int64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int64_t g = class_rows[start + idx];
        const BatchProb &tp = tab[row_prob[g]];
        const int64_t total = sym_bitmap_row<IA, IB>(s, tid, g - tp.row_off, tp.ncols_b, tp.a_rpt,
                                                     direct_lists<IB>(tp.a_col, tp.b_rpt, tp.b_end), tp.b_col);
        if (tid == 0) row_size[g] = (int32_t)total;
        __syncthreads();
    }
}

// The heavy rows' spill space in the arena, after the stage's C (the next
// stage's C may reuse it): a table of (spill offset, list-offset offset)
// per heavy row in class order, then every row's two spill buffers (2 *
// nprod columns, then 2 * nprod values) and its list offsets (lists + 1).
// A space that does not fit sets the overflow flag; the need counts towards
// the required arena size either way.
template <typename IA>
__global__ __launch_bounds__(1024) void k_b_heavy_plan(const BatchProb *tab, const int32_t *row_prob,
                                                       const int64_t *row_nprod, const int32_t *class_rows,
                                                       const Ctl *ctl, BatchStatus *st, char *arena,
                                                       int64_t arena_bytes) {
    const int64_t n = ctl->count[kClassHeavy];
    if (n == 0) return;
    __shared__ int64_t scr[Team<1024>::kWaves + 1];
    const int tid = threadIdx.x;
    const int64_t start = class_start(ctl, kClassHeavy);
    auto sizes = [&](int64_t i, int64_t &e, int64_t &f) {
        const int64_t g = class_rows[start + i];
        const BatchProb &tp = tab[row_prob[g]];
        const int64_t r = g - tp.row_off;
        e = 2 * row_nprod[g];
        f = ld_rpt<IA>(tp.a_rpt, r + 1) - ld_rpt<IA>(tp.a_rpt, r) + 1;
    };
    int64_t e_sum = 0, f_sum = 0;
    for (int64_t i = tid; i < n; i += 1024) {
        int64_t e, f;
        sizes(i, e, f);
        e_sum += e;
        f_sum += f;
    }
    const int64_t E = Team<1024>::sum(e_sum, scr, tid);
    const int64_t F = Team<1024>::sum(f_sum, scr, tid);
    auto al = [](int64_t x) { return (x + 255) / 256 * 256; };
    const int64_t o_tab = al(st->spill_base);
    const int64_t o_col = o_tab + al(16 * n);
    const int64_t o_val = o_col + al(4 * E);
    const int64_t o_leaf = o_val + al(8 * E);
    const int64_t end = o_leaf + al(4 * F);
    __syncthreads();  // every thread has read spill_base
    if (tid == 0) {
        if (end > st->required) st->required = end;
        if (end > arena_bytes) {
            atomicOr(&st->flags, (int)kBatchOverflow);
        } else {
            st->h_tab = reinterpret_cast<int64_t *>(arena + o_tab);
            st->h_col = reinterpret_cast<int32_t *>(arena + o_col);
            st->h_val = reinterpret_cast<double *>(arena + o_val);
            st->h_leaf = reinterpret_cast<int32_t *>(arena + o_leaf);
        }
    }
    if (end > arena_bytes) return;
    int64_t *htab = reinterpret_cast<int64_t *>(arena + o_tab);
    int64_t ce = 0, cf = 0;
    for (int64_t b = 0; b < n; b += 1024) {
        const int64_t i = b + tid;
        int64_t e = 0, f = 0;
        if (i < n) sizes(i, e, f);
        int64_t te, tf;
        const int64_t xe = Team<1024>::excl_scan(e, &te, scr, tid);
        const int64_t xf = Team<1024>::excl_scan(f, &tf, scr, tid);
        if (i < n) {
            gstore(htab + 2 * i, ce + xe);
            gstore(htab + 2 * i + 1, cf + xf);
        }
        ce += te;
        cf += tf;
    }
}

// the numeric pass of the heavy rows: one 512-thread workgroup merges a
// whole row (LDS nodes, spilled nodes merged through HBM), as in the single
// product
template <typename IA, typename IB, bool SLOT>
__global__ __launch_bounds__(kBatchHeavyThreads, 4) void k_b_num_heavy(const BatchProb *tab, const int32_t *row_prob,
                                                                       const int64_t *row_nprod,
                                                                       const int32_t *class_rows, Ctl *ctl,
                                                                       const BatchStatus *st, int lds_cap,
                                                                       NumOut no_in) {
    constexpr int T = kBatchHeavyThreads;
    constexpr int kCap = 4 * T;
    if (ctl->count[kClassHeavy] == 0) return;  // no heavy row in this stage
    NumOut no = no_in;
    no.bound = SLOT ? 1 : 0;
    constexpr size_t kUnion = sizeof(NumLds<T, kCap>) > sizeof(MergeLds<T>) ? sizeof(NumLds<T, kCap>)
                                                                            : sizeof(MergeLds<T>);
    __shared__ __align__(16) unsigned char raw[kUnion];
    __shared__ HeavyState<T> hs;
    auto &node_lds = *reinterpret_cast<NumLds<T, kCap> *>(raw);
    auto &mrg = *reinterpret_cast<MergeLds<T> *>(raw);
    if (st->flags & (kBatchOverflow | kBatchRowProducts)) return;
    const int tid = threadIdx.x;
    const int64_t count = ctl->count[kClassHeavy];
    const int64_t start = class_start(ctl, kClassHeavy);
    const int64_t *htab = st->h_tab;
    int32_t *hcol = st->h_col;
    double *hval = st->h_val;
    int32_t *hleaf = st->h_leaf;
    for (int64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int64_t g = class_rows[start + idx];
        const BatchProb &tp = tab[row_prob[g]];
        const int64_t row = g - wave_uniform(tp.row_off);
        const void *a_rpt = tp.a_rpt;
        const int64_t a0 = ld_rpt<IA>(a_rpt, row);
        const int64_t L = wave_uniform(ld_rpt<IA>(a_rpt, row + 1) - a0);
        const int64_t nprod = wave_uniform(gload(row_nprod + g));
        const int64_t so = wave_uniform(gload(htab + 2 * idx)), lo = wave_uniform(gload(htab + 2 * idx + 1));
        heavy_walk<IA, IB, T>(node_lds, mrg, hs, tid, row, 0, L, -1, nprod, hleaf + lo, hcol + so, hval + so,
                              lds_cap, nullptr, a_rpt, direct_lists<IB>(tp.a_col, tp.b_rpt, tp.b_end), tp.a_val, tp.b_col,
                              tp.b_val, tp.c_rpt, tp.c_col, tp.c_val, ctl, no, g);
    }
}

// Upper-bound slots of a batched stage (every row's slot holds its
// products; S2 is their prefix sum over the stage's rows): the region that
// the stage's C may take at most (every problem's arrays at their largest,
// from where the stage's C starts), then the slots' columns and values.
// The numeric kernels then write into the slots through the problems' C
// fields, and the compaction moves every row to C once its size is known.
__global__ __launch_bounds__(1024) void k_b_slot_plan(BatchProb *tab, int np, int64_t *S2, int64_t R,
                                                      BatchStatus *st, char *arena, int64_t arena_bytes,
                                                      int64_t data_off, int keep) {
    __shared__ int64_t scr[Team<1024>::kWaves + 1];
    auto al = [](int64_t x) { return (x + 255) / 256 * 256; };
    const int64_t used = st->arena_used;
    const int64_t base = al(used > data_off ? used : data_off);
    int64_t cb = 0;
    for (int p = threadIdx.x; p < np; p += 1024) {
        const int64_t n = S2[tab[p].row_off + tab[p].rows] - S2[tab[p].row_off];
        cb += al(4 * n) + al(8 * n);
    }
    const int64_t cbound = keep ? 0 : Team<1024>::sum(cb, scr, (int)threadIdx.x);
    const int64_t total = S2[R];
    const int64_t o_col = base + cbound;
    const int64_t o_val = o_col + al(4 * total);
    const int64_t end = o_val + al(8 * total);
    __syncthreads();  // every thread has read arena_used
    if (threadIdx.x == 0) {
        if (end > st->required) st->required = end;
        st->spill_base = end;  // heavy rows' spill space after the slots
        st->slots_end = end;
        if (end > arena_bytes) {
            atomicOr(&st->flags, (int)kBatchOverflow);
        } else {
            st->s_col = reinterpret_cast<int32_t *>(arena + o_col);
            st->s_val = reinterpret_cast<double *>(arena + o_val);
        }
    }
    if (end > arena_bytes) return;
    for (int p = threadIdx.x; p < np; p += 1024) {
        tab[p].c_rpt = S2 + tab[p].row_off;
        tab[p].c_col = reinterpret_cast<int32_t *>(arena + o_col);
        tab[p].c_val = reinterpret_cast<double *>(arena + o_val);
    }
}

// Compaction after upper-bound slots: the rows [g0, g0 + 256) of a
// workgroup pass are consecutive in C (stage-wide offsets S) and in the
// slots (S2); every thread takes every 256th entry of their C range and
// finds its row by a search over the rows' first offsets in LDS.
constexpr int kCompactUnroll = 8;
__global__ __launch_bounds__(256) void k_b_compact(const BatchProb *tab, const int32_t *row_prob, const int64_t *S2,
                                                   const int64_t *S, int64_t R, const BatchStatus *st) {
    __shared__ int64_t c_beg[257];
    __shared__ int64_t src[256], cap[256];  // slot offset and size of every row
    __shared__ int64_t dcol[256], dval[256];  // addresses of the rows' first entries in C
    if (st->flags & (kBatchOverflow | kBatchRowProducts)) return;
    const int32_t *scol = st->s_col;
    const double *sval = st->s_val;
    const int t = threadIdx.x;
    for (int64_t g0 = (int64_t)blockIdx.x * 256; g0 < R; g0 += (int64_t)gridDim.x * 256) {
        const int n = R - g0 < 256 ? (int)(R - g0) : 256;
        if (t < n) {
            const int64_t g = g0 + t;
            const BatchProb &pr = tab[row_prob[g]];
            const int64_t cb = S[g];
            const int64_t local = cb - S[pr.row_off];
            c_beg[t] = cb;
            src[t] = S2[g];
            cap[t] = S2[g + 1] - S2[g];
            dcol[t] = reinterpret_cast<int64_t>(pr.c_col + local);
            dval[t] = reinterpret_cast<int64_t>(pr.c_val + local);
        }
        if (t == 0) c_beg[n] = S[g0 + n];
        __syncthreads();
        const int64_t q0 = c_beg[0], q1 = c_beg[n];
        // kCompactUnroll entries per thread at a time, software-pipelined:
        // the next block's loads are issued before this block's stores
        int r[kCompactUnroll];
        int64_t off[kCompactUnroll];
        int32_t c[kCompactUnroll];
        double v[kCompactUnroll];
        auto load = [&](int64_t qb, int *rr, int64_t *oo, int32_t *cc, double *vv) {
#pragma unroll
            for (int u = 0; u < kCompactUnroll; ++u) {
                const int64_t q = qb + u * 256 + t;
                rr[u] = -1;
                oo[u] = 0;
                cc[u] = 0;
                vv[u] = 0.0;
                if (q < q1) {
                    const int ru = upper_bound(c_beg, n, q) - 1;
                    oo[u] = q - c_beg[ru];
                    // (a row never outgrows its slot of all its products)
                    if (oo[u] < cap[ru]) {
                        rr[u] = ru;
                        cc[u] = gload(scol + src[ru] + oo[u]);
                        vv[u] = gload(sval + src[ru] + oo[u]);
                    }
                }
            }
        };
        load(q0, r, off, c, v);
        for (int64_t qb = q0; qb < q1; qb += 256 * kCompactUnroll) {
            int nr[kCompactUnroll];
            int64_t noff[kCompactUnroll];
            int32_t nc[kCompactUnroll];
            double nv[kCompactUnroll];
            load(qb + 256 * kCompactUnroll, nr, noff, nc, nv);
#pragma unroll
            for (int u = 0; u < kCompactUnroll; ++u) {
                if (r[u] >= 0) {
                    gstore(reinterpret_cast<int32_t *>(dcol[r[u]]) + off[u], c[u]);
                    gstore(reinterpret_cast<double *>(dval[r[u]]) + off[u], v[u]);
                }
                r[u] = nr[u];
                off[u] = noff[u];
                c[u] = nc[u];
                v[u] = nv[u];
            }
        }
        __syncthreads();
    }
}

// caller-visible descriptors of the outputs (byte offsets into the arena)
// A stage whose problems are all operands only (SPG_PROBLEM_OPERAND_ONLY)
// keeps its upper-bound slots: every row of problem p is described by its
// first and end position in the stage's slot arrays, written into p's row
// pointer region of the arena (starts at c_rpt[0 .. rows), ends at
// c_end[0 .. rows), c_end = c_rpt + rows + 1), and the later problems read
// it through those two arrays (Lists::b_end).  The slots stay where they are:
// the arena fill moves past them.
__global__ __launch_bounds__(256) void k_b_keep_slots(BatchProb *tab, const int64_t *row_off, int np, int64_t R,
                                                      const int64_t *S2, const int32_t *row_size, char *arena,
                                                      BatchStatus *st) {
    __shared__ ProbLookup lk;
    load_lookup(lk, row_off, np);
    if (st->flags & (kBatchOverflow | kBatchRowProducts)) return;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < R; g += (int64_t)gridDim.x * blockDim.x) {
        const int p = find_prob(lk, row_off, np, g);
        const BatchProb &pr = tab[p];
        const int64_t r = g - pr.row_off;
        int64_t *beg = reinterpret_cast<int64_t *>(arena + pr.rpt_off);
        gstore(beg + r, S2[g]);
        gstore(beg + (pr.rows + 1) + r, S2[g] + (int64_t)row_size[g]);
    }
}

// then the kept problems' fields (the next launch: every row above has read them)

__global__ __launch_bounds__(256) void k_b_keep_fields(BatchProb *tab, int np, char *arena, BatchStatus *st) {
    if (st->flags & (kBatchOverflow | kBatchRowProducts)) return;
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        BatchProb &pr = tab[p];
        int64_t *beg = reinterpret_cast<int64_t *>(arena + pr.rpt_off);
        pr.c_rpt = beg;
        pr.c_end = beg + pr.rows + 1;
        pr.nnz = -2;
        pr.col_off = -1;
        pr.val_off = -1;
    }
    __syncthreads();
    if (threadIdx.x == 0) st->arena_used = st->slots_end;
}

__global__ void k_b_describe(const BatchProb *all, int n, spg_batched_out *out, const BatchStatus *st) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const BatchProb &p = all[i];
        spg_batched_out o;
        o.rows = p.rows;
        o.cols = p.ncols_b;
        o.nnz = (st->flags & (kBatchOverflow | kBatchRowProducts)) ? -1 : p.nnz;  // -2: kept in slots
        o.rpt_off = p.rpt_off;
        o.col_off = p.col_off;
        o.val_off = p.val_off;
        out[i] = o;
    }
}

// start of a batched stage: its control block cleared, and whether an
// earlier stage has already failed (overflow or heavy row) fixed for the
// whole stage
__global__ void k_b_stage_begin(Ctl *ctl, BatchStatus *st) {
    // the previous stage's device errors are kept in the status
    if (threadIdx.x == 0) st->err |= ctl->err;
    __syncthreads();
    int64_t *p = reinterpret_cast<int64_t *>(ctl);
    const int n = (int)(sizeof(Ctl) / sizeof(int64_t));
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
    if (threadIdx.x == 0) st->skip = st->flags != 0;
}

__global__ void k_b_zero_status(BatchStatus *st, Ctl *ctl) {
    if (threadIdx.x == 0) {
        st->flags = 0;
        st->skip = 0;
        st->required = 0;
        st->arena_used = 0;
        st->nprod = 0;
        st->err = 0;
        st->h_tab = nullptr;
        st->h_col = nullptr;
        st->h_val = nullptr;
        st->h_leaf = nullptr;
        st->spill_base = 0;
        st->s_col = nullptr;
        st->s_val = nullptr;
        st->slots_end = 0;
        ctl->err = 0;
    }
}

// the numeric launches of a batched stage (every class; empty classes return at once)
template <typename IA, typename IB, bool SLOT, typename G>
static void batched_numeric_launches(const BatchStage &bs, const Workspace &ws, const Thresholds &th,
                                     const NumOut &no, G &&grid_for, int num_cu, hipStream_t s) {
    const int np = bs.nprob;
    const int64_t *ro = bs.row_off;
    BatchProb *tab = bs.tab;
    const IB *ebs = static_cast<const IB *>(ws.ent_bs);
    hipLaunchKernelGGL((k_b_num_copy<IA, IB, SLOT>), grid_for(8, 4), dim3(256), 0, s, (int)kClassCopy, tab, ro, np,
                       ws.class_rows, ws.ctl, bs.status, no);
    if (th.windows)
        hipLaunchKernelGGL((k_b_num_win<IA, IB, SLOT>), grid_for(8, 4), dim3(256), 0, s, (int)kClassWaveSmall, tab,
                           ws.row_prob, ebs, ws.ent_len, ws.row_class, ws.class_rows, ws.ctl, bs.status, no);
    else
        hipLaunchKernelGGL((k_b_num_lds<64, 4, kCapWaveSmall, IA, IB, SLOT>), grid_for(8, 4), dim3(256), 0, s,
                           (int)kClassWaveSmall, tab, ro, np, ws.class_rows, ws.ctl, bs.status, no);
    if (th.multi)
        hipLaunchKernelGGL((k_b_num_mw<IA, IB, SLOT>), grid_for(5, 4), dim3(256), 0, s, (int)kClassMulti, tab,
                           ws.row_prob, ebs, ws.ent_len, ws.row_class, ws.class_rows, ws.ctl, bs.status, no);
    hipLaunchKernelGGL((k_b_num_lds<64, 4, kCapWave, IA, IB, SLOT>), grid_for(4, 4), dim3(256), 0, s, (int)kClassWave,
                       tab, ro, np, ws.class_rows, ws.ctl, bs.status, no);
    hipLaunchKernelGGL((k_b_num_lds<256, 1, kCapGroup, IA, IB, SLOT>), grid_for(4, 4), dim3(256), 0, s,
                       (int)kClassGroup, tab, ro, np, ws.class_rows, ws.ctl, bs.status, no);
    hipLaunchKernelGGL((k_b_num_lds<1024, 1, kCapBlock, IA, IB, SLOT>), grid_for(1, 16), dim3(1024), 0, s,
                       (int)kClassBlock, tab, ro, np, ws.class_rows, ws.ctl, bs.status, no);
    hipLaunchKernelGGL((k_b_num_heavy<IA, IB, SLOT>), dim3((unsigned)(2 * num_cu)), dim3(kBatchHeavyThreads), 0, s, tab,
                       ws.row_prob, ws.row_nprod, ws.class_rows, ws.ctl, bs.status, bs.heavy_lds_cap, no);
}

// The launches of one batched stage.  Precise sizes: analysis, binning,
// the symbolic pass of every class, scan, C's place in the arena (then the
// heavy rows' spill space), row pointers, the numeric pass into C.  Upper
// bounds: analysis (slot = products), binning, scan, slots in the arena
// (then the spill space), the numeric pass into the slots, scan of the exact
// sizes, C's place, row pointers, compaction.
template <typename IA, typename IB>
static void batched_stage_launches(const BatchStage &bs, const Workspace &ws, const Thresholds &th, int num_cu,
                                   int64_t grid_waves, hipStream_t s) {
    const int np = bs.nprob;
    const int64_t R = bs.rows;
    const int64_t *ro = bs.row_off;
    BatchProb *tab = bs.tab;
    const unsigned ga = (unsigned)(R > 0 ? ((R + 255) / 256 < 2048 ? (R + 255) / 256 : 2048) : 1);
    // the analysis: four chunks of 64 rows per workgroup pass
    const unsigned gc = (unsigned)(bs.chunks > 0 ? ((bs.chunks + 3) / 4 < 2048 ? (bs.chunks + 3) / 4 : 2048) : 1);
    auto grid_for = [&](int per_cu, int waves_per_wg) {
        int64_t g = (int64_t)num_cu * per_cu;
        if (grid_waves > 0) g = grid_waves / waves_per_wg > 0 ? grid_waves / waves_per_wg : 1;
        return dim3((unsigned)g);
    };
    const IB *ebs = static_cast<const IB *>(ws.ent_bs);
    hipLaunchKernelGGL(k_b_stage_begin, dim3(1), dim3(64), 0, s, ws.ctl, bs.status);
    if (bs.link) hipLaunchKernelGGL(k_b_link, dim3(1), dim3(256), 0, s, bs.all, bs.first, np);
    hipLaunchKernelGGL((k_b_analysis<IA, IB>), dim3(gc), dim3(256), 0, s, tab, bs.chunk_off, np, bs.chunks, th,
                       ws.row_nprod, ws.row_class, ws.row_size, ws.ctl, bs.status, ws.row_prob,
                       static_cast<IB *>(ws.ent_bs), ws.ent_len, bs.upper);
    hipLaunchKernelGGL(k_bin, dim3(ga), dim3(256), 0, s, R, nullptr, ws.row_class, ws.class_rows, ws.ctl);
    NumOut no;
    no.bound = 0;
    no.row_size = nullptr;
    no.ovf_rows = nullptr;
    no.M = R;
    if (!bs.upper) {
        if (th.windows)
            hipLaunchKernelGGL((k_b_sym_win<IA, IB>), grid_for(8, 4), dim3(256), 0, s, (int)kClassWaveSmall, tab,
                               ws.row_prob, ebs, ws.ent_len, ws.row_class, ws.class_rows, ws.row_size, ws.ctl);
        else
            hipLaunchKernelGGL((k_b_sym_hash<64, 4, 2 * kCapWaveSmall, IA, IB>), grid_for(8, 4), dim3(256), 0, s,
                               (int)kClassWaveSmall, tab, ro, np, ws.class_rows, ws.row_size, ws.ctl);
        if (th.multi)
            hipLaunchKernelGGL((k_b_sym_mw<IA, IB>), grid_for(8, 4), dim3(256), 0, s, (int)kClassMulti, tab,
                               ws.row_prob, ebs, ws.ent_len, ws.row_class, ws.class_rows, ws.row_size, ws.ctl);
        hipLaunchKernelGGL((k_b_sym_hash<64, 4, 2 * kCapWave, IA, IB>), grid_for(4, 4), dim3(256), 0, s,
                           (int)kClassWave, tab, ro, np, ws.class_rows, ws.row_size, ws.ctl);
        hipLaunchKernelGGL((k_b_sym_hash<256, 1, 2 * kCapGroup, IA, IB>), grid_for(4, 4), dim3(256), 0, s,
                           (int)kClassGroup, tab, ro, np, ws.class_rows, ws.row_size, ws.ctl);
        hipLaunchKernelGGL((k_b_sym_hash<1024, 1, 2 * kCapBlock, IA, IB>), grid_for(1, 16), dim3(1024), 0, s,
                           (int)kClassBlock, tab, ro, np, ws.class_rows, ws.row_size, ws.ctl);
        hipLaunchKernelGGL((k_b_sym_bitmap<IA, IB>), dim3((unsigned)num_cu), dim3(kHeavyThreads), 0, s, tab,
                           ws.row_prob, ws.class_rows, ws.row_size, ws.ctl);
        (void)launch_scan(R, ws.row_size, ws.tile_sum, bs.S, &ws.ctl->nnz, s);
        hipLaunchKernelGGL(k_b_distribute, dim3(1), dim3(1024), 0, s, tab, np, bs.S, bs.arena, bs.arena_bytes,
                           bs.data_off, bs.status);
        hipLaunchKernelGGL(k_b_heavy_plan<IA>, dim3(1), dim3(1024), 0, s, tab, ws.row_prob, ws.row_nprod,
                           ws.class_rows, ws.ctl, bs.status, bs.arena, bs.arena_bytes);
        hipLaunchKernelGGL(k_b_rpt, dim3(ga), dim3(256), 0, s, tab, ro, np, R, bs.S, bs.status);
    } else {
        (void)launch_scan(R, ws.row_size, ws.tile_sum, bs.S2, &ws.ctl->nnz, s);
        hipLaunchKernelGGL(k_b_slot_plan, dim3(1), dim3(1024), 0, s, tab, np, bs.S2, R, bs.status, bs.arena,
                           bs.arena_bytes, bs.data_off, bs.keep);
        hipLaunchKernelGGL(k_b_heavy_plan<IA>, dim3(1), dim3(1024), 0, s, tab, ws.row_prob, ws.row_nprod,
                           ws.class_rows, ws.ctl, bs.status, bs.arena, bs.arena_bytes);
        no.bound = 1;
        no.row_size = ws.row_size;
        no.ovf_rows = bs.ovf;
    }
    if (bs.upper) batched_numeric_launches<IA, IB, true>(bs, ws, th, no, grid_for, num_cu, s);
    else batched_numeric_launches<IA, IB, false>(bs, ws, th, no, grid_for, num_cu, s);
    if (bs.upper && bs.keep) {
        // operands only: the slots stay, described by their first and end positions
        hipLaunchKernelGGL(k_b_keep_slots, dim3(ga), dim3(256), 0, s, tab, ro, np, R, bs.S2, ws.row_size, bs.arena,
                           bs.status);
        hipLaunchKernelGGL(k_b_keep_fields, dim3(1), dim3(256), 0, s, tab, np, bs.arena, bs.status);
    } else if (bs.upper) {
        (void)launch_scan(R, ws.row_size, ws.tile_sum, bs.S, &ws.ctl->nnz, s);
        hipLaunchKernelGGL(k_b_distribute, dim3(1), dim3(1024), 0, s, tab, np, bs.S, bs.arena, bs.arena_bytes,
                           bs.data_off, bs.status);
        hipLaunchKernelGGL(k_b_rpt, dim3(ga), dim3(256), 0, s, tab, ro, np, R, bs.S, bs.status);
        hipLaunchKernelGGL(k_b_compact, dim3(ga), dim3(256), 0, s, tab, ws.row_prob, bs.S2, bs.S, R, bs.status);
    }
}

hipError_t launch_batched_stage(const BatchStage &bs, const Workspace &ws, const Thresholds &th, int num_cu,
                                int64_t grid_waves, hipStream_t s) {
    if (bs.a_rpt_bytes == 4 && bs.b_rpt_bytes == 4)
        batched_stage_launches<int32_t, int32_t>(bs, ws, th, num_cu, grid_waves, s);
    else if (bs.a_rpt_bytes == 4)
        batched_stage_launches<int32_t, int64_t>(bs, ws, th, num_cu, grid_waves, s);
    else if (bs.b_rpt_bytes == 4)
        batched_stage_launches<int64_t, int32_t>(bs, ws, th, num_cu, grid_waves, s);
    else
        batched_stage_launches<int64_t, int64_t>(bs, ws, th, num_cu, grid_waves, s);
    return hipGetLastError();
}

hipError_t launch_batched_begin(BatchStatus *st, Ctl *ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_b_zero_status, dim3(1), dim3(64), 0, s, st, ctl);
    return hipGetLastError();
}

hipError_t launch_batched_describe(const BatchProb *all, int n, spg_batched_out *out, const BatchStatus *st,
                                   hipStream_t s) {
    hipLaunchKernelGGL(k_b_describe, dim3((unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1)), dim3(256), 0, s,
                       all, n, out, st);
    return hipGetLastError();
}

}  // namespace brm
