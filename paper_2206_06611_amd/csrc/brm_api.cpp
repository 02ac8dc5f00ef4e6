// Host side of the C ABI declared in include/spgemm.h: argument checks, the
// handle's device workspace, and the launch sequence of the symbolic and
// numeric passes of the precise allocation (Section III-D.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "brm_internal.h"
#include "spgemm.h"

using namespace brm;

// Workspace of spgemm_batched_noalloc: a fixed array in device memory that
// every GPU the library runs on holds from the library's load until the
// process ends.  Host code never uses this name as an address: its device
// address is read once per device (scratch_address) and passed on.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};

// The device address of `scratch` on `device`, which must be current:
// looked up on the first call for that device, kept afterwards.
hipError_t scratch_address(int device, void **ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

struct spg_handle_s {
    int device = 0;
    int num_cu = 256;
    std::string err;
    // options
    int64_t validate = 0;
    int64_t wave_small_max = kCapWaveSmall;
    int64_t wave_max = kCapWave;
    int64_t group_max = kCapGroup;
    int64_t block_max = kCapBlock;
    int64_t force = -1;
    int64_t heavy_lds_max = kHeavyLdsCapMax;
    int64_t heavy_threads = 0;         // 0: chosen per batch; 512 or 1024
    int64_t spill_budget_mb = 0;       // 0: 128 GiB, or 60% of the device memory free at the call
    int64_t grid_waves = 0;
    int64_t group_rows = 1;  // kernel of the wave-small class (see SPG_OPT_GROUP_ROWS)
    int plan_group_rows = 1;  // the one the last symbolic pass classified for
    // workspace
    void *ws_mem = nullptr;
    size_t ws_bytes = 0;
    Ctl *ctl = nullptr;
    Ctl *ctl_host = nullptr;  // pinned
    // device address of ctl_host (mapped, coherent): the row-pointer scan
    // writes the control block there; null: it is read back by a copy
    Ctl *ctl_host_dev = nullptr;
    // heavy-row spill pool and per-row descriptors
    void *spill_mem = nullptr;
    size_t spill_bytes = 0;
    void *hdesc_mem = nullptr;
    size_t hdesc_bytes = 0;
    // plan left by the last symbolic call
    bool plan_valid = false;
    const void *pa_rpt = nullptr, *pb_rpt = nullptr;
    const int32_t *pa_col = nullptr, *pb_col = nullptr;
    int64_t pM = -1, pK = -1, pN = -1, pnnzA = -1, pnnzB = -1;
    int64_t counts[8] = {0};
    int64_t nnz = 0, nprod = 0;
    int64_t heavy_batches = 0;
    int64_t spill_allocs = 0;  // allocations of the spill pool
    int64_t heavy_wide = 0;    // heavy batches of the last numeric call run by 1024-thread workgroups
    int64_t heavy_split = 0;   // products per subtree item of a split heavy row (0: automatic, -1: never)
    int64_t heavy_split_rows = 0;  // heavy rows split into subtrees in the last numeric call
    void *hitem_mem = nullptr;     // heavy work items, top merges, subtree results, tickets
    size_t hitem_bytes = 0;
    // learned allocation
    int64_t alloc = 0;          // 0 precise, 1 learned, 2 upper bound
    int64_t accumulator = 0;    // 0 BRMerge, 1 hash table (comparator)
    int64_t learned_force = 0;  // testing: 1 = every predicted row at its lower bound
    int64_t b_err = 0;                 // device errors of the last batched call
    int64_t batch_alloc = SPG_BATCH_PRECISE;  // sizes of the batched stages: symbolic pass or upper bounds
    int64_t heavy_margin_milli = 200;  // extra margin (thousandths) of rows beyond one workgroup's LDS
    bool plan_learned = false;
    int64_t stored_order = 1;   // SPG_OPT_STORED_ORDER
    bool plan_order = false;    // the last symbolic pass kept the wave-small rows' order
    void *order_mem = nullptr;  // that order: [64 M] bytes, then [64 M] columns
    size_t order_bytes = 0;
    void *lw_mem = nullptr;     // per-row learned workspace
    size_t lw_bytes = 0;
    void *slot_mem = nullptr;   // predicted slots (column and value arrays)
    size_t slot_bytes = 0;
    Ctl *ctl2 = nullptr;        // control block of the exact fallback
    int64_t pred_total = 0, ovf_light = 0, ovf_heavy = 0;
    // predictor state (device): params, adam m, v, gradient, norm[12], loss, act, partial
    float *mlp = nullptr;
    size_t mlp_act_rows = 0;
    float *mlp_act = nullptr;
    bool mlp_ready = false;
    float delta = 0.0f;
    int64_t adam_t = 0;
    // batched products: own buffers (referenced by the captured graph)
    void *b_mem = nullptr;       // workspace rows | S | row offsets | table | status | ctl
    size_t b_bytes = 0;
    BatchProb *b_host = nullptr; // pinned host copy of the table
    size_t b_host_n = 0;
    int64_t *b_row_off_host = nullptr;
    size_t b_row_off_n = 0;
    BatchStatus *b_status_host = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<int64_t> graph_sig;
    std::vector<int64_t> seen_sig;  // the last batch launched directly (captured when it comes again)
    int64_t graph_captures = 0, graph_launches = 0, batched_direct = 0;
    // device address of the static scratch array on this handle's device
    // (the allocation-free batched call); null when it could not be read
    void *scratch = nullptr;
    std::string scratch_err;
};

struct LearnedWs {
    float *feats;       // [M * 6]
    int32_t *lo, *hi;   // [M]
    int8_t *predicted;  // [M]
    int32_t *pred_size; // [M]
    int64_t *slot_off;  // [M + 1]
    int32_t *ovf_rows;  // [2 M]
    int32_t *b_ends;    // [4 K] per row of B: first and last column (-1 / -1 when empty), length, start
};

namespace {

int fail(spg_handle h, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    return code;
}

#define HIP_TRY(h, expr)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail((h), SPG_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// a row whose product count does not fit int32 (the analysis routes it to
// no kernel and raises kErrRowProducts)
int fail_row_products(spg_handle h) {
    return fail(h, SPG_ERR_CAPACITY, "a row of C has 2^31 or more products (limit 2^31-1 per row); "
                                     "products per row are counted in int32 by the row kernels");
}

int check_csr(spg_handle h, const spg_csr *X, const char *name, bool need_val) {
    if (!X) return fail(h, SPG_ERR_ARG, "%s is NULL", name);
    if (X->rows < 0 || X->cols < 0 || X->nnz < 0)
        return fail(h, SPG_ERR_ARG, "%s has a negative size", name);
    if (X->rpt_bytes != 4 && X->rpt_bytes != 8)
        return fail(h, SPG_ERR_ARG, "%s.rpt_bytes must be 4 or 8", name);
    if (X->rpt_bytes == 4 && X->nnz > INT32_MAX)
        return fail(h, SPG_ERR_ARG, "%s.nnz does not fit int32 row pointers", name);
    if (X->cols > INT32_MAX) return fail(h, SPG_ERR_ARG, "%s.cols exceeds int32 column indices", name);
    if (!X->rpt) return fail(h, SPG_ERR_ARG, "%s.rpt is NULL", name);
    if (X->nnz > 0 && !X->col) return fail(h, SPG_ERR_ARG, "%s.col is NULL", name);
    if (need_val && X->nnz > 0 && !X->val) return fail(h, SPG_ERR_ARG, "%s.val is NULL", name);
    return SPG_OK;
}

CsrView view(const spg_csr *X) {
    CsrView v;
    v.rows = X->rows;
    v.cols = X->cols;
    v.nnz = X->nnz;
    v.rpt = X->rpt;
    v.rpt_bytes = X->rpt_bytes;
    v.col = X->col;
    v.val = X->val;
    return v;
}

int ensure_workspace(spg_handle h, int64_t M, int64_t nnzA, Workspace *ws) {
    const int64_t ntiles = (M + kScanTile - 1) / kScanTile + 1;
    const size_t a = 256;
    size_t off_nprod = 0;
    size_t off_class = align_up(off_nprod + 8 * (size_t)M, a);
    size_t off_size = align_up(off_class + (size_t)M, a);
    size_t off_rows = align_up(off_size + 4 * (size_t)M, a);
    size_t off_tile = align_up(off_rows + 4 * (size_t)M, a);
    size_t off_ebs = align_up(off_tile + 8 * (size_t)ntiles, a);
    size_t off_elen = align_up(off_ebs + 8 * (size_t)nnzA, a);
    size_t total = align_up(off_elen + 4 * (size_t)nnzA, a);
    if (total > h->ws_bytes) {
        if (h->ws_mem) HIP_TRY(h, hipFree(h->ws_mem));
        h->ws_mem = nullptr;
        h->ws_bytes = 0;
        size_t want = std::max(total, h->ws_bytes * 3 / 2);
        if (hipMalloc(&h->ws_mem, want) != hipSuccess) {
            (void)hipGetLastError();
            return fail(h, SPG_ERR_NOMEM, "workspace allocation of %zu bytes failed", want);
        }
        h->ws_bytes = want;
    }
    char *base = static_cast<char *>(h->ws_mem);
    ws->row_nprod = reinterpret_cast<int64_t *>(base + off_nprod);
    ws->row_class = reinterpret_cast<uint8_t *>(base + off_class);
    ws->row_size = reinterpret_cast<int32_t *>(base + off_size);
    ws->class_rows = reinterpret_cast<int32_t *>(base + off_rows);
    ws->tile_sum = reinterpret_cast<int64_t *>(base + off_tile);
    ws->ent_bs = base + off_ebs;
    ws->ent_len = reinterpret_cast<int32_t *>(base + off_elen);
    ws->row_prob = nullptr;
    ws->ctl = h->ctl;
    return SPG_OK;
}

int grow(spg_handle h, void **mem, size_t *have, size_t need, const char *what) {
    if (need <= *have) return SPG_OK;
    if (*mem) HIP_TRY(h, hipFree(*mem));
    *mem = nullptr;
    *have = 0;
    if (hipMalloc(mem, need) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, SPG_ERR_NOMEM, "allocation of %zu bytes for %s failed", need, what);
    }
    *have = need;
    return SPG_OK;
}

// Heavy rows: read their sizes back, order them largest first, cut them into
// batches whose spill buffers fit the budget and run one launch per batch.
int run_heavy(spg_handle h, const CsrView &a, const CsrView &b, const Workspace &ws, const int32_t *heavy_rows,
              int64_t n, const int64_t *c_rpt, int32_t *c_col, double *c_val, const NumOut &no,
              Ctl *ctl, hipStream_t s) {
    // descriptors: info (3 x int64 per row) then rows (int32), spill_off, leaf_off (int64)
    const size_t info_b = align_up(24 * (size_t)n, 256);
    const size_t rows_b = align_up(4 * (size_t)n, 256);
    const size_t offs_b = align_up(8 * (size_t)n, 256);
    int rc;
    if ((rc = grow(h, &h->hdesc_mem, &h->hdesc_bytes, info_b + rows_b + 2 * offs_b + 8 * 4096, "heavy descriptors")))
        return rc;
    char *d = static_cast<char *>(h->hdesc_mem);
    int64_t *d_info = reinterpret_cast<int64_t *>(d);
    int32_t *d_rows = reinterpret_cast<int32_t *>(d + info_b);
    int64_t *d_soff = reinterpret_cast<int64_t *>(d + info_b + rows_b);
    int64_t *d_loff = reinterpret_cast<int64_t *>(d + info_b + rows_b + offs_b);
    HIP_TRY(h, launch_heavy_info(a, ws, heavy_rows, n, d_info, s));
    std::vector<int64_t> info(3 * (size_t)n);
    HIP_TRY(h, hipMemcpyAsync(info.data(), d_info, 24 * (size_t)n, hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    // rows ordered largest first, to within an eighth of an octave: one
    // counting-sort pass over logarithmic buckets of the product count (a
    // full comparison sort of ~3e5 rows cost ~40 ms of host time per call),
    // visiting the rows by row id so that the order, and with it the batches
    // and the spill pool they need, is the same on every call (the heavy rows
    // arrive in the class list's order, which is not); the order decides
    // batching and load balance only, never a result
    std::vector<int64_t> order((size_t)n);
    {
        std::vector<int32_t> at((size_t)a.rows, -1);  // info index of every heavy row
        for (int64_t i = 0; i < n; ++i) at[(size_t)info[3 * i]] = (int32_t)i;
        std::vector<uint8_t> bucket((size_t)n);
        int64_t cnt[257] = {0};
        for (int64_t i = 0; i < n; ++i) {
            const uint64_t v = (uint64_t)std::max<int64_t>(info[3 * i + 1], 1);
            const int lg = 63 - __builtin_clzll(v);
            const int frac = lg >= 3 ? (int)((v >> (lg - 3)) & 7) : (int)((v << (3 - lg)) & 7);
            const int bk = 255 - (8 * lg + frac);  // larger counts first
            bucket[(size_t)i] = (uint8_t)(bk < 0 ? 0 : bk);
            ++cnt[bucket[(size_t)i] + 1];
        }
        for (int k = 0; k < 256; ++k) cnt[k + 1] += cnt[k];
        for (int64_t r = 0; r < a.rows; ++r) {
            const int32_t i = at[(size_t)r];
            if (i >= 0) order[(size_t)cnt[bucket[(size_t)i]]++] = i;
        }
    }
    std::vector<int32_t> rows((size_t)n);
    std::vector<int64_t> soff((size_t)n), loff((size_t)n);
    std::vector<std::pair<int64_t, int64_t>> batches;  // [begin, end)
    size_t budget = (size_t)h->spill_budget_mb << 20;
    if (budget == 0) {
        // automatic: 128 GiB, or 60% of the device memory free now (C is
        // allocated by then) when that is less; fewer batches leave the
        // device idle less often at batch ends
        size_t free_b = 0, total_b = 0;
        HIP_TRY(h, hipMemGetInfo(&free_b, &total_b));
        budget = std::max<size_t>(std::min<size_t>(free_b / 10 * 6, (size_t)128 << 30), (size_t)1 << 30);
        // a pool the handle already holds is used whole
        budget = std::max(budget, h->spill_bytes);
    }
    // the pool holds every batch in turn: columns and values of the largest
    // batch's two spill buffers, then the largest batch's list offsets
    auto pool_bytes = [](size_t elems, size_t leafs) {
        return align_up(4 * elems, 256) + align_up(8 * elems, 256) + align_up(4 * leafs, 256) + 256;
    };
    // batches of consecutive rows in that order: the longest rows run side by
    // side in the first batch (a batch lasts as long as its longest row).  A
    // batch is cut where the pool would outgrow the budget, so a pool already
    // held is never reallocated by a call that fits it.
    size_t max_elems = 0, max_leaf = 0;
    size_t elems = 0, leafs = 0;
    int64_t b0 = 0;
    for (int64_t j = 0; j < n; ++j) {
        const int64_t i = order[(size_t)j];
        const int64_t np = info[3 * i + 1], nl = info[3 * i + 2];
        if (np >= INT32_MAX || nl >= INT32_MAX)
            return fail(h, SPG_ERR_CAPACITY, "row %lld has %lld products (limit 2^31-1 per row)",
                        (long long)info[3 * i], (long long)np);
        if (j > b0 && pool_bytes(std::max(max_elems, elems + 2 * (size_t)np),
                                 std::max(max_leaf, leafs + (size_t)nl + 1)) > budget) {
            batches.emplace_back(b0, j);
            b0 = j;
            elems = leafs = 0;
        }
        rows[(size_t)j] = (int32_t)info[3 * i];
        soff[(size_t)j] = (int64_t)elems;
        loff[(size_t)j] = (int64_t)leafs;
        elems += 2 * (size_t)np;
        leafs += (size_t)nl + 1;
        max_elems = std::max(max_elems, elems);
        max_leaf = std::max(max_leaf, leafs);
    }
    batches.emplace_back(b0, n);
    if (batches.size() > 4096) return fail(h, SPG_ERR_CAPACITY, "too many spill batches; raise the spill budget");
    // work items of every batch: whole rows, or, for a row much longer than
    // the batch's share per workgroup, aligned subtrees of its lists (the
    // levels above them merged by one launch per level), so that no single
    // row bounds its batch
    struct Plan {
        int64_t item0, nitem;  // items of the batch
        int threads;
        std::vector<std::pair<int64_t, int64_t>> levels;  // [first, count) of the top merges per level
    };
    std::vector<Plan> plans(batches.size());
    std::vector<HeavyItem> items;
    std::vector<HeavyTop> tops;
    int64_t nres = 0;
    int64_t split_rows = 0;
    for (size_t bi = 0; bi < batches.size(); ++bi) {
        const int64_t lo = batches[bi].first, hi = batches[bi].second;
        int64_t tot = 0, longest_row = 0;
        for (int64_t j = lo; j < hi; ++j) {
            const int64_t np = info[3 * order[(size_t)j] + 1];
            tot += np;
            longest_row = std::max(longest_row, np);
        }
        // products per subtree item: a quarter of a workgroup's share of
        // the batch (two 512-thread workgroups per CU), at least 2^18
        int64_t target = h->heavy_split;
        if (target == 0) target = std::max<int64_t>(tot / (8 * (int64_t)h->num_cu), (int64_t)1 << 18);
        std::vector<std::pair<int64_t, HeavyItem>> bitems;  // (estimated products, item)
        std::vector<std::vector<HeavyTop>> blevels;
        for (int64_t j = lo; j < hi; ++j) {
            const int64_t i = order[(size_t)j];
            const int64_t np = info[3 * i + 1], L = info[3 * i + 2];
            if (target < 0 || np <= 2 * target || L < 2) {
                bitems.push_back({np, HeavyItem{(int32_t)(j - lo), -1, 0, L, np}});
                continue;
            }
            // subtrees of 2^H lists, at least ceil(np / target) of them (at most 1024)
            const int64_t want = std::min<int64_t>((np + target - 1) / target, 1024);
            int H = 0;
            while (((L + ((int64_t)1 << (H + 1)) - 1) >> (H + 1)) >= want) ++H;
            const int64_t S = (L + ((int64_t)1 << H) - 1) >> H;
            if (S < 2) {
                bitems.push_back({np, HeavyItem{(int32_t)(j - lo), -1, 0, L, np}});
                continue;
            }
            ++split_rows;
            const int64_t base = nres;
            nres += S;
            for (int64_t q = 0; q < S; ++q) {
                const int64_t l0 = q << H, l1 = std::min((q + 1) << H, L);
                bitems.push_back({np * (l1 - l0) / L, HeavyItem{(int32_t)(j - lo), (int32_t)(base + q), l0, l1, np}});
            }
            // the levels above: node (r, q) keeps its result in slot base + (q << r)
            for (int r = 1; ((S + ((int64_t)1 << (r - 1)) - 1) >> (r - 1)) > 1; ++r) {
                const int64_t nprev = (S + ((int64_t)1 << (r - 1)) - 1) >> (r - 1);
                const int64_t ncur = (S + ((int64_t)1 << r) - 1) >> r;
                if ((int64_t)blevels.size() < r) blevels.resize((size_t)r);
                for (int64_t q = 0; q < ncur; ++q) {
                    const int64_t xq = 2 * q, yq = 2 * q + 1;
                    const bool root = ncur == 1;
                    if (yq >= nprev && !root) continue;  // promoted unchanged
                    HeavyTop t;
                    t.bi = (int32_t)(j - lo);
                    t.res_x = (int32_t)(base + (xq << (r - 1)));
                    t.res_y = yq < nprev ? (int32_t)(base + (yq << (r - 1))) : -1;
                    t.root = root ? 1 : 0;
                    t.lx = (xq << (r - 1)) << H;
                    t.ly = yq < nprev ? (yq << (r - 1)) << H : 0;
                    t.nprod = np;
                    blevels[(size_t)r - 1].push_back(t);
                }
            }
        }
        // largest items first
        std::stable_sort(bitems.begin(), bitems.end(),
                         [](const std::pair<int64_t, HeavyItem> &a, const std::pair<int64_t, HeavyItem> &b) {
                             return a.first > b.first;
                         });
        Plan &pl = plans[bi];
        pl.item0 = (int64_t)items.size();
        pl.nitem = (int64_t)bitems.size();
        for (auto &x : bitems) items.push_back(x.second);
        for (auto &lv : blevels) {
            pl.levels.push_back({(int64_t)tops.size(), (int64_t)lv.size()});
            tops.insert(tops.end(), lv.begin(), lv.end());
        }
        int threads = (int)h->heavy_threads;
        if (threads == 0) {
            // a batch lasts at least as long as its longest item, merged by
            // one workgroup: 1024-thread workgroups (one per CU, each about
            // 1.4x as fast on one row) when that item outweighs a 512-thread
            // workgroup's share of the batch by a margin, else 512-thread
            // workgroups (two per CU, more items side by side)
            const int64_t longest = bitems.empty() ? 0 : bitems.front().first;
            threads = (double)longest > 1.3 * (double)tot / (2.0 * (double)h->num_cu) ? 1024 : 512;
        }
        pl.threads = threads;
    }
    h->heavy_split_rows += split_rows;
    // items | tops | results | tickets (one per launch)
    int64_t nlaunch = 0;
    for (auto &pl : plans) nlaunch += 1 + (int64_t)pl.levels.size();
    const size_t it_b = align_up(sizeof(HeavyItem) * std::max<size_t>(items.size(), 1), 256);
    const size_t tp_b = align_up(sizeof(HeavyTop) * std::max<size_t>(tops.size(), 1), 256);
    const size_t rs_b = align_up(16 * (size_t)std::max<int64_t>(nres, 1), 256);
    const size_t tk_b = align_up(8 * (size_t)nlaunch, 256);
    if ((rc = grow(h, &h->hitem_mem, &h->hitem_bytes, it_b + tp_b + rs_b + tk_b, "heavy work items"))) return rc;
    char *hm = static_cast<char *>(h->hitem_mem);
    HeavyItem *d_items = reinterpret_cast<HeavyItem *>(hm);
    HeavyTop *d_tops = reinterpret_cast<HeavyTop *>(hm + it_b);
    int64_t *d_res = reinterpret_cast<int64_t *>(hm + it_b + tp_b);
    unsigned long long *d_tick = reinterpret_cast<unsigned long long *>(hm + it_b + tp_b + rs_b);
    HIP_TRY(h, hipMemcpy(d_rows, rows.data(), 4 * (size_t)n, hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_soff, soff.data(), 8 * (size_t)n, hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_loff, loff.data(), 8 * (size_t)n, hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_items, items.data(), sizeof(HeavyItem) * items.size(), hipMemcpyHostToDevice));
    if (!tops.empty())
        HIP_TRY(h, hipMemcpy(d_tops, tops.data(), sizeof(HeavyTop) * tops.size(), hipMemcpyHostToDevice));
    const size_t col_b = align_up(4 * max_elems, 256), val_b = align_up(8 * max_elems, 256);
    const size_t pool_need = pool_bytes(max_elems, max_leaf);
    if (pool_need > h->spill_bytes) ++h->spill_allocs;
    if ((rc = grow(h, &h->spill_mem, &h->spill_bytes, pool_need, "spill buffers"))) return rc;
    char *sp = static_cast<char *>(h->spill_mem);
    HIP_TRY(h, launch_zero_words(d_tick, nlaunch, s));
    // results start as empty lists in buffer 0 (read only after their subtree wrote them)
    if (nres > 0) HIP_TRY(h, launch_zero_words(reinterpret_cast<unsigned long long *>(d_res), 2 * nres, s));
    int64_t tick = 0;
    for (size_t bi = 0; bi < batches.size(); ++bi) {
        const int64_t lo = batches[bi].first;
        const Plan &pl = plans[bi];
        HeavyArgs ha;
        ha.ticket = d_tick + tick++;
        ha.rows = d_rows + lo;
        ha.spill_off = d_soff + lo;
        ha.leaf_off = d_loff + lo;
        ha.items = d_items + pl.item0;
        ha.nitems = pl.nitem;
        ha.res = d_res;
        ha.spill_col = reinterpret_cast<int32_t *>(sp);
        ha.spill_val = reinterpret_cast<double *>(sp + col_b);
        ha.leaf = reinterpret_cast<int32_t *>(sp + col_b + val_b);
        ha.threads = pl.threads;
        ha.lds_cap = (int)std::min<int64_t>(h->heavy_lds_max, 4 * (int64_t)pl.threads);
        // 1024 / threads workgroups per CU
        const int grid = (int)std::min<int64_t>(pl.nitem, (int64_t)(1024 / pl.threads) * h->num_cu);
        if (pl.threads == 1024) ++h->heavy_wide;
        HIP_TRY(h, launch_numeric_heavy(a, b, ws, ha, grid, c_rpt, c_col, c_val, ctl, no, s));
        for (const auto &lv : pl.levels) {
            ha.ticket = d_tick + tick++;
            HIP_TRY(h, launch_heavy_top(ha, d_tops + lv.first, lv.second,
                                        (int)std::min<int64_t>(lv.second, h->num_cu), c_rpt, c_col, c_val, ctl,
                                        no, s));
        }
    }
    h->heavy_batches += (int64_t)batches.size();
    return SPG_OK;
}

int ensure_learned_ws(spg_handle h, int64_t M, LearnedWs *lw, int64_t K = 0) {
    const size_t a = 256;
    size_t o_feat = 0;
    size_t o_lo = align_up(o_feat + 24 * (size_t)M, a);
    size_t o_hi = align_up(o_lo + 4 * (size_t)M, a);
    size_t o_pr = align_up(o_hi + 4 * (size_t)M, a);
    size_t o_ps = align_up(o_pr + (size_t)M, a);
    size_t o_so = align_up(o_ps + 4 * (size_t)M, a);
    size_t o_ov = align_up(o_so + 8 * (size_t)(M + 1), a);
    size_t o_be = align_up(o_ov + 8 * (size_t)M + 8, a);
    size_t total = align_up(o_be + 16 * (size_t)K + 16, a);
    int rc;
    if ((rc = grow(h, &h->lw_mem, &h->lw_bytes, total, "learned workspace"))) return rc;
    char *b = static_cast<char *>(h->lw_mem);
    lw->feats = reinterpret_cast<float *>(b + o_feat);
    lw->lo = reinterpret_cast<int32_t *>(b + o_lo);
    lw->hi = reinterpret_cast<int32_t *>(b + o_hi);
    lw->predicted = reinterpret_cast<int8_t *>(b + o_pr);
    lw->pred_size = reinterpret_cast<int32_t *>(b + o_ps);
    lw->slot_off = reinterpret_cast<int64_t *>(b + o_so);
    lw->ovf_rows = reinterpret_cast<int32_t *>(b + o_ov);
    lw->b_ends = reinterpret_cast<int32_t *>(b + o_be);
    if (!h->ctl2) {
        HIP_TRY(h, hipMalloc(&h->ctl2, sizeof(Ctl)));
        HIP_TRY(h, hipMemset(h->ctl2, 0, sizeof(Ctl)));
    }
    return SPG_OK;
}

// predictor buffers: params | m | v | grad | norm(12) | loss(4) | partial
constexpr size_t kMlpOffM = kMlpParams, kMlpOffV = 2 * kMlpParams, kMlpOffG = 3 * kMlpParams,
                 kMlpOffNorm = 4 * kMlpParams, kMlpOffLoss = kMlpOffNorm + 12,
                 kMlpOffPartial = kMlpOffLoss + 4,
                 kMlpFloats = kMlpOffPartial + (size_t)kMlpGradChunks * (kMlpParams + 1);

int ensure_mlp(spg_handle h) {
    if (!h->mlp) {
        if (hipMalloc(&h->mlp, sizeof(float) * kMlpFloats) != hipSuccess) {
            (void)hipGetLastError();
            return fail(h, SPG_ERR_NOMEM, "predictor state allocation failed");
        }
        HIP_TRY(h, hipMemset(h->mlp, 0, sizeof(float) * kMlpFloats));
        std::vector<float> norm(12, 0.0f);
        for (int j = 6; j < 12; ++j) norm[(size_t)j] = 1.0f;
        HIP_TRY(h, hipMemcpy(h->mlp + kMlpOffNorm, norm.data(), 48, hipMemcpyHostToDevice));
    }
    return SPG_OK;
}

int ensure_mlp_act(spg_handle h, int64_t rows) {
    if ((size_t)rows <= h->mlp_act_rows) return SPG_OK;
    if (h->mlp_act) HIP_TRY(h, hipFree(h->mlp_act));
    h->mlp_act = nullptr;
    h->mlp_act_rows = 0;
    if (hipMalloc(&h->mlp_act, sizeof(float) * kMlpActStride * (size_t)rows) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, SPG_ERR_NOMEM, "activation buffer allocation failed");
    }
    h->mlp_act_rows = (size_t)rows;
    return SPG_OK;
}

// windows: the wave-small class is served by the register-window kernels,
// which take only rows whose lists fit lane windows
Thresholds thresholds(spg_handle h, bool windows, bool multi = false) {
    Thresholds t;
    t.wave_small_max = h->wave_small_max;
    t.wave_max = h->wave_max;
    t.group_max = h->group_max;
    t.block_max = h->block_max;
    t.force = (int32_t)h->force;
    t.windows = windows ? 1 : 0;
    t.multi = windows && multi ? 1 : 0;
    return t;
}

bool uses_windows(int64_t group_rows) { return group_rows == 1 || group_rows == 2; }

int persistent_grid(spg_handle h, int cls, int64_t rows, int group_rows) {
    // workgroups per launch of the persistent row kernels
    int per_cu;
    int teams_per_wg;  // rows a workgroup takes per pass
    switch (cls) {
        case kClassCopy: per_cu = 8; teams_per_wg = 4; break;
        case kClassWaveSmall:
            per_cu = 8;
            teams_per_wg = uses_windows(group_rows) ? 4 * 64 : 4 * (group_rows > 1 ? group_rows : 1);  // chunks of 64 rows
            break;
        case kClassMulti: per_cu = 5; teams_per_wg = 4 * 64; break;  // chunks of 64 rows
        case kClassWave: per_cu = 4; teams_per_wg = 4; break;
        case kClassGroup: per_cu = 4; teams_per_wg = 1; break;
        case kClassBlock: per_cu = 1; teams_per_wg = 1; break;
        default: per_cu = 1; teams_per_wg = 1; break;
    }
    int64_t g = (int64_t)h->num_cu * per_cu;
    if (h->grid_waves > 0) {
        const int waves_per_wg = (cls == kClassBlock || cls == kClassHeavy) ? 16
                                 : (cls == kClassGroup)                     ? 4
                                                                            : 4;
        g = std::max<int64_t>(1, h->grid_waves / waves_per_wg);
    }
    if (rows >= 0) g = std::min<int64_t>(g, (rows + teams_per_wg - 1) / teams_per_wg);
    return (int)std::max<int64_t>(g, 1);
}

}  // namespace

extern "C" {

int spg_create(spg_handle *out, int device) {
    if (!out) return SPG_ERR_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return SPG_ERR_HIP;
    }
    spg_handle h = new (std::nothrow) spg_handle_s();
    if (!h) return SPG_ERR_NOMEM;
    h->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete h;
        return SPG_ERR_HIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) h->num_cu = prop.multiProcessorCount;
    if (hipMalloc(&h->ctl, sizeof(Ctl)) != hipSuccess ||
        hipHostMalloc(&h->ctl_host, sizeof(Ctl), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        if (h->ctl) (void)hipFree(h->ctl);
        delete h;
        return SPG_ERR_NOMEM;
    }
    std::memset(h->ctl_host, 0, sizeof(Ctl));
    if (hipHostGetDevicePointer(reinterpret_cast<void **>(&h->ctl_host_dev), h->ctl_host, 0) != hipSuccess) {
        (void)hipGetLastError();
        h->ctl_host_dev = nullptr;
    }
    {
        const hipError_t e = scratch_address(device, &h->scratch);
        if (e != hipSuccess) h->scratch_err = hipGetErrorString(e);
    }
    *out = h;
    return SPG_OK;
}

int spg_destroy(spg_handle h) {
    if (!h) return SPG_ERR_ARG;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    if (h->ws_mem) (void)hipFree(h->ws_mem);
    if (h->spill_mem) (void)hipFree(h->spill_mem);
    if (h->hdesc_mem) (void)hipFree(h->hdesc_mem);
    if (h->hitem_mem) (void)hipFree(h->hitem_mem);
    if (h->lw_mem) (void)hipFree(h->lw_mem);
    if (h->slot_mem) (void)hipFree(h->slot_mem);
    if (h->order_mem) (void)hipFree(h->order_mem);
    if (h->ctl2) (void)hipFree(h->ctl2);
    if (h->mlp) (void)hipFree(h->mlp);
    if (h->mlp_act) (void)hipFree(h->mlp_act);
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->b_mem) (void)hipFree(h->b_mem);
    if (h->b_host) (void)hipHostFree(h->b_host);
    if (h->b_row_off_host) (void)hipHostFree(h->b_row_off_host);
    if (h->b_status_host) (void)hipHostFree(h->b_status_host);
    if (h->ctl) (void)hipFree(h->ctl);
    if (h->ctl_host) (void)hipHostFree(h->ctl_host);
    delete h;
    return SPG_OK;
}

const char *spg_last_error(spg_handle h) { return h ? h->err.c_str() : "null handle"; }

int spg_set_option(spg_handle h, int key, int64_t value) {
    if (!h) return SPG_ERR_ARG;
    switch (key) {
        case SPG_OPT_VALIDATE: h->validate = value != 0; break;
        case SPG_OPT_WAVE_SMALL_MAX:
            if (value < 0 || value > kCapWaveSmall) return fail(h, SPG_ERR_ARG, "wave-small max out of range");
            h->wave_small_max = value;
            break;
        case SPG_OPT_WAVE_MAX:
            if (value < 0 || value > kCapWave) return fail(h, SPG_ERR_ARG, "wave max out of range");
            h->wave_max = value;
            break;
        case SPG_OPT_GROUP_MAX:
            if (value < 0 || value > kCapGroup) return fail(h, SPG_ERR_ARG, "group max out of range");
            h->group_max = value;
            break;
        case SPG_OPT_BLOCK_MAX:
            if (value < 0 || value > kCapBlock) return fail(h, SPG_ERR_ARG, "block max out of range");
            h->block_max = value;
            break;
        case SPG_OPT_FORCE_CLASS:
            if (value != -1 && (value < kClassWaveSmall || value > kClassMulti))
                return fail(h, SPG_ERR_ARG, "force class must be -1 or 2..7");
            h->force = value;
            break;
        case SPG_OPT_ACCUMULATOR:
            if (value != SPG_ACC_BRMERGE && value != SPG_ACC_HASH)
                return fail(h, SPG_ERR_ARG, "accumulator must be SPG_ACC_BRMERGE or SPG_ACC_HASH");
            h->accumulator = value;
            break;
        case SPG_OPT_HEAVY_LDS_MAX:
            if (value < 64 || value > kHeavyLdsCapMax) return fail(h, SPG_ERR_ARG, "heavy LDS max out of range");
            h->heavy_lds_max = value;
            break;
        case SPG_OPT_HEAVY_THREADS:
            if (value != 0 && value != 512 && value != 1024)
                return fail(h, SPG_ERR_ARG, "heavy threads must be 0 (automatic), 512 or 1024");
            h->heavy_threads = value;
            break;
        case SPG_OPT_HEAVY_SPLIT:
            if (value < -1) return fail(h, SPG_ERR_ARG, "heavy split must be -1 (never), 0 (automatic) or > 0");
            h->heavy_split = value;
            break;
        case SPG_OPT_SPILL_BUDGET_MB:
            if (value < 0) return fail(h, SPG_ERR_ARG, "spill budget must be >= 0 (0: automatic)");
            h->spill_budget_mb = value;
            break;
        case SPG_OPT_GRID_WAVES:
            if (value < 0) return fail(h, SPG_ERR_ARG, "grid waves must be >= 0");
            h->grid_waves = value;
            break;
        case SPG_OPT_GROUP_ROWS:
            if (value != 0 && value != 1 && value != 2 && value != kGroupRows)
                return fail(h, SPG_ERR_ARG, "group rows must be 0, 1, 2 or %d", kGroupRows);
            h->group_rows = value;
            break;
        case SPG_OPT_ALLOC:
            if (value != SPG_ALLOC_PRECISE && value != SPG_ALLOC_LEARNED && value != SPG_ALLOC_UPPER)
                return fail(h, SPG_ERR_ARG, "allocation must be SPG_ALLOC_PRECISE, SPG_ALLOC_LEARNED or SPG_ALLOC_UPPER");
            h->alloc = value;
            break;
        case SPG_OPT_LEARNED_HEAVY_MARGIN:
            if (value < 0 || value > 10000) return fail(h, SPG_ERR_ARG, "heavy margin must be 0..10000 (thousandths)");
            h->heavy_margin_milli = value;
            break;
        case SPG_OPT_STORED_ORDER:
            if (value != 0 && value != 1) return fail(h, SPG_ERR_ARG, "stored order must be 0 or 1");
            h->stored_order = value;
            break;
        case SPG_OPT_BATCH_ALLOC:
            if (value != SPG_BATCH_PRECISE && value != SPG_BATCH_UPPER)
                return fail(h, SPG_ERR_ARG, "batched allocation must be SPG_BATCH_PRECISE or SPG_BATCH_UPPER");
            h->batch_alloc = value;
            break;
        case SPG_OPT_LEARNED_FORCE:
            if (value != 0 && value != 1) return fail(h, SPG_ERR_ARG, "learned force must be 0 or 1");
            h->learned_force = value;
            break;
        default: return fail(h, SPG_ERR_ARG, "unknown option %d", key);
    }
    h->plan_valid = false;
    return SPG_OK;
}

int spg_get_option(spg_handle h, int key, int64_t *value) {
    if (!h || !value) return SPG_ERR_ARG;
    switch (key) {
        case SPG_OPT_VALIDATE: *value = h->validate; break;
        case SPG_OPT_WAVE_SMALL_MAX: *value = h->wave_small_max; break;
        case SPG_OPT_WAVE_MAX: *value = h->wave_max; break;
        case SPG_OPT_GROUP_MAX: *value = h->group_max; break;
        case SPG_OPT_BLOCK_MAX: *value = h->block_max; break;
        case SPG_OPT_FORCE_CLASS: *value = h->force; break;
        case SPG_OPT_HEAVY_LDS_MAX: *value = h->heavy_lds_max; break;
        case SPG_OPT_HEAVY_THREADS: *value = h->heavy_threads; break;
        case SPG_OPT_HEAVY_SPLIT: *value = h->heavy_split; break;
        case SPG_OPT_SPILL_BUDGET_MB: *value = h->spill_budget_mb; break;
        case SPG_OPT_GRID_WAVES: *value = h->grid_waves; break;
        case SPG_OPT_ALLOC: *value = h->alloc; break;
        case SPG_OPT_GROUP_ROWS: *value = h->group_rows; break;
        case SPG_OPT_LEARNED_FORCE: *value = h->learned_force; break;
        case SPG_OPT_LEARNED_HEAVY_MARGIN: *value = h->heavy_margin_milli; break;
        case SPG_OPT_BATCH_ALLOC: *value = h->batch_alloc; break;
        case SPG_OPT_STORED_ORDER: *value = h->stored_order; break;
        case SPG_OPT_ACCUMULATOR: *value = h->accumulator; break;
        default: return fail(h, SPG_ERR_ARG, "unknown option %d", key);
    }
    return SPG_OK;
}

int spg_get_stat(spg_handle h, int key, int64_t *value) {
    if (!h || !value) return SPG_ERR_ARG;
    if (key >= SPG_STAT_CLASS_ROWS0 && key < SPG_STAT_CLASS_ROWS0 + kNumClasses) {
        *value = h->counts[key - SPG_STAT_CLASS_ROWS0];
        return SPG_OK;
    }
    switch (key) {
        case SPG_STAT_NPROD: *value = h->nprod; return SPG_OK;
        case SPG_STAT_NNZ: *value = h->nnz; return SPG_OK;
        case SPG_STAT_HEAVY_BATCHES: *value = h->heavy_batches; return SPG_OK;
        case SPG_STAT_PRED_TOTAL: *value = h->pred_total; return SPG_OK;
        case SPG_STAT_GRAPH_CAPTURES: *value = h->graph_captures; return SPG_OK;
        case SPG_STAT_GRAPH_LAUNCHES: *value = h->graph_launches; return SPG_OK;
        case SPG_STAT_BATCHED_DIRECT: *value = h->batched_direct; return SPG_OK;
        case SPG_STAT_SPILL_POOL_BYTES: *value = (int64_t)h->spill_bytes; return SPG_OK;
        case SPG_STAT_SPILL_ALLOCS: *value = h->spill_allocs; return SPG_OK;
        case SPG_STAT_HEAVY_WIDE: *value = h->heavy_wide; return SPG_OK;
        case SPG_STAT_HEAVY_SPLIT_ROWS: *value = h->heavy_split_rows; return SPG_OK;
        case SPG_STAT_OVERFLOW_ROWS: *value = h->ovf_light + h->ovf_heavy; return SPG_OK;
        case SPG_STAT_OVERFLOW_HEAVY_ROWS: *value = h->ovf_heavy; return SPG_OK;
        case SPG_STAT_PREDICTED_ROWS: {
            int64_t n = 0;
            for (int c = kClassWaveSmall; c < kNumClasses; ++c) n += h->counts[c];
            *value = n;
            return SPG_OK;
        }
        case SPG_STAT_DEVICE_ERR: {
            HIP_TRY(h, hipSetDevice(h->device));
            HIP_TRY(h, hipDeviceSynchronize());
            int64_t e = 0, e2 = 0;
            HIP_TRY(h, hipMemcpy(&e, &h->ctl->err, sizeof e, hipMemcpyDeviceToHost));
            if (h->ctl2) HIP_TRY(h, hipMemcpy(&e2, &h->ctl2->err, sizeof e2, hipMemcpyDeviceToHost));
            *value = e | e2 | h->b_err;
            return SPG_OK;
        }
        default: return fail(h, SPG_ERR_ARG, "unknown statistic %d", key);
    }
}

int spgemm_symbolic(spg_handle h, const spg_csr *A, const spg_csr *B, int64_t *c_rpt,
                    int64_t *c_nnz, void *stream) {
    if (!h) return SPG_ERR_ARG;
    h->err.clear();
    h->b_err = 0;
    h->plan_valid = false;
    int rc;
    // learned and upper-bound allocation compute the rows' values into slots
    // during this call: they read the values, the precise method does not
    const bool slotted = h->alloc == SPG_ALLOC_LEARNED || h->alloc == SPG_ALLOC_UPPER;
    if ((rc = check_csr(h, A, "A", slotted)) || (rc = check_csr(h, B, "B", slotted))) return rc;
    if (!c_rpt || !c_nnz) return fail(h, SPG_ERR_ARG, "c_rpt / c_nnz is NULL");
    if (A->cols != B->rows)
        return fail(h, SPG_ERR_DIM, "A is %lld x %lld but B has %lld rows", (long long)A->rows,
                    (long long)A->cols, (long long)B->rows);
    if (A->rows > INT32_MAX) return fail(h, SPG_ERR_ARG, "A has more than 2^31-1 rows");
    HIP_TRY(h, hipSetDevice(h->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const CsrView a = view(A), b = view(B);
    const int64_t M = A->rows;
    Workspace ws;
    if ((rc = ensure_workspace(h, M, A->nnz, &ws))) return rc;

    HIP_TRY(h, launch_zero_ctl(h->ctl, s));
    if (h->validate) {
        HIP_TRY(h, launch_validate(a, A->cols, kErrRptA, kErrColA, h->ctl, s));
        HIP_TRY(h, launch_validate(b, B->cols, kErrRptB, kErrColB, h->ctl, s));
        HIP_TRY(h, hipMemcpyAsync(h->ctl_host, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        HIP_TRY(h, hipStreamSynchronize(s));
        if (h->ctl_host->err)
            return fail(h, SPG_ERR_INVALID_CSR, "invalid CSR input (error bits 0x%llx: 1/2 = A rpt/col, 4/8 = B rpt/col)",
                        (unsigned long long)h->ctl_host->err);
    }
    const bool learned = h->alloc == SPG_ALLOC_LEARNED;
    // the short-row kernels are fixed with the classification: the numeric
    // pass uses what this call chose
    int gr = (int)h->group_rows;
    // the register merges key columns in 26 bits
    if (uses_windows(gr) && B->cols >= ((int64_t)1 << 26)) gr = 0;
    h->plan_valid = false;
    h->plan_group_rows = gr;
    // the precise method's wave-small rows in register windows keep their merge order
    h->plan_order = false;
    if (!slotted && gr == 1 && h->stored_order && M > 0) {
        const size_t pb = align_up(64 * (size_t)M, 256);
        if ((rc = grow(h, &h->order_mem, &h->order_bytes, pb + 4 * 64 * (size_t)M, "window order"))) return rc;
        ws.order = static_cast<uint8_t *>(h->order_mem);
        ws.ucol = reinterpret_cast<int32_t *>(static_cast<char *>(h->order_mem) + pb);
        h->plan_order = true;
    }
    if (learned && !h->mlp_ready) return fail(h, SPG_ERR_NOT_TRAINED, "learned allocation needs a trained or loaded predictor");
    h->heavy_batches = 0;
    h->heavy_wide = 0;
    h->heavy_split_rows = 0;
    h->pred_total = h->ovf_light = h->ovf_heavy = 0;
    LearnedWs lw;
    RowFeatures rf{};
    if (slotted && (rc = ensure_learned_ws(h, M, &lw, learned ? B->rows : 0))) return rc;
    if (learned) {
        HIP_TRY(h, launch_row_ends(b, lw.b_ends, s));
        rf.b_ends = lw.b_ends;
        rf.feats = lw.feats;
        rf.lo = lw.lo;
        rf.hi = lw.hi;
        rf.predicted = lw.predicted;
        rf.ncols = B->cols;
    }
    if (M > 0) {
        const int g = (int)std::min<int64_t>((M + 255) / 256, 2048);
        // the learned allocation takes the predictor's features from the same pass
        // multi-register windows key columns in 21 bits
        const Thresholds th = thresholds(h, uses_windows(gr), B->cols <= ((int64_t)1 << 21));
        HIP_TRY(h, launch_analysis(a, b, th, ws, g, s, learned ? &rf : nullptr));
        HIP_TRY(h, launch_bin(M, ws, g, s));
        if (!slotted) {
            HIP_TRY(h, launch_symbolic(a, b, ws, kClassWaveSmall, persistent_grid(h, kClassWaveSmall, -1, gr), s, gr));
            // the multi-register, wave and group classes share one launch
            HIP_TRY(h, launch_symbolic_mid(a, b, ws, persistent_grid(h, kClassMulti, -1, gr),
                                           persistent_grid(h, kClassWave, -1, gr),
                                           persistent_grid(h, kClassGroup, -1, gr), s));
            // so do the block class and the heavy rows
            HIP_TRY(h, launch_symbolic_big(a, b, ws, persistent_grid(h, kClassBlock, -1, gr),
                                           persistent_grid(h, kClassHeavy, -1, gr), s));
        }
    }
    if (slotted) {
        // predicted sizes (or the product counts, an upper bound) -> slots;
        // numeric into the slots (exact lengths and overflowing rows
        // recorded); exact row pointers from the lengths
        HIP_TRY(h, launch_zero_ctl(h->ctl2, s));
        if (learned)
            HIP_TRY(h, launch_mlp_sizes(M, lw.feats, lw.predicted, lw.lo, lw.hi, ws.row_nprod, h->mlp,
                                        h->mlp + kMlpOffNorm, h->delta, (int)h->learned_force, h->block_max,
                                        (float)h->heavy_margin_milli / 1000.0f, lw.pred_size, s));
        else
            HIP_TRY(h, launch_upper_sizes(M, ws.row_nprod, lw.pred_size, s));
        HIP_TRY(h, launch_scan(M, lw.pred_size, ws.tile_sum, lw.slot_off, &h->ctl->pred_total, s, h->ctl,
                               h->ctl_host_dev));
        if (!h->ctl_host_dev) HIP_TRY(h, hipMemcpyAsync(h->ctl_host, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        HIP_TRY(h, hipStreamSynchronize(s));
        if (h->ctl_host->err & kErrRowProducts) return fail_row_products(h);
        for (int i = 0; i < 8; ++i) h->counts[i] = h->ctl_host->count[i];
        h->pred_total = h->ctl_host->pred_total;
        const size_t pt = (size_t)std::max<int64_t>(h->pred_total, 1);
        if ((rc = grow(h, &h->slot_mem, &h->slot_bytes, align_up(4 * pt, 256) + 8 * pt, "predicted slots")))
            return rc;
        int32_t *s_col = static_cast<int32_t *>(h->slot_mem);
        double *s_val = reinterpret_cast<double *>(static_cast<char *>(h->slot_mem) + align_up(4 * pt, 256));
        NumOut no;
        no.bound = 1;
        no.row_size = ws.row_size;
        no.ovf_rows = lw.ovf_rows;
        no.M = M;
        for (int cls : kLightClasses) {
            if (h->counts[cls] == 0) continue;
            HIP_TRY(h, launch_numeric(a, b, ws, cls, persistent_grid(h, cls, h->counts[cls], gr), lw.slot_off, s_col,
                                      s_val, no, s, gr));
        }
        if (h->counts[kClassHeavy] > 0) {
            int64_t first = 0;
            for (int c = 0; c < kClassHeavy; ++c) first += h->counts[c];
            if ((rc = run_heavy(h, a, b, ws, ws.class_rows + first, h->counts[kClassHeavy], lw.slot_off, s_col,
                                s_val, no, h->ctl, s)))
                return rc;
        }
    }
    HIP_TRY(h, launch_scan(M, ws.row_size, ws.tile_sum, c_rpt, &h->ctl->nnz, s, h->ctl, h->ctl_host_dev));
    if (!h->ctl_host_dev) HIP_TRY(h, hipMemcpyAsync(h->ctl_host, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    const Ctl &c = *h->ctl_host;
    if (c.err & kErrRowProducts) return fail_row_products(h);
    for (int i = 0; i < 8; ++i) h->counts[i] = c.count[i];
    h->nnz = c.nnz;
    h->nprod = c.nprod;
    h->ovf_light = c.ovf_light;
    h->ovf_heavy = c.ovf_heavy;
    *c_nnz = c.nnz;
    h->plan_valid = true;
    h->plan_learned = slotted;
    h->pa_rpt = A->rpt;
    h->pb_rpt = B->rpt;
    h->pa_col = A->col;
    h->pb_col = B->col;
    h->pM = A->rows;
    h->pK = A->cols;
    h->pN = B->cols;
    h->pnnzA = A->nnz;
    h->pnnzB = B->nnz;
    return SPG_OK;
}

int spgemm_row_products(spg_handle h, const spg_csr *A, const spg_csr *B, int64_t *row_nprod, void *stream) {
    if (!h) return SPG_ERR_ARG;
    h->err.clear();
    int rc;
    if ((rc = check_csr(h, A, "A", false)) || (rc = check_csr(h, B, "B", false))) return rc;
    if (A->rows > 0 && !row_nprod) return fail(h, SPG_ERR_ARG, "row_nprod is NULL");
    if (A->cols != B->rows)
        return fail(h, SPG_ERR_DIM, "A is %lld x %lld but B has %lld rows", (long long)A->rows,
                    (long long)A->cols, (long long)B->rows);
    if (A->rows > INT32_MAX) return fail(h, SPG_ERR_ARG, "A has more than 2^31-1 rows");
    HIP_TRY(h, hipSetDevice(h->device));
    // the analysis reuses the workspace of the last plan
    h->plan_valid = false;
    const int64_t M = A->rows;
    if (M == 0) return SPG_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace ws;
    if ((rc = ensure_workspace(h, M, A->nnz, &ws))) return rc;
    HIP_TRY(h, launch_zero_ctl(h->ctl, s));
    const int g = (int)std::min<int64_t>((M + 255) / 256, 2048);
    HIP_TRY(h, launch_analysis(view(A), view(B), thresholds(h, false), ws, g, s));
    HIP_TRY(h, hipMemcpyAsync(row_nprod, ws.row_nprod, sizeof(int64_t) * (size_t)M, hipMemcpyDeviceToDevice, s));
    return SPG_OK;
}

int spgemm_numeric(spg_handle h, const spg_csr *A, const spg_csr *B, const int64_t *c_rpt,
                   int32_t *c_col, double *c_val, void *stream) {
    if (!h) return SPG_ERR_ARG;
    h->err.clear();
    int rc;
    if ((rc = check_csr(h, A, "A", true)) || (rc = check_csr(h, B, "B", true))) return rc;
    if (!h->plan_valid || A->rpt != h->pa_rpt || B->rpt != h->pb_rpt || A->col != h->pa_col ||
        B->col != h->pb_col || A->rows != h->pM || A->cols != h->pK || B->cols != h->pN ||
        A->nnz != h->pnnzA || B->nnz != h->pnnzB)
        return fail(h, SPG_ERR_STATE, "spgemm_numeric needs a preceding spgemm_symbolic on the same A and B");
    if (!c_rpt || (h->nnz > 0 && (!c_col || !c_val))) return fail(h, SPG_ERR_ARG, "C arrays are NULL");
    HIP_TRY(h, hipSetDevice(h->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const CsrView a = view(A), b = view(B);
    Workspace ws;
    if ((rc = ensure_workspace(h, A->rows, A->nnz, &ws))) return rc;
    if (h->plan_order && !h->plan_learned) {
        ws.order = static_cast<uint8_t *>(h->order_mem);
        ws.ucol = reinterpret_cast<int32_t *>(static_cast<char *>(h->order_mem) +
                                              align_up(64 * (size_t)A->rows, 256));
    }
    h->heavy_batches = 0;
    h->heavy_wide = 0;
    h->heavy_split_rows = 0;
    NumOut exact;
    exact.bound = 0;
    exact.row_size = nullptr;
    exact.ovf_rows = nullptr;
    exact.M = A->rows;
    if (h->plan_learned) {
        // exact fallback for the rows that overflowed their slot, then the
        // other rows move from their slots to C
        const int64_t M = A->rows;
        LearnedWs lw;
        if ((rc = ensure_learned_ws(h, M, &lw))) return rc;
        if (h->ovf_light + h->ovf_heavy > 0) {
            // the light rows that overflowed go, by class, to their kernels
            // (the class lists of the symbolic pass are free by now)
            HIP_TRY(h, launch_fallback_ctl(h->ctl, h->ctl2, M, s));
            Workspace ws2 = ws;
            ws2.ctl = h->ctl2;
            if (h->ovf_light > 0) {
                HIP_TRY(h, launch_bin_list(h->ovf_light, lw.ovf_rows + (M - h->ovf_light), ws.row_class,
                                           ws.class_rows, h->ctl2, s));
                for (int cls : kLightClasses)
                    HIP_TRY(h, launch_numeric(a, b, ws2, cls, persistent_grid(h, cls, h->ovf_light, h->plan_group_rows),
                                              c_rpt, c_col, c_val, exact, s, h->plan_group_rows));
            }
            if (h->ovf_heavy > 0 &&
                (rc = run_heavy(h, a, b, ws, lw.ovf_rows + M, h->ovf_heavy, c_rpt, c_col, c_val, exact, h->ctl2, s)))
                return rc;
        }
        const size_t pt = (size_t)std::max<int64_t>(h->pred_total, 1);
        const int32_t *s_col = static_cast<const int32_t *>(h->slot_mem);
        const double *s_val =
            reinterpret_cast<const double *>(static_cast<const char *>(h->slot_mem) + align_up(4 * pt, 256));
        HIP_TRY(h, launch_compact(M, lw.slot_off, ws.row_size, c_rpt, s_col, s_val, c_col, c_val,
                                  (int)std::min<int64_t>((M + 3) / 4, (int64_t)h->num_cu * 8), s));
        return SPG_OK;
    }
    for (int cls : kLightClasses) {
        if (h->counts[cls] == 0) continue;
        if (h->accumulator == SPG_ACC_HASH && cls != kClassCopy) {
            HIP_TRY(h, launch_numeric_hash(a, b, ws, cls, h->num_cu, c_rpt, c_col, c_val, s));
            continue;
        }
        HIP_TRY(h, launch_numeric(a, b, ws, cls, persistent_grid(h, cls, h->counts[cls], h->plan_group_rows), c_rpt,
                                  c_col, c_val, exact, s, h->plan_group_rows));
    }
    if (h->counts[kClassHeavy] > 0) {
        int64_t first = 0;
        for (int c = 0; c < kClassHeavy; ++c) first += h->counts[c];
        return run_heavy(h, a, b, ws, ws.class_rows + first, h->counts[kClassHeavy], c_rpt, c_col, c_val, exact,
                         h->ctl, s);
    }
    return SPG_OK;
}

// ---- learned size predictor ------------------------------------------------

int spg_mlp_set_params(spg_handle h, const float *params, const float *norm, float delta) {
    if (!h || !params || !norm) return h ? fail(h, SPG_ERR_ARG, "params / norm is NULL") : SPG_ERR_ARG;
    for (int j = 0; j < 6; ++j)
        if (!(norm[6 + j] > 0.0f)) return fail(h, SPG_ERR_ARG, "feature standard deviations must be positive");
    HIP_TRY(h, hipSetDevice(h->device));
    int rc;
    if ((rc = ensure_mlp(h))) return rc;
    HIP_TRY(h, hipMemcpy(h->mlp, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(h->mlp + kMlpOffNorm, norm, sizeof(float) * 12, hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemset(h->mlp + kMlpOffM, 0, sizeof(float) * 2 * kMlpParams));
    h->adam_t = 0;
    h->delta = delta;
    h->mlp_ready = true;
    return SPG_OK;
}

int spg_mlp_get_params(spg_handle h, float *params, float *norm, float *delta) {
    if (!h) return SPG_ERR_ARG;
    if (!h->mlp) return fail(h, SPG_ERR_NOT_TRAINED, "no predictor parameters");
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, hipDeviceSynchronize());
    if (params) HIP_TRY(h, hipMemcpy(params, h->mlp, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    if (norm) HIP_TRY(h, hipMemcpy(norm, h->mlp + kMlpOffNorm, sizeof(float) * 12, hipMemcpyDeviceToHost));
    if (delta) *delta = h->delta;
    return SPG_OK;
}

int spg_mlp_features(spg_handle h, const spg_csr *A, const spg_csr *B, const int64_t *c_rpt, float *feats,
                     float *targets, int8_t *predicted, int32_t *lo, int32_t *hi, void *stream) {
    if (!h) return SPG_ERR_ARG;
    int rc;
    if ((rc = check_csr(h, A, "A", false)) || (rc = check_csr(h, B, "B", false))) return rc;
    if (A->cols != B->rows) return fail(h, SPG_ERR_DIM, "inner dimensions differ");
    if (!feats || !predicted || (targets && !c_rpt)) return fail(h, SPG_ERR_ARG, "feats / predicted / c_rpt is NULL");
    HIP_TRY(h, hipSetDevice(h->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const CsrView a = view(A), b = view(B);
    std::vector<int32_t> dummy;
    int32_t *lo_p = lo, *hi_p = hi;
    void *tmp = nullptr;
    if (!lo || !hi) {
        if (hipMalloc(&tmp, 8 * (size_t)std::max<int64_t>(A->rows, 1)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(h, SPG_ERR_NOMEM, "bound buffers");
        }
        lo_p = static_cast<int32_t *>(tmp);
        hi_p = lo_p + std::max<int64_t>(A->rows, 1);
    }
    hipError_t e = launch_features(a, b, feats, lo_p, hi_p, predicted, c_rpt, targets, s);
    if (tmp) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(tmp);
    }
    if (e != hipSuccess) return fail(h, SPG_ERR_HIP, "features: %s", hipGetErrorString(e));
    return SPG_OK;
}

int spg_mlp_forward(spg_handle h, const float *feats, int64_t n, float *y, void *stream) {
    if (!h || n < 0 || (n > 0 && (!feats || !y))) return h ? fail(h, SPG_ERR_ARG, "bad forward arguments") : SPG_ERR_ARG;
    if (!h->mlp_ready) return fail(h, SPG_ERR_NOT_TRAINED, "no predictor parameters");
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, launch_mlp_forward(n, feats, h->mlp, h->mlp + kMlpOffNorm, y, static_cast<hipStream_t>(stream)));
    return SPG_OK;
}

int spg_mlp_gradient(spg_handle h, const float *feats, const float *targets, int64_t n, float *grad, float *loss,
                     void *stream) {
    if (!h || n <= 0 || !feats || !targets || !grad) return h ? fail(h, SPG_ERR_ARG, "bad gradient arguments") : SPG_ERR_ARG;
    if (!h->mlp_ready) return fail(h, SPG_ERR_NOT_TRAINED, "no predictor parameters");
    HIP_TRY(h, hipSetDevice(h->device));
    int rc;
    if ((rc = ensure_mlp_act(h, n))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(h, launch_mlp_gradient(n, feats, targets, h->mlp, h->mlp + kMlpOffNorm, h->mlp_act,
                                   h->mlp + kMlpOffPartial, grad, h->mlp + kMlpOffLoss, s));
    if (loss) {
        HIP_TRY(h, hipMemcpyAsync(loss, h->mlp + kMlpOffLoss, sizeof(float), hipMemcpyDeviceToHost, s));
        HIP_TRY(h, hipStreamSynchronize(s));
    }
    return SPG_OK;
}

int spg_mlp_fit_normalization(spg_handle h, const float *feats, int64_t n, void *stream) {
    if (!h || n <= 0 || !feats) return h ? fail(h, SPG_ERR_ARG, "bad normalization arguments") : SPG_ERR_ARG;
    if (!h->mlp_ready) return fail(h, SPG_ERR_NOT_TRAINED, "set initial parameters first");
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, launch_feature_stats(n, feats, h->mlp + kMlpOffNorm, static_cast<hipStream_t>(stream)));
    return SPG_OK;
}

int spg_mlp_train(spg_handle h, const float *feats, const float *targets, int64_t n, int epochs, int batch,
                  float lr, void *stream) {
    if (!h || n <= 0 || !feats || !targets || epochs < 0 || batch <= 0 || !(lr > 0.0f))
        return h ? fail(h, SPG_ERR_ARG, "bad training arguments") : SPG_ERR_ARG;
    if (!h->mlp_ready) return fail(h, SPG_ERR_NOT_TRAINED, "set initial parameters first");
    HIP_TRY(h, hipSetDevice(h->device));
    int rc;
    if ((rc = ensure_mlp_act(h, batch))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    float *grad = h->mlp + kMlpOffG;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int64_t b0 = 0; b0 < n; b0 += batch) {
            const int64_t nb = std::min<int64_t>(batch, n - b0);
            HIP_TRY(h, launch_mlp_gradient(nb, feats + 6 * b0, targets + b0, h->mlp, h->mlp + kMlpOffNorm,
                                           h->mlp_act, h->mlp + kMlpOffPartial, grad, nullptr, s));
            ++h->adam_t;
            HIP_TRY(h, launch_adam(h->mlp, grad, h->mlp + kMlpOffM, h->mlp + kMlpOffV, h->adam_t, lr, s));
        }
    }
    return SPG_OK;
}

int spg_mlp_loss(spg_handle h, const float *feats, const float *targets, int64_t n, float *loss, void *stream) {
    if (!h || n <= 0 || !feats || !targets || !loss) return h ? fail(h, SPG_ERR_ARG, "bad loss arguments") : SPG_ERR_ARG;
    if (!h->mlp_ready) return fail(h, SPG_ERR_NOT_TRAINED, "no predictor parameters");
    HIP_TRY(h, hipSetDevice(h->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    float *y = nullptr;
    if (hipMalloc(&y, sizeof(float) * (size_t)n) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, SPG_ERR_NOMEM, "loss buffer");
    }
    hipError_t e = launch_mlp_forward(n, feats, h->mlp, h->mlp + kMlpOffNorm, y, s);
    if (e == hipSuccess) e = launch_mse(n, y, targets, h->mlp + kMlpOffLoss, s);
    if (e == hipSuccess) e = hipMemcpyAsync(loss, h->mlp + kMlpOffLoss, sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(y);
    if (e != hipSuccess) return fail(h, SPG_ERR_HIP, "loss: %s", hipGetErrorString(e));
    return SPG_OK;
}

int spg_mlp_calibrate(spg_handle h, const float *feats, const float *targets, int64_t n, double quantile,
                      float *delta, void *stream) {
    if (!h || n <= 0 || !feats || !targets || !(quantile >= 0.0 && quantile <= 1.0))
        return h ? fail(h, SPG_ERR_ARG, "bad calibration arguments") : SPG_ERR_ARG;
    if (!h->mlp_ready) return fail(h, SPG_ERR_NOT_TRAINED, "no predictor parameters");
    HIP_TRY(h, hipSetDevice(h->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    float *y = nullptr;
    if (hipMalloc(&y, sizeof(float) * (size_t)n) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, SPG_ERR_NOMEM, "calibration buffer");
    }
    std::vector<float> hy((size_t)n), ht((size_t)n);
    hipError_t e = launch_mlp_forward(n, feats, h->mlp, h->mlp + kMlpOffNorm, y, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hy.data(), y, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ht.data(), targets, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(y);
    if (e != hipSuccess) return fail(h, SPG_ERR_HIP, "calibration: %s", hipGetErrorString(e));
    // margin: the `quantile` quantile of (target - prediction)
    std::vector<float> r((size_t)n);
    for (size_t i = 0; i < (size_t)n; ++i) r[i] = ht[i] - hy[i];
    size_t k = (size_t)std::min<double>((double)(n - 1), std::ceil(quantile * (double)n) - 1.0 < 0 ? 0.0
                                                                   : std::ceil(quantile * (double)n) - 1.0);
    std::nth_element(r.begin(), r.begin() + (long)k, r.end());
    h->delta = std::max(0.0f, r[k]);
    if (delta) *delta = h->delta;
    return SPG_OK;
}

int spg_mlp_save(spg_handle h, const char *path) {
    if (!h || !path) return SPG_ERR_ARG;
    if (!h->mlp_ready) return fail(h, SPG_ERR_NOT_TRAINED, "no predictor parameters");
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, hipDeviceSynchronize());
    std::vector<float> buf(3 * kMlpParams + 12);
    HIP_TRY(h, hipMemcpy(buf.data(), h->mlp, sizeof(float) * 3 * kMlpParams, hipMemcpyDeviceToHost));
    HIP_TRY(h, hipMemcpy(buf.data() + 3 * kMlpParams, h->mlp + kMlpOffNorm, 48, hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(h, SPG_ERR_ARG, "cannot open %s", path);
    const char magic[8] = {'B', 'R', 'M', 'M', 'L', 'P', '0', '1'};
    const int64_t t = h->adam_t;
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&t, 8, 1, f) == 1 &&
              std::fwrite(&h->delta, 4, 1, f) == 1 && std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? SPG_OK : fail(h, SPG_ERR_ARG, "write to %s failed", path);
}

int spg_mlp_load(spg_handle h, const char *path) {
    if (!h || !path) return SPG_ERR_ARG;
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(h, SPG_ERR_ARG, "cannot open %s", path);
    char magic[8];
    int64_t t = 0;
    float delta = 0.0f;
    std::vector<float> buf(3 * kMlpParams + 12);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "BRMMLP01", 8) == 0 &&
              std::fread(&t, 8, 1, f) == 1 && std::fread(&delta, 4, 1, f) == 1 &&
              std::fread(buf.data(), 4, buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) return fail(h, SPG_ERR_ARG, "%s is not a predictor checkpoint", path);
    HIP_TRY(h, hipSetDevice(h->device));
    int rc;
    if ((rc = ensure_mlp(h))) return rc;
    HIP_TRY(h, hipMemcpy(h->mlp, buf.data(), sizeof(float) * 3 * kMlpParams, hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(h->mlp + kMlpOffNorm, buf.data() + 3 * kMlpParams, 48, hipMemcpyHostToDevice));
    h->adam_t = t;
    h->delta = delta;
    h->mlp_ready = true;
    return SPG_OK;
}

// ---- batched products ------------------------------------------------------

}  // extern "C"

namespace {

// What both batched entry points derive on the host from the problems: the
// stages (problems grouped by their dependencies), the arena's row-pointer
// section, and the byte layout of the stage workspace.
struct BatchedPlan {
    struct Stage { int first, n; int64_t rows, ents; int arb, brb; bool link; size_t roff; bool keep; };
    std::vector<Stage> st;
    std::vector<int64_t> ccols, rpt_off, stage_chunks;
    size_t roff_total = 0;
    int64_t rpt_end = 0, max_bcols = 0;
    // workspace layout: rows | S | row offsets | table | status | ctl | row problems | list descriptors
    size_t o_nprod, o_class, o_size, o_rows, o_tile, o_S, o_roff, o_tab, o_stat, o_ctl, o_prob, o_ebs, o_elen,
        o_S2, o_ovf, total;
    bool upper = false;  // upper-bound slots (o_S2, o_ovf used)
};

int plan_batched(spg_handle h, int count, const spg_problem *probs, void *arena, int64_t arena_bytes,
                 spg_batched_out *out, int64_t *required_bytes, BatchedPlan *pl) {
    if (count < 0 || (count > 0 && (!probs || !arena || !out)) || !required_bytes || arena_bytes < 0)
        return fail(h, SPG_ERR_ARG, "bad batched arguments");
    *required_bytes = 0;
    if (count == 0) return SPG_OK;
    if (reinterpret_cast<uintptr_t>(arena) % 256) return fail(h, SPG_ERR_ARG, "arena must be 256-byte aligned");
    int rc;
    // stages from the dependencies; problems must come in stage order
    std::vector<int> stage((size_t)count, 0);
    std::vector<int64_t> crows((size_t)count);
    pl->ccols.assign((size_t)count, 0);
    for (int p = 0; p < count; ++p) {
        const spg_problem &q = probs[p];
        if ((rc = check_csr(h, &q.A, "A", true))) return rc;
        if (q.flags & ~(int32_t)SPG_PROBLEM_OPERAND_ONLY) return fail(h, SPG_ERR_ARG, "problem %d: unknown flags", p);
        int64_t brows, bcols;
        if (q.b_from >= 0) {
            if (q.b_from >= p) return fail(h, SPG_ERR_ARG, "problem %d: b_from must name an earlier problem", p);
            stage[(size_t)p] = stage[(size_t)q.b_from] + 1;
            brows = crows[(size_t)q.b_from];
            bcols = pl->ccols[(size_t)q.b_from];
        } else {
            if ((rc = check_csr(h, &q.B, "B", true))) return rc;
            brows = q.B.rows;
            bcols = q.B.cols;
        }
        if (q.A.cols != brows) return fail(h, SPG_ERR_DIM, "problem %d: A.cols != B.rows", p);
        if (p > 0 && stage[(size_t)p] < stage[(size_t)p - 1])
            return fail(h, SPG_ERR_ARG, "problems must be ordered by stage (problem %d)", p);
        crows[(size_t)p] = q.A.rows;
        pl->ccols[(size_t)p] = bcols;
    }
    // stage ranges, row offsets, widths
    pl->st.clear();
    pl->roff_total = 0;
    for (int p = 0; p < count;) {
        int q = p;
        BatchedPlan::Stage si{p, 0, 0, 0, probs[p].A.rpt_bytes, probs[p].b_from >= 0 ? 8 : probs[p].B.rpt_bytes,
                              false, pl->roff_total, false};
        // a stage keeps its upper-bound slots when every problem of it is an operand only
        bool all_operands = h->batch_alloc == SPG_BATCH_UPPER;
        while (q < count && stage[(size_t)q] == stage[(size_t)p]) {
            const int brb = probs[q].b_from >= 0 ? 8 : probs[q].B.rpt_bytes;
            if (probs[q].A.rpt_bytes != si.arb || brb != si.brb)
                return fail(h, SPG_ERR_ARG, "problems of one stage must share row-pointer widths (problem %d)", q);
            si.rows += probs[q].A.rows;
            si.ents += probs[q].A.nnz;
            si.link = si.link || probs[q].b_from >= 0;
            all_operands = all_operands && (probs[q].flags & SPG_PROBLEM_OPERAND_ONLY);
            ++q;
        }
        si.n = q - p;
        si.keep = all_operands;
        pl->roff_total += (size_t)si.n + 1;
        pl->st.push_back(si);
        p = q;
    }
    int64_t max_rows = 0, max_ents = 0;
    for (auto &x : pl->st) {
        max_rows = std::max(max_rows, x.rows);
        max_ents = std::max(max_ents, x.ents);
    }
    pl->max_bcols = 0;
    for (int p = 0; p < count; ++p) pl->max_bcols = std::max(pl->max_bcols, pl->ccols[(size_t)p]);
    if (max_rows > INT32_MAX) return fail(h, SPG_ERR_ARG, "too many rows in one stage");
    // arena: row pointers first (sizes known now), then C's columns and values;
    // a problem of a stage that keeps its slots takes the starts and the ends of its rows
    pl->rpt_end = 0;
    pl->rpt_off.assign((size_t)count, 0);
    std::vector<char> kept((size_t)count, 0);
    for (const auto &x : pl->st)
        for (int i = 0; i < x.n; ++i) kept[(size_t)(x.first + i)] = x.keep ? 1 : 0;
    for (int p = 0; p < count; ++p) {
        pl->rpt_off[(size_t)p] = pl->rpt_end;
        pl->rpt_end += (int64_t)align_up((kept[(size_t)p] ? 16 : 8) * (size_t)(crows[(size_t)p] + 1), 256);
    }
    if (pl->rpt_end > arena_bytes) {
        *required_bytes = pl->rpt_end;
        return fail(h, SPG_ERR_CAPACITY, "arena smaller than the row pointers alone (%lld bytes)",
                    (long long)pl->rpt_end);
    }
    const size_t a = 256;
    pl->o_nprod = 0;
    pl->o_class = align_up(pl->o_nprod + 8 * (size_t)max_rows, a);
    pl->o_size = align_up(pl->o_class + (size_t)max_rows, a);
    pl->o_rows = align_up(pl->o_size + 4 * (size_t)max_rows, a);
    pl->o_tile = align_up(pl->o_rows + 4 * (size_t)max_rows, a);
    pl->o_S = align_up(pl->o_tile + 8 * (size_t)((max_rows + kScanTile - 1) / kScanTile + 1), a);
    pl->o_roff = align_up(pl->o_S + 8 * (size_t)(max_rows + 1), a);
    pl->o_tab = align_up(pl->o_roff + 16 * pl->roff_total, a);  // row offsets, then chunk offsets
    pl->o_stat = align_up(pl->o_tab + sizeof(BatchProb) * (size_t)count, a);
    pl->o_ctl = align_up(pl->o_stat + sizeof(BatchStatus), a);
    // the window kernels' inputs: the problem of every row, list descriptors
    pl->o_prob = align_up(pl->o_ctl + sizeof(Ctl), a);
    // upper-bound slots: their offsets and the (never filled) overflow list
    pl->upper = h->batch_alloc == SPG_BATCH_UPPER;
    const size_t ub = pl->upper ? 1 : 0;
    pl->o_ebs = align_up(pl->o_prob + 4 * (size_t)max_rows, a);
    pl->o_elen = align_up(pl->o_ebs + 8 * (size_t)max_ents, a);
    pl->o_S2 = align_up(pl->o_elen + 4 * (size_t)max_ents, a);
    pl->o_ovf = align_up(pl->o_S2 + ub * 8 * (size_t)(max_rows + 1), a);
    pl->total = align_up(pl->o_ovf + ub * 8 * (size_t)max_rows, a);
    return SPG_OK;
}

// The problem table and the row / chunk offsets of every stage, written
// into host buffers (tab[count], roff[2 * roff_total]).
void fill_batched_tables(const BatchedPlan &pl, const spg_problem *probs, char *arena_c, BatchProb *tab,
                         int64_t *roff, std::vector<int64_t> *stage_chunks) {
    stage_chunks->assign(pl.st.size(), 0);
    for (size_t si = 0; si < pl.st.size(); ++si) {
        const auto &x = pl.st[si];
        int64_t ro = 0, eo = 0, co = 0;
        for (int i = 0; i < x.n; ++i) {
            const int p = x.first + i;
            const spg_problem &q = probs[p];
            BatchProb &b = tab[p];
            std::memset(&b, 0, sizeof b);
            b.row_off = ro;
            b.rows = q.A.rows;
            b.ncols_b = pl.ccols[(size_t)p];
            b.a_rpt = q.A.rpt;
            b.a_col = q.A.col;
            b.a_val = q.A.val;
            if (q.b_from < 0) {
                b.b_rpt = q.B.rpt;
                b.b_col = q.B.col;
                b.b_val = q.B.val;
            }
            b.c_rpt = reinterpret_cast<int64_t *>(arena_c + pl.rpt_off[(size_t)p]);
            b.rpt_off = pl.rpt_off[(size_t)p];
            b.b_from = q.b_from;
            b.ent_off = eo;
            roff[x.roff + (size_t)i] = ro;
            roff[pl.roff_total + x.roff + (size_t)i] = co;
            ro += q.A.rows;
            eo += q.A.nnz;
            co += (q.A.rows + kBatchChunkRows - 1) / kBatchChunkRows;
        }
        roff[x.roff + (size_t)x.n] = ro;
        roff[pl.roff_total + x.roff + (size_t)x.n] = co;
        (*stage_chunks)[si] = co;
    }
}

Workspace batched_workspace(const BatchedPlan &pl, char *base) {
    Workspace ws;
    ws.row_nprod = reinterpret_cast<int64_t *>(base + pl.o_nprod);
    ws.row_class = reinterpret_cast<uint8_t *>(base + pl.o_class);
    ws.row_size = reinterpret_cast<int32_t *>(base + pl.o_size);
    ws.class_rows = reinterpret_cast<int32_t *>(base + pl.o_rows);
    ws.tile_sum = reinterpret_cast<int64_t *>(base + pl.o_tile);
    ws.ctl = reinterpret_cast<Ctl *>(base + pl.o_ctl);
    ws.row_prob = reinterpret_cast<int32_t *>(base + pl.o_prob);
    ws.ent_bs = base + pl.o_ebs;
    ws.ent_len = reinterpret_cast<int32_t *>(base + pl.o_elen);
    return ws;
}

// The launch sequence of a whole batch: status cleared, then every stage.
hipError_t launch_batched_all(spg_handle h, const BatchedPlan &pl, const std::vector<int64_t> &stage_chunks,
                              char *base, char *arena_c, int64_t arena_bytes, hipStream_t s) {
    const Workspace ws = batched_workspace(pl, base);
    int64_t *d_S = reinterpret_cast<int64_t *>(base + pl.o_S);
    int64_t *d_roff = reinterpret_cast<int64_t *>(base + pl.o_roff);
    BatchProb *d_tab = reinterpret_cast<BatchProb *>(base + pl.o_tab);
    BatchStatus *d_stat = reinterpret_cast<BatchStatus *>(base + pl.o_stat);
    hipError_t e = launch_batched_begin(d_stat, ws.ctl, s);
    // lane windows as in the single product (their keys bound B's columns)
    const bool win = uses_windows(h->group_rows) && pl.max_bcols < ((int64_t)1 << 26);
    const Thresholds th = thresholds(h, win, pl.max_bcols <= ((int64_t)1 << 21));
    for (size_t si = 0; si < pl.st.size() && e == hipSuccess; ++si) {
        const auto &x = pl.st[si];
        BatchStage bs;
        bs.all = d_tab;
        bs.tab = d_tab + x.first;
        bs.first = x.first;
        bs.nprob = x.n;
        bs.row_off = d_roff + x.roff;
        bs.chunk_off = d_roff + pl.roff_total + x.roff;
        bs.chunks = stage_chunks[si];
        bs.rows = x.rows;
        bs.a_rpt_bytes = x.arb;
        bs.b_rpt_bytes = x.brb;
        bs.link = x.link ? 1 : 0;
        bs.S = d_S;
        bs.arena = arena_c;
        bs.arena_bytes = arena_bytes;
        bs.data_off = pl.rpt_end;
        bs.status = d_stat;
        bs.heavy_lds_cap = (int)std::min<int64_t>(h->heavy_lds_max, 4 * (int64_t)kBatchHeavyThreads);
        bs.upper = pl.upper ? 1 : 0;
        bs.S2 = pl.upper ? reinterpret_cast<int64_t *>(base + pl.o_S2) : nullptr;
        bs.ovf = pl.upper ? reinterpret_cast<int32_t *>(base + pl.o_ovf) : nullptr;
        bs.keep = x.keep ? 1 : 0;
        e = launch_batched_stage(bs, ws, th, h->num_cu, h->grid_waves, s);
    }
    return e;
}

// The call's result from the batch status read back after the batch.
int finish_batched(spg_handle h, const BatchStatus &bst, const Ctl &ctl, const BatchedPlan &pl,
                   int64_t *required_bytes) {
    h->nprod = bst.nprod;
    for (int i = 0; i < kNumClasses; ++i) h->counts[i] = ctl.count[i];  // the last stage's rows
    h->b_err = bst.err | ctl.err;
    if (bst.flags & kBatchRowProducts) {
        *required_bytes = -1;
        return fail(h, SPG_ERR_CAPACITY, "a row has 2^31 or more products");
    }
    *required_bytes = std::max<int64_t>(bst.required, pl.rpt_end);
    if (bst.flags & kBatchOverflow)
        return fail(h, SPG_ERR_CAPACITY, "arena too small: %lld bytes needed", (long long)*required_bytes);
    return SPG_OK;
}

}  // namespace

extern "C" {

int spgemm_batched(spg_handle h, int count, const spg_problem *probs, void *arena, int64_t arena_bytes,
                   spg_batched_out *out, int64_t *required_bytes, void *stream) {
    if (!h) return SPG_ERR_ARG;
    h->err.clear();
    h->b_err = 0;
    BatchedPlan pl;
    int rc;
    if ((rc = plan_batched(h, count, probs, arena, arena_bytes, out, required_bytes, &pl))) return rc;
    if (count == 0) return SPG_OK;
    HIP_TRY(h, hipSetDevice(h->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    bool realloc = false;
    if (pl.total > h->b_bytes) {
        if (h->graph_exec) {
            HIP_TRY(h, hipStreamSynchronize(s));
            (void)hipGraphExecDestroy(h->graph_exec);
            h->graph_exec = nullptr;
        }
        if ((rc = grow(h, &h->b_mem, &h->b_bytes, pl.total, "batched workspace"))) return rc;
        realloc = true;
    }
    if ((size_t)count > h->b_host_n) {
        if (h->b_host) HIP_TRY(h, hipHostFree(h->b_host));
        h->b_host = nullptr;
        HIP_TRY(h, hipHostMalloc(reinterpret_cast<void **>(&h->b_host), sizeof(BatchProb) * (size_t)count,
                                 hipHostMallocDefault));
        h->b_host_n = (size_t)count;
    }
    if (2 * pl.roff_total > h->b_row_off_n) {
        if (h->b_row_off_host) HIP_TRY(h, hipHostFree(h->b_row_off_host));
        h->b_row_off_host = nullptr;
        HIP_TRY(h, hipHostMalloc(reinterpret_cast<void **>(&h->b_row_off_host), 16 * pl.roff_total,
                                 hipHostMallocDefault));
        h->b_row_off_n = 2 * pl.roff_total;
    }
    if (!h->b_status_host)
        HIP_TRY(h, hipHostMalloc(reinterpret_cast<void **>(&h->b_status_host), sizeof(BatchStatus), hipHostMallocDefault));
    if (!h->cap_stream) HIP_TRY(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    char *base = static_cast<char *>(h->b_mem);
    char *arena_c = static_cast<char *>(arena);
    std::vector<int64_t> stage_chunks;
    fill_batched_tables(pl, probs, arena_c, h->b_host, h->b_row_off_host, &stage_chunks);
    BatchProb *d_tab = reinterpret_cast<BatchProb *>(base + pl.o_tab);
    BatchStatus *d_stat = reinterpret_cast<BatchStatus *>(base + pl.o_stat);
    HIP_TRY(h, hipMemcpyAsync(d_tab, h->b_host, sizeof(BatchProb) * (size_t)count, hipMemcpyHostToDevice, s));
    HIP_TRY(h, hipMemcpyAsync(base + pl.o_roff, h->b_row_off_host, 16 * pl.roff_total, hipMemcpyHostToDevice, s));
    // graph signature: problems, arena, outputs, options
    std::vector<int64_t> sig;
    sig.push_back(count);
    for (int p = 0; p < count; ++p) {
        const spg_problem &q = probs[p];
        for (int64_t v : {q.A.rows, q.A.cols, q.A.nnz, (int64_t)q.A.rpt_bytes, (int64_t)q.b_from, (int64_t)q.flags,
                          q.B.rows, q.B.cols, q.B.nnz, (int64_t)q.B.rpt_bytes})
            sig.push_back(v);
        for (const void *ptr : {q.A.rpt, (const void *)q.A.col, (const void *)q.A.val, q.B.rpt,
                                (const void *)q.B.col, (const void *)q.B.val})
            sig.push_back((int64_t)reinterpret_cast<uintptr_t>(ptr));
    }
    for (int64_t v : {(int64_t)reinterpret_cast<uintptr_t>(arena), arena_bytes, h->wave_small_max, h->wave_max,
                      h->group_max, h->group_rows,
                      h->block_max, h->force, h->grid_waves, h->heavy_lds_max, h->batch_alloc,
                      (int64_t)reinterpret_cast<uintptr_t>(h->b_mem)})
        sig.push_back(v);
    const bool replay = !realloc && h->graph_exec && sig == h->graph_sig;
    if (!replay && sig != h->seen_sig) {
        // a batch seen for the first time: its kernels are launched directly
        // (capturing and instantiating a graph pays off only when it is
        // replayed); the same batch in the next call is captured
        h->seen_sig = sig;
        ++h->batched_direct;
        HIP_TRY(h, launch_batched_all(h, pl, stage_chunks, base, arena_c, arena_bytes, s));
    } else if (!replay) {
        if (h->graph_exec) {
            HIP_TRY(h, hipStreamSynchronize(s));
            (void)hipGraphExecDestroy(h->graph_exec);
            h->graph_exec = nullptr;
        }
        hipStream_t cs = h->cap_stream;
        HIP_TRY(h, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        hipError_t e = launch_batched_all(h, pl, stage_chunks, base, arena_c, arena_bytes, cs);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(h, SPG_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
        }
        e = hipGraphInstantiateWithFlags(&h->graph_exec, graph, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            h->graph_exec = nullptr;
            return fail(h, SPG_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
        }
        h->graph_sig = sig;
        ++h->graph_captures;
        HIP_TRY(h, hipGraphLaunch(h->graph_exec, s));
    } else {
        ++h->graph_launches;
        HIP_TRY(h, hipGraphLaunch(h->graph_exec, s));
    }
    HIP_TRY(h, launch_batched_describe(d_tab, count, out, d_stat, s));
    HIP_TRY(h, hipMemcpyAsync(h->b_status_host, d_stat, sizeof(BatchStatus), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipMemcpyAsync(h->ctl_host, base + pl.o_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    return finish_batched(h, *h->b_status_host, *h->ctl_host, pl, required_bytes);
}

int spgemm_batched_noalloc(spg_handle h, int count, const spg_problem *probs, void *arena, int64_t arena_bytes,
                           spg_batched_out *out, int64_t *required_bytes, void *stream) {
    if (!h) return SPG_ERR_ARG;
    h->err.clear();
    h->b_err = 0;
    BatchedPlan pl;
    int rc;
    if ((rc = plan_batched(h, count, probs, arena, arena_bytes, out, required_bytes, &pl))) return rc;
    if (count == 0) return SPG_OK;
    if (!h->scratch)
        return fail(h, SPG_ERR_HIP, "the device address of the static scratch array is unknown (%s)",
                    h->scratch_err.c_str());
    if (pl.total > (size_t)kNoAllocScratchBytes)
        return fail(h, SPG_ERR_SCRATCH,
                    "this batch needs %zu bytes of workspace; the allocation-free call has %lld "
                    "(29 bytes per row and 12 per entry of A of the largest stage, 16 more per row with "
                    "upper-bound slots, plus the tables)",
                    pl.total, (long long)kNoAllocScratchBytes);
    HIP_TRY(h, hipSetDevice(h->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    // host tables in ordinary host memory: the copies complete before the
    // stream synchronization at the end of this call, while they still exist
    std::vector<BatchProb> tab((size_t)count);
    std::vector<int64_t> roff(2 * pl.roff_total);
    std::vector<int64_t> stage_chunks;
    char *base = static_cast<char *>(h->scratch);
    char *arena_c = static_cast<char *>(arena);
    fill_batched_tables(pl, probs, arena_c, tab.data(), roff.data(), &stage_chunks);
    BatchProb *d_tab = reinterpret_cast<BatchProb *>(base + pl.o_tab);
    BatchStatus *d_stat = reinterpret_cast<BatchStatus *>(base + pl.o_stat);
    HIP_TRY(h, hipMemcpyAsync(d_tab, tab.data(), sizeof(BatchProb) * (size_t)count, hipMemcpyHostToDevice, s));
    HIP_TRY(h, hipMemcpyAsync(base + pl.o_roff, roff.data(), 16 * pl.roff_total, hipMemcpyHostToDevice, s));
    // launched directly: instantiating a graph may allocate
    HIP_TRY(h, launch_batched_all(h, pl, stage_chunks, base, arena_c, arena_bytes, s));
    HIP_TRY(h, launch_batched_describe(d_tab, count, out, d_stat, s));
    BatchStatus bst;
    Ctl ctl;
    HIP_TRY(h, hipMemcpyAsync(&bst, d_stat, sizeof(BatchStatus), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipMemcpyAsync(&ctl, base + pl.o_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    return finish_batched(h, bst, ctl, pl, required_bytes);
}

}  // extern "C"
