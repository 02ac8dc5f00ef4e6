// Host side of the C ABI declared in include/spgemm.h: argument checks, the
// handle's device workspace, and the launch sequence of the symbolic and
// numeric passes of the precise allocation (Section III-D.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "brm_internal.h"
#include "spgemm.h"

using namespace brm;

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
    int64_t heavy_lds_max = kCapBlock;
    int64_t spill_budget_mb = 16384;
    int64_t grid_waves = 0;
    // workspace
    void *ws_mem = nullptr;
    size_t ws_bytes = 0;
    Ctl *ctl = nullptr;
    Ctl *ctl_host = nullptr;  // pinned
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

int ensure_workspace(spg_handle h, int64_t M, Workspace *ws) {
    const int64_t ntiles = (M + kScanTile - 1) / kScanTile + 1;
    const size_t a = 256;
    size_t off_nprod = 0;
    size_t off_class = align_up(off_nprod + 8 * (size_t)M, a);
    size_t off_size = align_up(off_class + (size_t)M, a);
    size_t off_rows = align_up(off_size + 4 * (size_t)M, a);
    size_t off_tile = align_up(off_rows + 4 * (size_t)M, a);
    size_t total = align_up(off_tile + 8 * (size_t)ntiles, a);
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
int run_heavy(spg_handle h, const CsrView &a, const CsrView &b, const Workspace &ws,
              const int64_t *c_rpt, int32_t *c_col, double *c_val, hipStream_t s) {
    const int64_t n = h->counts[kClassHeavy];
    int64_t first = 0;
    for (int c = 0; c < kClassHeavy; ++c) first += h->counts[c];
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
    unsigned long long *d_ticket = reinterpret_cast<unsigned long long *>(d + info_b + rows_b + 2 * offs_b);
    HIP_TRY(h, launch_heavy_info(a, ws, first, n, d_info, s));
    std::vector<int64_t> info(3 * (size_t)n);
    HIP_TRY(h, hipMemcpyAsync(info.data(), d_info, 24 * (size_t)n, hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    std::vector<int64_t> order((size_t)n);
    for (int64_t i = 0; i < n; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t x, int64_t y) { return info[3 * x + 1] > info[3 * y + 1]; });
    std::vector<int32_t> rows((size_t)n);
    std::vector<int64_t> soff((size_t)n), loff((size_t)n);
    std::vector<std::pair<int64_t, int64_t>> batches;  // [begin, end)
    const size_t budget = (size_t)h->spill_budget_mb << 20;
    size_t max_elems = 0, max_leaf = 0;
    size_t used = 0, elems = 0, leafs = 0;
    int64_t b0 = 0;
    for (int64_t j = 0; j < n; ++j) {
        const int64_t i = order[(size_t)j];
        const int64_t np = info[3 * i + 1], nl = info[3 * i + 2];
        if (np >= INT32_MAX || nl >= INT32_MAX)
            return fail(h, SPG_ERR_CAPACITY, "row %lld has %lld products (limit 2^31-1 per row)",
                        (long long)info[3 * i], (long long)np);
        const size_t need = 24 * (size_t)np + 4 * (size_t)(nl + 1);
        if (j > b0 && used + need > budget) {
            batches.emplace_back(b0, j);
            b0 = j;
            used = elems = leafs = 0;
        }
        rows[(size_t)j] = (int32_t)info[3 * i];
        soff[(size_t)j] = (int64_t)elems;
        loff[(size_t)j] = (int64_t)leafs;
        elems += 2 * (size_t)np;
        leafs += (size_t)nl + 1;
        used += need;
        max_elems = std::max(max_elems, elems);
        max_leaf = std::max(max_leaf, leafs);
    }
    batches.emplace_back(b0, n);
    if (batches.size() > 4096) return fail(h, SPG_ERR_CAPACITY, "too many spill batches; raise the spill budget");
    HIP_TRY(h, hipMemcpy(d_rows, rows.data(), 4 * (size_t)n, hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_soff, soff.data(), 8 * (size_t)n, hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_loff, loff.data(), 8 * (size_t)n, hipMemcpyHostToDevice));
    const size_t col_b = align_up(4 * max_elems, 256), val_b = align_up(8 * max_elems, 256);
    if ((rc = grow(h, &h->spill_mem, &h->spill_bytes, col_b + val_b + align_up(4 * max_leaf, 256) + 256, "spill buffers")))
        return rc;
    char *sp = static_cast<char *>(h->spill_mem);
    HIP_TRY(h, launch_zero_words(d_ticket, (int64_t)batches.size(), s));
    for (size_t bi = 0; bi < batches.size(); ++bi) {
        const int64_t lo = batches[bi].first, hi = batches[bi].second;
        HeavyArgs ha;
        ha.ticket = d_ticket + bi;
        ha.rows = d_rows + lo;
        ha.spill_off = d_soff + lo;
        ha.leaf_off = d_loff + lo;
        ha.nrows = hi - lo;
        ha.spill_col = reinterpret_cast<int32_t *>(sp);
        ha.spill_val = reinterpret_cast<double *>(sp + col_b);
        ha.leaf = reinterpret_cast<int32_t *>(sp + col_b + val_b);
        ha.lds_cap = (int)h->heavy_lds_max;
        const int grid = (int)std::min<int64_t>(hi - lo, h->num_cu);
        HIP_TRY(h, launch_numeric_heavy(a, b, ha, grid, c_rpt, c_col, c_val, h->ctl, s));
    }
    h->heavy_batches = (int64_t)batches.size();
    return SPG_OK;
}

Thresholds thresholds(spg_handle h) {
    Thresholds t;
    t.wave_small_max = h->wave_small_max;
    t.wave_max = h->wave_max;
    t.group_max = h->group_max;
    t.block_max = h->block_max;
    t.force = (int32_t)h->force;
    return t;
}

int persistent_grid(spg_handle h, int cls, int64_t rows) {
    // workgroups per launch of the persistent row kernels
    int per_cu;
    int teams_per_wg;
    switch (cls) {
        case kClassCopy: per_cu = 8; teams_per_wg = 4; break;
        case kClassWaveSmall: per_cu = 8; teams_per_wg = 4; break;
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
        hipHostMalloc(&h->ctl_host, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        if (h->ctl) (void)hipFree(h->ctl);
        delete h;
        return SPG_ERR_NOMEM;
    }
    std::memset(h->ctl_host, 0, sizeof(Ctl));
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
            if (value != -1 && (value < kClassWaveSmall || value > kClassHeavy))
                return fail(h, SPG_ERR_ARG, "force class must be -1 or 2..6");
            h->force = value;
            break;
        case SPG_OPT_HEAVY_LDS_MAX:
            if (value < 64 || value > kCapBlock) return fail(h, SPG_ERR_ARG, "heavy LDS max out of range");
            h->heavy_lds_max = value;
            break;
        case SPG_OPT_SPILL_BUDGET_MB:
            if (value < 1) return fail(h, SPG_ERR_ARG, "spill budget must be positive");
            h->spill_budget_mb = value;
            break;
        case SPG_OPT_GRID_WAVES:
            if (value < 0) return fail(h, SPG_ERR_ARG, "grid waves must be >= 0");
            h->grid_waves = value;
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
        case SPG_OPT_SPILL_BUDGET_MB: *value = h->spill_budget_mb; break;
        case SPG_OPT_GRID_WAVES: *value = h->grid_waves; break;
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
        case SPG_STAT_DEVICE_ERR: {
            HIP_TRY(h, hipSetDevice(h->device));
            HIP_TRY(h, hipDeviceSynchronize());
            int64_t e = 0;
            HIP_TRY(h, hipMemcpy(&e, &h->ctl->err, sizeof e, hipMemcpyDeviceToHost));
            *value = e;
            return SPG_OK;
        }
        default: return fail(h, SPG_ERR_ARG, "unknown statistic %d", key);
    }
}

int spgemm_symbolic(spg_handle h, const spg_csr *A, const spg_csr *B, int64_t *c_rpt,
                    int64_t *c_nnz, void *stream) {
    if (!h) return SPG_ERR_ARG;
    h->err.clear();
    h->plan_valid = false;
    int rc;
    if ((rc = check_csr(h, A, "A", false)) || (rc = check_csr(h, B, "B", false))) return rc;
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
    if ((rc = ensure_workspace(h, M, &ws))) return rc;

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
    if (M > 0) {
        const int g = (int)std::min<int64_t>((M + 255) / 256, 2048);
        HIP_TRY(h, launch_analysis(a, b, thresholds(h), ws, g, s));
        HIP_TRY(h, launch_bin(M, ws, g, s));
        for (int cls = kClassWaveSmall; cls <= kClassHeavy; ++cls)
            HIP_TRY(h, launch_symbolic(a, b, ws, cls, persistent_grid(h, cls, -1), s));
    }
    HIP_TRY(h, launch_scan(M, ws, c_rpt, s));
    HIP_TRY(h, hipMemcpyAsync(h->ctl_host, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    const Ctl &c = *h->ctl_host;
    for (int i = 0; i < 8; ++i) h->counts[i] = c.count[i];
    h->nnz = c.nnz;
    h->nprod = c.nprod;
    *c_nnz = c.nnz;
    h->plan_valid = true;
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
    if ((rc = ensure_workspace(h, A->rows, &ws))) return rc;
    h->heavy_batches = 0;
    for (int cls = kClassCopy; cls <= kClassBlock; ++cls) {
        if (h->counts[cls] == 0) continue;
        HIP_TRY(h, launch_numeric(a, b, ws, cls, h->counts[cls], persistent_grid(h, cls, h->counts[cls]),
                                  c_rpt, c_col, c_val, s));
    }
    if (h->counts[kClassHeavy] > 0) return run_heavy(h, a, b, ws, c_rpt, c_col, c_val, s);
    return SPG_OK;
}

}  // extern "C"
