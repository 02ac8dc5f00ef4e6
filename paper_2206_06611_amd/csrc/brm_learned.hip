// Learned allocation: a small perceptron predicts the size of every row of C
// from per-row features, so that the numeric pass can run without the
// symbolic pass into slots sized by the prediction (the temporary matrix of
// the upper-bound allocation, Section II-B.2 and Section III-D.1, with a
// learned bound in place of the product count).  Rows whose exact length
// exceeds their slot are recomputed exactly into C afterwards; all other rows
// are compacted from the slots into C.
//
// Network: 6 -> 64 -> 64 -> 1, ReLU, float32.  Parameters are one float
// vector: W1[6][64], b1[64], W2[64][64], b2[64], W3[64], b3[1] (row-major).
// Training: mean squared error on log(nnz(C_i) / nprod_i), Adam.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "brm_device.h"
#include "brm_internal.h"

namespace brm {

namespace {

template <typename I>
__device__ __forceinline__ int64_t ld_rpt_l(const void *p, int64_t i) {
    return (int64_t)(reinterpret_cast<const I *>(p)[i]);
}

}  // namespace

// ---------------------------------------------------------------------------
// features (row_features6); exact bounds of the row size: the longest list
// (a row of C holds at least its distinct columns) and min(products, span)
// ---------------------------------------------------------------------------
template <typename IA, typename IB>
__global__ __launch_bounds__(256) void k_features(int64_t M, const void *a_rpt, const int32_t *a_col,
                                                  const void *b_rpt, const int32_t *b_col, int64_t ncols,
                                                  float *feats, int32_t *lo, int32_t *hi,
                                                  int8_t *predicted, const int64_t *c_rpt,
                                                  float *targets) {
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t base0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1));
    for (int64_t base = base0; base < M; base += stride) {
        const int64_t i = base + lane;
        const bool in = i < M;
        int64_t a0 = 0, a1 = 0;
        if (in) {
            a0 = ld_rpt_l<IA>(a_rpt, i);
            a1 = ld_rpt_l<IA>(a_rpt, i + 1);
        }
        int64_t np = 0, mx = 0, mn = INT64_MAX, first = INT64_MAX, last = -1;
        const bool longrow = in && (a1 - a0) > 32;
        if (in && !longrow) {
            for (int64_t p = a0; p < a1; ++p) {
                const int32_t k = a_col[p];
                const int64_t bs = ld_rpt_l<IB>(b_rpt, k), be = ld_rpt_l<IB>(b_rpt, k + 1);
                const int64_t n = be - bs;
                np += n;
                mx = n > mx ? n : mx;
                mn = n < mn ? n : mn;
                if (n > 0) {
                    const int64_t f = b_col[bs], l = b_col[be - 1];
                    first = f < first ? f : first;
                    last = l > last ? l : last;
                }
            }
        }
        uint64_t lm = wave_ballot(longrow);
        while (lm) {
            const int src = __builtin_ctzll(lm);
            const int64_t r0 = __shfl(a0, src, kWave), r1 = __shfl(a1, src, kWave);
            int64_t pnp = 0, pmx = 0, pmn = INT64_MAX, pf = INT64_MAX, pl = -1;
            for (int64_t p = r0 + lane; p < r1; p += kWave) {
                const int32_t k = a_col[p];
                const int64_t bs = ld_rpt_l<IB>(b_rpt, k), be = ld_rpt_l<IB>(b_rpt, k + 1);
                const int64_t n = be - bs;
                pnp += n;
                pmx = n > pmx ? n : pmx;
                pmn = n < pmn ? n : pmn;
                if (n > 0) {
                    const int64_t f = b_col[bs], l = b_col[be - 1];
                    pf = f < pf ? f : pf;
                    pl = l > pl ? l : pl;
                }
            }
            pnp = wave_sum(pnp);
#pragma unroll
            for (int d = kWave / 2; d >= 1; d >>= 1) {
                const int64_t omx = __shfl_xor(pmx, d, kWave), omn = __shfl_xor(pmn, d, kWave);
                const int64_t of = __shfl_xor(pf, d, kWave), ol = __shfl_xor(pl, d, kWave);
                pmx = omx > pmx ? omx : pmx;
                pmn = omn < pmn ? omn : pmn;
                pf = of < pf ? of : pf;
                pl = ol > pl ? ol : pl;
            }
            if (lane == src) {
                np = pnp;
                mx = pmx;
                mn = pmn;
                first = pf;
                last = pl;
            }
            lm &= lm - 1;
        }
        if (in) {
            const int64_t L = a1 - a0;
            const int64_t span = last >= first ? last - first + 1 : 0;
            if (L == 0) mn = 0;
            row_features6(feats + 6 * i, L, np, mx, mn, span, ncols);
            const bool pred = np > 0 && L >= 2;
            predicted[i] = pred ? 1 : 0;
            lo[i] = (int32_t)(np == 0 ? 0 : (L == 1 ? np : mx));
            hi[i] = (int32_t)(np == 0 ? 0 : (L == 1 ? np : (np < span ? np : span)));
            if (targets) {
                const int64_t nc = c_rpt[i + 1] - c_rpt[i];
                targets[i] = pred ? logf((float)((double)nc / (double)np)) : 0.0f;
            }
        }
    }
}

hipError_t launch_features(const CsrView &A, const CsrView &B, float *feats, int32_t *lo, int32_t *hi,
                           int8_t *predicted, const int64_t *c_rpt, float *targets, hipStream_t s) {
    if (A.rows == 0) return hipSuccess;
    const unsigned g = (unsigned)((A.rows + 255) / 256 < 2048 ? (A.rows + 255) / 256 : 2048);
#define BRM_F(IA, IB)                                                                            \
    hipLaunchKernelGGL((k_features<IA, IB>), dim3(g), dim3(256), 0, s, A.rows, A.rpt, A.col,       \
                       B.rpt, B.col, B.cols, feats, lo, hi, predicted, c_rpt, targets)
    if (A.rpt_bytes == 4 && B.rpt_bytes == 4) BRM_F(int32_t, int32_t);
    else if (A.rpt_bytes == 4) BRM_F(int32_t, int64_t);
    else if (B.rpt_bytes == 4) BRM_F(int64_t, int32_t);
    else BRM_F(int64_t, int64_t);
#undef BRM_F
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// forward pass, one row per thread, parameters broadcast from LDS
// ---------------------------------------------------------------------------
constexpr int kIn = 6, kH = 64;
constexpr int oW1 = 0, oB1 = oW1 + kIn * kH, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH, kParams = oB3 + 1;
static_assert(kParams == 4673, "parameter layout");

struct MlpLds {
    float w[kParams];
    float mean[kIn], inv_std[kIn];
};

__device__ __forceinline__ void load_mlp(MlpLds &s, const float *params, const float *norm) {
    for (int i = threadIdx.x; i < kParams; i += blockDim.x) s.w[i] = params[i];
    if (threadIdx.x < kIn) {
        s.mean[threadIdx.x] = norm[threadIdx.x];
        s.inv_std[threadIdx.x] = 1.0f / norm[kIn + threadIdx.x];
    }
    __syncthreads();
}

// One row through the network, one thread per row.  The weights are read
// from global memory at wavefront-uniform addresses, so they arrive through
// scalar loads and every multiply-add takes its weight from a scalar
// register (no LDS traffic).  The hidden layer is formed in outer-product
// order: hidden unit k of layer 1 is computed when needed and added into
// all 64 accumulators of layer 2, so only those 64 stay in vector registers;
// each accumulator still sums k = 0 .. 63 in order, from its bias.  Fused
// multiply-adds: the predictor only sizes slots, its rounding never reaches C.
__device__ __forceinline__ float mlp_eval(const float *__restrict__ w, const float *__restrict__ norm,
                                          const float *raw) {
    float x[kIn];
#pragma unroll
    for (int j = 0; j < kIn; ++j) x[j] = (raw[j] - norm[j]) / norm[kIn + j];
    float acc[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) acc[j] = w[oB2 + j];
#pragma unroll 1
    for (int k = 0; k < kH; ++k) {
        float a = w[oB1 + k];
#pragma unroll
        for (int j = 0; j < kIn; ++j) a = __builtin_fmaf(x[j], w[oW1 + j * kH + k], a);
        const float hk = a > 0.0f ? a : 0.0f;
#pragma unroll
        for (int j = 0; j < kH; ++j) acc[j] = __builtin_fmaf(hk, w[oW2 + k * kH + j], acc[j]);
    }
    float y = w[oB3];
#pragma unroll
    for (int j = 0; j < kH; ++j) y = __builtin_fmaf(acc[j] > 0.0f ? acc[j] : 0.0f, w[oW3 + j], y);
    return y;
}

// Row sizes for the learned allocation: exact for rows with no product or a
// single list, clamp(ceil(nprod exp(y + delta)), lo, hi) otherwise.  `force`
// (testing only): 1 predicts every such row at its lower bound.
__global__ __launch_bounds__(256) void k_mlp_sizes(int64_t M, const float *feats, const int8_t *predicted,
                                                   const int32_t *lo, const int32_t *hi,
                                                   const int64_t *row_nprod, const float *__restrict__ params,
                                                   const float *__restrict__ norm, float delta, int force,
                                                   int64_t heavy_min, float heavy_margin, int32_t *pred_size) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t sz;
        // products over the columns they span (a log1p feature): with fewer
        // than one expected repeat among the products (products^2 / span <
        // 1), the exact upper bound min(products, span) is as tight as a
        // prediction could be and never overflows: no network needed
        const double per_col = expm1((double)feats[6 * i + 5]);
        if (!predicted[i]) {
            sz = lo[i];
        } else if (force == 1) {
            sz = lo[i];
        } else if ((double)row_nprod[i] * per_col < 1.0) {
            sz = hi[i];
        } else {
            const float y = mlp_eval(params, norm, feats + 6 * i);
            // rows merged through spill buffers get a wider margin: re-merging
            // one that overflows costs far more than its extra slot entries
            const double m = (double)delta + (row_nprod[i] > heavy_min ? (double)heavy_margin : 0.0);
            const double e = ceil((double)row_nprod[i] * exp((double)y + m));
            sz = e > (double)hi[i] ? hi[i] : (e < (double)lo[i] ? lo[i] : (int64_t)e);
        }
        pred_size[i] = (int32_t)sz;
    }
}

hipError_t launch_mlp_sizes(int64_t M, const float *feats, const int8_t *predicted, const int32_t *lo,
                            const int32_t *hi, const int64_t *row_nprod, const float *params,
                            const float *norm, float delta, int force, int64_t heavy_min, float heavy_margin,
                            int32_t *pred_size, hipStream_t s) {
    if (M == 0) return hipSuccess;
    const unsigned g = (unsigned)((M + 255) / 256 < 4096 ? (M + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_mlp_sizes, dim3(g), dim3(256), 0, s, M, feats, predicted, lo, hi, row_nprod,
                       params, norm, delta, force, heavy_min, heavy_margin, pred_size);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_mlp_forward(int64_t n, const float *feats,
                                                     const float *__restrict__ params,
                                                     const float *__restrict__ norm, float *y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = mlp_eval(params, norm, feats + 6 * i);
}

hipError_t launch_mlp_forward(int64_t n, const float *feats, const float *params, const float *norm,
                              float *y, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned g = (unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_mlp_forward, dim3(g), dim3(256), 0, s, n, feats, params, norm, y);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// training: per-row forward and backward to activations, then one thread per
// parameter sums its gradient over the batch in row order (deterministic),
// then Adam
// ---------------------------------------------------------------------------
// act layout per row r: x[6], h1[64] (post-ReLU), h2[64] (post-ReLU),
// d1[64] (dLoss/dz1), d2[64] (dLoss/dz2), dy
constexpr int kActStride = kIn + 4 * kH + 1;

__global__ __launch_bounds__(128) void k_mlp_backprop_rows(int64_t n, const float *feats,
                                                           const float *targets, const float *params,
                                                           const float *norm, float *act) {
    __shared__ MlpLds s;
    load_mlp(s, params, norm);
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    float *a = act + r * kActStride;
    float x[kIn];
#pragma unroll
    for (int j = 0; j < kIn; ++j) {
        x[j] = (feats[6 * r + j] - s.mean[j]) * s.inv_std[j];
        a[j] = x[j];
    }
    float h1[kH];
#pragma unroll
    for (int k = 0; k < kH; ++k) {
        float z = s.w[oB1 + k];
#pragma unroll
        for (int j = 0; j < kIn; ++j) z += x[j] * s.w[oW1 + j * kH + k];
        h1[k] = z > 0.0f ? z : 0.0f;
        a[kIn + k] = h1[k];
    }
    float y = s.w[oB3];
    for (int j = 0; j < kH; ++j) {
        float z = s.w[oB2 + j];
#pragma unroll
        for (int k = 0; k < kH; ++k) z += h1[k] * s.w[oW2 + k * kH + j];
        const float h2 = z > 0.0f ? z : 0.0f;
        a[kIn + kH + j] = h2;
        y += h2 * s.w[oW3 + j];
    }
    const float dy = 2.0f * (y - targets[r]) / (float)n;
    a[kIn + 4 * kH] = dy;
    // dLoss/dz2_j = dy W3_j [z2_j > 0]
    float d2[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        d2[j] = a[kIn + kH + j] > 0.0f ? dy * s.w[oW3 + j] : 0.0f;
        a[kIn + 3 * kH + j] = d2[j];
    }
    // dLoss/dz1_k = sum_j d2_j W2_kj [z1_k > 0]
    for (int k = 0; k < kH; ++k) {
        float t = 0.0f;
#pragma unroll
        for (int j = 0; j < kH; ++j) t += d2[j] * s.w[oW2 + k * kH + j];
        a[kIn + 2 * kH + k] = h1[k] > 0.0f ? t : 0.0f;
    }
}

// gradient of parameter p: a sum over the batch rows of a product of two
// activations.  The batch is cut into chunks of rows; each chunk's partial
// sums (and the chunk's squared error, in slot kParams) are added in chunk
// order afterwards, so the result does not depend on scheduling.
constexpr int kGradChunks = 64;

__device__ __forceinline__ void grad_operands(int p, int &ia, int &ib) {
    // grad_p = sum_r act[ia] * act[ib]  (ib < 0: factor 1)
    if (p < oB1) {
        ia = p / kH;                        // x_j
        ib = kIn + 2 * kH + p % kH;         // d1_k
    } else if (p < oW2) {
        ia = kIn + 2 * kH + (p - oB1);
        ib = -1;
    } else if (p < oB2) {
        ia = kIn + (p - oW2) / kH;          // h1_k
        ib = kIn + 3 * kH + (p - oW2) % kH; // d2_j
    } else if (p < oW3) {
        ia = kIn + 3 * kH + (p - oB2);
        ib = -1;
    } else if (p < oB3) {
        ia = kIn + kH + (p - oW3);          // h2_j
        ib = kIn + 4 * kH;                  // dy
    } else {
        ia = kIn + 4 * kH;
        ib = -1;
    }
}

__global__ __launch_bounds__(256) void k_mlp_grad_partial(int64_t n, const float *act, float *partial) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (n + kGradChunks - 1) / kGradChunks;
    const int64_t r0 = (int64_t)blockIdx.y * per;
    const int64_t r1 = (r0 + per) < n ? (r0 + per) : n;
    if (p > kParams) return;
    float g = 0.0f;
    if (p == kParams) {
        // squared error: dy_r = 2 (y_r - t_r) / n
        for (int64_t r = r0; r < r1; ++r) {
            const float d = act[r * kActStride + kIn + 4 * kH] * (float)n * 0.5f;
            g += d * d;
        }
    } else {
        int ia, ib;
        grad_operands(p, ia, ib);
        for (int64_t r = r0; r < r1; ++r) {
            const float *a = act + r * kActStride;
            g += ib < 0 ? a[ia] : a[ia] * a[ib];
        }
    }
    partial[(int64_t)blockIdx.y * (kParams + 1) + p] = g;
}

__global__ __launch_bounds__(256) void k_mlp_grad_reduce(int64_t n, const float *partial, float *grad,
                                                         float *loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kParams) return;
    float g = 0.0f;
    for (int c = 0; c < kGradChunks; ++c) g += partial[(int64_t)c * (kParams + 1) + p];
    if (p < kParams) grad[p] = g;
    else if (loss) *loss = n ? g / (float)n : 0.0f;
}

hipError_t launch_mlp_gradient(int64_t n, const float *feats, const float *targets, const float *params,
                               const float *norm, float *act, float *partial, float *grad, float *loss,
                               hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_mlp_backprop_rows, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, n, feats,
                           targets, params, norm, act);
    hipLaunchKernelGGL(k_mlp_grad_partial, dim3((kParams + 1 + 255) / 256, kGradChunks), dim3(256), 0, s, n,
                       act, partial);
    hipLaunchKernelGGL(k_mlp_grad_reduce, dim3((kParams + 1 + 255) / 256), dim3(256), 0, s, n, partial, grad,
                       loss);
    return hipGetLastError();
}

// Adam (Kingma & Ba 2015): step t >= 1
__global__ void k_adam(float *params, const float *grad, float *m, float *v, int64_t t, float lr,
                       float beta1, float beta2, float eps) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    const float g = grad[p];
    const float mm = beta1 * m[p] + (1.0f - beta1) * g;
    const float vv = beta2 * v[p] + (1.0f - beta2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mhat = mm / (1.0f - powf(beta1, (float)t));
    const float vhat = vv / (1.0f - powf(beta2, (float)t));
    params[p] -= lr * mhat / (sqrtf(vhat) + eps);
}

hipError_t launch_adam(float *params, const float *grad, float *m, float *v, int64_t t, float lr,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, params, grad, m, v, t, lr, 0.9f,
                       0.999f, 1e-8f);
    return hipGetLastError();
}

// feature normalisation: mean and standard deviation over n rows (one
// workgroup, fixed summation order)
__global__ __launch_bounds__(1024) void k_feature_stats(int64_t n, const float *feats, float *norm) {
    __shared__ double scr[Team<1024>::kWaves + 1];
    for (int j = 0; j < kIn; ++j) {
        double s1 = 0.0, s2 = 0.0;
        for (int64_t r = threadIdx.x; r < n; r += 1024) {
            const double x = feats[6 * r + j];
            s1 += x;
            s2 += x * x;
        }
        s1 = Team<1024>::sum(s1, scr, threadIdx.x);
        s2 = Team<1024>::sum(s2, scr, threadIdx.x);
        if (threadIdx.x == 0) {
            const double mean = n ? s1 / (double)n : 0.0;
            const double var = n ? s2 / (double)n - mean * mean : 0.0;
            norm[j] = (float)mean;
            norm[kIn + j] = (float)sqrt(var > 1e-12 ? var : 1.0);
        }
    }
}

hipError_t launch_feature_stats(int64_t n, const float *feats, float *norm, hipStream_t s) {
    hipLaunchKernelGGL(k_feature_stats, dim3(1), dim3(1024), 0, s, n, feats, norm);
    return hipGetLastError();
}

// mean squared error over n rows (one workgroup, fixed summation order)
__global__ __launch_bounds__(1024) void k_mse(int64_t n, const float *y, const float *t, float *out) {
    __shared__ double scr[Team<1024>::kWaves + 1];
    double acc = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += 1024) {
        const double d = (double)y[r] - (double)t[r];
        acc += d * d;
    }
    acc = Team<1024>::sum(acc, scr, threadIdx.x);
    if (threadIdx.x == 0) *out = n ? (float)(acc / (double)n) : 0.0f;
}

hipError_t launch_mse(int64_t n, const float *y, const float *t, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(1024), 0, s, n, y, t, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// compaction: rows that fit their predicted slot move from the slots to C
// (one wavefront per row)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_compact(int64_t M, const int64_t *slot_off, const int32_t *row_size,
                                                 const int64_t *c_rpt, const int32_t *s_col,
                                                 const double *s_val, int32_t *c_col, double *c_val) {
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; i < M; i += waves) {
        const int64_t so = slot_off[i];
        const int64_t cap = slot_off[i + 1] - so;
        const int64_t n = row_size[i];
        if (n > cap) continue;  // recomputed by the exact fallback
        const int64_t co = c_rpt[i];
        for (int64_t j = lane; j < n; j += kWave) {
            c_col[co + j] = s_col[so + j];
            c_val[co + j] = s_val[so + j];
        }
    }
}

hipError_t launch_compact(int64_t M, const int64_t *slot_off, const int32_t *row_size, const int64_t *c_rpt,
                          const int32_t *s_col, const double *s_val, int32_t *c_col, double *c_val,
                          int grid, hipStream_t s) {
    if (M == 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact, dim3(grid), dim3(256), 0, s, M, slot_off, row_size, c_rpt, s_col, s_val,
                       c_col, c_val);
    return hipGetLastError();
}

// Control block of the exact fallback: light overflow rows sit at
// [M - n_light, M) of the overflow list and are run by the 4096-product
// workgroup class, heavy ones at [M, M + n_heavy) by the heavy path.
__global__ void k_fallback_ctl(const Ctl *src, Ctl *dst, int64_t M) {
    if (threadIdx.x != 0) return;
    for (int c = 0; c < 8; ++c) {
        dst->count[c] = 0;
        dst->cursor[c] = 0;
    }
    // the light rows' counts per class are added by the binning of their list
    dst->count[kClassHeavy] = src->ovf_heavy;
    dst->err = 0;
    dst->ovf_light = dst->ovf_heavy = 0;
}

hipError_t launch_fallback_ctl(const Ctl *src, Ctl *dst, int64_t M, hipStream_t s) {
    hipLaunchKernelGGL(k_fallback_ctl, dim3(1), dim3(64), 0, s, src, dst, M);
    return hipGetLastError();
}

}  // namespace brm
