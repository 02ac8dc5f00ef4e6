// Device-side building blocks shared by the SpGEMM kernels: wavefront
// primitives (64 lanes on CDNA), team-wide scans for teams of one wavefront or
// one workgroup, and binary searches over sorted column arrays.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace brm {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Number of set bits of `mask` in the lanes below the calling lane.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __ballot(p); }

// A value every lane of the wavefront holds alike, moved to a scalar
// register: loops and branches on it become scalar branches instead of
// exec-masked vector code.
__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t wave_uniform(int64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Orders LDS traffic between the lanes of one wavefront (no s_barrier).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Loads and stores through pointers known to address global memory (device
// buffers): pointers read from memory (a problem table) are otherwise
// generic, and their flat accesses count against the LDS counter as well, so
// that every LDS wait also waits for them.
template <typename T>
__device__ __forceinline__ T gload(const T *p) {
    using GP = const __attribute__((address_space(1))) T *;
    return *(GP)p;
}
template <typename T>
__device__ __forceinline__ void gstore(T *p, T v) {
    using GP = __attribute__((address_space(1))) T *;
    *(GP)p = v;
}

template <typename Tv>
__device__ __forceinline__ Tv wave_incl_scan(Tv x) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        Tv y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

template <typename Tv>
__device__ __forceinline__ Tv wave_sum(Tv x) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

// The size predictor's six inputs for a row of C: log1p(lists), log((1 +
// products) / N), log1p(longest list), log1p(shortest list), log(column span
// / N) and log1p(products / span), N the column count of B (taken as at
// least 1, a span of 0 as 1).  Products and span relative to the column space
// keep the features comparable between matrices of different sizes.
__device__ __forceinline__ void row_features6(float *f, int64_t L, int64_t np, int64_t mx, int64_t mn,
                                              int64_t span, int64_t ncols) {
    const double n = (double)(ncols > 0 ? ncols : 1);
    f[0] = log1pf((float)L);
    f[1] = logf((float)((1.0 + (double)np) / n));
    f[2] = log1pf((float)mx);
    f[3] = log1pf((float)mn);
    f[4] = logf((float)((double)(span > 0 ? span : 1) / n));
    f[5] = log1pf(span > 0 ? (float)((double)np / (double)span) : 0.0f);
}

// A team is either one wavefront (T == 64) or a whole workgroup (T > 64).
template <int T>
struct Team {
    static_assert(T % kWave == 0, "team size must be a multiple of the wavefront");
    static constexpr int kWaves = T / kWave;

    __device__ __forceinline__ static void sync() {
        if constexpr (T == kWave)
            wave_sync();
        else
            __syncthreads();
    }

    // Exclusive prefix sum over the team in thread order; *total gets the sum.
    // `scratch` needs kWaves entries of LDS (unused for one wavefront).
    template <typename Tv>
    __device__ __forceinline__ static Tv excl_scan(Tv x, Tv *total, Tv *scratch, int tid) {
        Tv incl = wave_incl_scan(x);
        if constexpr (T == kWave) {
            *total = __shfl(incl, kWave - 1, kWave);
            return incl - x;
        } else {
            const int w = tid / kWave;
            if (lane_id() == kWave - 1) scratch[w] = incl;
            __syncthreads();
            Tv before = 0, all = 0;
#pragma unroll
            for (int i = 0; i < kWaves; ++i) {
                Tv s = scratch[i];
                before += (i < w) ? s : Tv(0);
                all += s;
            }
            __syncthreads();
            *total = all;
            return before + incl - x;
        }
    }

    template <typename Tv>
    __device__ __forceinline__ static Tv sum(Tv x, Tv *scratch, int tid) {
        Tv s = wave_sum(x);
        if constexpr (T == kWave) {
            return s;
        } else {
            if (lane_id() == 0) scratch[tid / kWave] = s;
            __syncthreads();
            Tv all = 0;
#pragma unroll
            for (int i = 0; i < kWaves; ++i) all += scratch[i];
            __syncthreads();
            return all;
        }
    }
};

// First index in [0, n) whose value is >= key (n if none).
template <typename Tk>
__device__ __forceinline__ int lower_bound(const Tk *a, int n, Tk key) {
    int lo = 0;
    while (n > 0) {
        int half = n >> 1;
        if (a[lo + half] < key) {
            lo += half + 1;
            n -= half + 1;
        } else {
            n = half;
        }
    }
    return lo;
}

// First index in [0, n) whose value is > key (n if none).
template <typename Tk>
__device__ __forceinline__ int upper_bound(const Tk *a, int n, Tk key) {
    int lo = 0;
    while (n > 0) {
        int half = n >> 1;
        if (!(key < a[lo + half])) {
            lo += half + 1;
            n -= half + 1;
        } else {
            n = half;
        }
    }
    return lo;
}

template <typename Tk>
__device__ __forceinline__ int64_t lower_bound64(const Tk *a, int64_t n, Tk key) {
    int64_t lo = 0;
    while (n > 0) {
        int64_t half = n >> 1;
        if (a[lo + half] < key) {
            lo += half + 1;
            n -= half + 1;
        } else {
            n = half;
        }
    }
    return lo;
}

template <typename Tk>
__device__ __forceinline__ int64_t upper_bound64(const Tk *a, int64_t n, Tk key) {
    int64_t lo = 0;
    while (n > 0) {
        int64_t half = n >> 1;
        if (!(key < a[lo + half])) {
            lo += half + 1;
            n -= half + 1;
        } else {
            n = half;
        }
    }
    return lo;
}

}  // namespace brm
