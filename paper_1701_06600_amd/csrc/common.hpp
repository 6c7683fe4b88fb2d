// Shared device helpers: Philox4x64-10, index mapping, BF16 rounding, small
// complex arithmetic, reductions.  gfx950 (wave64) only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cprand.h"

namespace cprand {

constexpr int kWave = 64;
constexpr int kMaxOrder = CPRAND_MAX_ORDER;
constexpr int kMaxRank = CPRAND_MAX_RANK;

// Philox stream tags (second key word).
constexpr uint64_t kTagSigns = 3;
constexpr uint64_t kTagSamples = 5;
constexpr uint64_t kTagFit = 6;

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
// (x0,x1,x2,x3) -> (hi(M1 x2)^x1^k0, lo(M1 x2), hi(M0 x0)^x3^k1, lo(M0 x0)),
// key bumped by the Weyl constants between rounds.
struct u64x4 {
    uint64_t v[4];
};

__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

__host__ __device__ inline u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                               uint64_t c3, uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t lo0 = M0 * c0, hi0 = mulhi64(M0, c0);
        uint64_t lo1 = M1 * c2, hi1 = mulhi64(M1, c2);
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    u64x4 out;
    out.v[0] = c0;
    out.v[1] = c1;
    out.v[2] = c2;
    out.v[3] = c3;
    return out;
}

// Row drawn from an integer proposal table: first i with cdf[i+1] > target.
__device__ inline int64_t cdf_search(const uint64_t *__restrict__ cdf, int64_t I, uint64_t target) {
    int64_t lo = 0, hi = I - 1;  // answer in [lo, hi]
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (cdf[mid + 1] > target)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Dimensions/strides/pointers passed by value to kernels.
struct ModeInfo {
    int32_t order;
    int32_t n;
    int64_t dims[kMaxOrder];
    int64_t strides[kMaxOrder];
};

struct FactorPtrs {
    const void *p[kMaxOrder];
};

struct CdfPtrs {
    const uint64_t *p[kMaxOrder];
};

// Word j (0..3) of a Philox block, by selects (a runtime index into the
// block would put it in scratch memory).
__device__ inline uint64_t u64x4_get(const u64x4 &b, int j) {
    return j == 0 ? b.v[0] : j == 1 ? b.v[1] : j == 2 ? b.v[2] : b.v[3];
}

// Draw the multi-index of sample s (modes != n) and its importance weight.
// idx_out[m] receives the row of mode m (undefined for m == n).  The mode
// loop is unrolled to kMaxOrder so that idx_out stays in registers.
__device__ inline double draw_sample(const ModeInfo &mi, uint64_t seed, uint64_t t, int64_t s,
                                     const CdfPtrs &cdf, bool use_cdf, int64_t *idx_out) {
    double w = 1.0;
    int k = 0;
    u64x4 blk;
#pragma unroll
    for (int m = 0; m < kMaxOrder; ++m) {
        if (m >= mi.order) break;
        if (m == mi.n) continue;
        if ((k & 3) == 0) blk = philox4x64_10((uint64_t)s, t, (uint64_t)mi.n, (uint64_t)(k >> 2), seed, kTagSamples);
        const uint64_t u = u64x4_get(blk, k & 3);
        const int64_t I = mi.dims[m];
        if (use_cdf) {
            const uint64_t *c = cdf.p[m];
            const uint64_t Q = c[I];
            const int64_t i = cdf_search(c, I, mulhi64(u, Q));
            idx_out[m] = i;
            const uint64_t qi = c[i + 1] - c[i];
            w = w * ((double)Q / ((double)I * (double)qi));
        } else {
            idx_out[m] = (int64_t)mulhi64(u, (uint64_t)I);
        }
        ++k;
    }
    return w;
}

// ---------------------------------------------------------------------------
// BF16 (round to nearest even; NaN kept quiet).
__host__ __device__ inline uint16_t f32_to_bf16_rne(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf16_to_f32(uint16_t h) {
    uint32_t u = ((uint32_t)h) << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// ---------------------------------------------------------------------------
// Block-wide FP64 sum with a fixed reduction order (deterministic).
template <int NT>
__device__ inline double block_sum(double v, double *sh) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < NT / kWave; ++i) r += sh[i];
    }
    __syncthreads();
    return r;  // valid on thread 0
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace cprand
