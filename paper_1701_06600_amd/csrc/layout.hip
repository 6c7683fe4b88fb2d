// Mode-major copies: the tensor re-laid with mode n innermost, every mode-n
// fiber contiguous and padded to ld elements (a multiple of the 16-byte
// vector), optionally converted (FP32 -> BF16 round-to-nearest-even, or
// between real types).  A one-time HBM pass; LDS-tiled transpose so both
// the reads (along mode 0) and the writes (along mode n) are coalesced.
#include <type_traits>

#include "kernels.hpp"

namespace cprand {

struct c64 {
    float re, im;
};
struct c128 {
    double re, im;
};

template <typename Ti, typename To>
__device__ inline To convert(Ti v) {
    return (To)v;
}
template <>
__device__ inline uint16_t convert<float, uint16_t>(float v) {
    return f32_to_bf16_rne(v);
}
template <>
__device__ inline uint16_t convert<double, uint16_t>(double v) {
    return f32_to_bf16_rne((float)v);
}
template <>
__device__ inline c64 convert<c64, c64>(c64 v) {
    return v;
}
template <>
__device__ inline c128 convert<c128, c128>(c128 v) {
    return v;
}
template <typename T>
__device__ inline T zero_of() {
    return T{};
}

// n == 0: fibers are already contiguous; re-pad to ld.
template <typename Ti, typename To>
__global__ __launch_bounds__(256) void repad_kernel(const Ti *X, To *Y, int64_t L, int64_t ld,
                                                    int64_t K) {
    const int64_t tot = ld * K;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / ld, i = e - k * ld;
        Y[e] = (i < L) ? convert<Ti, To>(X[i + L * k]) : zero_of<To>();
    }
}

// n > 0: X viewed as [J][L][K] (j fastest) -> Y as [ld][J][K] (i fastest).
constexpr int kT = 64;
template <typename Ti, typename To>
__global__ __launch_bounds__(256) void transpose_kernel(const Ti *X, To *Y, int64_t J, int64_t L,
                                                        int64_t ld, int64_t K, int64_t jt) {
    __shared__ To tile[kT][kT + 1];
    const int64_t bx = blockIdx.x;
    const int64_t k = bx / jt, j0 = (bx - k * jt) * kT;
    const int64_t i0 = (int64_t)blockIdx.y * kT;
    const int tx = threadIdx.x & (kT - 1), ty = threadIdx.x >> 6;
    for (int q = ty; q < kT; q += 4) {
        const int64_t i = i0 + q, j = j0 + tx;
        To v = zero_of<To>();
        if (i < L && j < J) v = convert<Ti, To>(X[j + J * (i + L * k)]);
        tile[q][tx] = v;
    }
    __syncthreads();
    for (int q = ty; q < kT; q += 4) {
        const int64_t j = j0 + q, i = i0 + tx;
        if (j < J && i < ld) Y[i + ld * (j + J * k)] = tile[tx][q];
    }
}

// The same transpose for 8-byte elements (complex64) when J, L and ld are
// even and both buffers 16-byte aligned: every access moves two elements
// (16 bytes), a row of the 64 x 64 tile is 32 lanes.
__global__ __launch_bounds__(256) void transpose_pair_kernel(const c64 *X, c64 *Y, int64_t J, int64_t L, int64_t ld,
                                                             int64_t K, int64_t jt) {
    __shared__ c64 tile[kT][kT + 1];
    const int64_t bx = blockIdx.x;
    const int64_t k = bx / jt, j0 = (bx - k * jt) * kT;
    const int64_t i0 = (int64_t)blockIdx.y * kT;
    const int c2 = threadIdx.x & 31, r = threadIdx.x >> 5;  // pair column, row within a pass of 8 rows
    float4 v[kT / 8];
#pragma unroll
    for (int p = 0; p < kT / 8; ++p) {
        const int64_t i = i0 + r + 8 * p, j = j0 + 2 * c2;
        v[p] = float4{0.f, 0.f, 0.f, 0.f};
        if (i < L && j < J) v[p] = *(const float4 *)(X + j + J * (i + L * k));
    }
#pragma unroll
    for (int p = 0; p < kT / 8; ++p) {
        tile[r + 8 * p][2 * c2] = c64{v[p].x, v[p].y};
        tile[r + 8 * p][2 * c2 + 1] = c64{v[p].z, v[p].w};
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < kT / 8; ++p) {
        const int64_t j = j0 + r + 8 * p, i = i0 + 2 * c2;
        if (j < J && i < ld) {
            const c64 a = tile[2 * c2][r + 8 * p], b = tile[2 * c2 + 1][r + 8 * p];
            *(float4 *)(Y + i + ld * (j + J * k)) = float4{a.re, a.im, b.re, b.im};
        }
    }
}

template <typename Ti, typename To>
static hipError_t launch_lc(const ModeInfo &xi, const void *X, int32_t n, int64_t ld, void *Y,
                            hipStream_t st) {
    int64_t J = 1, K = 1;
    for (int m = 0; m < n; ++m) J *= xi.dims[m];
    for (int m = n + 1; m < xi.order; ++m) K *= xi.dims[m];
    const int64_t L = xi.dims[n];
    if (n == 0) {
        const int64_t tot = ld * K;
        const int nb = (int)std::min<int64_t>(65536, ceil_div(tot, 256));
        hipLaunchKernelGGL((repad_kernel<Ti, To>), dim3(nb), dim3(256), 0, st, (const Ti *)X,
                           (To *)Y, L, ld, K);
    } else {
        const int64_t jt = ceil_div(J, kT);
        dim3 grid((unsigned)(jt * K), (unsigned)ceil_div(ld, kT));
        constexpr bool pairable = std::is_same<Ti, c64>::value && std::is_same<To, c64>::value;
        if (pairable && J % 2 == 0 && L % 2 == 0 && ld % 2 == 0 && ld == L && (((uintptr_t)X) & 15) == 0 &&
            (((uintptr_t)Y) & 15) == 0)
            hipLaunchKernelGGL(transpose_pair_kernel, grid, dim3(256), 0, st, (const c64 *)X, (c64 *)Y, J, L, ld, K,
                               jt);
        else
            hipLaunchKernelGGL((transpose_kernel<Ti, To>), grid, dim3(256), 0, st, (const Ti *)X,
                               (To *)Y, J, L, ld, K, jt);
    }
    return hipGetLastError();
}

hipError_t launch_layout_copy(const ModeInfo &xi, const void *X, int xkind, int32_t n, int64_t ld,
                              void *Y, int ykind, hipStream_t st) {
    if (xkind == K_F32 && ykind == K_F32) return launch_lc<float, float>(xi, X, n, ld, Y, st);
    if (xkind == K_F32 && ykind == K_BF16) return launch_lc<float, uint16_t>(xi, X, n, ld, Y, st);
    if (xkind == K_F64 && ykind == K_F64) return launch_lc<double, double>(xi, X, n, ld, Y, st);
    if (xkind == K_F64 && ykind == K_F32) return launch_lc<double, float>(xi, X, n, ld, Y, st);
    if (xkind == K_F64 && ykind == K_BF16) return launch_lc<double, uint16_t>(xi, X, n, ld, Y, st);
    if (xkind == K_C64 && ykind == K_C64) return launch_lc<c64, c64>(xi, X, n, ld, Y, st);
    if (xkind == K_C128 && ykind == K_C128) return launch_lc<c128, c128>(xi, X, n, ld, Y, st);
    return hipErrorInvalidValue;
}

}  // namespace cprand
