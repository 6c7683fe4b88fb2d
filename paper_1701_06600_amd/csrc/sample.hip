// Sample multi-indices for one mode step (Section 3.2): uniform with
// replacement, or importance draws from integer proposal tables.
#include "kernels.hpp"

namespace cprand {

__global__ __launch_bounds__(256) void sample_kernel(ModeInfo mi, int32_t S, uint64_t seed,
                                                     uint64_t t, const uint64_t *t_dev,
                                                     CdfPtrs cdf, int use_cdf, int32_t *idx,
                                                     double *w) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const uint64_t tt = t_dev ? *t_dev : t;
    int64_t row[kMaxOrder];
    const double ws = draw_sample(mi, seed, tt, s, cdf, use_cdf != 0, row);
#pragma unroll
    for (int m = 0; m < kMaxOrder; ++m)
        if (m < mi.order) idx[s * mi.order + m] = (m == mi.n) ? -1 : (int32_t)row[m];
    if (w) w[s] = ws;
}

hipError_t launch_sample(const ModeInfo &mi, int32_t S, uint64_t seed, uint64_t t,
                         const uint64_t *t_dev, const CdfPtrs *cdf, int32_t *idx, double *w,
                         hipStream_t st) {
    if (S <= 0) return hipSuccess;
    CdfPtrs c{};
    if (cdf) c = *cdf;
    const int nt = 256;
    const int nb = (int)ceil_div(S, nt);
    hipLaunchKernelGGL(sample_kernel, dim3(nb), dim3(nt), 0, st, mi, S, seed, t, t_dev, c,
                       cdf ? 1 : 0, idx, w);
    return hipGetLastError();
}

// Every mode step of iterations 0 .. T-1 at once: blockIdx.y = t * order + n,
// indices at idx + blockIdx.y * S * order, weights at w + blockIdx.y * S.
__global__ __launch_bounds__(256) void sample_all_kernel(ModeInfo mi, int32_t S, uint64_t seed, CdfPtrs cdf,
                                                         int use_cdf, int32_t *idx, double *w) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const int y = (int)blockIdx.y;
    const uint64_t t = (uint64_t)(y / mi.order);
    mi.n = y % mi.order;
    int64_t row[kMaxOrder];
    const double ws = draw_sample(mi, seed, t, s, cdf, use_cdf != 0, row);
    int32_t *ix = idx + (int64_t)y * S * mi.order;
#pragma unroll
    for (int m = 0; m < kMaxOrder; ++m)
        if (m < mi.order) ix[s * mi.order + m] = (m == mi.n) ? -1 : (int32_t)row[m];
    if (w) w[(int64_t)y * S + s] = ws;
}

hipError_t launch_sample_all(const ModeInfo &mi, int32_t S, int32_t T, uint64_t seed, const CdfPtrs *cdf,
                             int32_t *idx, double *w, hipStream_t st) {
    if (S <= 0 || T <= 0) return hipSuccess;
    if ((int64_t)T * mi.order > 65535) return hipErrorInvalidValue;
    CdfPtrs c{};
    if (cdf) c = *cdf;
    const int nt = 256;
    hipLaunchKernelGGL(sample_all_kernel, dim3((unsigned)ceil_div(S, nt), (unsigned)(T * mi.order)), dim3(nt), 0,
                       st, mi, S, seed, c, cdf ? 1 : 0, idx, w);
    return hipGetLastError();
}

}  // namespace cprand
