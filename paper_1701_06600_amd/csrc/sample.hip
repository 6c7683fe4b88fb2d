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

}  // namespace cprand
