// Sampled fit estimate (Section 3.4) and the tensor norm.
//
// One thread per sampled entry: it regenerates the entry's multi-index from
// Philox (so the set is the same at every call), loads the tensor element,
// evaluates the model entry sum_r lambda_r prod_m A^(m)(i_m, r) from the
// L2-resident factor rows and squares the error; FP64 throughout, fixed-order
// block sums, and a one-block final kernel.
#include <math.h>

#include <type_traits>

#include "kernels.hpp"

namespace cprand {

constexpr int kFitThreads = 256;

__device__ inline void load_elem(const void *X, int kind, int64_t o, double &re, double &im) {
    im = 0.0;
    switch (kind) {
        case K_F64: re = ((const double *)X)[o]; break;
        case K_F32: re = (double)((const float *)X)[o]; break;
        case K_BF16: re = (double)bf16_to_f32(((const uint16_t *)X)[o]); break;
        case K_C64:
            re = (double)((const float *)X)[2 * o];
            im = (double)((const float *)X)[2 * o + 1];
            break;
        default:
            re = ((const double *)X)[2 * o];
            im = ((const double *)X)[2 * o + 1];
            break;
    }
}

// Multi-index and tensor value of fit sample p (Philox counter (p, 0, 0, block)).
__device__ inline void fit_entry(const FitArgs &a, int64_t p, int64_t *row, double &xr, double &xi) {
    const int N = a.mi.order;
    u64x4 blk;
    int64_t off = 0;
#pragma unroll
    for (int k = 0; k < kMaxOrder; ++k) {
        if (k >= N) break;
        if ((k & 3) == 0) blk = philox4x64_10((uint64_t)p, 0, 0, (uint64_t)(k >> 2), a.seed, kTagFit);
        row[k] = (int64_t)mulhi64(u64x4_get(blk, k & 3), (uint64_t)a.mi.dims[k]);
        off += row[k] * a.mi.strides[k];
    }
    load_elem(a.X, a.kind, off, xr, xi);
}

__global__ __launch_bounds__(kFitThreads) void fit_set_kernel(FitArgs a, int32_t *frow, double *fx) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.P_hat) return;
    int64_t row[kMaxOrder];
    double xr, xi;
    fit_entry(a, p, row, xr, xi);
    for (int k = 0; k < a.mi.order; ++k) frow[p * a.mi.order + k] = (int32_t)row[k];
    fx[2 * p] = xr;
    fx[2 * p + 1] = xi;
}

hipError_t launch_fit_set(const FitArgs &a, int32_t *frow, double *fx, hipStream_t st) {
    hipLaunchKernelGGL(fit_set_kernel, dim3((unsigned)ceil_div(a.P_hat, kFitThreads)), dim3(kFitThreads), 0, st, a,
                       frow, fx);
    return hipGetLastError();
}

// Factor entry (r) of row `row` of mode m, real and imaginary parts.
__device__ inline void factor_entry(const FitArgs &a, int m, int64_t row, int r, double &ar, double &ai) {
    const int64_t o = row * a.R + r;
    if (!a.cplx) {
        ar = a.fdouble ? ((const double *)a.A.p[m])[o] : (double)((const float *)a.A.p[m])[o];
        ai = 0.0;
    } else if (a.fdouble) {
        ar = ((const double *)a.A.p[m])[2 * o];
        ai = ((const double *)a.A.p[m])[2 * o + 1];
    } else {
        ar = (double)((const float *)a.A.p[m])[2 * o];
        ai = (double)((const float *)a.A.p[m])[2 * o + 1];
    }
}

__global__ __launch_bounds__(kFitThreads) void fit_partial_kernel(FitArgs a) {
    __shared__ double sh[kFitThreads / kWave];
    __shared__ int s_last;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e2 = 0.0;
    if (p < a.P_hat) {
        const int N = a.mi.order;
        int64_t row[kMaxOrder];
        double xr, xi;
        if (a.frow) {
            for (int k = 0; k < N; ++k) row[k] = a.frow[p * N + k];
            xr = a.fx[2 * p];
            xi = a.fx[2 * p + 1];
        } else {
            fit_entry(a, p, row, xr, xi);
        }
        // model entry sum_r lambda_r prod_m A^(m)(i_m, r), four ranks at a time
        // so that their factor loads are in flight together (same order of
        // operations as one rank at a time)
        double mr = 0.0, mi = 0.0;
        for (int r0 = 0; r0 < a.R; r0 += 4) {
            double zr[4], zi[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                zr[u] = r0 + u < a.R ? a.lambda[r0 + u] : 0.0;
                zi[u] = 0.0;
            }
#pragma unroll
            for (int m = 0; m < kMaxOrder; ++m) {
                if (m >= N) break;
                double ar[4], ai[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (r0 + u < a.R)
                        factor_entry(a, m, row[m], r0 + u, ar[u], ai[u]);
                    else
                        ar[u] = ai[u] = 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (!a.cplx) {
                        zr[u] *= ar[u];
                    } else {
                        const double nr = zr[u] * ar[u] - zi[u] * ai[u], ni = zr[u] * ai[u] + zi[u] * ar[u];
                        zr[u] = nr;
                        zi[u] = ni;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (r0 + u < a.R) {
                    mr += zr[u];
                    mi += zi[u];
                }
        }
        const double dr = xr - mr, di = xi - mi;
        e2 = dr * dr + di * di;
    }
    const double s = block_sum<kFitThreads>(e2, sh);
    if (threadIdx.x == 0) {
        a.part[blockIdx.x] = s;
        s_last = 0;
        if (a.counter) {
            // publish the partial, then let the last block finish (the
            // device-scope fences order the partial stores of every block
            // before the last block's reads, across L2 slices)
            __threadfence();
            const unsigned ticket = atomicAdd(a.counter, 1u);
            s_last = ticket == gridDim.x - 1;
        }
    }
    __syncthreads();
    if (s_last && threadIdx.x < kWave) {
        __threadfence();
        const volatile double *vp = a.part;
        double tot = 0.0;
        for (unsigned b = threadIdx.x; b < gridDim.x; b += kWave) tot += vp[b];
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) tot += __shfl_down(tot, off, kWave);
        if (threadIdx.x == 0) {
            const double f = 1.0 - sqrt(a.P * (tot / (double)a.P_hat)) / *a.normX;
            const uint64_t t = a.t_dev ? *a.t_dev : 0;
            if (a.fit_out) *a.fit_out = f;
            if (a.hist) a.hist[t] = f;
            if (a.hist_host) a.hist_host[t] = f;
            if (a.t_dev) *a.t_dev = t + 1;
            *a.counter = 0u;
        }
    }
}

hipError_t launch_fit_partial(const FitArgs &a, int32_t *nblocks, hipStream_t st) {
    const int nb = (int)ceil_div(a.P_hat, kFitThreads);
    *nblocks = nb;
    hipLaunchKernelGGL(fit_partial_kernel, dim3(nb), dim3(kFitThreads), 0, st, a);
    return hipGetLastError();
}

__global__ void fit_final_kernel(const double *part, int32_t nparts, int32_t P_hat, double P,
                                 const double *normX, double *fit_out, double *hist,
                                 const uint64_t *t_dev) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += part[i];
    const double mu = s / (double)P_hat;
    const double f = 1.0 - sqrt(P * mu) / *normX;
    if (fit_out) *fit_out = f;
    if (hist) hist[t_dev ? *t_dev : 0] = f;
}

hipError_t launch_fit_final(const double *part, int32_t nparts, int32_t P_hat, double P,
                            const double *normX, double *fit_out, double *hist,
                            const uint64_t *t_dev, hipStream_t st) {
    hipLaunchKernelGGL(fit_final_kernel, dim3(1), dim3(64), 0, st, part, nparts, P_hat, P, normX,
                       fit_out, hist, t_dev);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sum of squares; every block covers a fixed contiguous range of the logical
// (column-major) element order, so the result does not depend on timing.
constexpr int kNormBlocks = 1024;

__global__ __launch_bounds__(256) void normsq_kernel(ModeInfo mi, const void *X, int kind,
                                                     int64_t P, int contiguous, double *part) {
    __shared__ double sh[256 / kWave];
    const int64_t per = ceil_div(P, (int64_t)gridDim.x);
    const int64_t b0 = (int64_t)blockIdx.x * per, b1 = min(P, b0 + per);
    double acc = 0.0;
    for (int64_t e = b0 + threadIdx.x; e < b1; e += blockDim.x) {
        int64_t off = e;
        if (!contiguous) {
            int64_t rem = e;
            off = 0;
            for (int m = 0; m < mi.order; ++m) {
                const int64_t im = rem % mi.dims[m];
                rem /= mi.dims[m];
                off += im * mi.strides[m];
            }
        }
        double re, im;
        load_elem(X, kind, off, re, im);
        acc += re * re + im * im;
    }
    const double s = block_sum<256>(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Contiguous, 16-byte aligned data of real or complex FP32 / FP64: the sum of
// squares of all scalar components.  Block b covers a fixed range of 16-byte
// vectors (four loads in flight per thread); block 0 also adds the scalar
// tail past the last whole vector.
template <typename T>
__global__ __launch_bounds__(256) void normsq_vec_kernel(const T *x, int64_t ncomp, double *part) {
    __shared__ double sh[256 / kWave];
    typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type V;
    constexpr int VL = 16 / sizeof(T);
    const int64_t nvec = ncomp / VL;
    const int64_t per = ceil_div(nvec, (int64_t)gridDim.x);
    const int64_t b0 = (int64_t)blockIdx.x * per, b1 = min(nvec, b0 + per);
    const V *v = (const V *)x;
    double acc = 0.0;
    for (int64_t e = b0 + threadIdx.x; e < b1; e += 4 * (int64_t)blockDim.x) {
        V q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t k = e + u * (int64_t)blockDim.x;
            q[u] = k < b1 ? v[k] : V{};
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const T *c = (const T *)&q[u];
#pragma unroll
            for (int j = 0; j < VL; ++j) acc += (double)c[j] * (double)c[j];
        }
    }
    if (blockIdx.x == 0)
        for (int64_t e = nvec * VL + threadIdx.x; e < ncomp; e += blockDim.x) acc += (double)x[e] * (double)x[e];
    const double s = block_sum<256>(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

hipError_t launch_normsq_partial(const ModeInfo &mi, const void *X, int kind, double *part,
                                 int32_t *nparts, hipStream_t st) {
    {
        int64_t P = 1, expect = 1;
        bool contiguous = true;
        for (int m = 0; m < mi.order; ++m) {
            if (mi.strides[m] != expect) contiguous = false;
            expect *= mi.dims[m];
            P *= mi.dims[m];
        }
        if (contiguous && (((uintptr_t)X) & 15) == 0 && kind != K_BF16) {
            const bool cplx = kind == K_C64 || kind == K_C128;
            const int64_t ncomp = P * (cplx ? 2 : 1);
            *nparts = kNormBlocks;
            if (kind == K_F32 || kind == K_C64)
                hipLaunchKernelGGL(normsq_vec_kernel<float>, dim3(kNormBlocks), dim3(256), 0, st, (const float *)X,
                                   ncomp, part);
            else
                hipLaunchKernelGGL(normsq_vec_kernel<double>, dim3(kNormBlocks), dim3(256), 0, st, (const double *)X,
                                   ncomp, part);
            return hipGetLastError();
        }
    }
    int64_t P = 1, expect = 1;
    bool contiguous = true;
    for (int m = 0; m < mi.order; ++m) {
        if (mi.strides[m] != expect) contiguous = false;
        expect *= mi.dims[m];
        P *= mi.dims[m];
    }
    *nparts = kNormBlocks;
    hipLaunchKernelGGL(normsq_kernel, dim3(kNormBlocks), dim3(256), 0, st, mi, X, kind, P,
                       contiguous ? 1 : 0, part);
    return hipGetLastError();
}

__global__ void sqrt_sum_kernel(const double *part, int32_t n, double *out) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = sqrt(s);
}

hipError_t launch_sqrt_sum(const double *part, int32_t nparts, double *out, hipStream_t st) {
    hipLaunchKernelGGL(sqrt_sum_kernel, dim3(1), dim3(64), 0, st, part, nparts, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ void fill_u64_kernel(uint64_t *p, uint64_t v) {
    if (threadIdx.x == 0) *p = v;
}
__global__ void inc_u64_kernel(uint64_t *p) {
    if (threadIdx.x == 0) *p += 1;
}
// Copy the factors and lambda after an outer iteration into one of two
// buffers, chosen by the iteration just finished ((*t_dev - 1) mod 2): the
// loop can launch the next iteration before it reads this one's fit estimate.
__global__ __launch_bounds__(256) void snapshot_kernel(SnapArgs a) {
    const uint64_t t = *a.t_dev - 1;
    uint32_t *dst = (uint32_t *)(t & 1 ? a.dst1 : a.dst0);
    int64_t off = 0;
    for (int m = 0; m <= a.nsrc; ++m) {
        const uint32_t *src = (const uint32_t *)(m < a.nsrc ? a.src[m] : (const void *)a.lambda);
        const int64_t w = m < a.nsrc ? a.words[m] : 2 * (int64_t)a.R;
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < w; e += (int64_t)gridDim.x * blockDim.x)
            dst[off + e] = src[e];
        off += w;
    }
}

hipError_t launch_snapshot(const SnapArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(snapshot_kernel, dim3(32), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t v, hipStream_t st) {
    hipLaunchKernelGGL(fill_u64_kernel, dim3(1), dim3(64), 0, st, p, v);
    return hipGetLastError();
}
hipError_t launch_inc_u64(uint64_t *p, hipStream_t st) {
    hipLaunchKernelGGL(inc_u64_kernel, dim3(1), dim3(64), 0, st, p);
    return hipGetLastError();
}

}  // namespace cprand
