// Sampled fit estimate (Section 3.4) and the tensor norm.
//
// Each entry's multi-index comes from Philox (so the set is the same at every
// call) or from the fit set drawn once per run; sixteen lanes evaluate its
// model entry sum_r lambda_r prod_m A^(m)(i_m, r) from the L2-resident factor
// rows and the error is squared; FP64 throughout, fixed-order block sums, and
// the last block (or a one-block kernel) sums the block partials.
#include <math.h>

#include <type_traits>

#include "kernels.hpp"

namespace cprand {

constexpr int kFitThreads = 256;
constexpr int kFitLanes = 16;
static_assert(kFitSamplesPerBlock * kMaxOrder % kFitThreads == 0 && kFitSamplesPerBlock * 2 % kFitThreads == 0,
              "whole staging loads per thread");
static_assert(kFitSamplesPerBlock % (kFitThreads / kFitLanes) == 0, "whole entries per lane group");

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


constexpr int kFitGroups = kFitThreads / kFitLanes;          // lane groups per block
constexpr int kFitJ = kFitSamplesPerBlock / kFitGroups;      // entries per lane group

// Model entries of a lane group's kFitJ entries (grp + kFitGroups j), lane
// taking ranks lane, lane + 16, ...: per mode, the kFitJ factor loads are
// issued together (entry indices past the block's last entry are clamped and
// their sums dropped), FP64 products in the order lambda_r, A^(1), A^(2), ...
template <typename FT, bool CPLX>
__device__ __forceinline__ void fit_model(const FitArgs &a, const int32_t *s_row, int ne, int lane, int grp,
                                          double (&mr)[kFitJ], double (&mi)[kFitJ]) {
    const int N = a.mi.order, R = a.R;
#pragma unroll
    for (int j = 0; j < kFitJ; ++j) mr[j] = mi[j] = 0.0;
    for (int r = lane; r < R; r += kFitLanes) {
        double zr[kFitJ], zi[kFitJ];
        const double lam = a.lambda[r];
#pragma unroll
        for (int j = 0; j < kFitJ; ++j) {
            zr[j] = lam;
            zi[j] = 0.0;
        }
#pragma unroll
        for (int m = 0; m < kMaxOrder; ++m) {  // static m: the factor pointers are scalar kernel arguments
            if (m >= N) break;
            const FT *Am = (const FT *)a.A.p[m];
            FT vr[kFitJ], vi[kFitJ];
#pragma unroll
            for (int j = 0; j < kFitJ; ++j) {
                const int q = min(grp + kFitGroups * j, ne - 1);
                const int64_t o = (int64_t)s_row[q * N + m] * R + r;
                if (CPLX) {
                    vr[j] = Am[2 * o];
                    vi[j] = Am[2 * o + 1];
                } else {
                    vr[j] = Am[o];
                }
            }
#pragma unroll
            for (int j = 0; j < kFitJ; ++j) {
                if (CPLX) {
                    const double ar = (double)vr[j], ai = (double)vi[j];
                    const double nr = zr[j] * ar - zi[j] * ai, ni = zr[j] * ai + zi[j] * ar;
                    zr[j] = nr;
                    zi[j] = ni;
                } else {
                    zr[j] *= (double)vr[j];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kFitJ; ++j) {
            mr[j] += zr[j];
            mi[j] += zi[j];
        }
    }
}

// A block takes kFitSamplesPerBlock entries: their rows and tensor values are
// staged in LDS with coalesced loads (or drawn from Philox), then each group
// of sixteen lanes evaluates sixteen entries, lane k taking ranks k, k + 16,
// ...: the factor loads of all sixteen entries are independent, so they are
// in flight together, and the entry sums are closed with lane shuffles.
// Few blocks keep the ticket counter of the single-launch finish cheap.
__global__ __launch_bounds__(kFitThreads) void fit_partial_kernel(FitArgs a) {
    __shared__ double sh[kFitThreads / kWave];
    __shared__ int s_last;
    __shared__ int32_t s_row[kFitSamplesPerBlock * kMaxOrder];
    __shared__ double s_x[kFitSamplesPerBlock * 2];
    __shared__ double s_w[kFitSamplesPerBlock];
    const int tid = threadIdx.x;
    const int N = a.mi.order;
    const int64_t p0 = (int64_t)blockIdx.x * kFitSamplesPerBlock;
    const int ne = (int)min((int64_t)kFitSamplesPerBlock, (int64_t)a.P_hat - p0);
    // State copy: word g of every segment (factors, then lambda) is loaded
    // here, with the staging loads, and stored after them; words past the
    // grid's size go in a plain loop.  Iteration *t_dev is read before this
    // block takes its ticket, so before the last block advances it.
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + tid, gs = (int64_t)gridDim.x * blockDim.x;
    const int nseg = a.snap.nsrc > 0 ? a.snap.nsrc + 1 : 0;
    uint32_t snapv[kMaxOrder + 1];
    uint64_t snap_t = 0;
    if (nseg > 0) snap_t = *a.t_dev;
#pragma unroll
    for (int m = 0; m <= kMaxOrder; ++m) {
        if (m >= nseg) break;
        const uint32_t *src = (const uint32_t *)(m < a.snap.nsrc ? a.snap.src[m] : (const void *)a.snap.lambda);
        const int64_t w = m < a.snap.nsrc ? a.snap.words[m] : 2 * (int64_t)a.snap.R;
        snapv[m] = g < w ? src[g] : 0u;
    }
    if (a.frow) {  // every load of the staging in flight at once
        constexpr int kRowLoads = kFitSamplesPerBlock * kMaxOrder / kFitThreads;
        constexpr int kXLoads = kFitSamplesPerBlock * 2 / kFitThreads;
        int32_t rv[kRowLoads];
        double xv[kXLoads];
#pragma unroll
        for (int u = 0; u < kRowLoads; ++u) {
            const int e = tid + u * kFitThreads;
            rv[u] = e < ne * N ? a.frow[p0 * N + e] : 0;
        }
#pragma unroll
        for (int u = 0; u < kXLoads; ++u) {
            const int e = tid + u * kFitThreads;
            xv[u] = e < 2 * ne ? a.fx[2 * p0 + e] : 0.0;
        }
        if (a.fw)
            for (int e = tid; e < ne; e += kFitThreads) s_w[e] = a.fw[p0 + e];
#pragma unroll
        for (int u = 0; u < kRowLoads; ++u) s_row[tid + u * kFitThreads] = rv[u];
#pragma unroll
        for (int u = 0; u < kXLoads; ++u) s_x[tid + u * kFitThreads] = xv[u];
    }
    if (nseg > 0) {
        uint32_t *dst = (uint32_t *)(snap_t & 1 ? a.snap.dst1 : a.snap.dst0);
        int64_t off = 0;
#pragma unroll
        for (int m = 0; m <= kMaxOrder; ++m) {
            if (m >= nseg) break;
            const uint32_t *src = (const uint32_t *)(m < a.snap.nsrc ? a.snap.src[m] : (const void *)a.snap.lambda);
            const int64_t w = m < a.snap.nsrc ? a.snap.words[m] : 2 * (int64_t)a.snap.R;
            if (g < w) dst[off + g] = snapv[m];
            for (int64_t e = g + gs; e < w; e += gs) dst[off + e] = src[e];
            off += w;
        }
    }
    if (!a.frow && tid < ne) {
        int64_t row[kMaxOrder];
        double xr, xi;
        fit_entry(a, p0 + tid, row, xr, xi);
#pragma unroll
        for (int k = 0; k < kMaxOrder; ++k)
            if (k < N) s_row[tid * N + k] = (int32_t)row[k];
        s_x[2 * tid] = xr;
        s_x[2 * tid + 1] = xi;
    }
    __syncthreads();
    // model entries sum_r lambda_r prod_m A^(m)(i_m, r) of entries grp + 16 j
    const int lane = tid & (kFitLanes - 1), grp = tid / kFitLanes;
    double mr[kFitJ], mi[kFitJ];
    if (a.cplx) {
        if (a.fdouble)
            fit_model<double, true>(a, s_row, ne, lane, grp, mr, mi);
        else
            fit_model<float, true>(a, s_row, ne, lane, grp, mr, mi);
    } else {
        if (a.fdouble)
            fit_model<double, false>(a, s_row, ne, lane, grp, mr, mi);
        else
            fit_model<float, false>(a, s_row, ne, lane, grp, mr, mi);
    }
    double e2 = 0.0;
#pragma unroll
    for (int j = 0; j < kFitJ; ++j) {
#pragma unroll
        for (int off = kFitLanes / 2; off > 0; off >>= 1) {
            mr[j] += __shfl_xor(mr[j], off, kFitLanes);
            mi[j] += __shfl_xor(mi[j], off, kFitLanes);
        }
        const int q = grp + kFitGroups * j;
        if (lane == 0 && q < ne) {
            const double dr = s_x[2 * q] - mr[j], di = s_x[2 * q + 1] - mi[j];
            const double sq = dr * dr + di * di;
            e2 += (a.frow && a.fw) ? s_w[q] * sq : sq;
        }
    }
    const double s = block_sum<kFitThreads>(e2, sh);
    if (tid == 0) {
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
    if (s_last) {
        __threadfence();
        const volatile double *vp = a.part;
        double tot = 0.0;
        for (unsigned b = tid; b < gridDim.x; b += kFitThreads) tot += vp[b];
        tot = block_sum<kFitThreads>(tot, sh);
        if (tid == 0) {
            const double f = 1.0 - sqrt(a.P * (tot / (double)a.P_hat)) / *a.normX;
            const uint64_t t = a.t_dev ? *a.t_dev : a.t;
            if (a.fit_out) *a.fit_out = f;
            if (a.hist) a.hist[t] = f;
            if (a.hist_host) a.hist_host[t] = f;
            if (a.t_dev) *a.t_dev = t + 1;
            *a.counter = 0u;
        }
    }
}

hipError_t launch_fit_partial(const FitArgs &a, int32_t *nblocks, hipStream_t st) {
    const int nb = (int)fit_partials(a.P_hat);
    *nblocks = nb;
    hipLaunchKernelGGL(fit_partial_kernel, dim3(nb), dim3(kFitThreads), 0, st, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(kFitThreads) void fit_final_kernel(const double *part, int32_t nparts, int32_t P_hat,
                                                               double P, const double *normX, double *fit_out,
                                                               double *hist, const uint64_t *t_dev) {
    __shared__ double sh[kFitThreads / kWave];
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kFitThreads) s += part[i];
    s = block_sum<kFitThreads>(s, sh);
    if (threadIdx.x != 0) return;
    const double mu = s / (double)P_hat;
    const double f = 1.0 - sqrt(P * mu) / *normX;
    if (fit_out) *fit_out = f;
    if (hist) hist[t_dev ? *t_dev : 0] = f;
}

hipError_t launch_fit_final(const double *part, int32_t nparts, int32_t P_hat, double P,
                            const double *normX, double *fit_out, double *hist,
                            const uint64_t *t_dev, hipStream_t st) {
    hipLaunchKernelGGL(fit_final_kernel, dim3(1), dim3(kFitThreads), 0, st, part, nparts, P_hat, P, normX,
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

__global__ __launch_bounds__(256) void sqrt_sum_kernel(const double *part, int32_t n, double *out) {
    __shared__ double sh[256 / kWave];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    s = block_sum<256>(s, sh);
    if (threadIdx.x == 0) *out = sqrt(s);
}

hipError_t launch_sqrt_sum(const double *part, int32_t nparts, double *out, hipStream_t st) {
    hipLaunchKernelGGL(sqrt_sum_kernel, dim3(1), dim3(256), 0, st, part, nparts, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ void fill_u64_kernel(uint64_t *p, uint64_t v) {
    if (threadIdx.x == 0) *p = v;
}
__global__ void inc_u64_kernel(uint64_t *p) {
    if (threadIdx.x == 0) *p += 1;
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
