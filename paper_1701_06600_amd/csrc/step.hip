// Everything after the gather of one mode step, in one workgroup, when the
// mode's I_n x R blocks fit in LDS: sum the MTTKRP and Gram partials, (MIX)
// unmix the product with D_n F_n^* (Alg. 4 unmix, applied to the I_n x R
// product), invert V (FP64), solve A = W V^{-1} (Alg. 3), optionally refine
// once against FP32 data, normalise the columns into lambda, and (MIX) remix
// the new factor, A-hat = F_n D_n A (Alg. 4).  Replaces five launches per
// mode step at the sizes where the step is latency-bound.
#include "fft_device.hpp"
#include "kernels.hpp"
#include "solve_device.hpp"

namespace cprand {

constexpr int kStepThreads = 512;
constexpr int kColParts = 16;
constexpr int kMaxParts = 8;  // partial products summed here (the gathers use at most this many chunks)

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    typedef float4 type;
};
template <>
struct Vec16<double> {
    typedef double2 type;
};
__device__ inline float vget(const float4 &v, int u) { return u == 0 ? v.x : u == 1 ? v.y : u == 2 ? v.z : v.w; }
__device__ inline double vget(const double2 &v, int u) { return u == 0 ? v.x : v.y; }

template <typename T>
__global__ __launch_bounds__(kStepThreads) void step_finish_kernel(StepArgs a, FftPlan fp) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int In = a.In, R = a.R, ld = R + 1;
    const int tid = threadIdx.x;
    double *B1 = (double *)lds;
    double *B2 = B1 + R * ld;
    double *B3 = B2 + R * ld;
    double *cs = B3 + R * ld;            // 66
    double *tmp = cs + 66;               // max(R, kColParts * R)
    int *pairs = (int *)(tmp + kColParts * kMaxRank);  // 66
    double *Wd = (double *)(pairs + 68); // In x R
    double *Ad = Wd + (size_t)In * R;    // In x R
    cx<T> *t0 = (cx<T> *)(Ad + (size_t)In * R);  // MIX: In x ld, twice, + twiddles
    cx<T> *t1 = t0 + (size_t)In * ld;
    cx<T> *tw = t1 + (size_t)In * ld;

    // Partial products (at most kMaxParts) are added in partial order; the
    // loads of one element are issued together, two elements per pass.
    for (int p = tid; p < R * R; p += kStepThreads) {
        double v[kMaxParts];
#pragma unroll
        for (int c = 0; c < kMaxParts; ++c) v[c] = c < a.vparts ? a.vpart[(size_t)c * R * R + p] : 0.0;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < kMaxParts; ++c)
            if (c < a.vparts) acc += v[c];
        const int i = p / R, j = p - i * R;
        B1[i * ld + j] = acc;
        B3[i * ld + j] = acc;
    }
    constexpr int VL = 16 / sizeof(T);  // values per 16-byte load
    typedef typename Vec16<T>::type V16;
    if (!a.mix && a.wsi == 1 && In % VL == 0 && a.wsr % VL == 0 && a.wps % VL == 0) {
        // (i .. i+VL-1, r) of every partial in one 16-byte load each
        const T *w = (const T *)a.W;
        const int ng = R * (In / VL);
        for (int g = tid; g < ng; g += kStepThreads) {
            const int r = g / (In / VL), i0 = (g - r * (In / VL)) * VL;
            V16 v[kMaxParts];
#pragma unroll
            for (int p = 0; p < kMaxParts; ++p)
                v[p] = p < a.wparts ? *(const V16 *)(w + (int64_t)p * a.wps + (int64_t)r * a.wsr + i0) : V16{};
#pragma unroll
            for (int u = 0; u < VL; ++u) {
                double acc = 0.0;
#pragma unroll
                for (int p = 0; p < kMaxParts; ++p)
                    if (p < a.wparts) acc += (double)vget(v[p], u);
                Wd[(i0 + u) * R + r] = acc;
            }
        }
    } else if (a.mix && In % VL == 0) {
        // real and imaginary rows of column c, VL consecutive l per load
        const T *y = (const T *)a.W;
        const size_t cstride = (size_t)2 * R * In;
        const int ng = R * (In / VL);
        for (int g = tid; g < ng; g += kStepThreads) {
            const int c = g / (In / VL), l0 = (g - c * (In / VL)) * VL;
            V16 vr[kMaxParts], vi[kMaxParts];
#pragma unroll
            for (int p = 0; p < kMaxParts; ++p) {
                vr[p] = p < a.wparts ? *(const V16 *)(y + p * cstride + (size_t)c * In + l0) : V16{};
                vi[p] = p < a.wparts ? *(const V16 *)(y + p * cstride + (size_t)(R + c) * In + l0) : V16{};
            }
#pragma unroll
            for (int u = 0; u < VL; ++u) {
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int p = 0; p < kMaxParts; ++p)
                    if (p < a.wparts) {
                        re += (double)vget(vr[p], u);
                        im += (double)vget(vi[p], u);
                    }
                t0[(l0 + u) * ld + c] = {(T)re, (T)im};
            }
        }
        for (int e = tid; e < In; e += kStepThreads) tw[e] = ((const cx<T> *)fp.tw)[e];
    } else if (!a.mix) {
        const T *w = (const T *)a.W;
        for (int e0 = tid; e0 < In * R; e0 += 2 * kStepThreads) {
            T v[2][kMaxParts];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int e = e0 + h * kStepThreads;
                const int i = e / R, r = e - i * R;
#pragma unroll
                for (int p = 0; p < kMaxParts; ++p)
                    v[h][p] = (e < In * R && p < a.wparts) ? w[(int64_t)p * a.wps + (int64_t)i * a.wsi + (int64_t)r * a.wsr]
                                                          : (T)0;
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int e = e0 + h * kStepThreads;
                double acc = 0.0;
#pragma unroll
                for (int p = 0; p < kMaxParts; ++p)
                    if (p < a.wparts) acc += (double)v[h][p];
                if (e < In * R) Wd[e] = acc;
            }
        }
    } else {
        const T *y = (const T *)a.W;
        const size_t cstride = (size_t)2 * R * In;
        for (int e0 = tid; e0 < In * R; e0 += 2 * kStepThreads) {
            T vr[2][kMaxParts], vi[2][kMaxParts];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int e = e0 + h * kStepThreads;
                const int c = e / In, l = e - c * In;
                const bool ok = e < In * R;
#pragma unroll
                for (int p = 0; p < kMaxParts; ++p) {
                    vr[h][p] = (ok && p < a.wparts) ? y[p * cstride + (size_t)c * In + l] : (T)0;
                    vi[h][p] = (ok && p < a.wparts) ? y[p * cstride + (size_t)(R + c) * In + l] : (T)0;
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int e = e0 + h * kStepThreads;
                const int c = e / In, l = e - c * In;
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int p = 0; p < kMaxParts; ++p)
                    if (p < a.wparts) {
                        re += (double)vr[h][p];
                        im += (double)vi[h][p];
                    }
                if (e < In * R) t0[l * ld + c] = {(T)re, (T)im};
            }
        }
        for (int e = tid; e < In; e += kStepThreads) tw[e] = ((const cx<T> *)fp.tw)[e];
    }
    __syncthreads();
    const int failed = spd_inverse(B1, B2, B3, tmp, R, ld, cs, pairs);
    if (tid == 0 && a.info && failed) *a.info = CPRAND_W_PINV;
    const T scale = (T)(1.0 / sqrt((double)In));
    if (a.mix) {
        const cx<T> *res = fft_tile_rt<T, 1>(t0, t1, fp, ld, R, tw);
        for (int e = tid; e < In * R; e += kStepThreads) {
            const int l = e / R, c = e - l * R;
            Wd[e] = (double)((T)a.sign[l] * res[l * ld + c].re * scale);
        }
        __syncthreads();
    }
    for (int e = tid; e < In * R; e += kStepThreads) {
        const int i = e / R, r = e - i * R;
        double s = 0.0;
        for (int k = 0; k < R; ++k) s += Wd[i * R + k] * B1[k * ld + r];
        Ad[e] = s;
    }
    __syncthreads();
    if (a.Wref) {
        for (int e = tid; e < In * R; e += kStepThreads) {
            const int i = e / R, r = e - i * R;
            float v[kMaxParts];
#pragma unroll
            for (int p = 0; p < kMaxParts; ++p)
                v[p] = p < a.wrefparts ? a.Wref[(int64_t)p * a.rps + (int64_t)i * a.rsi + (int64_t)r * a.rsr] : 0.f;
            double s = 0.0;
#pragma unroll
            for (int p = 0; p < kMaxParts; ++p)
                if (p < a.wrefparts) s += (double)v[p];
            for (int k = 0; k < R; ++k) s -= Ad[i * R + k] * B3[k * ld + r];
            Wd[e] = s;
        }
        __syncthreads();
        for (int e = tid; e < In * R; e += kStepThreads) {
            const int i = e / R, r = e - i * R;
            double s = 0.0;
            for (int k = 0; k < R; ++k) s += Wd[i * R + k] * B1[k * ld + r];
            Ad[e] += s;
        }
        __syncthreads();
    }
    // column norms of the stored (T-rounded) values, fixed-order partial sums
    for (int e = tid; e < kColParts * R; e += kStepThreads) {
        const int r = e / kColParts, part = e - r * kColParts;
        double s = 0.0;
        for (int i = part; i < In; i += kColParts) {
            const double v = (double)(T)Ad[i * R + r];
            s += v * v;
        }
        tmp[r * kColParts + part] = s;
    }
    __syncthreads();
    if (tid < R) {
        double s = 0.0;
        for (int part = 0; part < kColParts; ++part) s += tmp[tid * kColParts + part];
        const double l = sqrt(s);
        B2[tid] = l;  // B2 is free after the inversion
        a.lambda[tid] = l;
    }
    __syncthreads();
    T *A = (T *)a.A;
    for (int e = tid; e < In * R; e += kStepThreads) {
        const int r = e % R;
        const double l = B2[r];
        const T v = (T)Ad[e];
        const T nv = l > 0.0 ? (T)((double)v / l) : v;
        A[e] = nv;
        if (a.mix) t0[(e / R) * ld + r] = {(T)a.sign[e / R] * nv, (T)0};
    }
    if (a.mix) {
        __syncthreads();
        const cx<T> *res = fft_tile_rt<T, -1>(t0, t1, fp, ld, R, tw);
        T *Ah = (T *)a.Ahat;
        for (int e = tid; e < In * R; e += kStepThreads) {
            const int l = e / R, c = e - l * R;
            const cx<T> v = res[l * ld + c];
            Ah[2 * (size_t)e] = v.re * scale;
            Ah[2 * (size_t)e + 1] = v.im * scale;
        }
    }
}

size_t step_finish_lds(int32_t In, int32_t R, bool mix, bool dbl) {
    const size_t ld = (size_t)R + 1;
    size_t b = sizeof(double) * (3 * (size_t)R * ld + 66 + (size_t)kColParts * kMaxRank) + sizeof(int) * 68;
    b += sizeof(double) * 2 * (size_t)In * R;
    if (mix) b += (dbl ? 16 : 8) * ((size_t)2 * In * ld + In);
    return b;
}

hipError_t launch_step_finish(const StepArgs &a, const FftPlan *fp, bool dbl, hipStream_t st) {
    if (a.vparts > kMaxParts || a.wparts > kMaxParts || (a.Wref && a.wrefparts > kMaxParts)) return hipErrorInvalidValue;
    const size_t lds = step_finish_lds(a.In, a.R, a.mix, dbl);
    FftPlan f{};
    if (fp) f = *fp;
    if (dbl)
        hipLaunchKernelGGL(step_finish_kernel<double>, dim3(1), dim3(kStepThreads), lds, st, a, f);
    else
        hipLaunchKernelGGL(step_finish_kernel<float>, dim3(1), dim3(kStepThreads), lds, st, a, f);
    return hipGetLastError();
}

}  // namespace cprand
