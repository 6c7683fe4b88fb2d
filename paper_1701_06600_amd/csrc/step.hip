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
constexpr int kColParts = 8;

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

    for (int p = tid; p < R * R; p += kStepThreads) {
        double acc = 0.0;
        for (int c = 0; c < a.vparts; ++c) acc += a.vpart[(size_t)c * R * R + p];
        const int i = p / R, j = p - i * R;
        B1[i * ld + j] = acc;
        B3[i * ld + j] = acc;
    }
    if (!a.mix) {
        for (int e = tid; e < In * R; e += kStepThreads) {
            const int i = e / R, r = e - i * R;
            double acc = 0.0;
            for (int p = 0; p < a.wparts; ++p) {
                const int64_t o = (int64_t)p * a.wps + (int64_t)i * a.wsi + (int64_t)r * a.wsr;
                acc += a.wdouble ? ((const double *)a.W)[o] : (double)((const float *)a.W)[o];
            }
            Wd[e] = acc;
        }
    } else {
        const T *y = (const T *)a.W;
        const size_t cstride = (size_t)2 * R * In;
        for (int e = tid; e < In * R; e += kStepThreads) {
            const int c = e / In, l = e - c * In;
            double re = 0.0, im = 0.0;
            for (int p = 0; p < a.wparts; ++p) {
                re += (double)y[p * cstride + (size_t)c * In + l];
                im += (double)y[p * cstride + (size_t)(R + c) * In + l];
            }
            t0[l * ld + c] = {(T)re, (T)im};
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
            double s = 0.0;
            for (int p = 0; p < a.wrefparts; ++p)
                s += (double)a.Wref[(int64_t)p * a.rps + (int64_t)i * a.rsi + (int64_t)r * a.rsr];
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
