// Sampled least-squares solve through the normal equations (Alg. 3 solve
// step; Section 3.2 cost discussion), FP64 throughout, and the column
// normalisation that yields lambda.
//
// Every workgroup sums the Gram partials and inverts V in LDS (solve_device.hpp);
// the factorisation is repeated per workgroup (R <= 64) so that no extra
// launch or grid synchronisation is needed.  The workgroup then solves its
// block of rows, A_i = W_i V^{-1}, optionally takes one step of iterative
// refinement against the FP32 normal equations (A += (W_ref - A V_ref) V^{-1},
// the residual formed with the FP32 blocks and corrected with the inverse
// already computed), and writes per-block column sums of squares for the
// normalisation kernel.
#include "kernels.hpp"
#include "solve_device.hpp"

namespace cprand {

constexpr int kSolveRows = 32;

__device__ inline double ldw(const void *W, bool dbl, int64_t o) {
    return dbl ? ((const double *)W)[o] : (double)((const float *)W)[o];
}

template <int NT>
__global__ __launch_bounds__(NT) void solve_kernel(SolveArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int R = a.R, ld = R + 1;
    const int tid = threadIdx.x;
    double *B1 = (double *)lds;          // V -> V^{-1}
    double *B2 = B1 + R * ld;            // scratch
    double *B3 = B2 + R * ld;            // V
    double *Ws = B3 + R * ld;            // kSolveRows x ld
    double *A0 = Ws + kSolveRows * ld;   // kSolveRows x ld
    double *cs = A0 + kSolveRows * ld;   // 66
    int *pairs = (int *)(cs + 66);       // 66

    for (int p = tid; p < R * R; p += NT) {
        double acc = 0.0;
        for (int c = 0; c < a.vparts; ++c) acc += a.vpart[(size_t)c * R * R + p];
        const int i = p / R, j = p - i * R;
        B1[i * ld + j] = acc;
        B3[i * ld + j] = acc;
    }
    // rows of this block (independent of the inversion)
    const int i0 = blockIdx.x * kSolveRows;
    const int nr = min(kSolveRows, a.In - i0);
    for (int e = tid; e < nr * R; e += NT) {
        const int ii = e / R, r = e - ii * R;
        double acc = 0.0;
        for (int p = 0; p < a.wparts; ++p)
            acc += ldw(a.W, a.wdouble, (int64_t)p * a.wps + (int64_t)(i0 + ii) * a.wsi + (int64_t)r * a.wsr);
        Ws[ii * ld + r] = acc;
    }
    __syncthreads();
    const int failed = spd_inverse(B1, B2, B3, A0, R, ld, cs, pairs);
    if (tid == 0 && blockIdx.x == 0 && a.info) {
        if (failed)
            *a.info = CPRAND_W_PINV;
        else if (!a.info_sticky)
            *a.info = 0;
    }
    for (int e = tid; e < nr * R; e += NT) {
        const int ii = e / R, r = e - ii * R;
        double s = 0.0;
        for (int k = 0; k < R; ++k) s += Ws[ii * ld + k] * B1[k * ld + r];
        A0[ii * ld + r] = s;
    }
    __syncthreads();
    if (a.Wref) {
        // B3 <- V_ref: the residual is that of the FP32 normal equations
        for (int p = tid; p < R * R; p += NT) {
            double acc = 0.0;
            for (int c = 0; c < a.vrefparts; ++c) acc += a.vref[(size_t)c * R * R + p];
            B3[(p / R) * ld + p % R] = acc;
        }
        __syncthreads();
        for (int e = tid; e < nr * R; e += NT) {
            const int ii = e / R, r = e - ii * R;
            double s = 0.0;
            for (int p = 0; p < a.wrefparts; ++p)
                s += (double)a.Wref[(int64_t)p * a.rps + (int64_t)(i0 + ii) * a.rsi + (int64_t)r * a.rsr];
            for (int k = 0; k < R; ++k) s -= A0[ii * ld + k] * B3[k * ld + r];
            Ws[ii * ld + r] = s;
        }
        __syncthreads();
        for (int e = tid; e < nr * R; e += NT) {
            const int ii = e / R, r = e - ii * R;
            double s = 0.0;
            for (int k = 0; k < R; ++k) s += Ws[ii * ld + k] * B1[k * ld + r];
            A0[ii * ld + r] += s;
        }
        __syncthreads();
    }
    for (int e = tid; e < nr * R; e += NT) {
        const int ii = e / R, r = e - ii * R;
        const double v = A0[ii * ld + r];
        const int64_t o = (int64_t)(i0 + ii) * R + r;
        if (a.adouble)
            ((double *)a.A)[o] = v;
        else
            ((float *)a.A)[o] = (float)v;
    }
    for (int r = tid; r < R; r += NT) {
        double s = 0.0;
        for (int ii = 0; ii < nr; ++ii) {
            const double v = a.adouble ? A0[ii * ld + r] : (double)(float)A0[ii * ld + r];
            s += v * v;
        }
        a.colsq_part[(size_t)blockIdx.x * R + r] = s;
    }
}

hipError_t launch_solve(const SolveArgs &a, int32_t *nblocks, hipStream_t st) {
    const int nb = (int)ceil_div(a.In, kSolveRows);
    *nblocks = nb;
    const int ld = a.R + 1;
    const size_t lds = sizeof(double) * ((size_t)3 * a.R * ld + (size_t)2 * kSolveRows * ld + 66) + sizeof(int) * 66;
    if (a.R <= 16)
        hipLaunchKernelGGL(solve_kernel<64>, dim3(nb), dim3(64), lds, st, a);
    else
        hipLaunchKernelGGL(solve_kernel<256>, dim3(nb), dim3(256), lds, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void normalize_kernel(int32_t In, int32_t R, T *A, const double *colsq, int32_t nb,
                                                        double *lambda) {
    __shared__ double s_lam[kMaxRank];
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += colsq[(size_t)b * R + r];
        const double l = sqrt(s);
        s_lam[r] = l;
        if (blockIdx.x == 0) lambda[r] = l;
    }
    __syncthreads();
    const int64_t tot = (int64_t)In * R;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e % R);
        const double l = s_lam[r];
        if (l > 0.0) A[e] = (T)((double)A[e] / l);
    }
}

hipError_t launch_normalize(int32_t In, int32_t R, void *A, bool adouble, const double *colsq_part, int32_t nblocks,
                            double *lambda, hipStream_t st) {
    const int64_t tot = (int64_t)In * R;
    const int nb = (int)std::min<int64_t>(64, ceil_div(tot, 256));
    if (adouble)
        hipLaunchKernelGGL(normalize_kernel<double>, dim3(nb), dim3(256), 0, st, In, R, (double *)A, colsq_part,
                           nblocks, lambda);
    else
        hipLaunchKernelGGL(normalize_kernel<float>, dim3(nb), dim3(256), 0, st, In, R, (float *)A, colsq_part,
                           nblocks, lambda);
    return hipGetLastError();
}

}  // namespace cprand
