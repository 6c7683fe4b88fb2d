// Sampled least-squares solve through the normal equations (Alg. 3 solve
// step; Section 3.2 cost discussion), FP64 throughout, and the column
// normalisation that yields lambda.
//
// Every workgroup sums the Gram partials, factors V = L L^T (Cholesky) in
// LDS and forms V^{-1} = L^{-T} L^{-1}; the factorisation is repeated per
// workgroup (R <= 64, a few microseconds) so that no extra launch or grid
// synchronisation is needed.  If a pivot falls below 1e-12 of the largest
// diagonal entry, V is instead diagonalised by parallel cyclic Jacobi
// rotations and inverted on its numerically non-zero eigenvalues
// (pseudo-inverse), and *info is set.  The workgroup then solves its block
// of rows, A_i = W_i V^{-1}, optionally refines once against an FP32
// right-hand side, and writes per-block column sums of squares.
#include <math.h>

#include "kernels.hpp"

namespace cprand {

constexpr int kSolveRows = 32;
constexpr int kSolveThreads = 256;

__device__ inline double ldw(const void *W, bool dbl, int64_t o) {
    return dbl ? ((const double *)W)[o] : (double)((const float *)W)[o];
}

// Parallel cyclic Jacobi on the symmetric R x R matrix M (stride ld) with
// eigenvectors accumulated in Q; on exit the diagonal of M holds the
// eigenvalues.  Round-robin pairing: R is padded to an even count and in
// each of the Rp-1 steps every index is paired once.
__device__ void jacobi_eig(double *M, double *Q, int R, int ld, double *cs, int *pairs) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int Rp = R + (R & 1);
    for (int e = tid; e < R * ld; e += nt) {
        const int i = e / ld, j = e - i * ld;
        Q[e] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 30; ++sweep) {
        // off-diagonal norm test
        __shared__ double s_off, s_diag;
        if (tid == 0) {
            double off = 0.0, dg = 0.0;
            for (int i = 0; i < R; ++i)
                for (int j = 0; j < R; ++j) {
                    const double v = M[i * ld + j];
                    if (i == j)
                        dg += v * v;
                    else
                        off += v * v;
                }
            s_off = off;
            s_diag = dg;
        }
        __syncthreads();
        if (!(s_off > 1e-30 * s_diag)) break;
        for (int step = 0; step < Rp - 1; ++step) {
            // pair (p, q) number k: positions k and Rp-1-k of a rotating list
            // where slot 0 is fixed and the others rotate by `step`.
            for (int k = tid; k < Rp / 2; k += nt) {
                int a = k, b = Rp - 1 - k;
                auto pos = [&](int slot) { return slot == 0 ? 0 : 1 + (slot - 1 + step) % (Rp - 1); };
                int p = pos(a), q = pos(b);
                if (p > q) {
                    int tmp = p;
                    p = q;
                    q = tmp;
                }
                double c = 1.0, s = 0.0;
                if (q < R) {
                    const double apq = M[p * ld + q];
                    if (apq != 0.0) {
                        const double tau = (M[q * ld + q] - M[p * ld + p]) / (2.0 * apq);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                }
                pairs[2 * k] = p;
                pairs[2 * k + 1] = q;
                cs[2 * k] = c;
                cs[2 * k + 1] = s;
            }
            __syncthreads();
            // rows: M <- J^T M
            for (int e = tid; e < (Rp / 2) * R; e += nt) {
                const int k = e / R, j = e - k * R;
                const int p = pairs[2 * k], q = pairs[2 * k + 1];
                if (q >= R) continue;
                const double c = cs[2 * k], s = cs[2 * k + 1];
                const double mp = M[p * ld + j], mq = M[q * ld + j];
                M[p * ld + j] = c * mp - s * mq;
                M[q * ld + j] = s * mp + c * mq;
            }
            __syncthreads();
            // columns: M <- M J, Q <- Q J
            for (int e = tid; e < (Rp / 2) * R; e += nt) {
                const int k = e / R, i = e - k * R;
                const int p = pairs[2 * k], q = pairs[2 * k + 1];
                if (q >= R) continue;
                const double c = cs[2 * k], s = cs[2 * k + 1];
                const double mp = M[i * ld + p], mq = M[i * ld + q];
                M[i * ld + p] = c * mp - s * mq;
                M[i * ld + q] = s * mp + c * mq;
                const double qp = Q[i * ld + p], qq = Q[i * ld + q];
                Q[i * ld + p] = c * qp - s * qq;
                Q[i * ld + q] = s * qp + c * qq;
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(kSolveThreads) void solve_kernel(SolveArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int R = a.R, ld = R + 1;
    const int tid = threadIdx.x, nt = blockDim.x;
    double *B1 = (double *)lds;          // V -> L -> V^{-1}
    double *B2 = B1 + R * ld;            // L^{-1} (or Jacobi eigenvectors)
    double *B3 = B2 + R * ld;            // copy of V
    double *Ws = B3 + R * ld;            // kSolveRows x ld: W rows, then A rows
    double *A0 = Ws + kSolveRows * ld;   // kSolveRows x ld (refinement)
    double *cs = A0 + kSolveRows * ld;   // 2 * 33
    int *pairs = (int *)(cs + 2 * 33);   // 2 * 33
    __shared__ int s_fail;
    __shared__ double s_maxdiag;

    // V = sum of the Gram partials (fixed order)
    for (int p = tid; p < R * R; p += nt) {
        double acc = 0.0;
        for (int c = 0; c < a.vparts; ++c) acc += a.vpart[(size_t)c * R * R + p];
        const int i = p / R, j = p - i * R;
        B1[i * ld + j] = acc;
        B3[i * ld + j] = acc;
    }
    if (tid == 0) s_fail = 0;
    __syncthreads();
    if (tid == 0) {
        double mx = 0.0;
        for (int i = 0; i < R; ++i) mx = fmax(mx, B1[i * ld + i]);
        s_maxdiag = mx;
        if (!(mx > 0.0) || !isfinite(mx)) s_fail = 1;
    }
    __syncthreads();

    // Cholesky, right-looking, lower triangle of B1
    for (int k = 0; k < R && !s_fail; ++k) {
        if (tid == 0) {
            const double d = B1[k * ld + k];
            if (!(d > 1e-12 * s_maxdiag))
                s_fail = 1;
            else
                B1[k * ld + k] = sqrt(d);
        }
        __syncthreads();
        if (s_fail) break;
        const double dk = B1[k * ld + k];
        for (int i = k + 1 + tid; i < R; i += nt) B1[i * ld + k] /= dk;
        __syncthreads();
        const int m = R - k - 1;
        for (int e = tid; e < m * m; e += nt) {
            const int i = k + 1 + e / m, j = k + 1 + e % m;
            if (j <= i) B1[i * ld + j] -= B1[i * ld + k] * B1[j * ld + k];
        }
        __syncthreads();
    }
    __syncthreads();

    if (!s_fail) {
        // L^{-1} by columns (forward substitution), into B2 (lower)
        for (int j = tid; j < R; j += nt) {
            for (int i = 0; i < j; ++i) B2[i * ld + j] = 0.0;
            for (int i = j; i < R; ++i) {
                double s = (i == j) ? 1.0 : 0.0;
                for (int k = j; k < i; ++k) s -= B1[i * ld + k] * B2[k * ld + j];
                B2[i * ld + j] = s / B1[i * ld + i];
            }
        }
        __syncthreads();
        // V^{-1} = L^{-T} L^{-1} into B1
        for (int e = tid; e < R * R; e += nt) {
            const int i = e / R, j = e - i * R;
            const int k0 = i > j ? i : j;
            double s = 0.0;
            for (int k = k0; k < R; ++k) s += B2[k * ld + i] * B2[k * ld + j];
            B1[i * ld + j] = s;
        }
        __syncthreads();
    } else {
        // pseudo-inverse through the eigen-decomposition of V
        for (int e = tid; e < R * ld; e += nt) B1[e] = B3[e];
        __syncthreads();
        jacobi_eig(B1, B2, R, ld, cs, pairs);
        __shared__ double s_lmax;
        if (tid == 0) {
            double mx = 0.0;
            for (int i = 0; i < R; ++i) mx = fmax(mx, fabs(B1[i * ld + i]));
            s_lmax = mx;
        }
        __syncthreads();
        // eigenvalues to Ws row 0 (temporarily)
        for (int i = tid; i < R; i += nt) {
            const double l = B1[i * ld + i];
            Ws[i] = (l > 1e-12 * s_lmax) ? 1.0 / l : 0.0;
        }
        __syncthreads();
        for (int e = tid; e < R * R; e += nt) {
            const int i = e / R, j = e - i * R;
            double s = 0.0;
            for (int k = 0; k < R; ++k) s += B2[i * ld + k] * Ws[k] * B2[j * ld + k];
            B1[i * ld + j] = s;
        }
        __syncthreads();
    }
    if (tid == 0 && blockIdx.x == 0 && a.info) {
        if (s_fail)
            *a.info = CPRAND_W_PINV;
        else if (!a.info_sticky)
            *a.info = 0;
    }

    // rows of this block
    const int i0 = blockIdx.x * kSolveRows;
    const int nr = min(kSolveRows, a.In - i0);
    for (int e = tid; e < nr * R; e += nt) {
        const int ii = e / R, r = e - ii * R;
        double acc = 0.0;
        for (int p = 0; p < a.wparts; ++p)
            acc += ldw(a.W, a.wdouble, (int64_t)p * a.wps + (int64_t)(i0 + ii) * a.wsi + (int64_t)r * a.wsr);
        Ws[ii * ld + r] = acc;
    }
    __syncthreads();
    for (int e = tid; e < nr * R; e += nt) {
        const int ii = e / R, r = e - ii * R;
        double s = 0.0;
        for (int k = 0; k < R; ++k) s += Ws[ii * ld + k] * B1[k * ld + r];
        A0[ii * ld + r] = s;
    }
    __syncthreads();
    if (a.Wref) {
        // residual right-hand side W_ref - A0 V, then A0 += resid V^{-1}
        for (int e = tid; e < nr * R; e += nt) {
            const int ii = e / R, r = e - ii * R;
            double s = 0.0;
            for (int p = 0; p < a.wrefparts; ++p)
                s += (double)a.Wref[(int64_t)p * a.rps + (int64_t)(i0 + ii) * a.rsi + (int64_t)r * a.rsr];
            for (int k = 0; k < R; ++k) s -= A0[ii * ld + k] * B3[k * ld + r];
            Ws[ii * ld + r] = s;
        }
        __syncthreads();
        for (int e = tid; e < nr * R; e += nt) {
            const int ii = e / R, r = e - ii * R;
            double s = 0.0;
            for (int k = 0; k < R; ++k) s += Ws[ii * ld + k] * B1[k * ld + r];
            A0[ii * ld + r] += s;
        }
        __syncthreads();
    }
    for (int e = tid; e < nr * R; e += nt) {
        const int ii = e / R, r = e - ii * R;
        const double v = A0[ii * ld + r];
        const int64_t o = (int64_t)(i0 + ii) * R + r;
        if (a.adouble)
            ((double *)a.A)[o] = v;
        else
            ((float *)a.A)[o] = (float)v;
    }
    for (int r = tid; r < R; r += nt) {
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
    const size_t lds = sizeof(double) * ((size_t)3 * a.R * ld + (size_t)2 * kSolveRows * ld + 66) +
                       sizeof(int) * 66;
    hipLaunchKernelGGL(solve_kernel, dim3(nb), dim3(kSolveThreads), lds, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void normalize_kernel(int32_t In, int32_t R, T *A,
                                                        const double *colsq, int32_t nb,
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
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e % R);
        const double l = s_lam[r];
        if (l > 0.0) A[e] = (T)((double)A[e] / l);
    }
}

hipError_t launch_normalize(int32_t In, int32_t R, void *A, bool adouble, const double *colsq_part,
                            int32_t nblocks, double *lambda, hipStream_t st) {
    const int64_t tot = (int64_t)In * R;
    const int nb = (int)std::min<int64_t>(64, ceil_div(tot, 256));
    if (adouble)
        hipLaunchKernelGGL(normalize_kernel<double>, dim3(nb), dim3(256), 0, st, In, R, (double *)A,
                           colsq_part, nblocks, lambda);
    else
        hipLaunchKernelGGL(normalize_kernel<float>, dim3(nb), dim3(256), 0, st, In, R, (float *)A,
                           colsq_part, nblocks, lambda);
    return hipGetLastError();
}

}  // namespace cprand
