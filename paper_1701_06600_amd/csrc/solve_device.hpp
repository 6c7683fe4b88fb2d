// Device-side FP64 inversion of the R x R normal matrix, shared by the
// solve kernel (solve.hip) and the fused mode-step kernel (step.hip).
//
// V is factored as L L^T (right-looking Cholesky in LDS) and V^{-1} =
// L^{-T} L^{-1} is formed explicitly.  If a pivot falls below 1e-12 of the
// largest diagonal entry, V is diagonalised by parallel cyclic Jacobi
// rotations (round-robin pairing, R/2 disjoint rotations per step) and
// inverted on its eigenvalues above 1e-12 of the largest: the
// pseudo-inverse, which gives the minimum-norm least-squares solution.
#pragma once

#include <math.h>

#include "common.hpp"

namespace cprand {

// Jacobi eigen-decomposition of the symmetric M (stride ld) with
// eigenvectors accumulated in Q; on exit diag(M) holds the eigenvalues.
__device__ inline void jacobi_eig(double *M, double *Q, int R, int ld, double *cs, int *pairs) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int Rp = R + (R & 1);
    __shared__ double s_off, s_diag;
    for (int e = tid; e < R * ld; e += nt) {
        const int i = e / ld, j = e - i * ld;
        Q[e] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 30; ++sweep) {
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
            for (int k = tid; k < Rp / 2; k += nt) {
                // slot 0 fixed, slots 1..Rp-1 rotated by `step`; pair k is (slot k, slot Rp-1-k)
                auto pos = [&](int slot) { return slot == 0 ? 0 : 1 + (slot - 1 + step) % (Rp - 1); };
                int p = pos(k), q = pos(Rp - 1 - k);
                if (p > q) {
                    const int tmp = p;
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
            for (int e = tid; e < (Rp / 2) * R; e += nt) {  // M <- J^T M
                const int k = e / R, j = e - k * R;
                const int p = pairs[2 * k], q = pairs[2 * k + 1];
                if (q >= R) continue;
                const double c = cs[2 * k], s = cs[2 * k + 1];
                const double mp = M[p * ld + j], mq = M[q * ld + j];
                M[p * ld + j] = c * mp - s * mq;
                M[q * ld + j] = s * mp + c * mq;
            }
            __syncthreads();
            for (int e = tid; e < (Rp / 2) * R; e += nt) {  // M <- M J, Q <- Q J
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

// Scratch for spd_inverse: B1, B2, B3 (R x ld doubles each), tmp (>= R
// doubles), cs (2*33 doubles), pairs (2*33 ints).  On entry B1 = B3 = V;
// on exit B1 = V^{-1} (or the pseudo-inverse), B3 = V.  Returns 1 when the
// pseudo-inverse was used.  All threads of the block must call it.
__device__ inline int spd_inverse(double *B1, double *B2, const double *B3, double *tmp, int R, int ld, double *cs,
                                  int *pairs) {
    const int tid = threadIdx.x, nt = blockDim.x;
    __shared__ int s_fail;
    __shared__ double s_maxdiag, s_lmax;
    if (tid == 0) {
        double mx = 0.0;
        for (int i = 0; i < R; ++i) mx = fmax(mx, B1[i * ld + i]);
        s_maxdiag = mx;
        s_fail = (!(mx > 0.0) || !isfinite(mx)) ? 1 : 0;
    }
    __syncthreads();
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
    const int failed = s_fail;
    if (!failed) {
        for (int j = tid; j < R; j += nt) {  // L^{-1} by columns into B2
            for (int i = 0; i < j; ++i) B2[i * ld + j] = 0.0;
            for (int i = j; i < R; ++i) {
                double s = (i == j) ? 1.0 : 0.0;
                for (int k = j; k < i; ++k) s -= B1[i * ld + k] * B2[k * ld + j];
                B2[i * ld + j] = s / B1[i * ld + i];
            }
        }
        __syncthreads();
        for (int e = tid; e < R * R; e += nt) {  // V^{-1} = L^{-T} L^{-1}
            const int i = e / R, j = e - i * R;
            const int k0 = i > j ? i : j;
            double s = 0.0;
            for (int k = k0; k < R; ++k) s += B2[k * ld + i] * B2[k * ld + j];
            B1[i * ld + j] = s;
        }
        __syncthreads();
    } else {
        for (int e = tid; e < R * ld; e += nt) B1[e] = B3[e];
        __syncthreads();
        jacobi_eig(B1, B2, R, ld, cs, pairs);
        if (tid == 0) {
            double mx = 0.0;
            for (int i = 0; i < R; ++i) mx = fmax(mx, fabs(B1[i * ld + i]));
            s_lmax = mx;
        }
        __syncthreads();
        for (int i = tid; i < R; i += nt) {
            const double l = B1[i * ld + i];
            tmp[i] = (l > 1e-12 * s_lmax) ? 1.0 / l : 0.0;
        }
        __syncthreads();
        for (int e = tid; e < R * R; e += nt) {
            const int i = e / R, j = e - i * R;
            double s = 0.0;
            for (int k = 0; k < R; ++k) s += B2[i * ld + k] * tmp[k] * B2[j * ld + k];
            B1[i * ld + j] = s;
        }
        __syncthreads();
    }
    return failed;
}

}  // namespace cprand
