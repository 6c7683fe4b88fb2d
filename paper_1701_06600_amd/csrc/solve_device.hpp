// Device-side FP64 inversion of the R x R normal matrix, shared by the
// solve kernel (solve.hip), the fused mode-step kernel (step.hip) and the
// proposal statistics (proposal.hip).
//
// V is inverted in place by Gauss-Jordan elimination without pivoting (the
// pivots of a symmetric positive definite matrix are the diagonal entries of
// its successive Schur complements, the squares of its Cholesky diagonal):
// R steps, each a parallel rank-one update of all R^2 entries between two
// barriers.  If a pivot falls below 1e-12 of the largest diagonal entry of V,
// V is diagonalised by parallel cyclic Jacobi rotations (round-robin
// pairing, R/2 disjoint rotations per step) and inverted on its eigenvalues
// above 1e-12 of the largest: the pseudo-inverse, which gives the
// minimum-norm least-squares solution.
#pragma once

#include <math.h>

#include "common.hpp"

namespace cprand {

// Sum of v over the block into *out (valid after the call on every thread),
// in a fixed order: wave sums by shuffles, then the wave sums in wave order.
// `sh` holds one double per wave; the block size is a multiple of kWave.
__device__ inline double block_sum_dyn(double v, double *sh) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < nw; ++i) r += sh[i];
    return r;
}

// Jacobi eigen-decomposition of the symmetric M (stride ld) with
// eigenvectors accumulated in Q; on exit diag(M) holds the eigenvalues.
__device__ inline void jacobi_eig(double *M, double *Q, int R, int ld, double *cs, int *pairs) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int Rp = R + (R & 1);
    __shared__ double s_red[16];
    for (int e = tid; e < R * ld; e += nt) {
        const int i = e / ld, j = e - i * ld;
        Q[e] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, dg = 0.0;
        for (int e = tid; e < R * R; e += nt) {
            const int i = e / R, j = e - i * R;
            const double v = M[i * ld + j];
            if (i == j)
                dg += v * v;
            else
                off += v * v;
        }
        off = block_sum_dyn(off, s_red);
        dg = block_sum_dyn(dg, s_red);
        if (!(off > 1e-30 * dg)) break;
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

// Largest |diagonal entry| of M (R <= 64) on every thread, and whether any
// diagonal entry is not finite.  Wave 0 reduces by shuffles.
__device__ inline double diag_absmax(const double *M, int R, int ld, int *bad) {
    __shared__ double s_mx;
    __shared__ int s_bad;
    if (threadIdx.x < kWave) {
        const int l = threadIdx.x;
        const double d = l < R ? M[l * ld + l] : 0.0;
        const int nf = (l < R && !isfinite(d)) ? 1 : 0;
        double mx = fabs(d);
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, kWave));
        const int anybad = __any(nf);
        if (l == 0) {
            s_mx = mx;
            s_bad = anybad;
        }
    }
    __syncthreads();
    *bad = s_bad;
    return s_mx;
}

// Orders the LDS accesses of one wavefront: its lanes run in lockstep, so a
// fence at wavefront scope is all that separates a write from the reads of
// other lanes.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exact select by bit masks (keeps the elimination step free of branches).
__device__ inline double bsel(bool c, double a, double b) {
    const long long m = -(long long)c;
    return __longlong_as_double((__double_as_longlong(a) & m) | (__double_as_longlong(b) & ~m));
}

// One Gauss-Jordan step on pivot k for the entries a thread keeps in
// registers (v[q] at row ii[q], column jj[q]; valid[q] false for padding
// slots), given col[i] = M(i, k), rowp[j] = M(k, j) / M(k, k) and
// inv = 1 / M(k, k):  M(k, k) <- inv, M(k, j) <- rowp[j], M(i, k) <- -col[i] inv,
// M(i, j) <- M(i, j) - col[i] rowp[j].  Every candidate is computed and the
// right one selected; the new values are also stored to M (stride ld).
template <int Q>
__device__ inline void gj_update(double *v, const int *ii, const int *jj, const bool *valid, int k, double inv,
                                 const double *col, const double *rowp, double *M, int ld) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = ii[q], j = jj[q];
        const double ci = col[i], rj = rowp[j];
        const double other = fma(-ci, rj, v[q]);
        const double on_col = -ci * inv;
        const double on_row = bsel(j == k, inv, rj);
        const double nv = bsel(i == k, on_row, bsel(j == k, on_col, other));
        v[q] = nv;
        if (valid[q]) M[i * ld + j] = nv;
    }
}

template <int Q>
__device__ inline void gj_load(const double *M, int R, int ld, int t, int nt, double *v, int *ii, int *jj,
                               bool *valid) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int e = t + q * nt;
        valid[q] = e < R * R;
        const int i = valid[q] ? e / R : 0, j = valid[q] ? e - (e / R) * R : 0;
        ii[q] = i;
        jj[q] = j;
        v[q] = M[i * ld + j];
    }
}

// Gauss-Jordan elimination of B1 (R <= 16) by the first wavefront alone,
// entirely in registers: the matrix is padded to 16 x 16 with zeros (the
// padding is never a pivot and is left unchanged), lane l holds column
// l % 16 of rows l / 16 + 4 q (q < 4), and each step fetches the pivot, the
// pivot column and the pivot row from the owning lanes by shuffles.
// Returns 1 if a pivot falls below 1e-12 maxdiag (B1 is then untouched).
__device__ inline int gj_wave(double *B1, int R, int ld, double maxdiag) {
    const int l = threadIdx.x, j = l & 15, i0 = l >> 4;
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = i0 + 4 * q;
        v[q] = (i < R && j < R) ? B1[i * ld + j] : 0.0;
    }
    for (int k = 0; k < R; ++k) {
        const int kq = k >> 2;  // slot of row k (uniform)
        const double vk = kq == 0 ? v[0] : kq == 1 ? v[1] : kq == 2 ? v[2] : v[3];
        const double piv = __shfl(vk, ((k & 3) << 4) | k, kWave);
        if (!(piv > 1e-12 * maxdiag)) return 1;  // uniform across the wave
        const double inv = 1.0 / piv;
        const double rowp = __shfl(vk, ((k & 3) << 4) | j, kWave) * inv;  // M(k, j) / M(k, k)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + 4 * q;
            const double ci = __shfl(v[q], (l & 48) | k, kWave);  // M(i, k)
            const double other = fma(-ci, rowp, v[q]);
            const double on_col = -ci * inv;
            const double on_row = bsel(j == k, inv, rowp);
            v[q] = bsel(i == k, on_row, bsel(j == k, on_col, other));
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = i0 + 4 * q;
        if (i < R && j < R) B1[i * ld + j] = v[q];
    }
    return 0;
}

// Scratch for spd_inverse: B1, B2, B3 (R x ld doubles each), tmp (>= R
// doubles), cs (2*33 doubles), pairs (2*33 ints).  On entry B1 = B3 = V;
// on exit B1 = V^{-1} (or the pseudo-inverse), B3 = V.  Returns 1 when the
// pseudo-inverse was used.  All threads of the block must call it, and the
// block must have at least R*R / QMAX threads (R <= 16 uses the first wave
// only).  Each step copies the pivot row and column of B1 to LDS scratch
// (B2, tmp), then every thread updates its entries.
template <int QMAX>
__device__ inline int spd_inverse(double *B1, double *B2, const double *B3, double *tmp, int R, int ld, double *cs,
                                  int *pairs) {
    const int tid = threadIdx.x, nt = blockDim.x;
    int bad = 0;
    const double maxdiag = diag_absmax(B1, R, ld, &bad);
    int failed = (bad || !(maxdiag > 0.0)) ? 1 : 0;
    double *col = tmp, *row = B2;
    if (!failed && R <= 16) {
        __shared__ int s_failed;
        if (tid < kWave) {
            const int f = gj_wave(B1, R, ld, maxdiag);
            if (tid == 0) s_failed = f;
        }
        __syncthreads();
        failed = s_failed;
    } else if (!failed) {
        // each thread keeps up to QMAX entries; B1 stays current in LDS
        double v[QMAX];
        int ii[QMAX], jj[QMAX];
        bool valid[QMAX];
        gj_load<QMAX>(B1, R, ld, tid, nt, v, ii, jj, valid);
        for (int k = 0; k < R; ++k) {
            const double piv = B1[k * ld + k];
            if (!(piv > 1e-12 * maxdiag)) {  // same value on every thread: a uniform exit
                failed = 1;
                break;
            }
            const double inv = 1.0 / piv;
            if (tid < R) {
                col[tid] = B1[tid * ld + k];
                row[tid] = B1[k * ld + tid] * inv;
            }
            __syncthreads();
            gj_update<QMAX>(v, ii, jj, valid, k, inv, col, row, B1, ld);
            __syncthreads();
        }
    }
    if (!failed) return 0;
    __syncthreads();
    for (int e = tid; e < R * ld; e += nt) B1[e] = B3[e];
    __syncthreads();
    jacobi_eig(B1, B2, R, ld, cs, pairs);
    const double lmax = diag_absmax(B1, R, ld, &bad);
    for (int i = tid; i < R; i += nt) {
        const double l = B1[i * ld + i];
        tmp[i] = (l > 1e-12 * lmax) ? 1.0 / l : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < R * R; e += nt) {
        const int i = e / R, j = e - i * R;
        double s = 0.0;
        for (int k = 0; k < R; ++k) s += B2[i * ld + k] * tmp[k] * B2[j * ld + k];
        B1[i * ld + j] = s;
    }
    __syncthreads();
    return 1;
}

}  // namespace cprand
