// Device-side FP64 inversion of the R x R normal matrix, shared by the
// solve kernel (solve.hip), the fused mode-step kernel (step.hip) and the
// proposal statistics (proposal.hip).
//
// V is inverted in place by Gauss-Jordan elimination without pivoting (the
// pivots of a symmetric positive definite matrix are the diagonal entries of
// its successive Schur complements, the squares of its Cholesky diagonal):
// for R <= 16 by one wave in registers (R steps, shuffles between lanes, no
// barriers), above that blocked by 4 (ceil(R / 4) steps, each a rank-4
// update of the whole matrix between two barriers).  If a pivot falls below 1e-12 of the largest diagonal entry of V,
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
__device__ __forceinline__ void jacobi_eig(double *M, double *Q, int R, int ld, double *cs, int *pairs) {
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

// Exact select by bit masks (keeps the elimination step free of branches).
__device__ inline double bsel(bool c, double a, double b) {
    const long long m = -(long long)c;
    return __longlong_as_double((__double_as_longlong(a) & m) | (__double_as_longlong(b) & ~m));
}

// A double held by lane `lane` (a constant), as a wave-uniform value.
__device__ __forceinline__ double read_lane(double x, int lane) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, lane), hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// One scalar Gauss-Jordan step (pivot k) in the gj_wave_regs layout.
__device__ __forceinline__ void gj_wave_step(double (&v)[4], int k, double thr, int &bad) {
    const int l = threadIdx.x & (kWave - 1), j = l & 15, i0 = l >> 4;
    const double vk = v[k >> 2];
    const double piv = read_lane(vk, ((k & 3) << 4) | k);
    const double rk = __shfl(vk, ((k & 3) << 4) | j, kWave);  // M(k, j)
    double c[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) c[q] = __shfl(v[q], (l & 48) | k, kWave);  // M(i0 + 4 q, k)
    bad |= !(piv > thr);
    const double inv = 1.0 / piv;
    const double rowp = rk * inv;  // M(k, j) / M(k, k)
    const double on_row = bsel(j == k, inv, rowp);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = i0 + 4 * q;
        v[q] = bsel(i == k, on_row, bsel(j == k, -c[q] * inv, fma(-c[q], rowp, v[q])));
    }
}

// Gauss-Jordan elimination of B1 (R <= 16) by the first wavefront alone,
// entirely in registers: the matrix is padded to 16 x 16 with zeros (the
// padding is never a pivot and is left unchanged) and lane l holds column
// l % 16 of rows l / 16 + 4 q (q < 4).  Pivots are taken two at a time,
// K = {k, k+1} with P = M(K, K):
//   M(K, K) <- P^{-1},  M(K, j) <- P^{-1} M(K, j),  M(i, K) <- -M(i, K) P^{-1},
//   M(i, j) <- M(i, j) - M(i, K) P^{-1} M(K, j)      (i, j not in K),
// which equals two scalar steps; P comes by lane reads (the lanes are
// constants, the step loop being unrolled), the two pivot rows and columns by
// shuffles all issued together, so a pair costs one round of exchanges.  The
// scalar pivots M(k, k) and det P / M(k, k) are tested against 1e-12
// maxdiag; a failure is only recorded (no branch between the exchanges) and
// the elimination runs on to the end on meaningless values.  An odd last
// pivot takes a scalar step.  Returns 1 if any pivot failed (the same in
// every lane).
__device__ __forceinline__ int gj_wave_regs(double (&v)[4], int R, double maxdiag) {
    const int l = threadIdx.x & (kWave - 1), j = l & 15, i0 = l >> 4;
    const double thr = 1e-12 * maxdiag;
    int bad = 0;
#pragma unroll
    for (int k = 0; k < 16; k += 2) {
        if (k + 1 >= R) {
            if (k < R) gj_wave_step(v, k, thr, bad);
            break;
        }
        const int g0 = (k & 3) << 4, g1 = ((k + 1) & 3) << 4;  // lanes of rows k and k + 1
        const double vk = v[k >> 2];                            // rows k and k + 1 share the slot
        const double a = read_lane(vk, g0 | k), b = read_lane(vk, g0 | (k + 1));
        const double c = read_lane(vk, g1 | k), d = read_lane(vk, g1 | (k + 1));
        const double r0 = __shfl(vk, g0 | j, kWave), r1 = __shfl(vk, g1 | j, kWave);  // M(K, j)
        double c0[4], c1[4];                                                          // M(i, K)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            c0[q] = __shfl(v[q], (l & 48) | k, kWave);
            c1[q] = __shfl(v[q], (l & 48) | (k + 1), kWave);
        }
        const double det = fma(a, d, -b * c);
        bad |= !(a > thr) | !(det > thr * a);
        const double id = 1.0 / det;
        const double p00 = d * id, p01 = -b * id, p10 = -c * id, p11 = a * id;  // P^{-1}
        const double s0 = fma(p00, r0, p01 * r1), s1 = fma(p10, r0, p11 * r1);  // P^{-1} M(K, j)
        const bool jk0 = j == k, jk1 = j == k + 1;
        const double on_row0 = bsel(jk0, p00, bsel(jk1, p01, s0));
        const double on_row1 = bsel(jk0, p10, bsel(jk1, p11, s1));
        const double e0 = bsel(jk0, p00, p01), e1 = bsel(jk0, p10, p11);  // column j of P^{-1}
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + 4 * q;
            const double other = fma(-c0[q], s0, fma(-c1[q], s1, v[q]));
            const double on_col = -fma(c0[q], e0, c1[q] * e1);
            v[q] = bsel(i == k, on_row0, bsel(i == k + 1, on_row1, bsel(jk0 || jk1, on_col, other)));
        }
    }
    return bad;
}

__device__ __forceinline__ int gj_wave(double *B1, int R, int ld, double maxdiag) {
    const int l = threadIdx.x, j = l & 15, i0 = l >> 4;
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = i0 + 4 * q;
        v[q] = (i < R && j < R) ? B1[i * ld + j] : 0.0;
    }
    if (gj_wave_regs(v, R, maxdiag)) return 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = i0 + 4 * q;
        if (i < R && j < R) B1[i * ld + j] = v[q];
    }
    return 0;
}

// Gauss-Jordan inverse of B1, 16 < R <= C (C = 32 or 64), by the first four
// waves in registers, zero-padded to C x C (padding rows and columns stay
// zero).  Wave w holds rows w C/4 .. (w+1) C/4 - 1: lane l holds column
// l % C of rows w C/4 + l / C + (64 / C) q.  Pivots go two at a time with
// the block update of gj_wave_regs: the lanes holding rows k and k + 1 (one
// wave, as k is even and a wave holds an even number of rows) write them to
// rowbuf (double-buffered, 4 C doubles of LDS), one barrier, then every
// thread reads the 2 x 2 pivot block and its two row entries from there and
// takes M(i, k), M(i, k + 1) of its own rows from the lanes of its own wave
// that hold those columns (shuffles issued before the barrier).  An odd last
// pivot takes a scalar step.  The row loop is unrolled over a wave's rows so
// that the slots of the pivot rows are constants.  Returns 1 if a scalar
// pivot falls below 1e-12 maxdiag (every thread reads the same pivots, so
// all agree; B1 is then untouched).  Every thread of the block calls it
// (blockDim.x >= 256; further waves only meet the barriers).
template <int C>
__device__ __forceinline__ int gj_rows(double *B1, double *rowbuf, int R, int ld, double maxdiag) {
    constexpr int H = kWave / C;  // row groups in a wave
    constexpr int RW = C / 4;     // rows per wave
    constexpr int NQ = RW / H;    // rows per lane
    const int tid = threadIdx.x, w = tid / kWave, l = tid & (kWave - 1);
    const int j = l % C, h = l / C, src = h * C;
    const bool act = w < 4;
    const double thr = 1e-12 * maxdiag;
    int bad = 0;
    double v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = w * RW + h + H * q;
        v[q] = (act && i < R && j < R) ? B1[i * ld + j] : 0.0;
    }
    for (int kw = 0; kw < 4; ++kw) {
#pragma unroll
        for (int p = 0; p < RW / 2; ++p) {
            const int k = kw * RW + 2 * p;
            if (k >= R) goto done;  // uniform
            const int kh0 = (2 * p) % H, kq0 = (2 * p) / H, kh1 = (2 * p + 1) % H, kq1 = (2 * p + 1) / H;
            double *buf = rowbuf + (p & 1) * 2 * C;  // consecutive pairs alternate
            if (k + 1 >= R) {  // odd R: the last pivot alone
                if (w == kw && h == kh0) buf[j] = v[kq0];
                double c[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) c[q] = __shfl(v[q], src + k, kWave);
                __syncthreads();
                const double piv = buf[k], rk = buf[j];
                bad |= !(piv > thr);
                const double inv = 1.0 / piv;
                const double rowp = rk * inv;
                const double on_row = bsel(j == k, inv, rowp);
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const bool rowk = (q == kq0) && (w == kw) && (h == kh0);
                    v[q] = bsel(rowk, on_row, bsel(j == k, -c[q] * inv, fma(-c[q], rowp, v[q])));
                }
                goto done;
            }
            if (w == kw && h == kh0) buf[j] = v[kq0];
            if (w == kw && h == kh1) buf[C + j] = v[kq1];
            double c0[NQ], c1[NQ];  // M(i, k), M(i, k + 1) of this lane's rows
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                c0[q] = __shfl(v[q], src + k, kWave);
                c1[q] = __shfl(v[q], src + k + 1, kWave);
            }
            __syncthreads();
            const double a = buf[k], b = buf[k + 1], c = buf[C + k], d = buf[C + k + 1];
            const double r0 = buf[j], r1 = buf[C + j];
            const double det = fma(a, d, -b * c);
            bad |= !(a > thr) | !(det > thr * a);
            const double id = 1.0 / det;
            const double p00 = d * id, p01 = -b * id, p10 = -c * id, p11 = a * id;
            const double s0 = fma(p00, r0, p01 * r1), s1 = fma(p10, r0, p11 * r1);
            const bool jk0 = j == k, jk1 = j == k + 1;
            const double on_row0 = bsel(jk0, p00, bsel(jk1, p01, s0));
            const double on_row1 = bsel(jk0, p10, bsel(jk1, p11, s1));
            const double e0 = bsel(jk0, p00, p01), e1 = bsel(jk0, p10, p11);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const bool rowk0 = (q == kq0) && (w == kw) && (h == kh0);
                const bool rowk1 = (q == kq1) && (w == kw) && (h == kh1);
                const double other = fma(-c0[q], s0, fma(-c1[q], s1, v[q]));
                const double on_col = -fma(c0[q], e0, c1[q] * e1);
                v[q] = bsel(rowk0, on_row0, bsel(rowk1, on_row1, bsel(jk0 || jk1, on_col, other)));
            }
        }
    }
done:
    if (bad) return 1;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = w * RW + h + H * q;
        if (act && i < R && j < R) B1[i * ld + j] = v[q];
    }
    return 0;
}

// One wave, R <= 16, V already in registers in the gj_wave layout (lane l
// holds column l % 16 of rows l / 16 + 4 q; zero outside R x R): writes
// B3 = V, and B1 = V^{-1} when every pivot passes.  Returns 1 when the
// caller has to fall back (a non-finite or non-positive diagonal, or a
// failed pivot); B1 is then not written.  No barrier inside.
__device__ __forceinline__ int gj_wave_from_regs(double (&v)[4], double *B1, double *B3, int R, int ld) {
    const int l = threadIdx.x & (kWave - 1), j = l & 15, i0 = l >> 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = i0 + 4 * q;
        if (i < R && j < R) B3[i * ld + j] = v[q];
    }
    // the diagonal by lane reads (wave-uniform values, no exchange rounds)
    double mx = 0.0;
    bool nf = false;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i >= R) break;
        const double d = read_lane(v[i >> 2], ((i & 3) << 4) | i);
        nf = nf || !isfinite(d);
        mx = fmax(mx, fabs(d));
    }
    if (nf || !(mx > 0.0)) return 1;
    if (gj_wave_regs(v, R, mx)) return 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = i0 + 4 * q;
        if (i < R && j < R) B1[i * ld + j] = v[q];
    }
    return 0;
}

// The pseudo-inverse of V = B3 into B1 by a Jacobi eigen-decomposition
// (eigenvalues below 1e-12 of the largest dropped).  All threads of the block.
__device__ __forceinline__ void spd_pinv(double *B1, double *B2, const double *B3, double *tmp, int R, int ld,
                                         double *cs, int *pairs) {
    const int tid = threadIdx.x, nt = blockDim.x;
    int bad = 0;
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
}

// Scratch for spd_inverse: B1, B2, B3 (R x ld doubles each), tmp (>= R
// doubles), cs (2*33 doubles), pairs (2*33 ints).  On entry B1 = B3 = V;
// on exit B1 = V^{-1} (or the pseudo-inverse), B3 = V.  Returns 1 when the
// pseudo-inverse was used.  All threads of the block must call it; the block
// needs at least ceil(R / 4)^2 threads (256 for R = 64).
__device__ __forceinline__ int spd_inverse(double *B1, double *B2, const double *B3, double *tmp, int R, int ld, double *cs,
                                  int *pairs) {
    const int tid = threadIdx.x, nt = blockDim.x;
    int bad = 0;
    const double maxdiag = diag_absmax(B1, R, ld, &bad);
    int failed = (bad || !(maxdiag > 0.0)) ? 1 : 0;
    if (!failed && R <= 16) {
        __shared__ int s_failed;
        if (tid < kWave) {
            const int f = gj_wave(B1, R, ld, maxdiag);
            if (tid == 0) s_failed = f;
        }
        __syncthreads();
        failed = s_failed;
    } else if (!failed) {
        failed = R <= 32 ? gj_rows<32>(B1, B2, R, ld, maxdiag) : gj_rows<64>(B1, B2, R, ld, maxdiag);
        __syncthreads();
    }
    if (!failed) return 0;
    spd_pinv(B1, B2, B3, tmp, R, ld, cs, pairs);
    return 1;
}

}  // namespace cprand
