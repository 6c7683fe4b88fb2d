// Device-side FFT building blocks shared by the mixing kernels (fft.hip) and
// the fused mode-step kernel (step.hip): complex helpers, radix-2/3/4/5/7
// butterflies, the Stockham stage with run-time radices (two LDS tiles) and
// the compile-time in-place variant.  See fft.hip for the formulation.
#pragma once

#include "common.hpp"

namespace cprand {

template <typename T>
struct cx {
    T re, im;
};
template <typename T>
__device__ inline cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ inline cx<T> cadd(cx<T> a, cx<T> b) {
    return {a.re + b.re, a.im + b.im};
}
template <typename T>
__device__ inline cx<T> csub(cx<T> a, cx<T> b) {
    return {a.re - b.re, a.im - b.im};
}
template <typename T>
__device__ inline cx<T> cscale(cx<T> a, T s) {
    return {a.re * s, a.im * s};
}
// multiply by i*dir
template <int DIR, typename T>
__device__ inline cx<T> cmul_idir(cx<T> a) {
    return DIR > 0 ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}

struct FftPlan {
    int64_t L;
    int nrad;
    int rad[24];
    void *tw;  // device, L complex (float or double): exp(-2 pi i q / L)
};

// r-point DFT in place, sign DIR (-1 forward, +1 inverse).
template <typename T, int R, int DIR>
__device__ __forceinline__ void small_dft(cx<T> *v, const cx<T> *tw, int L) {
    if constexpr (R == 2) {
        cx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 3) {
        const T h = (T)0.86602540378443864676;  // sqrt(3)/2
        cx<T> a = v[0], b = v[1], c = v[2];
        cx<T> s = cadd(b, c), d = csub(b, c);
        cx<T> m = csub(a, cscale(s, (T)0.5));
        cx<T> q = cmul_idir<DIR>(cscale(d, h));
        v[0] = cadd(a, s);
        v[1] = cadd(m, q);
        v[2] = csub(m, q);
    } else if constexpr (R == 4) {
        cx<T> a = v[0], b = v[1], c = v[2], d = v[3];
        cx<T> s0 = cadd(a, c), d0 = csub(a, c), s1 = cadd(b, d), d1 = cmul_idir<DIR>(csub(b, d));
        v[0] = cadd(s0, s1);
        v[1] = cadd(d0, d1);
        v[2] = csub(s0, s1);
        v[3] = csub(d0, d1);
    } else if constexpr (R == 5) {
        const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
        const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
        cx<T> x0 = v[0];
        cx<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
        cx<T> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
        cx<T> a1 = cadd(x0, cadd(cscale(t1, c1), cscale(t2, c2)));
        cx<T> a2 = cadd(x0, cadd(cscale(t1, c2), cscale(t2, c1)));
        cx<T> b1 = cmul_idir<DIR>(cadd(cscale(t3, s1), cscale(t4, s2)));
        cx<T> b2 = cmul_idir<DIR>(csub(cscale(t3, s2), cscale(t4, s1)));
        v[0] = cadd(x0, cadd(t1, t2));
        v[1] = cadd(a1, b1);
        v[4] = csub(a1, b1);
        v[2] = cadd(a2, b2);
        v[3] = csub(a2, b2);
    } else {
        // direct R-point DFT from the length-L table: w^(a b) = tw[(a b mod R) L/R]
        cx<T> out[R];
        const int step = L / R;
#pragma unroll
        for (int a = 0; a < R; ++a) {
            cx<T> acc = v[0];
#pragma unroll
            for (int b = 1; b < R; ++b) {
                cx<T> w = tw[((a * b) % R) * step];
                if (DIR > 0) w.im = -w.im;
                acc = cadd(acc, cmul(v[b], w));
            }
            out[a] = acc;
        }
#pragma unroll
        for (int a = 0; a < R; ++a) v[a] = out[a];
    }
}

// ---------------------------------------------------------------------------
// Generic path: radices known at run time, ping-pong between two tiles.
// a = q b + r for 0 <= a < 2^22 and 1 <= b < 2^11: a float estimate of the
// quotient (off by at most one) and one correction; binv = 1.0f / b.
__device__ inline int divmod_small(int a, int b, float binv, int &r) {
    int q = (int)((float)a * binv);
    r = a - q * b;
    if (r < 0) {
        --q;
        r += b;
    } else if (r >= b) {
        ++q;
        r -= b;
    }
    return q;
}

template <typename T, int R, int DIR>
__device__ __forceinline__ void stage_rt(const cx<T> *in, cx<T> *out, int L, int ldt, int tc, int Ns, const cx<T> *tw) {
    const int nb = (L / R) * tc;
    const int twstep = L / (Ns * R);
    const int LR = L / R;
    const float tcinv = 1.0f / (float)tc, nsinv = 1.0f / (float)Ns;
    const int nt = blockDim.x;
    // two butterflies per pass so that both sets of LDS loads are in flight
    for (int id0 = threadIdx.x; id0 < nb; id0 += 2 * nt) {
        cx<T> v[2][R];
        int col[2], j[2], k[2];
        bool on[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int id = id0 + h * nt;
            on[h] = id < nb;
            j[h] = divmod_small(on[h] ? id : 0, tc, tcinv, col[h]);
            int kk;
            (void)divmod_small(j[h], Ns, nsinv, kk);
            k[h] = kk;
#pragma unroll
            for (int t = 0; t < R; ++t) v[h][t] = on[h] ? in[(j[h] + t * LR) * ldt + col[h]] : cx<T>{};
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int t = 1; t < R; ++t) {
                cx<T> w = tw[t * k[h] * twstep];
                if (DIR > 0) w.im = -w.im;
                v[h][t] = cmul(v[h][t], w);
            }
            small_dft<T, R, DIR>(v[h], tw, L);
            if (on[h]) {
                const int o = (j[h] - k[h]) * R + k[h];
#pragma unroll
                for (int t = 0; t < R; ++t) out[(o + t * Ns) * ldt + col[h]] = v[h][t];
            }
        }
    }
}

template <typename T, int DIR>
__device__ __forceinline__ cx<T> *fft_tile_rt(cx<T> *buf0, cx<T> *buf1, const FftPlan &fp, int ldt, int tc, const cx<T> *tw) {
    cx<T> *in = buf0, *out = buf1;
    int Ns = 1;
    const int L = (int)fp.L;
    for (int s = 0; s < fp.nrad; ++s) {
        const int r = fp.rad[s];
        switch (r) {
            case 2: stage_rt<T, 2, DIR>(in, out, L, ldt, tc, Ns, tw); break;
            case 3: stage_rt<T, 3, DIR>(in, out, L, ldt, tc, Ns, tw); break;
            case 4: stage_rt<T, 4, DIR>(in, out, L, ldt, tc, Ns, tw); break;
            case 5: stage_rt<T, 5, DIR>(in, out, L, ldt, tc, Ns, tw); break;
            default: stage_rt<T, 7, DIR>(in, out, L, ldt, tc, Ns, tw); break;
        }
        __syncthreads();
        Ns *= r;
        cx<T> *tmp = in;
        in = out;
        out = tmp;
    }
    return in;
}

// ---------------------------------------------------------------------------
// Compile-time path.
struct RadixList {
    int n;
    int r[16];
};
constexpr RadixList factor_len(int L) {
    RadixList f{};
    while (L % 4 == 0) {
        f.r[f.n++] = 4;
        L /= 4;
    }
    const int ps[4] = {2, 3, 5, 7};
    for (int i = 0; i < 4; ++i)
        while (L % ps[i] == 0) {
            f.r[f.n++] = ps[i];
            L /= ps[i];
        }
    return f;
}

template <typename T, int L, int TC, int NT, int DIR, int S = 0, int NS = 1>
__device__ __forceinline__ void fft_ct(cx<T> *buf, const cx<T> *tw) {
    constexpr RadixList RL = factor_len(L);
    if constexpr (S < RL.n) {
        constexpr int R = RL.r[S];
        constexpr int NB = (L / R) * TC;
        constexpr int ROUNDS = (NB + NT - 1) / NT;
        constexpr int LDT = TC + 1;
        constexpr int TWS = L / (NS * R);
        cx<T> v[ROUNDS][R];
#pragma unroll
        for (int q = 0; q < ROUNDS; ++q) {
            const int b = threadIdx.x + q * NT;
            if (NB % NT == 0 || b < NB) {
                const int j = b / TC, col = b % TC, k = j % NS;
#pragma unroll
                for (int t = 0; t < R; ++t) v[q][t] = buf[(j + t * (L / R)) * LDT + col];
#pragma unroll
                for (int t = 1; t < R; ++t) {
                    cx<T> w = tw[t * k * TWS];
                    if (DIR > 0) w.im = -w.im;
                    v[q][t] = cmul(v[q][t], w);
                }
                small_dft<T, R, DIR>(v[q], tw, L);
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < ROUNDS; ++q) {
            const int b = threadIdx.x + q * NT;
            if (NB % NT == 0 || b < NB) {
                const int j = b / TC, col = b % TC, k = j % NS;
                const int o = (j / NS) * NS * R + k;
#pragma unroll
                for (int t = 0; t < R; ++t) buf[(o + t * NS) * LDT + col] = v[q][t];
            }
        }
        __syncthreads();
        fft_ct<T, L, TC, NT, DIR, S + 1, NS * R>(buf, tw);
    }
}

}  // namespace cprand
