// Device pieces shared by the sampled MTTKRP kernels (the chunked form in
// mttkrp.hip and the streaming form in mttkrp_stream.hip): MFMA wrappers,
// the per-type load geometry, the kernel arguments, and the index and
// Khatri-Rao phases of a sample chunk (Alg. 2 and Alg. 3).
#pragma once
#include "kernels.hpp"

namespace cprand {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T>
struct AccT;
template <>
struct AccT<float> {
    typedef v4f type;
};
template <>
struct AccT<double> {
    typedef v4d type;
};

__device__ inline v4f mfma16(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline v4d mfma16(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T, bool CPLX>
struct Geo {
    static constexpr int NV = 16 / (int)sizeof(T);          // reals per 16-byte vector
    static constexpr int VE = CPLX ? NV / 2 : NV;          // fiber rows per lane per step
    static constexpr int RPW = 16 * VE;                    // rows per wave per step
};

constexpr int kUnroll = 8;  // k-steps (of 4 samples) whose fiber loads are in flight together
constexpr int kWholeFiberS = 4096;  // sample sets from this size on use whole-fiber workgroups

// LDS row stride (in T) for the B operand: >= 16*CT and, for float, an odd
// multiple of 16 words so that two B rows read by one half-wave hit
// disjoint banks.
__host__ __device__ constexpr int ldb_for(int ct, int tsize) {
    return tsize == 4 ? (ct % 2 ? 16 * ct : 16 * ct + 16) : 16 * ct + 2;
}

struct KArgs {
    ModeInfo mi;
    const void *X;
    FactorPtrs A;
    const int32_t *idx;
    const double *w;
    CdfPtrs cdf;
    int use_cdf;
    uint64_t seed, t;
    const uint64_t *t_dev;
    void *wpart;
    double *vpart;
    int32_t R, S, In, ncols, kc, rows_wg;
    int32_t per_split;  // streaming form: samples per split
};

// Fiber values of one MFMA batch: lane (li, lk) takes sample ks + 4u + lk
// (u < kUnroll) and rows row0 .. row0 + VE - 1 of its mode-n fiber.
template <typename T, bool CPLX, bool CONTIG>
__device__ __forceinline__ void load_fibers(T (&v)[kUnroll][16 / sizeof(T)], const T *xp, const int64_t *s_base,
                                            int ns, int ks, int row0, int lk, int In, int64_t sn) {
    typedef Geo<T, CPLX> G;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const int sl = ks + 4 * u + lk;
#pragma unroll
        for (int e = 0; e < G::NV; ++e) v[u][e] = (T)0;
        if (sl < ns && row0 < In) {
            const int64_t b = s_base[sl];
            if (CONTIG && row0 + G::VE <= In) {
                const T *src = xp + (b + row0) * (CPLX ? 2 : 1);
                if (sizeof(T) == 4) {
                    const float4 q = *(const float4 *)src;
                    v[u][0] = q.x;
                    v[u][1] = q.y;
                    v[u][2] = q.z;
                    v[u][3] = q.w;
                } else {
                    const double2 q = *(const double2 *)src;
                    v[u][0] = q.x;
                    v[u][1] = q.y;
                }
            } else {
#pragma unroll
                for (int c = 0; c < G::VE; ++c) {
                    if (row0 + c < In) {
                        const int64_t o = b + (int64_t)(row0 + c) * sn;
                        if (CPLX) {
                            v[u][2 * c] = xp[2 * o];
                            v[u][2 * c + 1] = xp[2 * o + 1];
                        } else {
                            v[u][c] = xp[o];
                        }
                    }
                }
            }
        }
    }
}


// (1) Multi-indices, weights and fiber base offsets of samples s0 ..
// s0 + ns - 1 into LDS; slots ns .. KC - 1 get zero weight and offset 0.
__device__ __forceinline__ void chunk_indices(const KArgs &a, uint64_t tt, int s0, int ns, int KC, int64_t *s_base,
                                              double *s_w, int32_t *s_idx, int tid) {
    const int N = a.mi.order, n = a.mi.n;
    for (int sl = tid; sl < KC; sl += blockDim.x) {
        int64_t row[kMaxOrder];
        double wv = 1.0;
        int64_t base = 0;
        // mode loops unrolled to kMaxOrder: row[] stays in registers
        if (sl < ns) {
            const int64_t s = (int64_t)s0 + sl;
            if (a.idx) {
#pragma unroll
                for (int m = 0; m < kMaxOrder; ++m)
                    if (m < N) row[m] = (m == n) ? 0 : a.idx[s * N + m];
                if (a.w) wv = a.w[s];
            } else {
                wv = draw_sample(a.mi, a.seed, tt, s, a.cdf, a.use_cdf != 0, row);
            }
#pragma unroll
            for (int m = 0; m < kMaxOrder; ++m)
                if (m < N && m != n) base += row[m] * a.mi.strides[m];
        } else {
#pragma unroll
            for (int m = 0; m < kMaxOrder; ++m) row[m] = 0;
            wv = 0.0;
        }
#pragma unroll
        for (int m = 0; m < kMaxOrder; ++m)
            if (m < N) s_idx[sl * N + m] = (m == n) ? 0 : (int32_t)row[m];
        s_base[sl] = base;
        s_w[sl] = wv;
    }
}

// (1) for given samples (a.idx set), without a row array: each index goes
// to LDS and into the base offset as it is read.
__device__ __forceinline__ void chunk_indices_given(const KArgs &a, int s0, int ns, int KC, int64_t *s_base,
                                                    double *s_w, int32_t *s_idx, int tid) {
    const int N = a.mi.order, n = a.mi.n;
    for (int sl = tid; sl < KC; sl += blockDim.x) {
        const bool in = sl < ns;
        const int64_t s = (int64_t)s0 + (in ? sl : 0);
        int64_t base = 0;
#pragma unroll
        for (int m = 0; m < kMaxOrder; ++m) {
            if (m >= N) break;  // uniform
            const int32_t i = (in && m != n) ? a.idx[s * N + m] : 0;
            s_idx[sl * N + m] = i;
            base += (int64_t)i * a.mi.strides[m];
        }
        s_base[sl] = base;
        s_w[sl] = in ? (a.w ? a.w[s] : 1.0) : 0.0;
    }
}

// (2) Sampled Khatri-Rao rows of the chunk's ns samples into the B operand
// tiles, up to four elements per thread per pass with all their factor loads
// issued before the products.  Loads run over the N-1 modes that take part
// (a uniform bound); elements past the end read element 0 and are not
// stored.  The product runs over the modes in order.  Real data: Zr gets the
// raw rows and (weighted) Bre the rows scaled by the sample weights; complex
// data: Y = X conj(Z) takes columns [0, R) real part, [R, 2R) imaginary part.
template <typename T, bool CPLX, bool WEIGHTED, int KE = 4>
__device__ __forceinline__ void chunk_krp(const KArgs &a, int ns, int LDB, const int32_t *s_idx, const double *s_w,
                                          T *Bre, T *Bim, T *Zr, int tid) {
    const int N = a.mi.order, n = a.mi.n, R = a.R;
    const int nthr = blockDim.x;
    const int nm = N - 1;
    const int tot = ns * R;
    // factor of the j-th mode that takes part, chosen by compares (a runtime
    // index into the argument's pointer array would copy it to scratch)
    const T *Aj[kMaxOrder - 1];
#pragma unroll
    for (int j = 0; j < kMaxOrder - 1; ++j) Aj[j] = (const T *)(j < n ? a.A.p[j] : a.A.p[j + 1]);
    const int ke = min(KE, (tot + nthr - 1) / nthr);  // passes fit the elements
    for (int e0 = tid; e0 < tot; e0 += ke * nthr) {
        T vr[KE][kMaxOrder - 1], vi[KE][kMaxOrder - 1];
#pragma unroll
        for (int h = 0; h < KE; ++h) {
            if (h >= ke) break;  // uniform
            const int e = min(e0 + h * nthr, tot - 1);
            const int sl = e / R, r = e - (e / R) * R;
#pragma unroll
            for (int j = 0; j < kMaxOrder - 1; ++j) {
                if (j >= nm) break;  // uniform
                const int m = j < n ? j : j + 1;
                const T *Am = Aj[j];
                const int64_t o = (int64_t)s_idx[sl * N + m] * R + r;
                if (CPLX) {
                    vr[h][j] = Am[2 * o];
                    vi[h][j] = Am[2 * o + 1];
                } else {
                    vr[h][j] = Am[o];
                }
            }
        }
#pragma unroll
        for (int h = 0; h < KE; ++h) {
            if (h >= ke) break;
            const int e = e0 + h * nthr;
            if (e >= tot) continue;
            const int sl = e / R, r = e - sl * R;
            if (!CPLX) {
                T z = (T)1;
#pragma unroll
                for (int j = 0; j < kMaxOrder - 1; ++j)
                    if (j < nm) z *= vr[h][j];
                Zr[sl * LDB + r] = z;
                if (WEIGHTED) Bre[sl * LDB + r] = (T)(s_w[sl] * (double)z);
            } else {
                T zr = (T)1, zi = (T)0;
#pragma unroll
                for (int j = 0; j < kMaxOrder - 1; ++j) {
                    if (j >= nm) break;
                    const T ar = vr[h][j], ai = vi[h][j];
                    const T nr = zr * ar - zi * ai;
                    const T ni = zr * ai + zi * ar;
                    zr = nr;
                    zi = ni;
                }
                Bre[sl * LDB + r] = zr;
                Bim[sl * LDB + r] = zi;
                Bre[sl * LDB + R + r] = -zi;
                Bim[sl * LDB + R + r] = zr;
            }
        }
    }
}

// Store one row group's output tile of column dst (dst = column base):
// output tile row i' of MFMA c is row rbase + VE i' + c, where lane (li, lk)
// holds tile rows i' = 4 lk + v (FP32 16x16x4) or lk + 4 v (FP64), v = 0..3.
// The lane's rows are consecutive runs (16 rows for FP32 with VE = 4, runs of
// 2 otherwise), written as 16- or 8-byte vectors when vec_ok (the column
// length keeps them aligned) and the run lies before row_end, else element
// by element.
template <typename T, int VE, typename Acc>
__device__ __forceinline__ void store_group(T *dst, const Acc (&acc)[VE], int rbase, int row_end, int lk,
                                            bool vec_ok) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        if (sizeof(T) == 4 && VE == 4) {
            const int r0 = rbase + 16 * lk + 4 * v;
            if (vec_ok && r0 + 4 <= row_end) {
                *(float4 *)(dst + r0) = float4{(float)acc[0][v], (float)acc[1][v], (float)acc[2][v], (float)acc[3][v]};
            } else {
#pragma unroll
                for (int c = 0; c < VE; ++c)
                    if (r0 + c < row_end) dst[r0 + c] = acc[c][v];
            }
        } else if (VE == 2) {
            const int r0 = sizeof(T) == 4 ? rbase + 8 * lk + 2 * v : rbase + 2 * lk + 8 * v;
            if (vec_ok && r0 + 2 <= row_end) {
                if (sizeof(T) == 4)
                    *(float2 *)(dst + r0) = float2{(float)acc[0][v], (float)acc[1][v]};
                else
                    *(double2 *)(dst + r0) = double2{(double)acc[0][v], (double)acc[1][v]};
            } else {
#pragma unroll
                for (int c = 0; c < VE; ++c)
                    if (r0 + c < row_end) dst[r0 + c] = acc[c][v];
            }
        } else {
#pragma unroll
            for (int c = 0; c < VE; ++c) {
                const int ip = sizeof(T) == 8 ? lk + 4 * v : 4 * lk + v;
                const int row = rbase + VE * ip + c;
                if (row < row_end) dst[row] = acc[c][v];
            }
        }
    }
}

// Streaming form (mttkrp_stream.hip): row groups per wave for a plan (0 when
// the accumulators exceed the register budget), the workgroups the chip
// holds at once, and the launch.
constexpr int kStreamLoads = 8;   // loads per batch (per lane, 16 bytes each)
constexpr int kStreamMaxR = 32;   // Gram: at most three tiles, one per wave
int stream_gw_host(int kind, int ct);
int stream_cap(int kind, int ct, size_t lds);
hipError_t launch_gather_stream(const GatherPlan &gp, const KArgs &k, bool weighted, hipStream_t st);

}  // namespace cprand
