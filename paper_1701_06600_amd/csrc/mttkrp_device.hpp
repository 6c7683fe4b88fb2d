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
// fast (contiguous fibers, I_n % VE == 0), and strided fibers: every load
// unconditional, no branch between them, so all stay in flight together; a
// lane past the chunk reads the chunk's last fiber (its B operand row is
// zero) and a row past the fiber reads the fiber's last vector or element
// (output rows that are never stored: each MFMA output row depends only on
// its own A row).
template <typename T, bool CPLX, bool CONTIG>
__device__ __forceinline__ void load_fibers(T (&v)[kUnroll][16 / sizeof(T)], const T *xp, const int64_t *s_base,
                                            int ns, int ks, int row0, int lk, int In, int64_t sn, bool fast) {
    typedef Geo<T, CPLX> G;
    if (CONTIG && fast) {
        int64_t b[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) b[u] = s_base[min(ks + 4 * u + lk, ns - 1)];
        const int rc = min(row0, In - G::VE);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const T *src = xp + (b[u] + rc) * (CPLX ? 2 : 1);
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
        }
        return;
    }
    if (!CONTIG) {
        // strided fibers: the same clamping, one load per element, all of
        // them unconditional (a load behind a branch is waited for at the
        // branch's end, which would serialize the batch)
        int64_t b[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) b[u] = s_base[min(ks + 4 * u + lk, ns - 1)];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int c = 0; c < G::VE; ++c) {
                const int64_t o = b[u] + (int64_t)min(row0 + c, In - 1) * sn;
                if (CPLX) {
                    v[u][2 * c] = xp[2 * o];
                    v[u][2 * c + 1] = xp[2 * o + 1];
                } else {
                    v[u][c] = xp[o];
                }
            }
        }
        return;
    }
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
                // every slot loaded (past the order: slot 0 again, the same
                // line), then selected: no branch between the loads, which
                // stay in flight together
                int32_t iv[kMaxOrder];
#pragma unroll
                for (int m = 0; m < kMaxOrder; ++m) iv[m] = a.idx[s * N + (m < N ? m : 0)];
#pragma unroll
                for (int m = 0; m < kMaxOrder; ++m) row[m] = (m < N && m != n) ? iv[m] : 0;
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
        int32_t iv[kMaxOrder];
#pragma unroll
        for (int m = 0; m < kMaxOrder; ++m) iv[m] = a.idx[s * N + (m < N ? m : 0)];  // no branch between loads
        int64_t base = 0;
#pragma unroll
        for (int m = 0; m < kMaxOrder; ++m) {
            if (m >= N) break;  // uniform
            const int32_t i = (in && m != n) ? iv[m] : 0;
            s_idx[sl * N + m] = i;
            base += (int64_t)i * a.mi.strides[m];
        }
        s_base[sl] = base;
        s_w[sl] = in ? (a.w ? a.w[s] : 1.0) : 0.0;
    }
}

// (2) Sampled Khatri-Rao rows of the chunk's ns samples into the B operand
// tiles, KE elements per thread per pass; each row is the product of the
// N-1 participating factor rows, taken over the modes in order.  Real data:
// Zr gets the raw rows and (weighted) Bre the rows scaled by the sample
// weights; complex data: Y = X conj(Z) takes columns [0, R) real part,
// [R, 2R) imaginary part.  ILV (complex only): row sl of Bre (stride LDB)
// holds the B operand pairs of its columns interleaved, (zr, zi) of column r
// at 2 r and (-zi, zr) of column R + r at 2 (R + r), with a zero pair at 4R
// for the padding columns.
//
// Mode-by-mode form (for kernels whose accumulators stay live meanwhile):
// per pass, the KE elements' factor values of one mode are loaded and
// multiplied in before the next mode's are loaded, so that the registers do
// not grow with the order; the products run over the modes in the same
// order as in chunk_krp (bit-identical rows).
template <typename T, bool CPLX, bool WEIGHTED, int KE, bool ILV>
__device__ __forceinline__ void chunk_krp_by_mode(const KArgs &a, int ns, int LDB, const int32_t *s_idx,
                                                  const double *s_w, T *Bre, T *Bim, T *Zr, int tid) {
    const int N = a.mi.order, n = a.mi.n, R = a.R;
    const int nthr = blockDim.x;
    const int nm = N - 1;
    const int tot = ns * R;
    // always KE elements per pass (past the end: the last element again,
    // not stored), so that no branch separates their loads
    for (int e0 = tid; e0 < tot; e0 += KE * nthr) {
        T zr[KE], zi[KE];
#pragma unroll
        for (int h = 0; h < KE; ++h) {
            zr[h] = (T)1;
            zi[h] = (T)0;
        }
#pragma unroll
        for (int j = 0; j < kMaxOrder - 1; ++j) {
            if (j >= nm) break;  // uniform
            const int m = j < n ? j : j + 1;
            const T *Am = (const T *)(j < n ? a.A.p[j] : a.A.p[j + 1]);
            T ar[KE], ai[KE];
#pragma unroll
            for (int h = 0; h < KE; ++h) {
                const int e = min(e0 + h * nthr, tot - 1);
                const int sl = e / R, r = e - (e / R) * R;
                const int64_t o = (int64_t)s_idx[sl * N + m] * R + r;
                if (CPLX) {
                    ar[h] = Am[2 * o];
                    ai[h] = Am[2 * o + 1];
                } else {
                    ar[h] = Am[o];
                }
            }
#pragma unroll
            for (int h = 0; h < KE; ++h) {
                if (!CPLX) {
                    zr[h] *= ar[h];
                } else {
                    const T nr = zr[h] * ar[h] - zi[h] * ai[h];
                    const T ni = zr[h] * ai[h] + zi[h] * ar[h];
                    zr[h] = nr;
                    zi[h] = ni;
                }
            }
        }
#pragma unroll
        for (int h = 0; h < KE; ++h) {
            const int e = e0 + h * nthr;
            if (e >= tot) continue;
            const int sl = e / R, r = e - sl * R;
            if (!CPLX) {
                Zr[sl * LDB + r] = zr[h];
                if (WEIGHTED) Bre[sl * LDB + r] = (T)(s_w[sl] * (double)zr[h]);
            } else if (ILV) {
                Bre[sl * LDB + 2 * r] = zr[h];
                Bre[sl * LDB + 2 * r + 1] = zi[h];
                Bre[sl * LDB + 2 * (R + r)] = -zi[h];
                Bre[sl * LDB + 2 * (R + r) + 1] = zr[h];
            } else {
                Bre[sl * LDB + r] = zr[h];
                Bim[sl * LDB + r] = zi[h];
                Bre[sl * LDB + R + r] = -zi[h];
                Bim[sl * LDB + R + r] = zr[h];
            }
        }
    }
}

// All N-1 modes at once (NM of them, a compile-time count): the KE
// elements' factor loads of every mode are issued together, one round trip
// per pass; always KE elements per pass (past the end: the last element
// again, not stored).
template <typename T, bool CPLX, bool WEIGHTED, int KE, bool ILV, int NM>
__device__ __forceinline__ void krp_modes(const KArgs &a, int ns, int LDB, const int32_t *s_idx, const double *s_w,
                                          T *Bre, T *Bim, T *Zr, int tid) {
    const int N = a.mi.order, n = a.mi.n, R = a.R;
    const int nthr = blockDim.x;
    const int tot = ns * R;
    // factor of the j-th mode that takes part, chosen by compares (a runtime
    // index into the argument's pointer array would copy it to scratch)
    const T *Aj[NM];
    int mj[NM];
#pragma unroll
    for (int j = 0; j < NM; ++j) {
        mj[j] = j < n ? j : j + 1;
        Aj[j] = (const T *)(j < n ? a.A.p[j] : a.A.p[j + 1]);
    }
    for (int e0 = tid; e0 < tot; e0 += KE * nthr) {
        T vr[KE][NM], vi[KE][NM];
#pragma unroll
        for (int h = 0; h < KE; ++h) {
            const int e = min(e0 + h * nthr, tot - 1);
            const int sl = e / R, r = e - (e / R) * R;
#pragma unroll
            for (int j = 0; j < NM; ++j) {
                const int64_t o = (int64_t)s_idx[sl * N + mj[j]] * R + r;
                if (CPLX) {
                    vr[h][j] = Aj[j][2 * o];
                    vi[h][j] = Aj[j][2 * o + 1];
                } else {
                    vr[h][j] = Aj[j][o];
                }
            }
        }
#pragma unroll
        for (int h = 0; h < KE; ++h) {
            const int e = e0 + h * nthr;
            if (e >= tot) continue;
            const int sl = e / R, r = e - sl * R;
            if (!CPLX) {
                T z = (T)1;
#pragma unroll
                for (int j = 0; j < NM; ++j) z *= vr[h][j];
                Zr[sl * LDB + r] = z;
                if (WEIGHTED) Bre[sl * LDB + r] = (T)(s_w[sl] * (double)z);
            } else {
                T zr = (T)1, zi = (T)0;
#pragma unroll
                for (int j = 0; j < NM; ++j) {
                    const T ar = vr[h][j], ai = vi[h][j];
                    const T nr = zr * ar - zi * ai;
                    const T ni = zr * ai + zi * ar;
                    zr = nr;
                    zi = ni;
                }
                if (ILV) {
                    Bre[sl * LDB + 2 * r] = zr;
                    Bre[sl * LDB + 2 * r + 1] = zi;
                    Bre[sl * LDB + 2 * (R + r)] = -zi;
                    Bre[sl * LDB + 2 * (R + r) + 1] = zr;
                } else {
                    Bre[sl * LDB + r] = zr;
                    Bim[sl * LDB + r] = zi;
                    Bre[sl * LDB + R + r] = -zi;
                    Bim[sl * LDB + R + r] = zr;
                }
            }
        }
    }
}

template <typename T, bool CPLX, bool WEIGHTED, int KE = 4, bool ILV = false>
__device__ __forceinline__ void chunk_krp(const KArgs &a, int ns, int LDB, const int32_t *s_idx, const double *s_w,
                                          T *Bre, T *Bim, T *Zr, int tid) {
    static_assert(kMaxOrder == 8, "one case per count of participating modes");
    switch (a.mi.order - 1) {  // uniform
        case 1: krp_modes<T, CPLX, WEIGHTED, KE, ILV, 1>(a, ns, LDB, s_idx, s_w, Bre, Bim, Zr, tid); break;
        case 2: krp_modes<T, CPLX, WEIGHTED, KE, ILV, 2>(a, ns, LDB, s_idx, s_w, Bre, Bim, Zr, tid); break;
        case 3: krp_modes<T, CPLX, WEIGHTED, KE, ILV, 3>(a, ns, LDB, s_idx, s_w, Bre, Bim, Zr, tid); break;
        case 4: krp_modes<T, CPLX, WEIGHTED, KE, ILV, 4>(a, ns, LDB, s_idx, s_w, Bre, Bim, Zr, tid); break;
        case 5: krp_modes<T, CPLX, WEIGHTED, KE, ILV, 5>(a, ns, LDB, s_idx, s_w, Bre, Bim, Zr, tid); break;
        case 6: krp_modes<T, CPLX, WEIGHTED, KE, ILV, 6>(a, ns, LDB, s_idx, s_w, Bre, Bim, Zr, tid); break;
        default: krp_modes<T, CPLX, WEIGHTED, KE, ILV, 7>(a, ns, LDB, s_idx, s_w, Bre, Bim, Zr, tid); break;
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

// The chunked MTTKRP of one workgroup (chunk blockIdx.y, row block
// blockIdx.x; see mttkrp.hip): W partial products of the chunk's rows into
// a.wpart, and Gram entries p (row-major R x R) with p mod gram_nrb ==
// gram_rb (R <= 16; for larger R, 16 x 16 tiles dealt likewise over
// (gram_rb, wave) pairs) into vp.  gram_nrb = 1 computes the whole Gram.
template <typename T, bool CPLX, int CT, bool CONTIG, bool WEIGHTED>
__device__ __forceinline__ void gather_chunk(const KArgs &a, unsigned char *lds, double *vp, int gram_rb,
                                             int gram_nrb) {
    typedef Geo<T, CPLX> G;
    typedef typename AccT<T>::type Acc;
    constexpr int LDB = ldb_for(CT, (int)sizeof(T));

    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int KC = a.kc;
    const int N = a.mi.order, n = a.mi.n;
    const int R = a.R;
    const int chunk = blockIdx.y;
    const int s0 = chunk * KC;
    const int ns = min(KC, a.S - s0);

    // ---- LDS carve-up
    int64_t *s_base = (int64_t *)lds;                      // KC
    double *s_w = (double *)(s_base + KC);                 // KC
    int32_t *s_idx = (int32_t *)(s_w + KC);                // KC x N
    T *Bre = (T *)(lds + (((size_t)KC * (16 + 4 * N) + 15) & ~(size_t)15));
    T *Bim = Bre + (size_t)KC * LDB;                       // complex only
    T *Zr = CPLX ? Bre : (WEIGHTED ? Bre + (size_t)KC * LDB : Bre);  // raw z (real)

    // ---- (1) indices, weights and fiber offsets.  Given samples never read
    // the device-side iteration counter: its load would be one more round
    // trip ahead of the index loads.
    if (a.idx) {  // uniform
        chunk_indices_given(a, s0, ns, KC, s_base, s_w, s_idx, tid);
    } else {
        const uint64_t tt = a.t_dev ? *a.t_dev : a.t;
        chunk_indices(a, tt, s0, ns, KC, s_base, s_w, s_idx, tid);
    }
    // zero the B operand tiles (padding columns and samples stay zero)
    {
        const int words = (int)(((size_t)KC * LDB * sizeof(T) * ((CPLX || WEIGHTED) ? 2 : 1)) / 4);
        uint32_t *p = (uint32_t *)Bre;
        for (int e = tid; e < words; e += nthr) p[e] = 0u;
    }
    __syncthreads();

    // ---- fiber loads (phase 4 below): the first two batches of this wave's
    // first row group are issued now, so their latency overlaps the
    // Khatri-Rao loads (a chunk of up to 8 kUnroll samples then meets no
    // fiber round trip after them)
    const int wv = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
    const int In = a.In;
    const int row_end = min(In, (int)(blockIdx.x + 1) * a.rows_wg);
    const T *xp = (const T *)a.X;
    const int64_t sn = a.mi.strides[n];
    T v[kUnroll][G::NV], v2[kUnroll][G::NV];
    const bool fast = In % G::VE == 0;
    const int rb0 = blockIdx.x * a.rows_wg + wv * G::RPW;
    const int npre = rb0 < row_end ? (ns > 4 * kUnroll ? 2 : 1) : 0;  // uniform per wave
    if (npre > 0) load_fibers<T, CPLX, CONTIG>(v, xp, s_base, ns, 0, rb0 + G::VE * li, lk, In, sn, fast);
    if (npre > 1) load_fibers<T, CPLX, CONTIG>(v2, xp, s_base, ns, 4 * kUnroll, rb0 + G::VE * li, lk, In, sn, fast);

    // ---- (2) sampled Khatri-Rao rows
    chunk_krp<T, CPLX, WEIGHTED>(a, ns, LDB, s_idx, s_w, Bre, Bim, Zr, tid);
    __syncthreads();

    // ---- (3) Gram of the chunk, V(r, q) = sum_k w_k z_k(r) z_k(q) (complex:
    // zr zr^T + zi zi^T) over the chunk's samples k, FP64, fixed order.
    // No barrier: waves without Gram work go on to the fiber products.
    const int nrb = gram_nrb, rb = gram_rb;
    // R <= 16: the one 16 x 16 tile on FP64 MFMA in row block 0, wave w
    // taking the k-steps w, w + 4, ...; the four partial tiles are summed in
    // wave order once the fiber products are done (below).  Lane (li, lk)
    // feeds A(r = li, k) and B(k, q = li) and holds V(lk + 4 v, li).
    v4d gacc = {0.0, 0.0, 0.0, 0.0};
    if (R <= 16) {
        if (rb == 0) {  // uniform per workgroup
            const bool rin = li < R;
            for (int kk = wv; kk < (ns + 3) / 4; kk += 4) {  // rows past ns are zero
                const int sl = 4 * kk + lk;
                if (!CPLX) {
                    double av = rin ? (double)Zr[sl * LDB + li] : 0.0;
                    if (WEIGHTED) av *= s_w[sl];
                    gacc = mfma16(av, rin ? (double)Zr[sl * LDB + li] : 0.0, gacc);
                } else {
                    const double zr = rin ? (double)Bre[sl * LDB + li] : 0.0;
                    const double zi = rin ? (double)Bim[sl * LDB + li] : 0.0;
                    gacc = mfma16(zr, zr, gacc);
                    gacc = mfma16(zi, zi, gacc);
                }
            }
        }
    } else {
        // FP64 MFMA 16x16x4: output tiles (rt, qt), qt >= rt, dealt to the
        // chunk's (row block, wave) pairs.  Lane (li, lk) feeds A(r = 16 rt +
        // li, k = 4 kk + lk) and B(k, q = 16 qt + li) and holds rows 16 rt + lk
        // + 4 v of column 16 qt + li.  Columns at or past R are masked (for
        // complex data they hold the imaginary block).
        const int wv3 = tid >> 6, l3 = tid & 63, li3 = l3 & 15, lk3 = l3 >> 4;
        const int nwv = nthr >> 6;
        const int nt16 = (R + 15) / 16;
        const int ntiles = nt16 * (nt16 + 1) / 2;
        const int ksteps = (ns + 3) / 4;  // rows past ns are zero (and have zero weight)
        for (int tix = rb + nrb * wv3; tix < ntiles; tix += nrb * nwv) {  // uniform per wave
            int rt = 0, rem = tix;
            while (rem >= nt16 - rt) {
                rem -= nt16 - rt;
                ++rt;
            }
            const int qt = rt + rem;
            const int r = rt * 16 + li3, q = qt * 16 + li3;
            const bool rin = r < R, qin = q < R;
            v4d acc = {0.0, 0.0, 0.0, 0.0};
            for (int kk = 0; kk < ksteps; ++kk) {
                const int sl = 4 * kk + lk3;
                if (!CPLX) {
                    double av = rin ? (double)Zr[sl * LDB + r] : 0.0;
                    if (WEIGHTED) av *= s_w[sl];
                    const double bv = qin ? (double)Zr[sl * LDB + q] : 0.0;
                    acc = mfma16(av, bv, acc);
                } else {
                    acc = mfma16(rin ? (double)Bre[sl * LDB + r] : 0.0, qin ? (double)Bre[sl * LDB + q] : 0.0, acc);
                    acc = mfma16(rin ? (double)Bim[sl * LDB + r] : 0.0, qin ? (double)Bim[sl * LDB + q] : 0.0, acc);
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = rt * 16 + lk3 + 4 * v, qq = qt * 16 + li3;
                if (rr < R && qq < R) {
                    vp[rr * R + qq] = acc[v];
                    if (rt != qt) vp[qq * R + rr] = acc[v];
                }
            }
        }
    }

    // ---- (4) fibers x Z_S on MFMA, one row group of G::RPW rows per wave at a
    // time (a workgroup covers rows_wg rows: one group per wave for short
    // sample chunks, whole fibers for long ones)
    T *wp = (T *)a.wpart + (size_t)chunk * a.ncols * In;
    int inreg = npre;  // batches of this row group already in registers
    for (int rowbase = rb0; rowbase < row_end; rowbase += (int)(blockDim.x >> 6) * G::RPW) {
    const int row0 = rowbase + G::VE * li;

    Acc acc[CT][G::VE];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int c = 0; c < G::VE; ++c) acc[ct][c] = Acc{0, 0, 0, 0};

    for (int ks = 0; ks < ns; ks += 4 * kUnroll) {
        const int b = ks / (4 * kUnroll);
        if (b >= inreg) {
            load_fibers<T, CPLX, CONTIG>(v, xp, s_base, ns, ks, row0, lk, In, sn, fast);
        } else if (b == 1) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                for (int e = 0; e < G::NV; ++e) v[u][e] = v2[u][e];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (ks + 4 * u >= ns) break;  // uniform: the rest of this pass is past the chunk
            const int sl = ks + 4 * u + lk;  // < KC: KC is a multiple of 4 and ns <= KC
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const T bre = Bre[sl * LDB + ct * 16 + li];
                if (!CPLX) {
#pragma unroll
                    for (int c = 0; c < G::VE; ++c) acc[ct][c] = mfma16(v[u][c], bre, acc[ct][c]);
                } else {
                    const T bim = Bim[sl * LDB + ct * 16 + li];
#pragma unroll
                    for (int c = 0; c < G::VE; ++c) {
                        acc[ct][c] = mfma16(v[u][2 * c], bre, acc[ct][c]);
                        acc[ct][c] = mfma16(v[u][2 * c + 1], bim, acc[ct][c]);
                    }
                }
            }
        }
    }

    // the row group's partial products, column by column
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const int col = ct * 16 + li;
        if (col < a.ncols)
            store_group<T, G::VE>(wp + (size_t)col * In, acc[ct], rowbase, row_end, lk,
                                  In % (sizeof(T) == 4 && G::VE == 4 ? 4 : 2) == 0);
    }
    inreg = 0;
    }  // row groups

    if (R <= 16 && rb == 0) {  // uniform per workgroup
        // the four waves' partial Gram tiles, summed in wave order through
        // LDS (the chunk's tiles are no longer read), then V(r, q) for
        // q >= r, mirrored so that V is exactly symmetric
        __syncthreads();
        double *gt = (double *)lds;
#pragma unroll
        for (int v4 = 0; v4 < 4; ++v4) gt[(wv * 64 + l) * 4 + v4] = gacc[v4];
        __syncthreads();
        if (wv == 0) {
#pragma unroll
            for (int v4 = 0; v4 < 4; ++v4) {
                double t = gt[l * 4 + v4];
#pragma unroll
                for (int w2 = 1; w2 < 4; ++w2) t += gt[(w2 * 64 + l) * 4 + v4];
                const int r = lk + 4 * v4, q = li;
                if (r < R && q < R && q >= r) {
                    vp[r * R + q] = t;
                    vp[q * R + r] = t;
                }
            }
        }
    }
}

// Streaming form (mttkrp_stream.hip): row groups per wave for a plan (0 when
// the accumulators exceed the register budget), the workgroups the chip
// holds at once, and the launch.
// row stride (in T) of the interleaved complex B operand rows in LDS:
// 4R + 2, padded when rows would start on the same LDS bank
__host__ __device__ inline int stream_ldz(int R, int tsize) {
    const int ld = 4 * R + 2;
    return (ld * tsize / 4) % 32 == 0 ? ld + 2 : ld;
}
constexpr int kStreamLoads = 8;   // loads per batch (per lane, 16 bytes each)
constexpr int kStreamMaxR = 32;   // Gram: at most three tiles, one per wave
KArgs make_kargs(const GatherPlan &gp, const GatherArgs &a);
int stream_gw_host(int kind, int ct);
int stream_cap(int kind, int ct, size_t lds);
hipError_t launch_gather_stream(const GatherPlan &gp, const KArgs &k, bool weighted, hipStream_t st);

}  // namespace cprand
