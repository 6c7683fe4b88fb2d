// The dense side of the paper's comparison: the full MTTKRP of CP-ALS
// (Alg. 1), W = X_(n) Z^(n) with Z^(n) the Khatri-Rao product of every
// factor but the n-th, the factor Gram matrices (Z^T Z is their Hadamard
// product, eq. KRGram) and the exact fit of Section 3.4,
//   ||X - X~||^2 = ||X||^2 - 2 <X, X~> + ||X~||^2,
//   <X, X~> = sum_r lambda_r sum_i A^(n)(i, r) W(i, r),
//   ||X~||^2 = lambda^T (G_1 * ... * G_N) lambda.
//
// Column-major X is read as [J][I_n][K] (J = product of the dims before n,
// K after); column q = (j, k), q = j + J k, of the unfolding holds the
// elements X[j + J i + J I_n k], i < I_n, and row q of Z^(n) is the
// Hadamard product of the factor rows at the indices q encodes.  The kernel
// is W = sum_q X(:, q) Z(q, :) on MFMA 16x16x4 with FP32 (FP64 for FP64
// data) accumulation.  A workgroup owns a range of q and a block of rows;
// per tile of 64 columns it issues its tensor loads, builds the 64 Khatri-
// Rao rows in LDS and runs the products.  Loads are 16-byte vectors: along
// the fiber when J = 1 (mode 0), along j otherwise (consecutive columns are
// contiguous there).  Every HBM byte of X is read once per launch.  Partial
// products of the q ranges are summed in FP64 in a fixed order.
#include <algorithm>

#include "kernels.hpp"

namespace cprand {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T>
struct FAcc;
template <>
struct FAcc<float> {
    typedef v4f type;
};
template <>
struct FAcc<double> {
    typedef v4d type;
};
__device__ inline v4f fmfma(float a, float b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ inline v4d fmfma(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

constexpr int kQT = 64;    // columns q per tile
constexpr int kWaves = 4;  // waves per workgroup

// LDS row stride of the Khatri-Rao tile (in T): >= 16 CT; for float an odd
// multiple of 16 words, so the four rows a wave reads hit distinct banks.
__host__ __device__ constexpr int full_ldb(int ct, int tsize) {
    return tsize == 4 ? (ct % 2 ? 16 * ct : 16 * ct + 16) : 16 * ct + 2;
}

struct FullArgs {
    ModeInfo mi;
    const void *X;
    FactorPtrs A;
    int32_t R, In;
    int64_t J, K, Q;    // Q = J K columns
    int64_t qchunk;     // columns per chunk (multiple of kQT)
    int32_t rows_wg;    // rows per workgroup
    void *wpart;        // [chunk][R][In] partial products, real type
};

// Rows per wave: VE rows per lane along the fiber (IV) or one 16-row MFMA
// tile per vector component (QV); both give 16 * VE rows.
template <typename T>
struct FGeo {
    static constexpr int VE = 16 / (int)sizeof(T);
    static constexpr int RPW = 16 * VE;
};

// IV: vectors along the fiber (J == 1).  QV: vectors along j (J % VE == 0).
// VEC false: scalar loads (any alignment).
template <typename T, int CT, bool IV, bool VEC>
__global__ __launch_bounds__(kWaves * 64) void full_mttkrp_kernel(FullArgs a) {
    typedef FGeo<T> G;
    typedef typename FAcc<T>::type Acc;
    constexpr int VE = G::VE;
    constexpr int LDB = full_ldb(CT, (int)sizeof(T));
    __shared__ __align__(16) T Zs[kQT * LDB];
    __shared__ int64_t qoff[kQT][kMaxOrder];  // factor element offsets (row * R) per column and mode
    const int tid = threadIdx.x;
    const int N = a.mi.order, n = a.mi.n, R = a.R, In = a.In;
    const int wv = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
    const int64_t qa = (int64_t)blockIdx.y * a.qchunk;
    const int64_t qb = min(a.Q, qa + a.qchunk);
    const int rw = blockIdx.x * a.rows_wg + wv * G::RPW;  // first row of this wave
    const T *X = (const T *)a.X;
    const int64_t J = a.J, JI = a.J * (int64_t)In;
    const bool small = a.Q < (int64_t)INT32_MAX;  // 32-bit column arithmetic

    Acc acc[CT][VE];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int c = 0; c < VE; ++c) acc[ct][c] = Acc{0, 0, 0, 0};

    // IV, VEC: load u of a tile (columns q0 + 4u + lk, rows rw + VE li ..),
    // unconditional (I_n % VE == 0 here): a column past the tile reads its
    // last column (its Khatri-Rao row is zero), a row past the fiber the
    // fiber's last vector (rows never stored).  Each tile's loads are issued
    // while the previous tile's products run: right after the MFMAs have
    // read v[u], v[u] is loaded with the next tile's vector.
    T v[16][VE];
    const bool wave_rows = rw < In;  // uniform per wave
    const int rc = min(rw + VE * (tid & 15), In - VE);
    auto load_iv = [&](int u, int64_t q0t, int nqt) {
        const T *src = X + (q0t + min(4 * u + lk, nqt - 1)) * (int64_t)In + rc;
        if constexpr (sizeof(T) == 4) {
            const float4 x = *(const float4 *)src;
            v[u][0] = x.x;
            v[u][1] = x.y;
            v[u][2] = x.z;
            v[u][3] = x.w;
        } else {
            const double2 x = *(const double2 *)src;
            v[u][0] = x.x;
            v[u][1] = x.y;
        }
    };
    if (IV && VEC && wave_rows && qa < qb) {
        const int nq0 = (int)min((int64_t)kQT, qb - qa);
#pragma unroll
        for (int u = 0; u < 16; ++u) load_iv(u, qa, nq0);
    }

    for (int64_t q0 = qa; q0 < qb; q0 += kQT) {
        const int nq = (int)min((int64_t)kQT, qb - q0);
        // ---- tensor loads of this tile, into registers
        // IV: v[u][c] = row rw + VE li + c of column q0 + 4u + lk.  QV: step u =
        // t (16 / VE) + s covers row tile t (rows rw + 16 t + li) and columns
        // q0 + 4 VE s + VE lk + c.  Both: 16 VE values per lane.
        constexpr int QS = 16 / VE;  // QV steps per tile
        if (IV && VEC) {
            // already in flight (issued with the previous tile's products)
        } else if (IV) {
            const int row0 = rw + VE * li;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int ql = 4 * u + lk;
#pragma unroll
                for (int c = 0; c < VE; ++c) v[u][c] = (T)0;
                if (ql < nq && row0 < In) {
                    const T *src = X + (q0 + ql) * (int64_t)In + row0;  // J == 1: column q at q * I_n
                    if (VEC && row0 + VE <= In) {
                        if constexpr (sizeof(T) == 4) {
                            const float4 x = *(const float4 *)src;
                            v[u][0] = x.x;
                            v[u][1] = x.y;
                            v[u][2] = x.z;
                            v[u][3] = x.w;
                        } else {
                            const double2 x = *(const double2 *)src;
                            v[u][0] = x.x;
                            v[u][1] = x.y;
                        }
                    } else {
#pragma unroll
                        for (int c = 0; c < VE; ++c)
                            if (row0 + c < In) v[u][c] = src[c];
                    }
                }
            }
        } else if (VEC) {
            // unconditional loads along j (J % VE == 0, so every tile and the
            // tile's column count are multiples of VE): clamped as above
#pragma unroll
            for (int t = 0; t < VE; ++t) {
                const int row = min(rw + 16 * t + li, In - 1);
#pragma unroll
                for (int s = 0; s < QS; ++s) {
                    const int u = QS * t + s;
                    const int64_t q = q0 + min(4 * VE * s + VE * lk, nq - VE);
                    const int64_t k = small ? (int64_t)((uint32_t)q / (uint32_t)J) : q / J;
                    const T *src = X + (q - k * J) + J * (int64_t)row + JI * k;
                    if constexpr (sizeof(T) == 4) {
                        const float4 x = *(const float4 *)src;
                        v[u][0] = x.x;
                        v[u][1] = x.y;
                        v[u][2] = x.z;
                        v[u][3] = x.w;
                    } else {
                        const double2 x = *(const double2 *)src;
                        v[u][0] = x.x;
                        v[u][1] = x.y;
                    }
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < VE; ++t) {
                const int row = rw + 16 * t + li;
#pragma unroll
                for (int s = 0; s < QS; ++s) {
                    const int u = QS * t + s;
                    const int ql = 4 * VE * s + VE * lk;
#pragma unroll
                    for (int c = 0; c < VE; ++c) v[u][c] = (T)0;
                    if (row < In && ql < nq) {
                        const int64_t q = q0 + ql;
                        const int64_t k = q / J, j = q - k * J;
                        const T *src = X + j + J * (int64_t)row + JI * k;
                        if (VEC && ql + VE <= nq) {  // J % VE == 0 and q % VE == 0: one k, aligned
                            if constexpr (sizeof(T) == 4) {
                                const float4 x = *(const float4 *)src;
                                v[u][0] = x.x;
                                v[u][1] = x.y;
                                v[u][2] = x.z;
                                v[u][3] = x.w;
                            } else {
                                const double2 x = *(const double2 *)src;
                                v[u][0] = x.x;
                                v[u][1] = x.y;
                            }
                        } else {
#pragma unroll
                            for (int c = 0; c < VE; ++c) {
                                if (ql + c < nq) {
                                    const int64_t qq = q + c;
                                    const int64_t kk = qq / J, jj = qq - kk * J;
                                    v[u][c] = X[jj + J * (int64_t)row + JI * kk];
                                }
                            }
                        }
                    }
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);  // the tensor loads stay issued together
        __syncthreads();  // the previous tile's Khatri-Rao rows are no longer read
        // ---- Khatri-Rao rows of the tile: factor offsets, then products
        for (int ql = tid; ql < kQT; ql += kWaves * 64) {
            int64_t q = q0 + ql;
            if (ql >= nq) q = q0;  // past the end: any valid column (its row is zeroed)
            if (small) {
                uint32_t j = (uint32_t)q % (uint32_t)J, k = (uint32_t)q / (uint32_t)J;
#pragma unroll
                for (int m = 0; m < kMaxOrder; ++m) {
                    if (m >= N) break;
                    uint32_t im = 0;
                    const uint32_t d = (uint32_t)a.mi.dims[m];
                    if (m < n) {
                        im = j % d;
                        j /= d;
                    } else if (m > n) {
                        im = k % d;
                        k /= d;
                    }
                    qoff[ql][m] = (int64_t)im * R;
                }
            } else {
                int64_t j = q % J, k = q / J;
#pragma unroll
                for (int m = 0; m < kMaxOrder; ++m) {
                    if (m >= N) break;
                    int64_t im = 0;
                    if (m < n) {
                        im = j % a.mi.dims[m];
                        j /= a.mi.dims[m];
                    } else if (m > n) {
                        im = k % a.mi.dims[m];
                        k /= a.mi.dims[m];
                    }
                    qoff[ql][m] = im * R;
                }
            }
        }
        __syncthreads();
        for (int e = tid; e < kQT * 16 * CT; e += kWaves * 64) {
            const int ql = e / (16 * CT), r = e - ql * (16 * CT);
            // every slot's factor value loaded (a mode past the order or the
            // skipped mode reads mode 0's or 1's row again, clamped column)
            // with no branch between the loads, then multiplied in mode order
            const int rc = min(r, R - 1);
            T f[kMaxOrder];
#pragma unroll
            for (int m = 0; m < kMaxOrder; ++m) {
                const bool take = m < N && m != n;
                const int m0 = n == 0 ? 1 : 0;  // a participating mode
                // compile-time indices into the pointer array (a run-time
                // index would copy it to scratch)
                const T *Am = (const T *)(take ? a.A.p[m] : (n == 0 ? a.A.p[1] : a.A.p[0]));
                f[m] = Am[qoff[ql][take ? m : m0] + rc];
            }
            T z = (T)1;
#pragma unroll
            for (int m = 0; m < kMaxOrder; ++m)
                if (m < N && m != n) z *= f[m];
            Zs[ql * LDB + r] = (ql < nq && r < R) ? z : (T)0;
        }
        __syncthreads();
        // ---- products
        if (rw < In) {
            if (IV) {
                auto mfma_u = [&](int u) {
                    const int ql = 4 * u + lk;
#pragma unroll
                    for (int ct = 0; ct < CT; ++ct) {
                        const T b = Zs[ql * LDB + ct * 16 + li];
#pragma unroll
                        for (int c = 0; c < VE; ++c) acc[ct][c] = fmfma(v[u][c], b, acc[ct][c]);
                    }
                };
                const int64_t qn = q0 + kQT;
                if (VEC && qn < qb) {
                    const int nqn = (int)min((int64_t)kQT, qb - qn);
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        mfma_u(u);
                        load_iv(u, qn, nqn);  // the next tile's vector into the register just read
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < 16; ++u) mfma_u(u);
                }
            } else {
#pragma unroll
                for (int t = 0; t < VE; ++t)
#pragma unroll
                    for (int s = 0; s < QS; ++s)
#pragma unroll
                        for (int c = 0; c < VE; ++c) {
                            const int ql = 4 * VE * s + VE * lk + c;
#pragma unroll
                            for (int ct = 0; ct < CT; ++ct)
                                acc[ct][t] = fmfma(v[QS * t + s][c], Zs[ql * LDB + ct * 16 + li], acc[ct][t]);
                        }
            }
        }
    }
    // ---- partial products of this column range: lane (li, lk) holds tile
    // rows i' = 4 lk + vv (FP32) or lk + 4 vv (FP64) of column 16 ct + li
    if (rw >= In) return;
    T *wp = (T *)a.wpart + (size_t)blockIdx.y * R * In;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const int col = ct * 16 + li;
        if (col >= R) continue;
#pragma unroll
        for (int vv = 0; vv < 4; ++vv)
#pragma unroll
            for (int c = 0; c < VE; ++c) {
                const int ip = sizeof(T) == 8 ? lk + 4 * vv : 4 * lk + vv;
                const int row = IV ? rw + VE * ip + c : rw + 16 * c + ip;
                if (row < In) wp[(size_t)col * In + row] = acc[ct][c][vv];
            }
    }
}

// W[i][r] = sum over chunks of wpart[chunk][r][i] in FP64: a workgroup takes
// 64 consecutive entries of the [R][In] order, its four waves the chunks
// c = wave, wave + 4, ... (coalesced 64-entry rows), and the four wave sums
// are added in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void full_reduce_kernel(const T *wpart, int32_t chunks, int32_t In, int32_t R,
                                                          double *W) {
    __shared__ double sh[4][64];
    const int l = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t n = (int64_t)In * R;
    const int64_t e = (int64_t)blockIdx.x * 64 + l;
    double s = 0.0;
    if (e < n)
        for (int c = g; c < chunks; c += 4) s += (double)wpart[(size_t)c * n + e];
    sh[g][l] = s;
    __syncthreads();
    if (g == 0 && e < n) {
        const int r = (int)(e / In), i = (int)(e - (int64_t)r * In);
        W[(int64_t)i * R + r] = (sh[0][l] + sh[1][l]) + (sh[2][l] + sh[3][l]);
    }
}

// Gram partials of one factor over a block of kGramRows rows: part[blk][r][q]
// for q >= r (FP64), the rows staged in LDS.
constexpr int kGramRows = 64;
template <typename T>
__global__ __launch_bounds__(256) void gram_part_kernel_full(const T *A, int32_t I, int32_t R, double *part) {
    __shared__ double rows[kGramRows * 65];
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * kGramRows;
    const int nr = min(kGramRows, I - i0);
    for (int e = tid; e < nr * R; e += 256) {
        const int i = e / R, r = e - i * R;
        rows[i * 65 + r] = (double)A[(int64_t)(i0 + i) * R + r];
    }
    __syncthreads();
    double *out = part + (size_t)blockIdx.x * R * R;
    for (int p = tid; p < R * R; p += 256) {
        const int r = p / R, q = p - r * R;
        if (q < r) continue;
        double s = 0.0;
        for (int i = 0; i < nr; ++i) s += rows[i * 65 + r] * rows[i * 65 + q];
        out[r * R + q] = s;
    }
}

// G = sum of the partials (fixed order), both triangles.
__global__ __launch_bounds__(256) void gram_finish_kernel_full(const double *part, int32_t nparts, int32_t R,
                                                               double *G) {
    for (int p = threadIdx.x; p < R * R; p += 256) {
        const int r = p / R, q = p - r * R;
        const int a = min(r, q), b = max(r, q);
        double s = 0.0;
        for (int k = 0; k < nparts; ++k) s += part[(size_t)k * R * R + a * R + b];
        G[p] = s;
    }
}

// V = Hadamard product of G[m], m != skip (skip = -1: all modes).
__global__ __launch_bounds__(256) void gram_hadamard_kernel(const double *G, int32_t order, int32_t R, int32_t skip,
                                                            double *V) {
    for (int p = threadIdx.x; p < R * R; p += 256) {
        double v = 1.0;
        for (int m = 0; m < order; ++m)
            if (m != skip) v *= G[(size_t)m * R * R + p];
        V[p] = v;
    }
}

// Exact fit from the mode-n MTTKRP W (FP64, row-major) of the model (lambda,
// factors), with A^(n) its mode-n factor and Gall the Hadamard product of
// every factor's Gram: F = 1 - sqrt(max(||X||^2 - 2 inner + model, 0)) / ||X||.
template <typename T>
__global__ __launch_bounds__(256) void fit_exact_kernel(const double *W, const T *An, int32_t In, int32_t R,
                                                        const double *lambda, const double *Gall,
                                                        const double *normX, double *fit_out) {
    __shared__ double sh[256 / 64];
    double inner = 0.0;
    for (int64_t e = threadIdx.x; e < (int64_t)In * R; e += 256) {
        const int r = (int)(e % R);
        inner += lambda[r] * (double)An[e] * W[e];
    }
    double model = 0.0;
    for (int p = threadIdx.x; p < R * R; p += 256) model += lambda[p / R] * lambda[p % R] * Gall[p];
    inner = block_sum<256>(inner, sh);
    __syncthreads();
    model = block_sum<256>(model, sh);
    if (threadIdx.x == 0) {
        const double nx = *normX;
        const double res = fmax(nx * nx - 2.0 * inner + model, 0.0);
        *fit_out = 1.0 - sqrt(res) / nx;
    }
}

}  // namespace

FullPlan plan_full(const ModeInfo &mi, int kind, int32_t R, bool aligned) {
    FullPlan f{};
    const int n = mi.n;
    f.In = (int32_t)mi.dims[n];
    f.R = R;
    f.kind = kind;
    f.J = 1;
    f.K = 1;
    for (int m = 0; m < n; ++m) f.J *= mi.dims[m];
    for (int m = n + 1; m < mi.order; ++m) f.K *= mi.dims[m];
    f.Q = f.J * f.K;
    const int ve = kind == K_F64 ? 2 : 4;
    f.iv = f.J == 1;
    f.vec = aligned && (f.iv ? f.In % ve == 0 : f.J % ve == 0);
    f.ct = (R + 15) / 16;
    const int rpw = 16 * ve;
    f.rows_wg = kWaves * rpw;
    f.row_blocks = (int32_t)ceil_div(f.In, f.rows_wg);
    // about the workgroups the chip holds at once (two per CU), so the
    // grid runs in one round and each workgroup walks many tiles, while the
    // partial products stay within about 2% of the tensor's bytes
    const int64_t tiles = ceil_div(f.Q, kQT);
    int64_t chunks = ceil_div(512, f.row_blocks);
    const int64_t cap = std::max<int64_t>(1, (f.Q * (int64_t)f.In) / ((int64_t)f.In * R * 50));
    chunks = std::max<int64_t>(1, std::min({chunks, cap, tiles}));
    f.qchunk = ceil_div(tiles, chunks) * kQT;
    f.chunks = (int32_t)ceil_div(f.Q, f.qchunk);
    return f;
}

template <typename T, int CT>
static hipError_t launch_full_t(const FullPlan &f, const FullArgs &a, hipStream_t st) {
    dim3 grid((unsigned)f.row_blocks, (unsigned)f.chunks);
    if (f.iv) {
        if (f.vec)
            hipLaunchKernelGGL((full_mttkrp_kernel<T, CT, true, true>), grid, dim3(kWaves * 64), 0, st, a);
        else
            hipLaunchKernelGGL((full_mttkrp_kernel<T, CT, true, false>), grid, dim3(kWaves * 64), 0, st, a);
    } else {
        if (f.vec)
            hipLaunchKernelGGL((full_mttkrp_kernel<T, CT, false, true>), grid, dim3(kWaves * 64), 0, st, a);
        else
            hipLaunchKernelGGL((full_mttkrp_kernel<T, CT, false, false>), grid, dim3(kWaves * 64), 0, st, a);
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_full_ct(const FullPlan &f, const FullArgs &a, hipStream_t st) {
    switch (f.ct) {
        case 1: return launch_full_t<T, 1>(f, a, st);
        case 2: return launch_full_t<T, 2>(f, a, st);
        case 3: return launch_full_t<T, 3>(f, a, st);
        default: return launch_full_t<T, 4>(f, a, st);
    }
}

hipError_t launch_mttkrp_full(const FullPlan &f, const ModeInfo &mi, const void *X, const FactorPtrs &A, void *wpart,
                              double *W, hipStream_t st) {
    FullArgs a{};
    a.mi = mi;
    a.X = X;
    a.A = A;
    a.R = f.R;
    a.In = f.In;
    a.J = f.J;
    a.K = f.K;
    a.Q = f.Q;
    a.qchunk = f.qchunk;
    a.rows_wg = f.rows_wg;
    a.wpart = wpart;
    hipError_t e = f.kind == K_F64 ? launch_full_ct<double>(f, a, st) : launch_full_ct<float>(f, a, st);
    if (e != hipSuccess) return e;
    const unsigned nb = (unsigned)ceil_div((int64_t)f.In * f.R, 64);
    if (f.kind == K_F64)
        hipLaunchKernelGGL(full_reduce_kernel<double>, dim3(nb), dim3(256), 0, st, (const double *)wpart, f.chunks,
                           f.In, f.R, W);
    else
        hipLaunchKernelGGL(full_reduce_kernel<float>, dim3(nb), dim3(256), 0, st, (const float *)wpart, f.chunks, f.In,
                           f.R, W);
    return hipGetLastError();
}

hipError_t launch_gram_full(const void *A, bool dbl, int32_t I, int32_t R, double *part, double *G, hipStream_t st) {
    const int nb = (int)ceil_div(I, kGramRows);
    if (dbl)
        hipLaunchKernelGGL(gram_part_kernel_full<double>, dim3(nb), dim3(256), 0, st, (const double *)A, I, R, part);
    else
        hipLaunchKernelGGL(gram_part_kernel_full<float>, dim3(nb), dim3(256), 0, st, (const float *)A, I, R, part);
    hipLaunchKernelGGL(gram_finish_kernel_full, dim3(1), dim3(256), 0, st, (const double *)part, nb, R, G);
    return hipGetLastError();
}

hipError_t launch_gram_hadamard(const double *G, int32_t order, int32_t R, int32_t skip, double *V, hipStream_t st) {
    hipLaunchKernelGGL(gram_hadamard_kernel, dim3(1), dim3(256), 0, st, G, order, R, skip, V);
    return hipGetLastError();
}

hipError_t launch_fit_exact(const double *W, const void *An, bool dbl, int32_t In, int32_t R, const double *lambda,
                            const double *Gall, const double *normX, double *fit_out, hipStream_t st) {
    if (dbl)
        hipLaunchKernelGGL(fit_exact_kernel<double>, dim3(1), dim3(256), 0, st, W, (const double *)An, In, R, lambda,
                           Gall, normX, fit_out);
    else
        hipLaunchKernelGGL(fit_exact_kernel<float>, dim3(1), dim3(256), 0, st, W, (const float *)An, In, R, lambda,
                           Gall, normX, fit_out);
    return hipGetLastError();
}

}  // namespace cprand
