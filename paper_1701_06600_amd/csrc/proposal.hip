// Importance-sampling proposals for the Khatri-Rao rows of one mode step (a
// project addition): per-row features of each factor, the 4-64-64-1 ReLU
// network (FP32, plain vector ALUs: 4.5 k multiply-adds per row), the exact
// per-factor marginals of Khatri-Rao leverage (closed form from the factor
// Grams), and the integer cumulative tables that the sampler searches.
// Training kernels: forward, softmax cross-entropy backward with per-block
// gradient sums, fixed-order reduction, Adam.
//
// Features of row i of A = A^(m) (I x R) for the product over the set K of
// modes other than n (m in K):  f1 = I |a_i|^2/|A|_F^2,
// f2 = (I/R) a_i^T G^{-1} a_i, f3 = (I/R) sum_r a_ir^2/G_rr (G = A^T A), and
// f4 = mean over k in K\{m} of the mean |cosine| between distinct columns of
// A^(k); the network reads (log f1, log f2, log f3, f4).  The exact marginal
// is L(i) = a_i^T (G_K^{-1} * prod_{k in K\{m}} G_k) a_i, G_K the Hadamard
// product of the Grams in K (* = Hadamard), and sums to R.
#include <math.h>

#include "kernels.hpp"
#include "solve_device.hpp"

namespace cprand {

constexpr int kH1 = 64, kH2 = 64, kIn = 4;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kH1 * kIn, kOffW2 = kOffB1 + kH1, kOffB2 = kOffW2 + kH2 * kH1,
              kOffW3 = kOffB2 + kH2, kOffB3 = kOffW3 + kH2, kParams = kOffB3 + 1;
static_assert(kParams == 4545, "parameter layout");
constexpr float kFeatEps = 1e-6f;

// ---------------------------------------------------------------------------
// Per-mode statistics: G = A^T A (FP64), G^{-1}, |A|_F^2, mean |cosine|.
// stats layout per mode (doubles): G [R*R], Ginv [R*R], frob2, cong.
//
// (1) gram_part_kernel: block (c, m) sums a_i a_i^T over chunk c of the
//     rows of A^(m) (at most kGramChunks chunks per mode), staging tiles of
//     kGramTile rows in LDS; upper triangle computed, mirrored on store.
// (2) stats_finish_kernel: block m != n adds the chunk partials in chunk
//     order, writes G, its trace and mean |cosine|, and inverts it; block n
//     (the mode of the step, otherwise idle) forms the Hadamard product of
//     the Grams of all modes but n and writes its inverse to Hinv (only
//     when Hinv is requested: the exact marginals need it).
constexpr int kGramChunks = 64, kGramTile = 64, kStatThreads = 256;

__global__ __launch_bounds__(kStatThreads) void gram_part_kernel(FactorPtrs A, ModeInfo mi, int32_t R,
                                                                  double *gpart) {
    __shared__ double tile[kGramTile][kMaxRank + 1];
    const int m = blockIdx.y, c = blockIdx.x, tid = threadIdx.x;
    if (m == mi.n) return;
    const int64_t I = mi.dims[m];
    const int nch = (int)min((int64_t)kGramChunks, ceil_div(I, kGramTile));
    if (c >= nch) return;
    const int64_t per = ceil_div(I, nch);
    const int64_t i0 = (int64_t)c * per, i1 = min(I, i0 + per);
    const float *a = (const float *)A.p[m];
    constexpr int kQ = kMaxRank * kMaxRank / kStatThreads;
    double acc[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) acc[q] = 0.0;
    for (int64_t t0 = i0; t0 < i1; t0 += kGramTile) {
        const int nr = (int)min((int64_t)kGramTile, i1 - t0);
        __syncthreads();
        for (int e = tid; e < nr * R; e += kStatThreads) {
            const int rr = e / R, cc = e - rr * R;
            tile[rr][cc] = (double)a[(t0 + rr) * R + cc];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const int e = tid + q * kStatThreads;
            const int r = e / R, s2 = e - r * R;
            if (e < R * R && r <= s2) {
                double v = acc[q];
                for (int rr = 0; rr < nr; ++rr) v += tile[rr][r] * tile[rr][s2];
                acc[q] = v;
            }
        }
    }
    double *gp = gpart + ((size_t)m * kGramChunks + c) * R * R;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const int e = tid + q * kStatThreads;
        const int r = e / R, s2 = e - r * R;
        if (e < R * R && r <= s2) {
            gp[r * R + s2] = acc[q];
            gp[s2 * R + r] = acc[q];
        }
    }
}

// Chunk partials of entry e, added in chunk order; loads issued eight at a time.
__device__ inline double gram_sum(const double *gpart, int m, int nch, int R, int e) {
    const double *gp = gpart + (size_t)m * kGramChunks * R * R + e;
    const size_t st = (size_t)R * R;
    double g = 0.0;
    int c = 0;
    for (; c + 8 <= nch; c += 8) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = gp[(c + k) * st];
#pragma unroll
        for (int k = 0; k < 8; ++k) g += v[k];
    }
    for (; c < nch; ++c) g += gp[c * st];
    return g;
}

__global__ __launch_bounds__(kStatThreads) void stats_finish_kernel(ModeInfo mi, int32_t R, const double *gpart,
                                                                     double *stats, double *Hinv) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ double s_red[kStatThreads / kWave];
    const int m = blockIdx.x, n = mi.n, N = mi.order, tid = threadIdx.x;
    const bool hblock = (m == n);
    if (hblock && !Hinv) return;
    const int ld = R + 1;
    double *B1 = (double *)lds, *B2 = B1 + R * ld, *B3 = B2 + R * ld, *cs = B3 + R * ld, *tmp = cs + 66;
    int *pairs = (int *)(tmp + kMaxRank);
    for (int e = tid; e < R * R; e += kStatThreads) {
        double g;
        if (!hblock) {
            g = gram_sum(gpart, m, (int)min((int64_t)kGramChunks, ceil_div(mi.dims[m], kGramTile)), R, e);
        } else {
            g = 1.0;
            for (int k = 0; k < N; ++k)
                if (k != n) g *= gram_sum(gpart, k, (int)min((int64_t)kGramChunks, ceil_div(mi.dims[k], kGramTile)), R, e);
        }
        B1[(e / R) * ld + e % R] = g;
        B3[(e / R) * ld + e % R] = g;
    }
    __syncthreads();
    double *st = stats + (size_t)m * mode_stats_doubles(R);
    if (!hblock) {
        double fr = 0.0, cg = 0.0;
        for (int e = tid; e < R * R; e += kStatThreads) {
            const int r = e / R, s2 = e - r * R;
            const double v = B3[r * ld + s2];
            st[e] = v;
            if (r == s2)
                fr += v;
            else
                cg += fabs(v) / sqrt(B3[r * ld + r] * B3[s2 * ld + s2]);
        }
        fr = block_sum_dyn(fr, s_red);
        cg = block_sum_dyn(cg, s_red);
        if (tid == 0) {
            st[2 * R * R] = fr;
            st[2 * R * R + 1] = R > 1 ? cg / ((double)R * (R - 1)) : 0.0;
        }
    }
    spd_inverse(B1, B2, B3, tmp, R, ld, cs, pairs);
    double *out = hblock ? Hinv : st + R * R;
    for (int e = tid; e < R * R; e += kStatThreads) out[e] = B1[(e / R) * ld + e % R];
}

// ---------------------------------------------------------------------------
__device__ inline float mlp_row(const float *P, const float x[4]) {
    float h1[kH1];
#pragma unroll
    for (int j = 0; j < kH1; ++j) {
        float s = P[kOffB1 + j];
#pragma unroll
        for (int k = 0; k < kIn; ++k) s += P[kOffW1 + j * kIn + k] * x[k];
        h1[j] = s > 0.f ? s : 0.f;
    }
    float z = P[kOffB3];
    for (int j = 0; j < kH2; ++j) {
        float s = P[kOffB2 + j];
#pragma unroll
        for (int k = 0; k < kH1; ++k) s += P[kOffW2 + j * kH1 + k] * h1[k];
        z += P[kOffW3 + j] * (s > 0.f ? s : 0.f);
    }
    return z;
}

// The network's output without its bias, restricted to second-layer units
// j = q, q + 4, ... (q < 4); the four parts sum to mlp_row(P, x) - b3.  W2p
// holds the second-layer weights with rows padded to kH1 + 1 floats, so the
// four lanes of a quad (four rows j) read different LDS banks.
__device__ inline float mlp_part(const float *P, const float *W2p, const float x[4], int q) {
    float h1[kH1];
#pragma unroll
    for (int j = 0; j < kH1; ++j) {
        float s = P[kOffB1 + j];
#pragma unroll
        for (int k = 0; k < kIn; ++k) s += P[kOffW1 + j * kIn + k] * x[k];
        h1[j] = s > 0.f ? s : 0.f;
    }
    float z = 0.f;
    for (int j = q; j < kH2; j += 4) {
        float w[kH1];  // the unit's weights, all reads issued before the sums
#pragma unroll
        for (int k = 0; k < kH1; ++k) w[k] = W2p[j * (kH1 + 1) + k];
        float s4[4] = {P[kOffB2 + j], 0.f, 0.f, 0.f};  // four independent chains
#pragma unroll
        for (int k = 0; k < kH1; ++k) s4[k & 3] += w[k] * h1[k];
        const float s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
        z += P[kOffW3 + j] * (s > 0.f ? s : 0.f);
    }
    return z;
}

// Row scores for every mode m != n: mode == LEARNED: the network's logit;
// mode == MARGINAL: log of the exact marginal; neither (no Hinv): log of the
// row's leverage in its own factor, a_i^T G_m^{-1} a_i.  Also (optionally) writes the
// feature rows and the exact targets L/R for training.  One workgroup of
// four waves per kScoreRows rows: G^{-1}, the marginal matrix H_m = Hinv *
// prod_{k in K\{m}} G_k (Hadamard products), the rows (transposed) and the
// network are staged in LDS; the quadratic forms run on FP64 MFMA over
// 16-row blocks shared by the waves, one thread per row forms the features,
// and four lanes per row evaluate the network.
struct RowArgs {
    FactorPtrs A;
    ModeInfo mi;
    int32_t R;
    const double *stats;
    const double *Hinv;     // inverse of the Hadamard product of the Grams in K (NULL: no marginals)
    const float *params;    // network (LEARNED)
    int32_t learned;
    float *score[kMaxOrder];  // per mode, I_m floats
    float *feat;            // rows x 4 (optional)
    float *target;          // rows (optional)
    int64_t row_off[kMaxOrder];  // first row of mode m in feat/target
};

constexpr int kScoreRows = 128, kScoreThreads = 256;
typedef double v4d_t __attribute__((ext_vector_type(4)));

__host__ __device__ inline int pad16(int R) { return (R + 15) & ~15; }

size_t row_scores_lds(int R, bool marg, bool learned) {
    const size_t RP = pad16(R);
    size_t b = sizeof(double) * (RP * RP * (marg ? 2 : 1) + R + 2 * kScoreRows) + sizeof(float) * RP * kScoreRows;
    if (learned) b += sizeof(float) * (kParams + 4 * kScoreRows + kH2 * (kH1 + 1));
    return b;
}

// Quadratic forms q_i = a_i^T M a_i for the block's rows: U = A_rows M on
// FP64 MFMA 16x16x4 (lane l: A operand A[l%16][l/16], B operand
// M[l/16][l%16], result U[l/16 + 4v][l%16]), then the row sums of U * A by
// shuffles over the 16 lanes that share a row, in a fixed order.  The
// 16-row blocks go round-robin over the waves of the block.
__device__ inline void quad_forms(const float *sRow, const double *M1, const double *M2, int RP, int nr, double *q1,
                                  double *q2) {
    const int w = threadIdx.x / kWave, l = threadIdx.x & (kWave - 1), li = l & 15, lk = l >> 4;
    for (int rb = w * 16; rb < nr; rb += (kScoreThreads / kWave) * 16) {
        double p1[4] = {0.0, 0.0, 0.0, 0.0}, p2[4] = {0.0, 0.0, 0.0, 0.0};
        for (int ct = 0; ct < RP; ct += 16) {
            v4d_t u1 = {0.0, 0.0, 0.0, 0.0}, u2 = {0.0, 0.0, 0.0, 0.0};
            for (int k0 = 0; k0 < RP; k0 += 4) {
                const int k = k0 + lk;
                const double av = (double)sRow[k * kScoreRows + rb + li];
                u1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, M1[k * RP + ct + li], u1, 0, 0, 0);
                if (M2) u2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, M2[k * RP + ct + li], u2, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double ar = (double)sRow[(ct + li) * kScoreRows + rb + lk + 4 * v];
                p1[v] += u1[v] * ar;
                p2[v] += u2[v] * ar;
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                p1[v] += __shfl_xor(p1[v], off, kWave);
                p2[v] += __shfl_xor(p2[v], off, kWave);
            }
            if (li == 0) {
                q1[rb + lk + 4 * v] = p1[v];
                q2[rb + lk + 4 * v] = p2[v];
            }
        }
    }
}

__global__ __launch_bounds__(kScoreThreads) void row_scores_kernel(RowArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int m = blockIdx.y, tid = threadIdx.x;
    if (m == a.mi.n) return;
    const int R = a.R, N = a.mi.order, RP = pad16(R);
    const int64_t I = a.mi.dims[m];
    const int64_t r0 = (int64_t)blockIdx.x * kScoreRows;
    if (r0 >= I) return;
    const bool marg = a.Hinv != nullptr;
    const size_t sz = mode_stats_doubles(R);
    double *sGi = (double *)lds;                  // [RP][RP], zero padded
    double *sH = sGi + RP * RP;                   // [RP][RP] (marginals only)
    double *sGd = sH + (marg ? RP * RP : 0);      // [R]
    double *sLev = sGd + R;                       // [kScoreRows]
    double *sMg = sLev + kScoreRows;              // [kScoreRows]
    float *sRow = (float *)(sMg + kScoreRows);    // [RP][kScoreRows], zero padded
    float *P = sRow + RP * kScoreRows;
    const double *G = a.stats + m * sz, *Gi = G + R * R;
    for (int e = tid; e < RP * RP; e += kScoreThreads) {
        const int r = e / RP, c = e - r * RP;
        const bool in = r < R && c < R;
        sGi[e] = in ? Gi[r * R + c] : 0.0;
        if (marg) {
            double h = 0.0;
            if (in) {
                h = a.Hinv[r * R + c];
                for (int k = 0; k < N; ++k)
                    if (k != a.mi.n && k != m) h *= a.stats[k * sz + r * R + c];
            }
            sH[e] = h;
        }
    }
    for (int r = tid; r < R; r += kScoreThreads) sGd[r] = G[r * R + r];
    if (a.learned) {
        constexpr int PU = (kParams + kScoreThreads - 1) / kScoreThreads;
        float t[PU];  // every load of this thread in flight before the first store
#pragma unroll
        for (int u = 0; u < PU; ++u) t[u] = a.params[min(tid + u * kScoreThreads, kParams - 1)];
        float *W2p = P + kParams + 4 * kScoreRows;  // second-layer weights, rows padded to kH1 + 1
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            const int e = tid + u * kScoreThreads;
            if (e < kParams) P[e] = t[u];
            const int w = e - kOffW2;
            if (w >= 0 && w < kH2 * kH1) W2p[(w / kH1) * (kH1 + 1) + w % kH1] = t[u];
        }
    }
    const int nr = (int)min((int64_t)kScoreRows, I - r0);
    for (int e = tid; e < RP * kScoreRows; e += kScoreThreads) sRow[e] = 0.f;
    __syncthreads();
    const float *A = (const float *)a.A.p[m] + r0 * R;
    for (int e = tid; e < nr * R; e += kScoreThreads) {
        const int rr = e / R, c = e - rr * R;
        sRow[c * kScoreRows + rr] = A[e];
    }
    double f4 = 0.0;
    int cnt = 0;
    for (int k = 0; k < N; ++k)
        if (k != a.mi.n && k != m) {
            f4 += a.stats[k * sz + 2 * R * R + 1];
            ++cnt;
        }
    f4 = cnt ? f4 / cnt : 0.0;
    __syncthreads();
    quad_forms(sRow, sGi, marg ? sH : nullptr, RP, nr, sLev, sMg);
    __syncthreads();
    float *sX = P + kParams;  // [kScoreRows][4] features (learned)
    if (tid < nr) {
        const int64_t i = r0 + tid;
        const double frob2 = G[2 * R * R];
        double rn = 0.0, cn = 0.0;
        for (int r = 0; r < R; ++r) {
            const double ar = (double)sRow[r * kScoreRows + tid];
            rn += ar * ar;
            cn += ar * ar / sGd[r];
        }
        const double lev = sLev[tid], mg = marg ? sMg[tid] : 0.0;
        const double f1 = (double)I * rn / frob2, f2 = (double)I / R * lev, f3 = (double)I / R * cn;
        const float x[4] = {logf((float)f1 + kFeatEps), logf((float)f2 + kFeatEps), logf((float)f3 + kFeatEps),
                            (float)f4};
        if (a.learned) {
#pragma unroll
            for (int k = 0; k < 4; ++k) sX[tid * 4 + k] = x[k];
        } else if (a.score[m]) {  // the exact marginal, or (no marginals) the factor's own leverage
            a.score[m][i] = logf((float)fmax(marg ? mg : lev, 1e-30));
        }
        if (a.feat) {
            float *f = a.feat + (a.row_off[m] + i) * 4;
            f[0] = x[0];
            f[1] = x[1];
            f[2] = x[2];
            f[3] = x[3];
        }
        if (a.target) a.target[a.row_off[m] + i] = (float)(mg / R);
    }
    if (!a.learned) return;
    __syncthreads();
    // the network, four lanes per row: each lane the first layer whole and a
    // quarter of the second-layer units with their output terms, summed over
    // the quad
    const int sub = tid & 3;
    for (int row = tid >> 2; row < nr; row += kScoreThreads / 4) {
        // keeps the compiler from hoisting the weight reads out of the row
        // loop (holding them would leave no registers for the inner loads)
        asm volatile("" ::: "memory");
        float x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = sX[row * 4 + k];
        float z = mlp_part(P, P + kParams + 4 * kScoreRows, x, sub);
        z += __shfl_xor(z, 1, kWave);
        z += __shfl_xor(z, 2, kWave);
        if (sub == 0 && a.score[m]) a.score[m][r0 + row] = z + P[kOffB3];
    }
}

// Per mode m != n: p = softmax(score), mixture (1-alpha) p + alpha/I,
// q = max(1, floor(p 2^32)) (at most 2^32-1), cdf = [0, prefix sums].
struct ScoreCdf {
    const float *score[kMaxOrder];
    uint64_t *cdf[kMaxOrder];
};

constexpr int kCdfThreads = 256;

__global__ __launch_bounds__(kCdfThreads) void cdf_kernel(ModeInfo mi, ScoreCdf sc, double alpha_val,
                                                          const double *alpha_dev) {
    __shared__ double s_red[kCdfThreads / kWave];
    __shared__ float s_mx[kCdfThreads / kWave];
    __shared__ uint64_t s_wsum[kCdfThreads / kWave];
    const int m = blockIdx.x;
    if (m == mi.n) return;
    const int64_t I = mi.dims[m];
    const float *z = sc.score[m];
    uint64_t *c = sc.cdf[m];
    const double alpha = alpha_dev ? *alpha_dev : alpha_val;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    constexpr int nw = kCdfThreads / kWave;
    // max of the scores
    float mx = -INFINITY;
    for (int64_t i = tid; i < I; i += kCdfThreads) mx = fmaxf(mx, z[i]);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, kWave));
    if (lane == 0) s_mx[wid] = mx;
    __syncthreads();
    mx = s_mx[0];
    for (int w = 1; w < nw; ++w) mx = fmaxf(mx, s_mx[w]);
    // softmax normaliser, fixed order
    double sum = 0.0;
    for (int64_t i = tid; i < I; i += kCdfThreads) sum += exp((double)z[i] - (double)mx);
    const double tot = block_sum_dyn(sum, s_red);
    // contiguous chunk per thread, integer weights, exclusive scan of the chunk sums
    const int64_t per = ceil_div(I, kCdfThreads);
    const int64_t i0 = tid * per, i1 = min(I, i0 + per);
    auto qof = [&](int64_t i) {
        const double p = (1.0 - alpha) * exp((double)z[i] - (double)mx) / tot + alpha / (double)I;
        double q = floor(p * 4294967296.0);
        q = fmin(fmax(q, 1.0), 4294967295.0);
        return (uint64_t)q;
    };
    uint64_t local = 0;
    for (int64_t i = i0; i < i1; ++i) local += qof(i);
    uint64_t incl = local;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t v = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += v;
    }
    if (lane == kWave - 1) s_wsum[wid] = incl;
    __syncthreads();
    uint64_t base = 0;
    for (int w = 0; w < wid; ++w) base += s_wsum[w];
    uint64_t run = base + incl - local;
    if (tid == 0) c[0] = 0;
    for (int64_t i = i0; i < i1; ++i) {
        run += qof(i);
        c[i + 1] = run;
    }
}

// ---------------------------------------------------------------------------
// training: forward+backward per row with per-block gradient sums.
// group_of[row] gives the group; the loss is the mean over groups of the
// cross-entropy, so dz = (p - t)/ngroups with p the group softmax.
__global__ __launch_bounds__(256) void mlp_logits_kernel(const float *params, const float *X, int64_t rows,
                                                         float *z) {
    __shared__ float P[kParams];
    for (int e = threadIdx.x; e < kParams; e += blockDim.x) P[e] = params[e];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    float x[4] = {X[i * 4], X[i * 4 + 1], X[i * 4 + 2], X[i * 4 + 3]};
    z[i] = mlp_row(P, x);
}

// one block per group: dz = (softmax(z) - t)/ngroups, loss partial per group
__global__ __launch_bounds__(256) void group_ce_kernel(const float *z, const float *t, const int64_t *goff,
                                                       int32_t ngroups, float *dz, double *gloss) {
    __shared__ double s[256];
    const int g = blockIdx.x;
    const int64_t b = goff[g], e = goff[g + 1];
    const int tid = threadIdx.x;
    float mx = -INFINITY;
    for (int64_t i = b + tid; i < e; i += blockDim.x) mx = fmaxf(mx, z[i]);
    __shared__ float sm[256];
    sm[tid] = mx;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (tid < o) sm[tid] = fmaxf(sm[tid], sm[tid + o]);
        __syncthreads();
    }
    mx = sm[0];
    double acc = 0.0;
    for (int64_t i = b + tid; i < e; i += blockDim.x) acc += exp((double)z[i] - (double)mx);
    s[tid] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (tid < o) s[tid] += s[tid + o];
        __syncthreads();
    }
    const double tot = s[0];
    __syncthreads();
    const double lt = log(tot);
    double l = 0.0;
    for (int64_t i = b + tid; i < e; i += blockDim.x) {
        const double lp = (double)z[i] - (double)mx - lt;
        dz[i] = (float)((exp(lp) - (double)t[i]) / ngroups);
        l -= (double)t[i] * lp;
    }
    s[tid] = l;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (tid < o) s[tid] += s[tid + o];
        __syncthreads();
    }
    if (tid == 0) gloss[g] = s[0] / ngroups;
}

constexpr int kGradRows = 96;

// Each block: its rows' contributions to the gradient, summed in a fixed
// order (one thread per parameter, looping over the block's rows).
__global__ __launch_bounds__(256) void mlp_grad_kernel(const float *params, const float *X, const float *dz,
                                                       int64_t rows, float *gpart) {
    __shared__ float P[kParams];
    __shared__ float sx[kGradRows][kIn];
    __shared__ float sh1[kGradRows][kH1 + 1];
    __shared__ float sh2[kGradRows][kH2 + 1];
    __shared__ float sd2[kGradRows][kH2 + 1];
    __shared__ float sd1[kGradRows][kH1 + 1];
    __shared__ float sdz[kGradRows];
    const int tid = threadIdx.x;
    for (int e = tid; e < kParams; e += blockDim.x) P[e] = params[e];
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * kGradRows;
    const int nr = (int)min((int64_t)kGradRows, rows - r0);
    if (tid < nr) {
        const int64_t i = r0 + tid;
        float x[4] = {X[i * 4], X[i * 4 + 1], X[i * 4 + 2], X[i * 4 + 3]};
        float h1[kH1];  // relu(a1); a1 > 0 exactly where h1 > 0
        for (int j = 0; j < kH1; ++j) {
            float s = P[kOffB1 + j];
            for (int k = 0; k < kIn; ++k) s += P[kOffW1 + j * kIn + k] * x[k];
            h1[j] = s > 0.f ? s : 0.f;
            sh1[tid][j] = h1[j];
        }
        const float d = dz[i];
        float dh1[kH1];
        for (int k = 0; k < kH1; ++k) dh1[k] = 0.f;
        for (int j = 0; j < kH2; ++j) {
            float w[kH1];  // row j of W2, read once (all reads issued together) for both products
#pragma unroll
            for (int k = 0; k < kH1; ++k) w[k] = P[kOffW2 + j * kH1 + k];
            float s = P[kOffB2 + j];
#pragma unroll
            for (int k = 0; k < kH1; ++k) s += w[k] * h1[k];
            sh2[tid][j] = s > 0.f ? s : 0.f;
            const float d2 = s > 0.f ? d * P[kOffW3 + j] : 0.f;
            sd2[tid][j] = d2;
#pragma unroll
            for (int k = 0; k < kH1; ++k) dh1[k] += d2 * w[k];
        }
        for (int k = 0; k < kH1; ++k) sd1[tid][k] = h1[k] > 0.f ? dh1[k] : 0.f;
        for (int k = 0; k < kIn; ++k) sx[tid][k] = x[k];
        sdz[tid] = d;
    }
    __syncthreads();
    float *gp = gpart + (size_t)blockIdx.x * kParams;
    for (int p = tid; p < kParams; p += blockDim.x) {
        float acc = 0.f;
        if (p < kOffB1) {
            const int j = p / kIn, k = p % kIn;
            for (int r = 0; r < nr; ++r) acc += sd1[r][j] * sx[r][k];
        } else if (p < kOffW2) {
            const int j = p - kOffB1;
            for (int r = 0; r < nr; ++r) acc += sd1[r][j];
        } else if (p < kOffB2) {
            const int j = (p - kOffW2) / kH1, k = (p - kOffW2) % kH1;
            for (int r = 0; r < nr; ++r) acc += sd2[r][j] * sh1[r][k];
        } else if (p < kOffW3) {
            const int j = p - kOffB2;
            for (int r = 0; r < nr; ++r) acc += sd2[r][j];
        } else if (p < kOffB3) {
            const int j = p - kOffW3;
            for (int r = 0; r < nr; ++r) acc += sdz[r] * sh2[r][j];
        } else {
            for (int r = 0; r < nr; ++r) acc += sdz[r];
        }
        gp[p] = acc;
    }
}

// The per-block gradients summed in two fixed-order stages.  Stage one,
// chunk c = blockIdx.y < nchunks: the parts b = c, c + nchunks, ... of
// parameter p, written in place over part c (which only this thread reads).
__global__ __launch_bounds__(256) void grad_chunk_kernel(float *gpart, int32_t nparts, int32_t nchunks) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
    if (p >= kParams || c >= nchunks) return;
    double acc = 0.0;
    for (int b = c; b < nparts; b += nchunks) acc += (double)gpart[(size_t)b * kParams + p];
    gpart[(size_t)c * kParams + p] = (float)acc;
}

// Stage two: the nchunks chunk sums in order.
__global__ __launch_bounds__(256) void grad_reduce_kernel(const float *gpart, int32_t nparts, float *grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    double acc = 0.0;
    for (int b = 0; b < nparts; ++b) acc += (double)gpart[(size_t)b * kParams + p];
    grad[p] = (float)acc;
}

__global__ __launch_bounds__(256) void adam_kernel(float *params, const float *grad, float *mom, float *vel,
                                                   int32_t step, float lr, float b1, float b2, float eps) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    const float g = grad[p];
    const float m = b1 * mom[p] + (1.f - b1) * g;
    const float v = b2 * vel[p] + (1.f - b2) * g * g;
    mom[p] = m;
    vel[p] = v;
    const float mh = m / (1.f - powf(b1, (float)step));
    const float vh = v / (1.f - powf(b2, (float)step));
    params[p] -= lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------------------------------
static size_t inv_lds(int R) {
    const int ld = R + 1;
    return sizeof(double) * ((size_t)3 * R * ld + 66 + kMaxRank) + sizeof(int) * 68;
}

size_t gram_part_doubles(int order, int R) { return (size_t)order * kGramChunks * R * R; }

hipError_t launch_mode_stats(const FactorPtrs &A, const ModeInfo &mi, int32_t R, double *stats, double *gpart,
                             double *Hinv, hipStream_t st) {
    hipLaunchKernelGGL(gram_part_kernel, dim3(kGramChunks, mi.order), dim3(kStatThreads), 0, st, A, mi, R, gpart);
    hipLaunchKernelGGL(stats_finish_kernel, dim3(mi.order), dim3(kStatThreads), inv_lds(R), st, mi, R,
                       (const double *)gpart, stats, Hinv);
    return hipGetLastError();
}

hipError_t launch_row_scores(const FactorPtrs &A, const ModeInfo &mi, int32_t R, const double *stats,
                             const double *Hinv, const float *params, bool learned, float *const *score, float *feat,
                             float *target, const int64_t *row_off, hipStream_t st) {
    RowArgs a{};
    a.A = A;
    a.mi = mi;
    a.R = R;
    a.stats = stats;
    a.Hinv = Hinv;
    a.params = params;
    a.learned = learned ? 1 : 0;
    int64_t maxI = 1;
    for (int m = 0; m < mi.order; ++m) {
        a.score[m] = score ? score[m] : nullptr;
        a.row_off[m] = row_off ? row_off[m] : 0;
        if (m != mi.n) maxI = std::max(maxI, mi.dims[m]);
    }
    a.feat = feat;
    a.target = target;
    dim3 grid((unsigned)ceil_div(maxI, kScoreRows), mi.order);
    hipLaunchKernelGGL(row_scores_kernel, grid, dim3(kScoreThreads), row_scores_lds(R, Hinv != nullptr, learned), st,
                       a);
    return hipGetLastError();
}

hipError_t launch_cdf(const ModeInfo &mi, float *const *score, double alpha, const double *alpha_dev,
                      uint64_t *const *cdf, hipStream_t st) {
    ScoreCdf sc{};
    for (int m = 0; m < mi.order; ++m) {
        sc.score[m] = score[m];
        sc.cdf[m] = cdf[m];
    }
    hipLaunchKernelGGL(cdf_kernel, dim3(mi.order), dim3(kCdfThreads), 0, st, mi, sc, alpha, alpha_dev);
    return hipGetLastError();
}

hipError_t launch_mlp_logits(const float *params, const float *X, int64_t rows, float *z, hipStream_t st) {
    hipLaunchKernelGGL(mlp_logits_kernel, dim3((unsigned)ceil_div(rows, 256)), dim3(256), 0, st, params, X, rows, z);
    return hipGetLastError();
}

hipError_t launch_group_ce(const float *z, const float *t, const int64_t *goff, int32_t ngroups, float *dz,
                           double *gloss, hipStream_t st) {
    hipLaunchKernelGGL(group_ce_kernel, dim3(ngroups), dim3(256), 0, st, z, t, goff, ngroups, dz, gloss);
    return hipGetLastError();
}

int32_t mlp_grad_blocks(int64_t rows) { return (int32_t)ceil_div(rows, kGradRows); }

hipError_t launch_mlp_grad(const float *params, const float *X, const float *dz, int64_t rows, float *gpart,
                           float *grad, hipStream_t st) {
    const int nb = mlp_grad_blocks(rows);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(nb), dim3(256), 0, st, params, X, dz, rows, gpart);
    const int nchunks = std::min(nb, 64);  // stage one reads nb parts, writes parts 0 .. nchunks-1
    const unsigned pb = (unsigned)ceil_div(kParams, 256);
    hipLaunchKernelGGL(grad_chunk_kernel, dim3(pb, nchunks), dim3(256), 0, st, gpart, nb, nchunks);
    hipLaunchKernelGGL(grad_reduce_kernel, dim3(pb), dim3(256), 0, st, gpart, nchunks, grad);
    return hipGetLastError();
}

hipError_t launch_adam(float *params, const float *grad, float *m, float *v, int32_t step, float lr, hipStream_t st) {
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)ceil_div(kParams, 256)), dim3(256), 0, st, params, grad, m, v, step,
                       lr, 0.9f, 0.999f, 1e-8f);
    return hipGetLastError();
}

}  // namespace cprand
