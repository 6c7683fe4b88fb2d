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
__global__ __launch_bounds__(256) void mode_stats_kernel(FactorPtrs A, ModeInfo mi, int32_t R, double *stats,
                                                         int32_t skip) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int m = blockIdx.x;
    if (m == skip) return;
    const int ld = R + 1;
    double *B1 = (double *)lds, *B2 = B1 + R * ld, *B3 = B2 + R * ld, *cs = B3 + R * ld, *tmp = cs + 66;
    int *pairs = (int *)(tmp + kMaxRank);
    const float *a = (const float *)A.p[m];
    const int64_t I = mi.dims[m];
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
        const int r = e / R, s = e - r * R;
        double acc = 0.0;
        for (int64_t i = 0; i < I; ++i) acc += (double)a[i * R + r] * (double)a[i * R + s];
        B1[r * ld + s] = acc;
        B3[r * ld + s] = acc;
    }
    __syncthreads();
    double *st = stats + (size_t)m * (2 * R * R + 2);
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) st[e] = B3[(e / R) * ld + e % R];
    if (threadIdx.x == 0) {
        double fr = 0.0, cg = 0.0;
        for (int r = 0; r < R; ++r) fr += B3[r * ld + r];
        for (int r = 0; r < R; ++r)
            for (int s = 0; s < R; ++s)
                if (r != s) cg += fabs(B3[r * ld + s]) / sqrt(B3[r * ld + r] * B3[s * ld + s]);
        st[2 * R * R] = fr;
        st[2 * R * R + 1] = R > 1 ? cg / ((double)R * (R - 1)) : 0.0;
    }
    spd_inverse(B1, B2, B3, tmp, R, ld, cs, pairs);
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) st[R * R + e] = B1[(e / R) * ld + e % R];
}

// H_m = inverse(Hadamard of the Grams in K) * Hadamard of the Grams in K\{m},
// for every m in K (K = all modes but n).  One workgroup.
__global__ __launch_bounds__(256) void marginal_h_kernel(ModeInfo mi, int32_t R, const double *stats, double *H) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int ld = R + 1, n = mi.n, N = mi.order;
    double *B1 = (double *)lds, *B2 = B1 + R * ld, *B3 = B2 + R * ld, *cs = B3 + R * ld, *tmp = cs + 66;
    int *pairs = (int *)(tmp + kMaxRank);
    const size_t sz = 2 * (size_t)R * R + 2;
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
        double g = 1.0;
        for (int k = 0; k < N; ++k)
            if (k != n) g *= stats[k * sz + e];
        B1[(e / R) * ld + e % R] = g;
        B3[(e / R) * ld + e % R] = g;
    }
    __syncthreads();
    spd_inverse(B1, B2, B3, tmp, R, ld, cs, pairs);
    for (int m = 0; m < N; ++m) {
        if (m == n) continue;
        for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
            double h = B1[(e / R) * ld + e % R];
            for (int k = 0; k < N; ++k)
                if (k != n && k != m) h *= stats[k * sz + e];
            H[(size_t)m * R * R + e] = h;
        }
    }
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

// Row scores for every mode m != n: mode == LEARNED: the network's logit;
// mode == MARGINAL: log of the exact marginal.  Also (optionally) writes the
// feature rows and the exact targets L/R for training.
struct RowArgs {
    FactorPtrs A;
    ModeInfo mi;
    int32_t R;
    const double *stats;
    const double *H;        // marginal matrices (may be NULL when not needed)
    const float *params;    // network (LEARNED)
    int32_t learned;
    float *score[kMaxOrder];  // per mode, I_m floats
    float *feat;            // rows x 4 (optional)
    float *target;          // rows (optional)
    int64_t row_off[kMaxOrder];  // first row of mode m in feat/target
};

__global__ __launch_bounds__(256) void row_scores_kernel(RowArgs a) {
    __shared__ float P[kParams];
    __shared__ double s_f4[kMaxOrder];
    const int m = blockIdx.y;
    if (m == a.mi.n) return;
    const int R = a.R, N = a.mi.order;
    const size_t sz = 2 * (size_t)R * R + 2;
    if (a.learned)
        for (int e = threadIdx.x; e < kParams; e += blockDim.x) P[e] = a.params[e];
    if (threadIdx.x == 0) {
        double c = 0.0;
        int cnt = 0;
        for (int k = 0; k < N; ++k)
            if (k != a.mi.n && k != m) {
                c += a.stats[k * sz + 2 * R * R + 1];
                ++cnt;
            }
        s_f4[0] = cnt ? c / cnt : 0.0;
    }
    __syncthreads();
    const int64_t I = a.mi.dims[m];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= I) return;
    const float *row = (const float *)a.A.p[m] + i * R;
    const double *G = a.stats + m * sz, *Gi = G + R * R;
    const double frob2 = G[2 * R * R];
    double rn = 0.0, lev = 0.0, cn = 0.0, marg = 0.0;
    for (int r = 0; r < R; ++r) {
        const double ar = (double)row[r];
        rn += ar * ar;
        cn += ar * ar / G[r * R + r];
        double gr = 0.0, hr = 0.0;
        for (int s = 0; s < R; ++s) {
            gr += Gi[r * R + s] * (double)row[s];
            if (a.H) hr += a.H[(size_t)m * R * R + r * R + s] * (double)row[s];
        }
        lev += ar * gr;
        marg += ar * hr;
    }
    const double f1 = (double)I * rn / frob2, f2 = (double)I / R * lev, f3 = (double)I / R * cn;
    float x[4] = {logf((float)f1 + kFeatEps), logf((float)f2 + kFeatEps), logf((float)f3 + kFeatEps),
                  (float)s_f4[0]};
    float sc;
    if (a.learned)
        sc = mlp_row(P, x);
    else
        sc = logf((float)fmax(marg, 1e-30));
    if (a.score[m]) a.score[m][i] = sc;
    if (a.feat) {
        float *f = a.feat + (a.row_off[m] + i) * 4;
        f[0] = x[0];
        f[1] = x[1];
        f[2] = x[2];
        f[3] = x[3];
    }
    if (a.target) a.target[a.row_off[m] + i] = (float)(marg / R);
}

// Per mode m != n: p = softmax(score), mixture (1-alpha) p + alpha/I,
// q = max(1, floor(p 2^32)) (at most 2^32-1), cdf = [0, prefix sums].
struct ScoreCdf {
    const float *score[kMaxOrder];
    uint64_t *cdf[kMaxOrder];
};

__global__ __launch_bounds__(256) void cdf_kernel(ModeInfo mi, ScoreCdf sc, double alpha_val, const double *alpha_dev) {
    __shared__ float s_red[256];
    __shared__ uint64_t s_scan[256];
    const int m = blockIdx.x;
    if (m == mi.n) return;
    const int64_t I = mi.dims[m];
    const float *z = sc.score[m];
    uint64_t *c = sc.cdf[m];
    const double alpha = alpha_dev ? *alpha_dev : alpha_val;
    const int tid = threadIdx.x, nt = blockDim.x;
    float mx = -INFINITY;
    for (int64_t i = tid; i < I; i += nt) mx = fmaxf(mx, z[i]);
    s_red[tid] = mx;
    __syncthreads();
    for (int o = nt / 2; o > 0; o >>= 1) {
        if (tid < o) s_red[tid] = fmaxf(s_red[tid], s_red[tid + o]);
        __syncthreads();
    }
    mx = s_red[0];
    __syncthreads();
    double sum = 0.0;
    for (int64_t i = tid; i < I; i += nt) sum += exp((double)z[i] - (double)mx);
    __shared__ double s_sum[256];
    s_sum[tid] = sum;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int t = 0; t < nt; ++t) s += s_sum[t];
        s_sum[0] = s;
    }
    __syncthreads();
    const double tot = s_sum[0];
    // contiguous chunk per thread, then an exclusive scan of the chunk sums
    const int64_t per = ceil_div(I, nt);
    const int64_t i0 = tid * per, i1 = min(I, i0 + per);
    uint64_t local = 0;
    for (int64_t i = i0; i < i1; ++i) {
        const double p = (1.0 - alpha) * exp((double)z[i] - (double)mx) / tot + alpha / (double)I;
        double q = floor(p * 4294967296.0);
        q = fmin(fmax(q, 1.0), 4294967295.0);
        local += (uint64_t)q;
    }
    s_scan[tid] = local;
    __syncthreads();
    if (tid == 0) {
        uint64_t run = 0;
        for (int t = 0; t < nt; ++t) {
            const uint64_t v = s_scan[t];
            s_scan[t] = run;
            run += v;
        }
        c[0] = 0;
    }
    __syncthreads();
    uint64_t run = s_scan[tid];
    for (int64_t i = i0; i < i1; ++i) {
        const double p = (1.0 - alpha) * exp((double)z[i] - (double)mx) / tot + alpha / (double)I;
        double q = floor(p * 4294967296.0);
        q = fmin(fmax(q, 1.0), 4294967295.0);
        run += (uint64_t)q;
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
        float a1[kH1], h1[kH1];
        for (int j = 0; j < kH1; ++j) {
            float s = P[kOffB1 + j];
            for (int k = 0; k < kIn; ++k) s += P[kOffW1 + j * kIn + k] * x[k];
            a1[j] = s;
            h1[j] = s > 0.f ? s : 0.f;
            sh1[tid][j] = h1[j];
        }
        const float d = dz[i];
        float dh1[kH1];
        for (int k = 0; k < kH1; ++k) dh1[k] = 0.f;
        for (int j = 0; j < kH2; ++j) {
            float s = P[kOffB2 + j];
            for (int k = 0; k < kH1; ++k) s += P[kOffW2 + j * kH1 + k] * h1[k];
            sh2[tid][j] = s > 0.f ? s : 0.f;
            const float d2 = s > 0.f ? d * P[kOffW3 + j] : 0.f;
            sd2[tid][j] = d2;
            for (int k = 0; k < kH1; ++k) dh1[k] += d2 * P[kOffW2 + j * kH1 + k];
        }
        for (int k = 0; k < kH1; ++k) sd1[tid][k] = a1[k] > 0.f ? dh1[k] : 0.f;
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

hipError_t launch_mode_stats(const FactorPtrs &A, const ModeInfo &mi, int32_t R, double *stats, int32_t skip,
                             hipStream_t st) {
    hipLaunchKernelGGL(mode_stats_kernel, dim3(mi.order), dim3(256), inv_lds(R), st, A, mi, R, stats, skip);
    return hipGetLastError();
}

hipError_t launch_marginal_h(const ModeInfo &mi, int32_t R, const double *stats, double *H, hipStream_t st) {
    hipLaunchKernelGGL(marginal_h_kernel, dim3(1), dim3(256), inv_lds(R), st, mi, R, stats, H);
    return hipGetLastError();
}

hipError_t launch_row_scores(const FactorPtrs &A, const ModeInfo &mi, int32_t R, const double *stats, const double *H,
                             const float *params, bool learned, float *const *score, float *feat, float *target,
                             const int64_t *row_off, hipStream_t st) {
    RowArgs a{};
    a.A = A;
    a.mi = mi;
    a.R = R;
    a.stats = stats;
    a.H = H;
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
    dim3 grid((unsigned)ceil_div(maxI, 256), mi.order);
    hipLaunchKernelGGL(row_scores_kernel, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_cdf(const ModeInfo &mi, float *const *score, double alpha, const double *alpha_dev,
                      uint64_t *const *cdf, hipStream_t st) {
    ScoreCdf sc{};
    for (int m = 0; m < mi.order; ++m) {
        sc.score[m] = score[m];
        sc.cdf[m] = cdf[m];
    }
    hipLaunchKernelGGL(cdf_kernel, dim3(mi.order), dim3(256), 0, st, mi, sc, alpha, alpha_dev);
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
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((unsigned)ceil_div(kParams, 256)), dim3(256), 0, st, gpart, nb, grad);
    return hipGetLastError();
}

hipError_t launch_adam(float *params, const float *grad, float *m, float *v, int32_t step, float lr, hipStream_t st) {
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)ceil_div(kParams, 256)), dim3(256), 0, st, params, grad, m, v, step,
                       lr, 0.9f, 0.999f, 1e-8f);
    return hipGetLastError();
}

}  // namespace cprand
