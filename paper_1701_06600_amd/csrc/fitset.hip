// The importance-weighted fit set (a project addition to the sampled fit
// estimate of Section 3.4, for unmixed tensors whose energy and residual sit
// in few slices).  Entries come from a defensive mixture: with probability
// beta from the product of per-mode proposals proportional to the mode slice
// energies of X, s_m(i) = sum of x^2 over the entries with index i in mode
// m (mixed with uniform by alpha, quantised to integers), and with
// probability 1 - beta uniformly.  Entry i carries w(i) = 1 / (P q(i)),
// q(i) = beta prod_m q_m(i_m)/Q_m + (1 - beta)/P, so the estimate
// P mean(w e^2) of ||E||^2 stays unbiased and w <= 1 / (1 - beta).
//
// Slice energies are summed in 64-bit fixed point (x^2 scaled by
// 2^62 / ||X||^2, so every slice sum fits): integer sums do not depend on
// the order of the atomic adds, so the tables, and with them the fit set,
// are the same at every run.
#include <math.h>

#include <algorithm>

#include "kernels.hpp"

namespace cprand {

constexpr int kEnergyThreads = 256;
constexpr int kEnergyLdsBins = 8192;  // sum of the dims up to which the bins live in LDS

__device__ inline double load_real(const void *X, int kind, int64_t o) {
    switch (kind) {
        case K_F64: return ((const double *)X)[o];
        case K_F32: return (double)((const float *)X)[o];
        default: return (double)bf16_to_f32(((const uint16_t *)X)[o]);
    }
}

// Grid-stride over the column-major element order; each thread takes runs
// of kRun consecutive elements, computes their mode indices once and steps
// them, and adds a run's fixed-point squares per bin (an add per element for
// mode 0, one per run and mode where the index does not change).
constexpr int kRun = 8;

__global__ __launch_bounds__(kEnergyThreads) void slice_energy_kernel(ModeInfo mi, const void *X, int kind,
                                                                      const double *normX, int64_t P,
                                                                      unsigned long long *bins, int nbins) {
    __shared__ unsigned long long lb[kEnergyLdsBins];
    const bool lds = nbins <= kEnergyLdsBins;
    if (lds)
        for (int e = threadIdx.x; e < nbins; e += kEnergyThreads) lb[e] = 0ull;
    __syncthreads();
    unsigned long long *b = lds ? lb : bins;
    const int N = mi.order;
    const double nx = *normX;
    const double scale = nx > 0.0 ? ldexp(1.0, 62) / (nx * nx * (1.0 + 1e-6)) : 0.0;
    int off[kMaxOrder];
    {
        int o = 0;
#pragma unroll
        for (int m = 0; m < kMaxOrder; ++m) {
            off[m] = o;
            if (m < N) o += (int)mi.dims[m];
        }
    }
    const int64_t nruns = ceil_div(P, kRun);
    for (int64_t r = (int64_t)blockIdx.x * kEnergyThreads + threadIdx.x; r < nruns;
         r += (int64_t)gridDim.x * kEnergyThreads) {
        const int64_t e0 = r * kRun;
        int64_t idx[kMaxOrder];
        int64_t rem = e0, o = 0;
#pragma unroll
        for (int m = 0; m < kMaxOrder; ++m) {
            if (m >= N) break;
            idx[m] = rem % mi.dims[m];
            rem /= mi.dims[m];
            o += idx[m] * mi.strides[m];
        }
        unsigned long long acc = 0ull;  // run sum of the modes >= 1 since their last change
        const int ne = (int)min((int64_t)kRun, P - e0);
        for (int j = 0; j < ne; ++j) {
            const double x = load_real(X, kind, o);
            const unsigned long long v = (unsigned long long)(x * x * scale + 0.5);
            atomicAdd(&b[off[0] + idx[0]], v);
            acc += v;
            if (j + 1 == ne) break;
            // step the mixed-radix index; modes >= 1 flush their run sum when they change
            ++idx[0];
            o += mi.strides[0];
            if (idx[0] == mi.dims[0]) {
                idx[0] = 0;
                o -= mi.strides[0] * mi.dims[0];
                int m = 1;
                for (; m < N; ++m) {
                    atomicAdd(&b[off[m] + idx[m]], acc);
                    ++idx[m];
                    o += mi.strides[m];
                    if (idx[m] < mi.dims[m]) break;
                    idx[m] = 0;
                    o -= mi.strides[m] * mi.dims[m];
                }
                for (++m; m < N; ++m) atomicAdd(&b[off[m] + idx[m]], acc);
                acc = 0ull;
            }
        }
        for (int m = 1; m < N && acc; ++m) atomicAdd(&b[off[m] + idx[m]], acc);
    }
    if (lds) {
        __syncthreads();
        for (int e = threadIdx.x; e < nbins; e += kEnergyThreads)
            if (lb[e]) atomicAdd(&bins[e], lb[e]);
    }
}

// One workgroup per mode: the integer proposal q_i = max(1, floor(p_i 2^32))
// of p_i = (1 - alpha) s(i)/sum(s) + alpha/I, and its table cdf[0] = 0,
// cdf[i+1] = cdf[i] + q_i.  With every s(i) = 0 the proposal is uniform.
constexpr int kTabThreads = 256;
__global__ __launch_bounds__(kTabThreads) void energy_cdf_kernel(ModeInfo mi, const unsigned long long *bins,
                                                                 double alpha, CdfPtrs cdf, double *energy_out,
                                                                 const double *normX) {
    __shared__ unsigned long long s_tot[kTabThreads / kWave];
    __shared__ uint64_t s_wsum[kTabThreads / kWave];
    const int m = blockIdx.x;
    int off = 0;
    for (int k = 0; k < m; ++k) off += (int)mi.dims[k];
    const int64_t I = mi.dims[m];
    const unsigned long long *s = bins + off;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    constexpr int nw = kTabThreads / kWave;
    unsigned long long t = 0ull;
    for (int64_t i = tid; i < I; i += kTabThreads) t += s[i];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) t += __shfl_xor(t, o, kWave);
    if (lane == 0) s_tot[wid] = t;
    __syncthreads();
    unsigned long long tot = 0ull;
    for (int w = 0; w < nw; ++w) tot += s_tot[w];
    const double nx = *normX;
    const double unscale = nx * nx * (1.0 + 1e-6) / ldexp(1.0, 62);
    if (energy_out)
        for (int64_t i = tid; i < I; i += kTabThreads) energy_out[off + i] = (double)s[i] * unscale;
    auto qof = [&](int64_t i) {
        const double p = tot ? (double)s[i] / (double)tot : 1.0 / (double)I;
        const double pm = (1.0 - alpha) * p + alpha / (double)I;
        double q = floor(pm * 4294967296.0);
        q = fmin(fmax(q, 1.0), 4294967295.0);
        return (uint64_t)q;
    };
    const int64_t per = ceil_div(I, kTabThreads);
    const int64_t i0 = tid * per, i1 = min(I, i0 + per);
    uint64_t local = 0;
    for (int64_t i = i0; i < i1; ++i) local += qof(i);
    uint64_t incl = local;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint64_t v = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += v;
    }
    if (lane == kWave - 1) s_wsum[wid] = incl;
    __syncthreads();
    uint64_t base = 0;
    for (int w = 0; w < wid; ++w) base += s_wsum[w];
    uint64_t run = base + incl - local;
    uint64_t *c = (uint64_t *)cdf.p[m];
    if (tid == 0) c[0] = 0;
    for (int64_t i = i0; i < i1; ++i) {
        run += qof(i);
        c[i + 1] = run;
    }
}

// Entry p of the weighted fit set: Philox counter (p, 1, 0, b) under key
// (seed, FIT); word j of the sequence (block j / 4, word j % 4): j = 0 picks
// the component (the product when (u >> 11) < beta_thr), j = k + 1 the row
// of mode k.  The weight's FP64 operations are not contracted into fused
// multiply-adds, so they round like the separate operations of the oracle.
__device__ inline double fit_weight(const int64_t *row, const ModeInfo &mi, const CdfPtrs &cdf, double beta,
                                    double P) {
#pragma clang fp contract(off)
    double prod = 1.0;
    for (int k = 0; k < mi.order; ++k) {
        const uint64_t *c = cdf.p[k];
        const double q = (double)(c[row[k] + 1] - c[row[k]]);
        const double Q = (double)c[mi.dims[k]];
        prod = prod * (q / Q);
    }
    return 1.0 / (beta * P * prod + (1.0 - beta));
}

__global__ __launch_bounds__(256) void fit_set_weighted_kernel(ModeInfo mi, const void *X, int kind, int32_t P_hat,
                                                               uint64_t seed, CdfPtrs cdf, uint64_t beta_thr,
                                                               double beta, double P, int32_t *frow, double *fx,
                                                               double *fw) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= P_hat) return;
    const int N = mi.order;
    int64_t row[kMaxOrder];
    int64_t o = 0;
    bool prod = false;
    u64x4 blk;
#pragma unroll
    for (int j = 0; j <= kMaxOrder; ++j) {
        if (j > N) break;
        if ((j & 3) == 0) blk = philox4x64_10((uint64_t)p, 1, 0, (uint64_t)(j >> 2), seed, kTagFit);
        const uint64_t u = u64x4_get(blk, j & 3);
        if (j == 0) {
            prod = (u >> 11) < beta_thr;
            continue;
        }
        const int k = j - 1;
        const int64_t I = mi.dims[k];
        if (prod) {
            const uint64_t *c = cdf.p[k];
            row[k] = cdf_search(c, I, mulhi64(u, c[I]));
        } else {
            row[k] = (int64_t)mulhi64(u, (uint64_t)I);
        }
        o += row[k] * mi.strides[k];
    }
    for (int k = 0; k < N; ++k) frow[p * N + k] = (int32_t)row[k];
    if (fx) {
        fx[2 * p] = load_real(X, kind, o);
        fx[2 * p + 1] = 0.0;
    }
    fw[p] = fit_weight(row, mi, cdf, beta, P);
}

__global__ void zero_u64_kernel(unsigned long long *p, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < n) p[e] = 0ull;
}

hipError_t launch_energy_tables(const ModeInfo &mi, const void *X, int kind, const double *normX,
                                unsigned long long *bins, double alpha, const CdfPtrs &cdf, double *energy_out,
                                hipStream_t st) {
    int nbins = 0;
    int64_t P = 1;
    for (int m = 0; m < mi.order; ++m) {
        nbins += (int)mi.dims[m];
        P *= mi.dims[m];
    }
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)ceil_div(nbins, 256)), dim3(256), 0, st, bins, (int64_t)nbins);
    const int64_t runs = ceil_div(P, kRun);
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(2048, ceil_div(runs, kEnergyThreads)));
    hipLaunchKernelGGL(slice_energy_kernel, dim3(nb), dim3(kEnergyThreads), 0, st, mi, X, kind, normX, P, bins, nbins);
    hipLaunchKernelGGL(energy_cdf_kernel, dim3(mi.order), dim3(kTabThreads), 0, st, mi,
                       (const unsigned long long *)bins, alpha, cdf, energy_out, normX);
    return hipGetLastError();
}

uint64_t fit_beta_threshold(double beta) {
    if (!(beta > 0.0)) return 0;
    if (beta >= 1.0) return (uint64_t)1 << 53;
    return (uint64_t)floor(beta * 9007199254740992.0);
}

hipError_t launch_fit_set_weighted(const ModeInfo &mi, const void *X, int kind, int32_t P_hat, uint64_t seed,
                                   const CdfPtrs &cdf, double beta, int32_t *frow, double *fx, double *fw,
                                   hipStream_t st) {
    double P = 1.0;
    for (int m = 0; m < mi.order; ++m) P *= (double)mi.dims[m];
    hipLaunchKernelGGL(fit_set_weighted_kernel, dim3((unsigned)ceil_div(P_hat, 256)), dim3(256), 0, st, mi, X, kind,
                       P_hat, seed, cdf, fit_beta_threshold(beta), beta, P, frow, fx, fw);
    return hipGetLastError();
}

}  // namespace cprand
