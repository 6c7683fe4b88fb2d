// Real orthogonal mixing for CPRAND-PREMIX (Section 3.3, Alg. 5): the
// orthonormal DCT-II, C[k][i] = s_k cos(pi k (2i + 1) / (2L)) with s_0 =
// sqrt(1/L) and s_k = sqrt(2/L), applied along every mode of a real tensor
// after the random signs, and the matching mix and unmix of factor matrices.
//
// Tensor passes compute the DCT through one complex FFT of the same length
// (Makhoul, "A fast cosine transform in one and multiple dimensions", IEEE
// TASSP 1980): with v[n] = x[2n] and v[L-1-n] = x[2n+1],
//   sum_i x[i] cos(pi k (2i + 1) / (2L)) = Re(exp(-i pi k / (2L)) V[k]),
// V the unnormalised DFT of v.  Two real fibers share one complex FFT (one
// in the real, one in the imaginary part of z); their spectra separate by
// conjugate symmetry, V1[k] = (Z[k] + conj Z[L-k]) / 2 and V2[k] = (Z[k] -
// conj Z[L-k]) / (2i).  The FFT stages are those of the CPRAND-MIX passes.
// Each pass reads and writes 1 real element per element of the tensor.
#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "fft_device.hpp"

namespace cprand {

// Post-rotation table of one length: (s_k cos(pi k/(2L)), s_k sin(pi k/(2L)))
// for k < L, computed on the host in FP64; cached per (device, L, precision).
static const void *dct_table_get(int64_t L, bool dbl, hipError_t *err) {
    static std::mutex mu;
    static std::map<std::tuple<int, int64_t, int>, void *> cache;
    *err = hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *err = e;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_tuple(dev, L, dbl ? 1 : 0);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    const size_t esz = dbl ? 16 : 8;
    std::vector<unsigned char> host(esz * L);
    for (int64_t k = 0; k < L; ++k) {
        const double s = k == 0 ? sqrt(1.0 / (double)L) : sqrt(2.0 / (double)L);
        const double a = M_PI * (double)k / (2.0 * (double)L);
        const double c = s * cos(a), sn = s * sin(a);
        if (dbl) {
            ((double *)host.data())[2 * k] = c;
            ((double *)host.data())[2 * k + 1] = sn;
        } else {
            ((float *)host.data())[2 * k] = (float)c;
            ((float *)host.data())[2 * k + 1] = (float)sn;
        }
    }
    void *d = nullptr;
    e = hipMalloc(&d, esz * L);
    if (e == hipSuccess) e = hipMemcpy(d, host.data(), esz * L, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        *err = e;
        return nullptr;
    }
    cache[key] = d;
    return d;
}

// One DCT-II pass along mode m over a tile of 2 TC real fibers.  The tensor
// Y is column-major [J][L][K] (J = product of the dims before m, K after);
// fiber q is (j = q % J, k = q / J), element l at j + J L k + J l.  FIRST
// (m = 0): read X through its own strides, multiply by the product of every
// mode's signs and write Y; otherwise Y is transformed in place.  LC > 0:
// compile-time length (in-place Stockham stages, one LDS tile), else the
// run-time radix schedule of fp (two tiles).
template <typename T, typename Tin, int LC, int TC, int NT, bool FIRST>
__global__ __launch_bounds__(NT) void dct_pass_kernel(FftPlan fp, const Tin *X, T *Y, int64_t J, int64_t K,
                                                      ModeInfo xi, int m, const int8_t *signs, const cx<T> *twg,
                                                      const cx<T> *csg) {
    extern __shared__ __align__(16) unsigned char lds[];
    constexpr int FC = 2 * TC;
    const int L = LC > 0 ? LC : (int)fp.L;
    const int ldt = TC + 1;
    cx<T> *b0 = (cx<T> *)lds;
    cx<T> *b1 = LC > 0 ? b0 : b0 + L * ldt;
    cx<T> *tw = b1 + L * ldt;
    cx<T> *cs = tw + L;
    __shared__ int64_t cout[FC];
    __shared__ int64_t cin[FIRST ? FC : 1];
    __shared__ T csign[FIRST ? FC : 1];
    const int tid = threadIdx.x;
    const int64_t ncols = J * K;
    const int64_t q0 = (int64_t)blockIdx.x * FC;
    const int nc = (int)min((int64_t)FC, ncols - q0);
    for (int e = tid; e < L; e += NT) {
        tw[e] = twg[e];
        cs[e] = csg[e];
    }
    for (int c = tid; c < FC; c += NT) {
        if (c >= nc) continue;
        const int64_t q = q0 + c;
        const int64_t j = q % J, k = q / J;
        cout[c] = j + J * L * k;
        if (FIRST) {  // m = 0: q runs over modes 1 .. order-1
            int64_t r = q, off = 0;
            T sg = (T)1;
            int soff = (int)xi.dims[0];
            for (int mm = 1; mm < xi.order; ++mm) {
                const int64_t im = r % xi.dims[mm];
                r /= xi.dims[mm];
                off += im * xi.strides[mm];
                sg *= (T)signs[soff + im];
                soff += (int)xi.dims[mm];
            }
            cin[c] = off;
            csign[c] = sg;
        }
    }
    __syncthreads();
    // fiber c -> real (even c) or imaginary (odd c) part of column c / 2, in
    // Makhoul's order; fibers past the end contribute zeros
    for (int e = tid; e < L * FC; e += NT) {
        int l, c;
        if (J == 1) {
            c = e / L;
            l = e - c * L;
        } else {
            l = e / FC;
            c = e - l * FC;
        }
        T v = (T)0;
        if (c < nc) {
            if (FIRST)
                v = (T)X[cin[c] + xi.strides[0] * (int64_t)l] * csign[c] * (T)signs[l];
            else
                v = Y[cout[c] + J * (int64_t)l];
        }
        const int p = (l & 1) ? (L - 1 - (l >> 1)) : (l >> 1);
        ((T *)&b0[p * ldt + (c >> 1)])[c & 1] = v;
    }
    __syncthreads();
    cx<T> *res;
    if constexpr (LC > 0) {
        fft_ct<T, LC, TC, NT, -1>(b0, tw);
        res = b0;
    } else {
        res = fft_tile_rt<T, -1>(b0, b1, fp, ldt, TC, tw);
    }
    for (int e = tid; e < L * FC; e += NT) {
        int k, c;
        if (J == 1) {
            c = e / L;
            k = e - c * L;
        } else {
            k = e / FC;
            c = e - k * FC;
        }
        if (c >= nc) continue;
        const int cc = c >> 1, mk = k == 0 ? 0 : L - k;
        const cx<T> zk = res[k * ldt + cc], zm = res[mk * ldt + cc];
        T a, b;
        if (c & 1) {  // V2 = (Z[k] - conj Z[L-k]) / (2i)
            a = zk.im + zm.im;
            b = zm.re - zk.re;
        } else {      // V1 = (Z[k] + conj Z[L-k]) / 2
            a = zk.re + zm.re;
            b = zk.im - zm.im;
        }
        const cx<T> w = cs[k];
        Y[cout[c] + J * (int64_t)k] = (T)0.5 * (w.re * a + w.im * b);
    }
}

// Software-pipelined form for long FP32 tensors (compile-time lengths): a
// persistent grid walks tiles of 2 TC real fibers, t = blockIdx.x,
// blockIdx.x + gridDim.x, ...; the 16-byte loads of the next tile are held
// in registers through the current tile's FFT, as in the CPRAND-MIX passes.
// FIRST (m = 0, fibers contiguous in X): vectors run along the fiber (4
// elements of one fiber); otherwise along j (4 neighbouring fibers, which lie
// in one k because J % 4 == 0).  A tile may straddle k: offsets are per
// fiber.  Makhoul's reordering is applied on the LDS write, the post-rotation
// on the store.  Fibers past the end read fiber 0 (zero sign, or output not
// stored).
template <int L, int TC, int NT, bool FIRST>
__global__ __launch_bounds__(NT) void dct_pass_pipe(const float *X, float *Y, int64_t J, int64_t K, ModeInfo xi,
                                                    const int8_t *signs, const cx<float> *twg, const cx<float> *csg,
                                                    double *normsq_part) {
    constexpr int LDT = TC + 1;
    constexpr int FC = 2 * TC;                // real fibers per tile
    constexpr int NV = L * FC / 4;            // float4 per tile
    constexpr int PF = (NV + NT - 1) / NT;    // float4 per thread
    static_assert(!FIRST || L % 4 == 0, "vectors along the fiber");
    __shared__ cx<float> buf[L * LDT];
    __shared__ cx<float> tw[L];
    __shared__ cx<float> cs[L];
    // tile offsets (and FIRST: input offsets and sign products) in three
    // slots: the slot written for the next tile was last read two iterations
    // ago, before the previous barrier
    __shared__ int64_t cout[3][FC];
    __shared__ int64_t cin[3][FIRST ? FC : 1];
    __shared__ float csign[3][FIRST ? FC : 1];
    __shared__ float lsign[FIRST ? L : 1];
    // FIRST: every sign vector staged in LDS once (when they fit), so the
    // per-tile sign products read no global memory
    constexpr int kSignLds = 2048;
    __shared__ int8_t sgl[FIRST ? kSignLds : 1];
    const int tid = threadIdx.x;
    const int64_t ncols = J * K;
    const int64_t ntiles = ceil_div(ncols, FC);
    const bool small = ncols < (int64_t)INT32_MAX;
    int nsg = 0;
    for (int mm = 0; mm < xi.order; ++mm) nsg += (int)xi.dims[mm];
    for (int e = tid; e < L; e += NT) {
        tw[e] = twg[e];
        cs[e] = csg[e];
        if (FIRST) lsign[e] = (float)signs[e];
    }
    if (FIRST && nsg <= kSignLds)
        for (int e = tid; e < nsg; e += NT) sgl[e] = signs[e];
    const int8_t *sgp = (FIRST && nsg <= kSignLds) ? sgl : signs;
    __syncthreads();  // the staged signs are read by the first tile's offsets below
    auto tile_info = [&](int64_t t, int slot) {
        for (int c = tid; c < FC; c += NT) {
            const int64_t q = t * FC + c;
            if (q >= ncols) {
                cout[slot][c] = 0;
                if (FIRST) {
                    cin[slot][c] = 0;
                    csign[slot][c] = 0.f;
                }
                continue;
            }
            if (small) {  // 32-bit index arithmetic (the divisions sit before a barrier)
                const uint32_t j = (uint32_t)q % (uint32_t)J, k = (uint32_t)q / (uint32_t)J;
                cout[slot][c] = (int64_t)j + J * L * (int64_t)k;
            } else {
                const int64_t j = q % J, k = q / J;
                cout[slot][c] = j + J * L * k;
            }
            if (FIRST) {  // m = 0: q runs over modes 1 .. order-1
                int64_t off = 0;
                float sg = 1.f;
                int soff = (int)xi.dims[0];
                if (small) {
                    uint32_t r = (uint32_t)q;
                    for (int mm = 1; mm < xi.order; ++mm) {
                        const uint32_t d = (uint32_t)xi.dims[mm];
                        const uint32_t im = r % d;
                        r /= d;
                        off += (int64_t)im * xi.strides[mm];
                        sg *= (float)sgp[soff + (int)im];
                        soff += (int)d;
                    }
                } else {
                    int64_t r = q;
                    for (int mm = 1; mm < xi.order; ++mm) {
                        const int64_t im = r % xi.dims[mm];
                        r /= xi.dims[mm];
                        off += im * xi.strides[mm];
                        sg *= (float)sgp[soff + im];
                        soff += (int)xi.dims[mm];
                    }
                }
                cin[slot][c] = off;
                csign[slot][c] = sg;
            }
        }
    };
    float4 r[PF];
    auto issue_loads = [&](int slot) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int e = tid + u * NT;
            r[u] = float4{0.f, 0.f, 0.f, 0.f};
            if (e < NV) {
                if (FIRST) {  // along the fiber: 4 elements of fiber c, a wave reading 1 KB runs
                    const int c = e / (L / 4), l4 = (e - c * (L / 4)) * 4;
                    r[u] = *(const float4 *)(X + cin[slot][c] + l4);
                } else {      // row l: fibers c4 .. c4 + 3
                    const int l = e / (FC / 4), c4 = (e - l * (FC / 4)) * 4;
                    r[u] = *(const float4 *)(Y + cout[slot][c4] + J * (int64_t)l);
                }
            }
        }
    };
    auto perm = [](int l) { return (l & 1) ? (L - 1 - (l >> 1)) : (l >> 1); };
    int64_t t = blockIdx.x;
    if (t >= ntiles) {
        if (FIRST && normsq_part && tid == 0) normsq_part[blockIdx.x] = 0.0;
        return;
    }
    double nacc = 0.0;  // FIRST: sum of squares of the raw input (signs do not change it)
    tile_info(t, 0);
    __syncthreads();
    issue_loads(0);
    for (int it = 0; t < ntiles; ++it, t += gridDim.x) {
        const int cur = it % 3, nxt = (it + 1) % 3;
        const int nc = (int)min((int64_t)FC, ncols - t * FC);
        const int64_t tn = t + gridDim.x;
        if (tn < ntiles) tile_info(tn, nxt);
        __syncthreads();  // the previous tile's output reads are done; tile_info(tn) is visible
        // registers (tile t) -> LDS in Makhoul's order: fiber c to the real
        // (even c) or imaginary (odd c) part of column c / 2
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int e = tid + u * NT;
            if (e >= NV) continue;
            const float4 v = r[u];
            if (FIRST) {
                const int c = e / (L / 4), l4 = (e - c * (L / 4)) * 4;
                const float sc = csign[cur][c];
                // fibers past the end read fiber 0 (their sign is zero)
                if (c < nc) nacc += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
                float *bf = (float *)buf + (c & 1);
                const int cc = c >> 1;
                bf[2 * (perm(l4 + 0) * LDT + cc)] = v.x * sc * lsign[l4 + 0];
                bf[2 * (perm(l4 + 1) * LDT + cc)] = v.y * sc * lsign[l4 + 1];
                bf[2 * (perm(l4 + 2) * LDT + cc)] = v.z * sc * lsign[l4 + 2];
                bf[2 * (perm(l4 + 3) * LDT + cc)] = v.w * sc * lsign[l4 + 3];
            } else {
                const int l = e / (FC / 4), c4 = (e - l * (FC / 4)) * 4;
                const int p = perm(l);
                buf[p * LDT + (c4 >> 1)] = {v.x, v.y};
                buf[p * LDT + (c4 >> 1) + 1] = {v.z, v.w};
            }
        }
        // the next tile's loads stay in flight through this tile's FFT
        if (tn < ntiles) issue_loads(nxt);
        __syncthreads();
        fft_ct<float, L, TC, NT, -1>(buf, tw);
        __syncthreads();
        // y_c[k] = (s_k / 2)(cos(pi k / 2L) a + sin(pi k / 2L) b), (a, b) from
        // Z[k] and Z[L - k] of column c / 2 (conjugate-symmetric split)
        auto out1 = [&](int c, int k) {
            const int cc = c >> 1, mk = k == 0 ? 0 : L - k;
            const cx<float> zk = buf[k * LDT + cc], zm = buf[mk * LDT + cc];
            float a, b;
            if (c & 1) {
                a = zk.im + zm.im;
                b = zm.re - zk.re;
            } else {
                a = zk.re + zm.re;
                b = zk.im - zm.im;
            }
            const cx<float> w = cs[k];
            return 0.5f * (w.re * a + w.im * b);
        };
        if (FIRST) {
            // one k per lane: consecutive lanes read consecutive LDS rows
            // (no bank conflicts) and write consecutive words of a fiber
            for (int e = tid; e < FC * L; e += NT) {
                const int c = e / L, k = e - c * L;
                if (c < nc) Y[cout[cur][c] + k] = out1(c, k);
            }
        } else {
            for (int e = tid; e < L * (FC / 4); e += NT) {
                const int k = e / (FC / 4), c4 = (e - k * (FC / 4)) * 4;
                if (c4 >= nc) continue;
                *(float4 *)(Y + cout[cur][c4] + J * (int64_t)k) = float4{out1(c4, k), out1(c4 + 1, k),
                                                                         out1(c4 + 2, k), out1(c4 + 3, k)};
            }
        }
    }
    if (FIRST && normsq_part) {
        __shared__ double sh[NT / kWave];
        nacc = block_sum<NT>(nacc, sh);
        if (tid == 0) normsq_part[blockIdx.x] = nacc;
    }
}

// resident workgroups of a kernel on the current device (cached per call
// site by the caller)
template <typename Kern>
static unsigned resident_blocks(Kern kernel, int nt, unsigned &per_cu) {
    if (per_cu == 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, nt, 0) != hipSuccess || n < 1) n = 1;
        per_cu = (unsigned)n;
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || cus < 1)
        cus = 256;
    return per_cu * (unsigned)cus;
}

// The pipelined pass when its vector accesses are legal: FIRST needs unit
// stride along mode 0, 16-byte aligned fiber starts in X and Y and L % 4 ==
// 0; the other passes need J % 4 == 0 and Y aligned.  Returns false (nothing
// launched) otherwise.
template <int L, int TC, int NT>
static bool launch_dct_pipe(const FftPlan *fp, const void *tab, const ModeInfo &xi, const void *X, void *Y,
                            bool first, const int8_t *signs, int64_t J, int64_t K, hipStream_t st, hipError_t *err,
                            MixExtras *ex) {
    const bool ya = (((uintptr_t)Y) & 15) == 0;
    const int64_t ntiles = ceil_div(J * K, 2 * TC);
    if (first) {
        if constexpr (L % 4 == 0) {
            bool ok = J == 1 && ya && (((uintptr_t)X) & 15) == 0 && xi.strides[0] == 1;
            for (int mm = 1; mm < xi.order; ++mm) ok = ok && xi.strides[mm] % 4 == 0;
            if (!ok) return false;
            static unsigned per_cu = 0;
            const unsigned np = (unsigned)std::min<int64_t>(ntiles, resident_blocks(dct_pass_pipe<L, TC, NT, true>,
                                                                                      NT, per_cu));
            double *nsp = (ex && np <= 4096) ? ex->normsq_part : nullptr;  // partial buffer: 4096 doubles
            hipLaunchKernelGGL((dct_pass_pipe<L, TC, NT, true>), dim3(np), dim3(NT), 0, st, (const float *)X,
                               (float *)Y, J, K, xi, signs, (const cx<float> *)fp->tw, (const cx<float> *)tab, nsp);
            if (nsp) ex->nparts = (int32_t)np;
            *err = hipGetLastError();
            return true;
        }
        return false;
    }
    if (J % 4 != 0 || !ya) return false;
    static unsigned per_cu = 0;
    const unsigned np = (unsigned)std::min<int64_t>(ntiles, resident_blocks(dct_pass_pipe<L, TC, NT, false>, NT,
                                                                              per_cu));
    hipLaunchKernelGGL((dct_pass_pipe<L, TC, NT, false>), dim3(np), dim3(NT), 0, st, (const float *)nullptr,
                       (float *)Y, J, K, xi, signs, (const cx<float> *)fp->tw, (const cx<float> *)tab,
                       (double *)nullptr);
    *err = hipGetLastError();
    return true;
}

template <typename T, typename Tin, int LC, int TC, int NT>
static hipError_t launch_dct_tiles(const FftPlan *fp, const void *tab, const ModeInfo &xi, const void *X, void *Y,
                                     int m, bool first, const int8_t *signs, int64_t J, int64_t K, hipStream_t st) {
    const int64_t L = fp->L;
    const size_t lds = ((LC > 0 ? 1 : 2) * (size_t)L * (TC + 1) + 2 * (size_t)L) * sizeof(cx<T>);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const int64_t nb = ceil_div(J * K, 2 * TC);
    if (first)
        hipLaunchKernelGGL((dct_pass_kernel<T, Tin, LC, TC, NT, true>), dim3((unsigned)nb), dim3(NT), lds, st, *fp,
                           (const Tin *)X, (T *)Y, J, K, xi, m, signs, (const cx<T> *)fp->tw, (const cx<T> *)tab);
    else
        hipLaunchKernelGGL((dct_pass_kernel<T, T, LC, TC, NT, false>), dim3((unsigned)nb), dim3(NT), lds, st, *fp,
                           (const T *)nullptr, (T *)Y, J, K, xi, m, signs, (const cx<T> *)fp->tw, (const cx<T> *)tab);
    return hipGetLastError();
}

// Run-time length: the widest tile (16, 4 or 1 column pairs) whose LDS
// stays within 64 KB, or within 160 KB for one column pair.
template <typename T, typename Tin>
static hipError_t launch_dct_generic(const FftPlan *fp, const void *tab, const ModeInfo &xi, const void *X, void *Y,
                                     int m, bool first, const int8_t *signs, int64_t J, int64_t K, hipStream_t st) {
    const size_t per = 2 * (size_t)fp->L * sizeof(cx<T>);
    auto lds = [&](int tc) { return per * (tc + 1) + per; };
    if (lds(16) <= 65536)
        return launch_dct_tiles<T, Tin, 0, 16, 256>(fp, tab, xi, X, Y, m, first, signs, J, K, st);
    if (lds(4) <= 65536)
        return launch_dct_tiles<T, Tin, 0, 4, 256>(fp, tab, xi, X, Y, m, first, signs, J, K, st);
    return launch_dct_tiles<T, Tin, 0, 1, 256>(fp, tab, xi, X, Y, m, first, signs, J, K, st);
}

hipError_t launch_dct_pass(const ModeInfo &xi, const void *X, int xkind, void *Y, bool dbl, int32_t m, bool first,
                           const int8_t *signs, hipStream_t st, MixExtras *ex) {
    if (ex) ex->nparts = 0;
    if (first && m != 0) return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    const FftPlan *fp = fft_plan_get(xi.dims[m], dbl, &e);
    if (!fp) return e == hipSuccess ? hipErrorInvalidValue : e;
    const void *tab = dct_table_get(xi.dims[m], dbl, &e);
    if (!tab) return e;
    int64_t J = 1, K = 1;
    for (int i = 0; i < m; ++i) J *= xi.dims[i];
    for (int i = m + 1; i < xi.order; ++i) K *= xi.dims[i];
    if (dbl) {
        if (first && xkind != K_F64) return hipErrorInvalidValue;
        return launch_dct_generic<double, double>(fp, tab, xi, X, Y, m, first, signs, J, K, st);
    }
    if (first && xkind == K_F64) return launch_dct_generic<float, double>(fp, tab, xi, X, Y, m, first, signs, J, K, st);
    if (first && xkind != K_F32) return hipErrorInvalidValue;
    switch (fp->L) {  // compile-time schedules for the common lengths (pipelined when the layout allows)
        case 60:
            if (launch_dct_pipe<60, 16, 512>(fp, tab, xi, X, Y, first, signs, J, K, st, &e, first ? ex : nullptr)) return e;
            return launch_dct_tiles<float, float, 60, 16, 512>(fp, tab, xi, X, Y, m, first, signs, J, K, st);
        case 150:
            if (launch_dct_pipe<150, 16, 512>(fp, tab, xi, X, Y, first, signs, J, K, st, &e, first ? ex : nullptr)) return e;
            return launch_dct_tiles<float, float, 150, 16, 512>(fp, tab, xi, X, Y, m, first, signs, J, K, st);
        case 400:
            if (launch_dct_pipe<400, 16, 1024>(fp, tab, xi, X, Y, first, signs, J, K, st, &e, first ? ex : nullptr)) return e;
            return launch_dct_tiles<float, float, 400, 16, 512>(fp, tab, xi, X, Y, m, first, signs, J, K, st);
        case 1000:  // 8 column pairs: the tile and its tables take ~95 KB of LDS
            if (launch_dct_pipe<1000, 8, 512>(fp, tab, xi, X, Y, first, signs, J, K, st, &e, first ? ex : nullptr)) return e;
            return launch_dct_tiles<float, float, 1000, 8, 512>(fp, tab, xi, X, Y, m, first, signs, J, K, st);
        default: return launch_dct_generic<float, float>(fp, tab, xi, X, Y, m, first, signs, J, K, st);
    }
}

// ---------------------------------------------------------------------------
// Factor mix A-hat = C D A (inverse: A = D C^T A-hat) for one I x R row-major
// matrix, as a direct product with the DCT matrix (I^2 R multiply-adds, FP64
// sums; a one-time step per mode).  One workgroup per output row; the row's
// DCT coefficients are formed in LDS in chunks, the argument reduced exactly
// as k (2i + 1) mod 4I before cospi.
template <typename T>
__global__ __launch_bounds__(256) void factor_dct_kernel(const T *in, const int8_t *sign, T *out, int I, int R,
                                                         int inverse) {
    constexpr int kChunk = 4096;
    __shared__ double coef[kChunk];
    __shared__ double part[4][64];
    const int tid = threadIdx.x, row = blockIdx.x;
    const int r = tid & 63, g = tid >> 6;
    const double s0 = sqrt(1.0 / (double)I), s1 = sqrt(2.0 / (double)I);
    double acc = 0.0;
    for (int j0 = 0; j0 < I; j0 += kChunk) {
        const int n = min(kChunk, I - j0);
        __syncthreads();
        for (int jj = tid; jj < n; jj += 256) {
            const int j = j0 + jj;
            const int k = inverse ? j : row, i = inverse ? row : j;
            const int64_t a = ((int64_t)k * (2 * (int64_t)i + 1)) % (4 * (int64_t)I);
            double c = (k == 0 ? s0 : s1) * cospi((double)a / (2.0 * (double)I));
            if (!inverse) c *= (double)sign[i];
            coef[jj] = c;
        }
        __syncthreads();
        if (r < R)
            for (int jj = g; jj < n; jj += 4) acc += coef[jj] * (double)in[(int64_t)(j0 + jj) * R + r];
    }
    part[g][r] = acc;
    __syncthreads();
    if (tid < R) {
        double v = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
        if (inverse) v *= (double)sign[row];
        out[(int64_t)row * R + tid] = (T)v;
    }
}

hipError_t launch_factor_dct(int32_t I, int32_t R, const void *in, const int8_t *sign, void *out, bool dbl,
                             bool inverse, hipStream_t st) {
    if (R < 1 || R > 64 || I < 1) return hipErrorInvalidValue;
    if (dbl)
        hipLaunchKernelGGL(factor_dct_kernel<double>, dim3(I), dim3(256), 0, st, (const double *)in, sign,
                           (double *)out, I, R, inverse ? 1 : 0);
    else
        hipLaunchKernelGGL(factor_dct_kernel<float>, dim3(I), dim3(256), 0, st, (const float *)in, sign,
                           (float *)out, I, R, inverse ? 1 : 0);
    return hipGetLastError();
}

}  // namespace cprand
