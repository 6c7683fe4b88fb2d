// Unitary mixed-radix FFTs for the mixing of Section 2.2 / Section 3.3
// (Alg. 4): the one-time mix of the tensor along every mode, the mix and
// unmix of factor matrices, and the unmix of a mode step's sampled MTTKRP.
//
// The transform is the Stockham autosort formulation (Govindaraju et al.,
// "High performance discrete Fourier transforms on graphics processors",
// SC'08) on a tile of TC fibers held in LDS: stage s with radix r reads
// element j + t*L/r (t < r), applies the twiddle exp(+-2 pi i t k/(Ns r)),
// k = j mod Ns, does an r-point DFT and writes element (j/Ns)*Ns*r + k + t*Ns;
// two LDS buffers alternate between stages.  Radices 2, 3, 4, 5, 7.
// Twiddles exp(-2 pi i q/L) are computed on the host in FP64 and uploaded.
// Strided modes move whole rows of TC neighbouring fibers (contiguous in
// memory), so reads and writes stay coalesced without a transpose.
#include <math.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "kernels.hpp"

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
template <typename T>
__device__ inline cx<T> cmul_idir(cx<T> a, int dir) {
    return dir > 0 ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}

struct FftPlan {
    int64_t L;
    int nrad;
    int rad[24];
    void *tw;  // device, L complex (float or double): exp(-2 pi i q / L)
};

// r-point DFT in place, sign dir (-1 forward, +1 inverse).
template <typename T, int R>
__device__ inline void small_dft(cx<T> *v, int dir, const cx<T> *tw, int64_t L) {
    if (R == 2) {
        cx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if (R == 3) {
        const T h = (T)0.86602540378443864676;  // sqrt(3)/2
        cx<T> a = v[0], b = v[1], c = v[2];
        cx<T> s = cadd(b, c), d = csub(b, c);
        cx<T> m = csub(a, cscale(s, (T)0.5));
        cx<T> q = cmul_idir(cscale(d, h), dir);
        v[0] = cadd(a, s);
        v[1] = cadd(m, q);
        v[2] = csub(m, q);
    } else if (R == 4) {
        cx<T> a = v[0], b = v[1], c = v[2], d = v[3];
        cx<T> s0 = cadd(a, c), d0 = csub(a, c), s1 = cadd(b, d), d1 = cmul_idir(csub(b, d), dir);
        v[0] = cadd(s0, s1);
        v[1] = cadd(d0, d1);
        v[2] = csub(s0, s1);
        v[3] = csub(d0, d1);
    } else if (R == 5) {
        const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
        const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
        cx<T> x0 = v[0];
        cx<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
        cx<T> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
        cx<T> a1 = cadd(x0, cadd(cscale(t1, c1), cscale(t2, c2)));
        cx<T> a2 = cadd(x0, cadd(cscale(t1, c2), cscale(t2, c1)));
        cx<T> b1 = cmul_idir(cadd(cscale(t3, s1), cscale(t4, s2)), dir);
        cx<T> b2 = cmul_idir(csub(cscale(t3, s2), cscale(t4, s1)), dir);
        v[0] = cadd(x0, cadd(t1, t2));
        v[1] = cadd(a1, b1);
        v[4] = csub(a1, b1);
        v[2] = cadd(a2, b2);
        v[3] = csub(a2, b2);
    } else {
        // direct R-point DFT with the length-L table: w^(a b) = tw[(a b mod R) L/R]
        cx<T> out[R];
        const int64_t step = L / R;
        for (int a = 0; a < R; ++a) {
            cx<T> acc = v[0];
            for (int b = 1; b < R; ++b) {
                cx<T> w = tw[((a * b) % R) * step];
                if (dir > 0) w.im = -w.im;
                acc = cadd(acc, cmul(v[b], w));
            }
            out[a] = acc;
        }
        for (int a = 0; a < R; ++a) v[a] = out[a];
    }
}

// One Stockham stage over TC columns: in/out are [L][ldt] column tiles.
template <typename T, int R>
__device__ inline void stage(const cx<T> *in, cx<T> *out, int64_t L, int ldt, int tc, int64_t Ns,
                             int dir, const cx<T> *tw) {
    const int64_t nb = (L / R) * tc;
    const int64_t twstep = L / (Ns * R);
    for (int64_t id = threadIdx.x; id < nb; id += blockDim.x) {
        const int col = (int)(id % tc);
        const int64_t j = id / tc;
        const int64_t k = j % Ns;
        cx<T> v[R];
#pragma unroll
        for (int t = 0; t < R; ++t) v[t] = in[(j + t * (L / R)) * ldt + col];
#pragma unroll
        for (int t = 1; t < R; ++t) {
            cx<T> w = tw[t * k * twstep];
            if (dir > 0) w.im = -w.im;
            v[t] = cmul(v[t], w);
        }
        small_dft<T, R>(v, dir, tw, L);
        const int64_t o = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int t = 0; t < R; ++t) out[(o + t * Ns) * ldt + col] = v[t];
    }
}

// Transform the tile in buf0 (result may end in buf0 or buf1; returned).
template <typename T>
__device__ cx<T> *fft_tile(cx<T> *buf0, cx<T> *buf1, const FftPlan &fp, int ldt, int tc, int dir,
                           const cx<T> *tw) {
    cx<T> *in = buf0, *out = buf1;
    int64_t Ns = 1;
    for (int s = 0; s < fp.nrad; ++s) {
        const int r = fp.rad[s];
        switch (r) {
            case 2: stage<T, 2>(in, out, fp.L, ldt, tc, Ns, dir, tw); break;
            case 3: stage<T, 3>(in, out, fp.L, ldt, tc, Ns, dir, tw); break;
            case 4: stage<T, 4>(in, out, fp.L, ldt, tc, Ns, dir, tw); break;
            case 5: stage<T, 5>(in, out, fp.L, ldt, tc, Ns, dir, tw); break;
            default: stage<T, 7>(in, out, fp.L, ldt, tc, Ns, dir, tw); break;
        }
        __syncthreads();
        Ns *= r;
        cx<T> *tmp = in;
        in = out;
        out = tmp;
    }
    return in;
}

// Columns per tile: two LDS buffers of L x (tc+1) complex within ~64 KB.
static int tile_cols(int64_t L, int esz) {
    int64_t tc = (int64_t)(65536 / (2 * esz)) / L - 1;
    if (tc > 16) tc = 16;
    if (tc < 1) tc = 1;
    return (int)tc;
}

// ---------------------------------------------------------------------------
// Tensor pass along mode m (J = prod of dims before m, K = after; column q
// of the flattened (j, k) range is fiber (j, k), element l at
// j + J*(l + L*k)).
template <typename T, typename Tin>
__global__ __launch_bounds__(256) void mix_pass_kernel(FftPlan fp, const Tin *X, cx<T> *Xh, int64_t J,
                                                       int64_t K, int tc, int first, ModeInfo xi,
                                                       int m, const int8_t *signs,
                                                       double *normsq_part) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int64_t L = fp.L;
    const int ldt = tc + 1;
    cx<T> *b0 = (cx<T> *)lds, *b1 = b0 + L * ldt;
    const cx<T> *tw = (const cx<T> *)fp.tw;
    __shared__ double sh[256 / kWave];
    __shared__ double s_colsign[16];
    const int64_t ncols = J * K;
    const int64_t q0 = (int64_t)blockIdx.x * tc;
    const int nc = (int)min((int64_t)tc, ncols - q0);

    // sign product of every mode except m for each column (first pass);
    // signs are stored mode after mode
    if (first) {
        for (int c = threadIdx.x; c < nc; c += blockDim.x) {
            int64_t j = (q0 + c) % J, k = (q0 + c) / J;
            double sg = 1.0;
            int64_t off = 0;
            for (int mm = 0; mm < xi.order; ++mm) {
                if (mm != m) {
                    int64_t im;
                    if (mm < m) {
                        im = j % xi.dims[mm];
                        j /= xi.dims[mm];
                    } else {
                        im = k % xi.dims[mm];
                        k /= xi.dims[mm];
                    }
                    sg *= (double)signs[off + im];
                }
                off += xi.dims[mm];
            }
            s_colsign[c] = sg;
        }
    }
    int64_t moff = 0;
    for (int mm = 0; mm < m; ++mm) moff += xi.dims[mm];
    __syncthreads();
    double acc = 0.0;
    // load
    for (int64_t e = threadIdx.x; e < L * tc; e += blockDim.x) {
        int64_t l, c;
        if (J == 1) {
            c = e / L;
            l = e - c * L;
        } else {
            l = e / tc;
            c = e - l * tc;
        }
        cx<T> v = {(T)0, (T)0};
        if (c < nc) {
            const int64_t q = q0 + c;
            const int64_t j = q % J, k = q / J;
            const int64_t o = j + J * (l + L * k);
            if (first) {
                const double x = (double)X[o];
                acc += x * x;
                v.re = (T)(x * s_colsign[c] * (double)signs[moff + l]);
            } else {
                v = Xh[o];
            }
        }
        b0[l * ldt + c] = v;
    }
    if (first && normsq_part) {
        const double s = block_sum<256>(acc, sh);
        if (threadIdx.x == 0) normsq_part[blockIdx.x] = s;
    }
    __syncthreads();
    cx<T> *res = fft_tile<T>(b0, b1, fp, ldt, tc, -1, tw);
    const T scale = (T)(1.0 / sqrt((double)L));
    for (int64_t e = threadIdx.x; e < L * tc; e += blockDim.x) {
        int64_t l, c;
        if (J == 1) {
            c = e / L;
            l = e - c * L;
        } else {
            l = e / tc;
            c = e - l * tc;
        }
        if (c < nc) {
            const int64_t q = q0 + c;
            const int64_t j = q % J, k = q / J;
            Xh[j + J * (l + L * k)] = cscale(res[l * ldt + c], scale);
        }
    }
}


// ---------------------------------------------------------------------------
// Factor mix (A-hat = F D A), inverse factor mix (A = Re(D F^* A-hat)) and
// the unmix of a mode step (W = D Re(F^* Y)).  Columns of an I x R
// row-major matrix are the transformed fibers.
template <typename T>
__global__ __launch_bounds__(256) void factor_mix_kernel(FftPlan fp, const T *in, const int8_t *sign,
                                                         T *out, int R, int tc, int inverse) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int64_t L = fp.L;
    const int ldt = tc + 1;
    cx<T> *b0 = (cx<T> *)lds, *b1 = b0 + L * ldt;
    const int r0 = blockIdx.x * tc;
    const int nc = min(tc, R - r0);
    for (int64_t e = threadIdx.x; e < L * tc; e += blockDim.x) {
        const int64_t l = e / tc;
        const int c = (int)(e - l * tc);
        cx<T> v = {(T)0, (T)0};
        if (c < nc) {
            const int64_t o = l * R + r0 + c;
            if (!inverse)
                v.re = (T)sign[l] * in[o];
            else
                v = {in[2 * o], in[2 * o + 1]};
        }
        b0[l * ldt + c] = v;
    }
    __syncthreads();
    cx<T> *res = fft_tile<T>(b0, b1, fp, ldt, tc, inverse ? 1 : -1, (const cx<T> *)fp.tw);
    const T scale = (T)(1.0 / sqrt((double)L));
    for (int64_t e = threadIdx.x; e < L * tc; e += blockDim.x) {
        const int64_t l = e / tc;
        const int c = (int)(e - l * tc);
        if (c >= nc) continue;
        const int64_t o = l * R + r0 + c;
        const cx<T> v = res[l * ldt + c];
        if (!inverse) {
            out[2 * o] = v.re * scale;
            out[2 * o + 1] = v.im * scale;
        } else {
            out[o] = (T)sign[l] * v.re * scale;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void unmix_kernel(FftPlan fp, const T *ypart, int chunks, int R,
                                                    const int8_t *sign, T *W, int rowmajor, int tc) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int64_t L = fp.L;
    const int ldt = tc + 1;
    cx<T> *b0 = (cx<T> *)lds, *b1 = b0 + L * ldt;
    const int r0 = blockIdx.x * tc;
    const int nc = min(tc, R - r0);
    const size_t cstride = (size_t)2 * R * L;
    for (int64_t e = threadIdx.x; e < L * tc; e += blockDim.x) {
        const int c = (int)(e / L);
        const int64_t l = e - (int64_t)c * L;
        double re = 0.0, im = 0.0;
        if (c < nc) {
            const int r = r0 + c;
            for (int p = 0; p < chunks; ++p) {
                re += (double)ypart[p * cstride + (size_t)r * L + l];
                im += (double)ypart[p * cstride + (size_t)(R + r) * L + l];
            }
        }
        b0[l * ldt + c] = {(T)re, (T)im};
    }
    __syncthreads();
    cx<T> *res = fft_tile<T>(b0, b1, fp, ldt, tc, 1, (const cx<T> *)fp.tw);
    const T scale = (T)(1.0 / sqrt((double)L));
    for (int64_t e = threadIdx.x; e < L * tc; e += blockDim.x) {
        const int64_t l = e / tc;
        const int c = (int)(e - l * tc);
        if (c >= nc) continue;
        const int r = r0 + c;
        const T v = (T)sign[l] * res[l * ldt + c].re * scale;
        if (rowmajor)
            W[l * R + r] = v;
        else
            W[(int64_t)r * L + l] = v;
    }
}

__global__ void signs_kernel(ModeInfo mi, uint64_t seed, int8_t *signs, int64_t total) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    int64_t i = e;
    int m = 0;
    while (i >= mi.dims[m]) {
        i -= mi.dims[m];
        ++m;
    }
    const u64x4 w = philox4x64_10((uint64_t)i, (uint64_t)m, 0, 0, seed, kTagSigns);
    signs[e] = (w.v[0] >> 63) ? (int8_t)-1 : (int8_t)1;
}

// ---------------------------------------------------------------------------
FftPlan *fft_plan_get(int64_t L, bool dbl, hipError_t *err) {
    static std::mutex mu;
    static std::map<std::tuple<int, int64_t, int>, FftPlan *> cache;
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
    FftPlan p{};
    p.L = L;
    int64_t rem = L;
    while (rem % 4 == 0 && p.nrad < 24) { p.rad[p.nrad++] = 4; rem /= 4; }
    const int primes[4] = {2, 3, 5, 7};
    for (int pi = 0; pi < 4; ++pi)
        while (rem % primes[pi] == 0 && p.nrad < 24) { p.rad[p.nrad++] = primes[pi]; rem /= primes[pi]; }
    if (rem != 1) {
        *err = hipErrorInvalidValue;
        return nullptr;
    }
    const size_t esz = dbl ? 16 : 8;
    std::vector<unsigned char> host(esz * L);
    for (int64_t q = 0; q < L; ++q) {
        const double ang = -2.0 * M_PI * (double)q / (double)L;
        const double c = cos(ang), s = sin(ang);
        if (dbl) {
            ((double *)host.data())[2 * q] = c;
            ((double *)host.data())[2 * q + 1] = s;
        } else {
            ((float *)host.data())[2 * q] = (float)c;
            ((float *)host.data())[2 * q + 1] = (float)s;
        }
    }
    e = hipMalloc(&p.tw, esz * L);
    if (e == hipSuccess) e = hipMemcpy(p.tw, host.data(), esz * L, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        *err = e;
        return nullptr;
    }
    FftPlan *heap = new FftPlan(p);
    cache[key] = heap;
    return heap;
}

static size_t tile_lds(int64_t L, int tc, size_t esz) { return 2 * (size_t)L * (tc + 1) * esz; }

hipError_t launch_mix_pass(const FftPlan *fp, bool dbl, const ModeInfo &xi, const void *X, int xkind,
                           void *Xhat, int32_t m, bool first, const int8_t *signs,
                           double *normsq_part, int32_t *nparts, hipStream_t st) {
    int64_t J = 1, K = 1;
    for (int i = 0; i < m; ++i) J *= xi.dims[i];
    for (int i = m + 1; i < xi.order; ++i) K *= xi.dims[i];
    const size_t esz = dbl ? 16 : 8;
    const int tc = tile_cols(fp->L, (int)esz);
    const int64_t nb = ceil_div(J * K, tc);
    if (nparts) *nparts = (int32_t)nb;
    const size_t lds = tile_lds(fp->L, tc, esz);
    if (dbl) {
        hipLaunchKernelGGL((mix_pass_kernel<double, double>), dim3((unsigned)nb), dim3(256), lds, st, *fp,
                           (const double *)X, (cx<double> *)Xhat, J, K, tc, first ? 1 : 0, xi, m, signs,
                           normsq_part);
    } else {
        if (first && xkind == K_F64)
            hipLaunchKernelGGL((mix_pass_kernel<float, double>), dim3((unsigned)nb), dim3(256), lds, st, *fp,
                               (const double *)X, (cx<float> *)Xhat, J, K, tc, 1, xi, m, signs, normsq_part);
        else
            hipLaunchKernelGGL((mix_pass_kernel<float, float>), dim3((unsigned)nb), dim3(256), lds, st, *fp,
                               (const float *)X, (cx<float> *)Xhat, J, K, tc, first ? 1 : 0, xi, m, signs,
                               normsq_part);
    }
    return hipGetLastError();
}

hipError_t launch_factor_mix(const FftPlan *fp, bool dbl, int32_t I, int32_t R, const void *in,
                             const int8_t *sign, void *out, bool inverse, hipStream_t st) {
    const size_t esz = dbl ? 16 : 8;
    const int tc = std::min(tile_cols(fp->L, (int)esz), (int)R);
    const int nb = (int)ceil_div(R, tc);
    const size_t lds = tile_lds(fp->L, tc, esz);
    if (dbl)
        hipLaunchKernelGGL(factor_mix_kernel<double>, dim3(nb), dim3(256), lds, st, *fp, (const double *)in,
                           sign, (double *)out, R, tc, inverse ? 1 : 0);
    else
        hipLaunchKernelGGL(factor_mix_kernel<float>, dim3(nb), dim3(256), lds, st, *fp, (const float *)in,
                           sign, (float *)out, R, tc, inverse ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_unmix(const FftPlan *fp, bool dbl, int32_t In, int32_t R, int32_t chunks,
                        const void *ypart, const int8_t *sign, void *W, bool w_rowmajor,
                        hipStream_t st) {
    const size_t esz = dbl ? 16 : 8;
    const int tc = std::min(tile_cols(fp->L, (int)esz), (int)R);
    const int nb = (int)ceil_div(R, tc);
    const size_t lds = tile_lds(fp->L, tc, esz);
    if (dbl)
        hipLaunchKernelGGL(unmix_kernel<double>, dim3(nb), dim3(256), lds, st, *fp, (const double *)ypart,
                           chunks, R, sign, (double *)W, w_rowmajor ? 1 : 0, tc);
    else
        hipLaunchKernelGGL(unmix_kernel<float>, dim3(nb), dim3(256), lds, st, *fp, (const float *)ypart,
                           chunks, R, sign, (float *)W, w_rowmajor ? 1 : 0, tc);
    return hipGetLastError();
}

hipError_t launch_signs(const ModeInfo &mi, uint64_t seed, int8_t *signs, hipStream_t st) {
    int64_t total = 0;
    for (int m = 0; m < mi.order; ++m) total += mi.dims[m];
    hipLaunchKernelGGL(signs_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, mi, seed, signs,
                       total);
    return hipGetLastError();
}

}  // namespace cprand
