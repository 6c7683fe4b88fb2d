// Everything after the gather of one mode step, in one workgroup, when the
// mode's I_n x R blocks fit in LDS: sum the MTTKRP and Gram partials, invert V
// (FP64), solve A = W V^{-1} (Alg. 3), optionally refine once against FP32
// data, and normalise the columns into lambda.  Replaces five launches per mode
// step at the sizes where the step is latency-bound.
//
// Under mixing the step stays in the mixed domain and needs no FFT.  With Y
// the I_n x R product of the mixed fibers and the conjugated mixed KRP rows,
// the real-constrained solution is A = Re(D_n F_n^* Y) V^{-1} (Alg. 4 unmix,
// eq. rcLS), and its remix A-hat = F_n D_n A (Alg. 4) equals
// (Z + P conj(Z)) / 2 with Z = Y V^{-1} and P the index reversal
// k -> (I_n - k) mod I_n: F_n D_n conj(D_n F_n^* Z) = F_n^2 conj(Z) because
// D_n is a real +-1 diagonal and the unitary DFT is symmetric, and F_n^2 = P.
// The column norms of A equal those of A-hat (unitary mixing), so lambda and
// the normalised A-hat come straight from Z.  The real factor is not formed
// here; the caller unmixes A-hat once when it needs A.
#include "kernels.hpp"
#include "solve_device.hpp"

namespace cprand {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kStepThreads = 512;
constexpr int kColParts = 16;
template <typename T>
struct Pair;
template <>
struct Pair<float> {
    typedef float2 type;
};
template <>
struct Pair<double> {
    typedef double2 type;
};
constexpr int kMixGroups = 3; // mixed products: (column, VL rows) groups per thread per pass, loads in flight together
static_assert(kColParts * kMaxRank >= kStepThreads, "tmp holds one double per thread");

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    typedef float4 type;
};
template <>
struct Vec16<double> {
    typedef double2 type;
};
__device__ inline float vget(const float4 &v, int u) { return u == 0 ? v.x : u == 1 ? v.y : u == 2 ? v.z : v.w; }
__device__ inline double vget(const double2 &v, int u) { return u == 0 ? v.x : v.y; }

// MIX: the mixed-domain step, a compile-time parameter so that each
// instance holds only its own path (the kernel runs as one workgroup on one
// CU, so its code is fetched cold at every launch: less of it is faster)
template <typename T, bool MIX>
__global__ __launch_bounds__(kStepThreads) void step_finish_kernel(StepArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int In = a.In, R = a.R, ld = R + 1;
    const int tid = threadIdx.x;
    double *B1 = (double *)lds;
    double *B2 = B1 + R * ld;
    double *B3 = B2 + R * ld;
    double *cs = B3 + R * ld;            // 66
    double *tmp = cs + 66;               // kColParts * kMaxRank (>= one per thread)
    int *pairs = (int *)(tmp + kColParts * kMaxRank);  // 66
    double *Wd = (double *)(pairs + 68); // In x R: W (MIX: Re Y)
    double *Ad = Wd + (size_t)In * R;    // In x R: A (MIX: Re A-hat)
    double *Wi = Ad + (size_t)In * R;    // MIX: Im Y
    double *Ai = Wi + (size_t)In * R;    // MIX: Im A-hat

    // Partial products (at most kMaxParts) are added in partial order.  Gram
    // element tid is loaded here and summed after the product loads below
    // have been issued, so both are in flight together.
    auto gram_sum = [&](int p, const double (&v)[kMaxParts]) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < kMaxParts; ++c)
            if (c < a.vparts) acc += v[c];
        const int i = p / R, j = p - i * R;
        B1[i * ld + j] = acc;
        B3[i * ld + j] = acc;
    };
    // R <= 16: wave 0 loads and sums V in the register layout of the one-wave
    // Gauss-Jordan inverse (below) and inverts it while the other waves load
    // and sum the product partials; larger R: Gram element tid is loaded here
    // and summed after the product loads have been issued.
    const bool wave_inv = R <= 16;
    __shared__ int s_failed;
    double vv[kMaxParts];
    if (!wave_inv) {
#pragma unroll
        for (int c = 0; c < kMaxParts; ++c)
            vv[c] = (tid < R * R && c < a.vparts) ? a.vpart[(size_t)c * R * R + tid] : 0.0;
    }
    // R <= 16: wave 0 sums the Gram partials into the register layout of the
    // one-wave inverse, and the inverse runs while the other waves load the
    // products.  Real factors: the product loads wait for the Gram sums (a
    // barrier), so that the few Gram loads do not queue behind them (measured
    // faster); the mixed path, with twice the product loads, starts them at
    // once (measured faster there).
    double vw[4] = {0.0, 0.0, 0.0, 0.0};
    if (wave_inv) {
        if (tid < kWave) {
            const int j = tid & 15, i0 = tid >> 4;
            double vq[4][kMaxParts];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = i0 + 4 * q;
                const int e = (i < R && j < R) ? i * R + j : 0;
#pragma unroll
                for (int c = 0; c < kMaxParts; ++c) {
                    const int cc = c < a.vparts ? c : 0;
                    vq[q][c] = a.vpart[(size_t)cc * R * R + e];
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = i0 + 4 * q;
                double acc = 0.0;
#pragma unroll
                for (int c = 0; c < kMaxParts; ++c)
                    if (c < a.vparts) acc += vq[q][c];
                vw[q] = (i < R && j < R) ? acc : 0.0;
            }
        }
        if (!MIX) __syncthreads();
    }
    // The product partials: all threads, or (R <= 16) waves 1.. while wave 0
    // inverts V.
    const int yt = wave_inv ? tid - kWave : tid, ys = wave_inv ? kStepThreads - kWave : kStepThreads;
    if (yt >= 0) {
        constexpr int VL = 16 / sizeof(T);  // values per 16-byte load
        typedef typename Vec16<T>::type V16;
        if (!MIX && a.wsi == 1 && In % VL == 0 && a.wsr % VL == 0 && a.wps % VL == 0) {
            // (i .. i+VL-1, r) of every partial in one 16-byte load each
            const T *w = (const T *)a.W;
            const int ng = R * (In / VL);
            for (int g = yt; g < ng; g += ys) {
                const int r = g / (In / VL), i0 = (g - r * (In / VL)) * VL;
                V16 v[kMaxParts];
    #pragma unroll
                for (int p = 0; p < kMaxParts; ++p)
                    v[p] = p < a.wparts ? *(const V16 *)(w + (int64_t)p * a.wps + (int64_t)r * a.wsr + i0) : V16{};
    #pragma unroll
                for (int u = 0; u < VL; ++u) {
                    double acc = 0.0;
    #pragma unroll
                    for (int p = 0; p < kMaxParts; ++p)
                        if (p < a.wparts) acc += (double)vget(v[p], u);
                    Wd[(i0 + u) * R + r] = acc;
                }
            }
        } else if (MIX && In % VL == 0) {
            // real and imaginary rows of column c, VL consecutive l per load; two
            // groups per thread per pass, all their loads in flight together
            const T *y = (const T *)a.W;
            const size_t cstride = (size_t)2 * R * In;
            const int ng = R * (In / VL);
            for (int g0 = yt; g0 < ng; g0 += kMixGroups * ys) {
                V16 vr[kMixGroups][kMaxParts], vi[kMixGroups][kMaxParts];
    #pragma unroll
                for (int h = 0; h < kMixGroups; ++h) {
                    const int g = g0 + h * ys;
                    const int c = g / (In / VL), l0 = (g - c * (In / VL)) * VL;
    #pragma unroll
                    for (int p = 0; p < kMaxParts; ++p) {
                        const bool ok = g < ng && p < a.wparts;
                        vr[h][p] = ok ? *(const V16 *)(y + p * cstride + (size_t)c * In + l0) : V16{};
                        vi[h][p] = ok ? *(const V16 *)(y + p * cstride + (size_t)(R + c) * In + l0) : V16{};
                    }
                }
    #pragma unroll
                for (int h = 0; h < kMixGroups; ++h) {
                    const int g = g0 + h * ys;
                    if (g >= ng) continue;
                    const int c = g / (In / VL), l0 = (g - c * (In / VL)) * VL;
    #pragma unroll
                    for (int u = 0; u < VL; ++u) {
                        double re = 0.0, im = 0.0;
    #pragma unroll
                        for (int p = 0; p < kMaxParts; ++p)
                            if (p < a.wparts) {
                                re += (double)vget(vr[h][p], u);
                                im += (double)vget(vi[h][p], u);
                            }
                        Wd[(l0 + u) * R + c] = re;
                        Wi[(l0 + u) * R + c] = im;
                    }
                }
            }
        } else if (!MIX) {
            const T *w = (const T *)a.W;
            for (int e0 = yt; e0 < In * R; e0 += 2 * ys) {
                T v[2][kMaxParts];
    #pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int e = e0 + h * ys;
                    const int i = e / R, r = e - i * R;
    #pragma unroll
                    for (int p = 0; p < kMaxParts; ++p)
                        v[h][p] = (e < In * R && p < a.wparts) ? w[(int64_t)p * a.wps + (int64_t)i * a.wsi + (int64_t)r * a.wsr]
                                                              : (T)0;
                }
    #pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int e = e0 + h * ys;
                    double acc = 0.0;
    #pragma unroll
                    for (int p = 0; p < kMaxParts; ++p)
                        if (p < a.wparts) acc += (double)v[h][p];
                    if (e < In * R) Wd[e] = acc;
                }
            }
        } else {
            const T *y = (const T *)a.W;
            const size_t cstride = (size_t)2 * R * In;
            for (int e0 = yt; e0 < In * R; e0 += 2 * ys) {
                T vr[2][kMaxParts], vi[2][kMaxParts];
    #pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int e = e0 + h * ys;
                    const int c = e / In, l = e - c * In;
                    const bool ok = e < In * R;
    #pragma unroll
                    for (int p = 0; p < kMaxParts; ++p) {
                        vr[h][p] = (ok && p < a.wparts) ? y[p * cstride + (size_t)c * In + l] : (T)0;
                        vi[h][p] = (ok && p < a.wparts) ? y[p * cstride + (size_t)(R + c) * In + l] : (T)0;
                    }
                }
    #pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int e = e0 + h * ys;
                    const int c = e / In, l = e - c * In;
                    double re = 0.0, im = 0.0;
    #pragma unroll
                    for (int p = 0; p < kMaxParts; ++p)
                        if (p < a.wparts) {
                            re += (double)vr[h][p];
                            im += (double)vi[h][p];
                        }
                    if (e < In * R) {
                        Wd[l * R + c] = re;
                        Wi[l * R + c] = im;
                    }
                }
            }
        }
    }
    int failed;
    if (wave_inv) {
        if (tid < kWave) {  // the whole of wave 0
            const int f = gj_wave_from_regs(vw, B1, B3, R, ld);
            if (tid == 0) s_failed = f;
        }
        __syncthreads();
        failed = s_failed;
        if (failed) spd_pinv(B1, B2, B3, tmp, R, ld, cs, pairs);
    } else {
        if (tid < R * R) gram_sum(tid, vv);
        for (int p = tid + kStepThreads; p < R * R; p += kStepThreads) {
            double v[kMaxParts];
#pragma unroll
            for (int c = 0; c < kMaxParts; ++c) v[c] = c < a.vparts ? a.vpart[(size_t)c * R * R + p] : 0.0;
            gram_sum(p, v);
        }
        __syncthreads();
        failed = spd_inverse(B1, B2, B3, tmp, R, ld, cs, pairs);
    }
    if (tid == 0 && a.info && failed) *a.info = CPRAND_W_PINV;
    if (MIX) {
        // A-hat (unnormalised) = Y_s V^{-1} with Y_s = (Y + P conj Y) / 2:
        // rows k and I_n - k of Y_s are conjugates (rows 0 and I_n / 2 pair
        // with themselves), so one thread takes the pair, reads both rows of
        // Y and writes both rows of A-hat.  Thread t keeps rank r = t mod R
        // and rows t / R, t / R + kstride, ..., and sums |A-hat|^2 of its
        // rows; the column norms are then closed in a fixed order.
        const int half = In / 2 + 1;
        if (R <= 16) {
            // FP64 MFMA 16x16x4 over tiles of 16 row pairs: lane (li, lk)
            // feeds A(row li, k lk) = Y_s(tile row li, 4c + lk) and
            // B(k lk, col li) = V^{-1}(4c + lk, li), and holds output rows
            // lk + 4v, column li; per-wave column sums of |A-hat|^2
            const int wv = tid / kWave, l = tid & (kWave - 1), li = l & 15, lk = l >> 4;
            constexpr int nw = kStepThreads / kWave;
            double bo[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int jj = 4 * c + lk;
                bo[c] = (jj < R && li < R) ? B1[jj * ld + li] : 0.0;
            }
            double nsq = 0.0;
            const int ntile = (half + 15) / 16;
            for (int tile = wv; tile < ntile; tile += nw) {  // uniform per wave
                const int k = tile * 16 + li;
                const bool kin = k < half;
                const int kk = (k == 0 || !kin) ? 0 : In - k;
                v4d dre = {0.0, 0.0, 0.0, 0.0}, dim = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int jj = 4 * c + lk;
                    double are = 0.0, aim = 0.0;
                    if (kin && jj < R) {
                        are = 0.5 * (Wd[k * R + jj] + Wd[kk * R + jj]);
                        aim = 0.5 * (Wi[k * R + jj] - Wi[kk * R + jj]);
                    }
                    dre = __builtin_amdgcn_mfma_f64_16x16x4f64(are, bo[c], dre, 0, 0, 0);
                    dim = __builtin_amdgcn_mfma_f64_16x16x4f64(aim, bo[c], dim, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int ko = tile * 16 + lk + 4 * v;
                    if (ko < half && li < R) {
                        const int kko = ko == 0 ? 0 : In - ko;
                        const double sr = dre[v], si = dim[v];
                        Ad[ko * R + li] = sr;
                        Ai[ko * R + li] = si;
                        const double q2 = sr * sr + si * si;
                        nsq += q2;
                        if (kko != ko) {
                            Ad[kko * R + li] = sr;
                            Ai[kko * R + li] = -si;
                            nsq += q2;
                        }
                    }
                }
            }
            nsq += __shfl_xor(nsq, 16, kWave);
            nsq += __shfl_xor(nsq, 32, kWave);
            if (lk == 0) tmp[wv * 16 + li] = nsq;
            __syncthreads();
            if (tid < R) {
                double s = 0.0;
                for (int w = 0; w < nw; ++w) s += tmp[w * 16 + tid];
                const double l = sqrt(s);
                B2[tid] = l;
                B2[R + tid] = l > 0.0 ? 1.0 / l : 1.0;  // B2 holds R (R + 1) >= 2 R doubles
                a.lambda[tid] = l;
                if (a.snap_lambda) a.snap_lambda[tid] = l;
            }
            __syncthreads();
        } else {
            const int kstride = kStepThreads / R;
            double nsq = 0.0;
            if (tid < kstride * R) {
                const int r = tid % R;
                for (int k = tid / R; k < half; k += kstride) {
                    const int kk = k == 0 ? 0 : In - k;
                    double sr = 0.0, si = 0.0;
                    for (int j = 0; j < R; ++j) {
                        const double h = B1[j * ld + r];
                        sr += (Wd[k * R + j] + Wd[kk * R + j]) * h;
                        si += (Wi[k * R + j] - Wi[kk * R + j]) * h;
                    }
                    sr *= 0.5;
                    si *= 0.5;
                    Ad[k * R + r] = sr;
                    Ai[k * R + r] = si;
                    const double q2 = sr * sr + si * si;
                    nsq += q2;
                    if (kk != k) {
                        Ad[kk * R + r] = sr;
                        Ai[kk * R + r] = -si;
                        nsq += q2;
                    }
                }
            }
            tmp[tid] = nsq;
            __syncthreads();
            if (tid < R) {
                double s = 0.0;
                for (int k0 = 0; k0 < kstride; ++k0) s += tmp[k0 * R + tid];
                const double l = sqrt(s);
                B2[tid] = l;
                B2[R + tid] = l > 0.0 ? 1.0 / l : 1.0;  // B2 holds R (R + 1) >= 2 R doubles
                a.lambda[tid] = l;
                if (a.snap_lambda) a.snap_lambda[tid] = l;
            }
            __syncthreads();
        }
        typedef typename Pair<T>::type P2;  // one complex entry per store
        P2 *Ah = (P2 *)a.Ahat;
        P2 *Sn = (P2 *)a.snapA;
        for (int e = tid; e < In * R; e += kStepThreads) {
            const double q = B2[R + e % R];
            P2 z;
            z.x = (T)(Ad[e] * q);
            z.y = (T)(Ai[e] * q);
            Ah[e] = z;
            if (Sn) Sn[e] = z;
        }
        return;
    }
    if (R <= 16) {
        // A = W V^{-1} on FP64 MFMA 16x16x4 (as for the mixed solve), tiles
        // of 16 rows dealt to the waves: lane (li, lk) feeds A(row li, k lk)
        // = W(tile row li, 4c + lk) and B(k lk, col li) = V^{-1}(4c + lk, li)
        // and holds rows lk + 4v of column li
        const int wv = tid / kWave, l = tid & (kWave - 1), li = l & 15, lk = l >> 4;
        constexpr int nw = kStepThreads / kWave;
        double bo[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int jj = 4 * c + lk;
            bo[c] = (jj < R && li < R) ? B1[jj * ld + li] : 0.0;
        }
        const int ntile = (In + 15) / 16;
        for (int tile = wv; tile < ntile; tile += nw) {  // uniform per wave
            const int i = tile * 16 + li;
            v4d d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int jj = 4 * c + lk;
                const double av = (i < In && jj < R) ? Wd[i * R + jj] : 0.0;
                d = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bo[c], d, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int io = tile * 16 + lk + 4 * v;
                if (io < In && li < R) Ad[io * R + li] = d[v];
            }
        }
    } else {
        for (int e = tid; e < In * R; e += kStepThreads) {
            const int i = e / R, r = e - i * R;
            double s = 0.0;
            for (int k = 0; k < R; ++k) s += Wd[i * R + k] * B1[k * ld + r];
            Ad[e] = s;
        }
    }
    __syncthreads();
    if (a.Wref) {
        // B3 <- V_ref, the Gram of the FP32 rows: the residual is that of the
        // FP32 normal equations, the correction uses the inverse above
        for (int p = tid; p < R * R; p += kStepThreads) {
            double acc = 0.0;
            for (int c = 0; c < a.vrefparts; ++c) acc += a.vref[(size_t)c * R * R + p];
            B3[(p / R) * ld + p % R] = acc;
        }
        __syncthreads();
        for (int e = tid; e < In * R; e += kStepThreads) {
            const int i = e / R, r = e - i * R;
            float v[kMaxParts];
#pragma unroll
            for (int p = 0; p < kMaxParts; ++p)
                v[p] = p < a.wrefparts ? a.Wref[(int64_t)p * a.rps + (int64_t)i * a.rsi + (int64_t)r * a.rsr] : 0.f;
            double s = 0.0;
#pragma unroll
            for (int p = 0; p < kMaxParts; ++p)
                if (p < a.wrefparts) s += (double)v[p];
            for (int k = 0; k < R; ++k) s -= Ad[i * R + k] * B3[k * ld + r];
            Wd[e] = s;
        }
        __syncthreads();
        for (int e = tid; e < In * R; e += kStepThreads) {
            const int i = e / R, r = e - i * R;
            double s = 0.0;
            for (int k = 0; k < R; ++k) s += Wd[i * R + k] * B1[k * ld + r];
            Ad[e] += s;
        }
        __syncthreads();
    }
    // column norms of the stored (T-rounded) values, fixed-order partial sums
    for (int e = tid; e < kColParts * R; e += kStepThreads) {
        const int r = e / kColParts, part = e - r * kColParts;
        double s = 0.0;
        for (int i = part; i < In; i += kColParts) {
            const double v = (double)(T)Ad[i * R + r];
            s += v * v;
        }
        tmp[r * kColParts + part] = s;
    }
    __syncthreads();
    if (tid < R) {
        double s = 0.0;
        for (int part = 0; part < kColParts; ++part) s += tmp[tid * kColParts + part];
        const double l = sqrt(s);
        B2[tid] = l;  // B2 is free after the inversion
        B2[R + tid] = l > 0.0 ? 1.0 / l : 1.0;
        a.lambda[tid] = l;
        if (a.snap_lambda) a.snap_lambda[tid] = l;
    }
    __syncthreads();
    T *A = (T *)a.A;
    for (int e = tid; e < In * R; e += kStepThreads) {
        const T nv = (T)((double)(T)Ad[e] * B2[R + e % R]);
        A[e] = nv;
        if (a.snapA) ((T *)a.snapA)[e] = nv;
    }
}

size_t step_finish_lds(int32_t In, int32_t R, bool mix) {
    const size_t ld = (size_t)R + 1;
    size_t b = sizeof(double) * (3 * (size_t)R * ld + 66 + (size_t)kColParts * kMaxRank) + sizeof(int) * 68;
    b += sizeof(double) * (mix ? 4 : 2) * (size_t)In * R;
    return b;
}

hipError_t launch_step_finish(const StepArgs &a, bool dbl, hipStream_t st) {
    if (a.vparts > kMaxParts || a.wparts > kMaxParts || (a.Wref && a.wrefparts > kMaxParts)) return hipErrorInvalidValue;
    if (a.Wref && (!a.vref || a.vrefparts < 1)) return hipErrorInvalidValue;
    if (a.mix && !a.Ahat) return hipErrorInvalidValue;
    const size_t lds = step_finish_lds(a.In, a.R, a.mix);
    if (dbl && a.mix)
        hipLaunchKernelGGL((step_finish_kernel<double, true>), dim3(1), dim3(kStepThreads), lds, st, a);
    else if (dbl)
        hipLaunchKernelGGL((step_finish_kernel<double, false>), dim3(1), dim3(kStepThreads), lds, st, a);
    else if (a.mix)
        hipLaunchKernelGGL((step_finish_kernel<float, true>), dim3(1), dim3(kStepThreads), lds, st, a);
    else
        hipLaunchKernelGGL((step_finish_kernel<float, false>), dim3(1), dim3(kStepThreads), lds, st, a);
    return hipGetLastError();
}

}  // namespace cprand
