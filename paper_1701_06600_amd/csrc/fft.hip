// Unitary mixed-radix FFTs for the mixing of Section 2.2 / Section 3.3
// (Alg. 4): the one-time mix of the tensor along every mode, the mix and
// unmix of factor matrices, and the unmix of a mode step's sampled MTTKRP.
//
// The transform is the Stockham autosort formulation (Govindaraju et al.,
// "High performance discrete Fourier transforms on graphics processors",
// SC'08) applied to a tile of TC fibers held in LDS as [L][TC+1] complex:
// stage s with radix r takes elements j + t*L/r (t < r), multiplies by the
// twiddle exp(+-2 pi i t k/(Ns r)) with k = j mod Ns, does an r-point DFT and
// stores element (j/Ns)*Ns*r + k + t*Ns.  Twiddles exp(-2 pi i q/L) are
// computed on the host in FP64 and uploaded; kernels copy them to LDS.
//
// Tensor passes use a compile-time radix schedule for the common lengths:
// every stage reads its butterfly inputs into registers, synchronises and
// writes the outputs back in place, so one LDS tile suffices and all
// register indexing is static.  Other {2,3,5,7}-smooth lengths use a generic
// path with two LDS tiles.  Strided modes move rows of TC neighbouring
// fibers (TC*8 contiguous bytes), so reads and writes stay coalesced without
// a transpose.
#include <math.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "fft_device.hpp"

namespace cprand {

// Tensor pass along mode m.  The tensor is [J][L][K] (J = product of the
// dims before m, K after); flattened column q of the J*K fibers is fiber
// (j = q % J, k = q / J) with element l at j + J*L*k + J*l.  FIRST: read the
// real input, apply the product of all sign vectors, write complex.
// VEC: 16-byte global accesses (4 real inputs along a contiguous fiber in
// the first pass; 2 neighbouring complex fibers per row in strided passes,
// where every tile lies inside one k and starts 16-byte aligned).
template <typename Tin, int L, int TC, int NT, bool FIRST, bool VEC>
__global__ __launch_bounds__(NT) void mix_pass_ct(const Tin *X, cx<float> *Xh, int64_t J, int64_t K, ModeInfo xi,
                                                  int m, const int8_t *signs, const cx<float> *twg) {
    constexpr int LDT = TC + 1;
    __shared__ cx<float> buf[L * LDT];
    __shared__ cx<float> tw[L];
    __shared__ int64_t cbase[TC];
    __shared__ float csign[TC];
    const int tid = threadIdx.x;
    const int64_t ncols = J * K;
    const int64_t q0 = (int64_t)blockIdx.x * TC;
    const int nc = (int)min((int64_t)TC, ncols - q0);
    for (int e = tid; e < L; e += NT) tw[e] = twg[e];
    int moff = 0;
    if (FIRST)
        for (int mm = 0; mm < m; ++mm) moff += (int)xi.dims[mm];
    for (int c = tid; c < TC; c += NT) {
        if (c < nc) {
            const int64_t q = q0 + c;
            int64_t j = q % J, k = q / J;
            cbase[c] = j + J * L * k;
            if (FIRST) {
                float sg = 1.0f;
                int off = 0;
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
                        sg *= (float)signs[off + im];
                    }
                    off += (int)xi.dims[mm];
                }
                csign[c] = sg;
            }
        }
    }
    __syncthreads();
    const float scale = (float)(1.0 / sqrt((double)L));
    if (VEC && FIRST) {
        static_assert(L % 4 == 0 || !VEC || !FIRST, "vector first pass needs L % 4 == 0");
        for (int e = tid; e < L * TC / 4; e += NT) {
            const int c = e / (L / 4), l4 = (e - c * (L / 4)) * 4;
            float4 v = {0.f, 0.f, 0.f, 0.f};
            if (c < nc) v = *(const float4 *)((const float *)X + cbase[c] + l4);
            const float sc = c < nc ? csign[c] : 0.f;
            buf[(l4 + 0) * LDT + c] = {v.x * sc * (float)signs[moff + l4 + 0], 0.f};
            buf[(l4 + 1) * LDT + c] = {v.y * sc * (float)signs[moff + l4 + 1], 0.f};
            buf[(l4 + 2) * LDT + c] = {v.z * sc * (float)signs[moff + l4 + 2], 0.f};
            buf[(l4 + 3) * LDT + c] = {v.w * sc * (float)signs[moff + l4 + 3], 0.f};
        }
    } else if (VEC) {
        for (int e = tid; e < L * TC / 2; e += NT) {
            const int l = e / (TC / 2), c = (e - l * (TC / 2)) * 2;
            float4 v = {0.f, 0.f, 0.f, 0.f};
            if (c < nc) v = *(const float4 *)(Xh + cbase[c] + J * (int64_t)l);
            buf[l * LDT + c] = {v.x, v.y};
            buf[l * LDT + c + 1] = {v.z, v.w};
        }
    } else {
        for (int e = tid; e < L * TC; e += NT) {
            int l, c;
            if (J == 1) {
                c = e / L;
                l = e - c * L;
            } else {
                l = e / TC;
                c = e - l * TC;
            }
            cx<float> v = {0.f, 0.f};
            if (c < nc) {
                const int64_t o = cbase[c] + J * (int64_t)l;
                if (FIRST) {
                    v.re = (float)X[o] * csign[c] * (float)signs[moff + l];
                } else {
                    v = Xh[o];
                }
            }
            buf[l * LDT + c] = v;
        }
    }
    __syncthreads();
    fft_ct<float, L, TC, NT, -1>(buf, tw);
    if (VEC && FIRST) {
        for (int e = tid; e < L * TC / 2; e += NT) {
            const int c = e / (L / 2), l2 = (e - c * (L / 2)) * 2;
            if (c < nc) {
                const cx<float> a = buf[l2 * LDT + c], b = buf[(l2 + 1) * LDT + c];
                *(float4 *)(Xh + cbase[c] + l2) = {a.re * scale, a.im * scale, b.re * scale, b.im * scale};
            }
        }
        return;
    }
    if (VEC) {
        for (int e = tid; e < L * TC / 2; e += NT) {
            const int l = e / (TC / 2), c = (e - l * (TC / 2)) * 2;
            if (c < nc) {
                const cx<float> a = buf[l * LDT + c], b = buf[l * LDT + c + 1];
                *(float4 *)(Xh + cbase[c] + J * (int64_t)l) = {a.re * scale, a.im * scale, b.re * scale, b.im * scale};
            }
        }
        return;
    }
    for (int e = tid; e < L * TC; e += NT) {
        int l, c;
        if (J == 1) {
            c = e / L;
            l = e - c * L;
        } else {
            l = e / TC;
            c = e - l * TC;
        }
        if (c < nc) Xh[cbase[c] + J * (int64_t)l] = cscale(buf[l * LDT + c], scale);
    }
}

// Non-temporal 16-byte store (the written tensor is not read again before it
// has left the caches).
typedef float ntv4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void store_nt(void *p, float4 v) {
    __builtin_nontemporal_store(ntv4{v.x, v.y, v.z, v.w}, (ntv4 *)p);
}

// Software-pipelined form of the 16-byte passes above for long tensors: a
// persistent grid (a few workgroups per CU) walks the tiles t = blockIdx.x,
// blockIdx.x + gridDim.x, ...; the global loads of the next tile are issued
// into registers before the FFT of the current tile, so HBM traffic overlaps
// the LDS work.  The first pass (real input) transforms two real fibers
// with one complex FFT, x in the real and y in the imaginary part of
// z = x + i y, and splits the result by conjugate symmetry:
//   X(k) = (Z(k) + conj Z(L-k)) / 2,  Y(k) = (Z(k) - conj Z(L-k)) / (2 i),
// so a tile holds 2 TC fibers and the FFT work per element halves.  Other
// passes: same arithmetic and output as mix_pass_ct, with non-temporal stores
// (measured faster for these passes, slower for the first).
template <int L, int TC, int NT, bool FIRST>
__global__ __launch_bounds__(NT) void mix_pass_pipe(const float *X, cx<float> *Xh, int64_t J, int64_t K, ModeInfo xi,
                                                    int m, const int8_t *signs, const cx<float> *twg,
                                                    double *normsq_part, cx<float> *copy) {
    constexpr int LDT = TC + 1;
    constexpr int FC = FIRST ? 2 * TC : TC;              // fibers per tile
    constexpr int NV = FIRST ? L * FC / 4 : L * TC / 2;  // float4 per tile
    constexpr int PF = (NV + NT - 1) / NT;                // float4 per thread
    __shared__ cx<float> buf[L * LDT];
    __shared__ cx<float> tw[L];
    // tile offsets and signs in three slots: the slot written for the next
    // tile was last read two iterations ago, before the previous barrier
    __shared__ int64_t cbase[3][FC];
    __shared__ float csign[3][FC];
    __shared__ float lsign[FIRST ? L : 1];
    // FIRST: every sign vector staged in LDS once (when they fit), so the
    // per-tile sign products read no global memory
    constexpr int kSignLds = 2048;
    __shared__ int8_t sgl[FIRST ? kSignLds : 1];
    const int tid = threadIdx.x;
    const int64_t ncols = J * K;
    const int64_t ntiles = ceil_div(ncols, FC);
    for (int e = tid; e < L; e += NT) tw[e] = twg[e];
    int moff = 0, nsg = 0;
    if (FIRST) {
        for (int mm = 0; mm < m; ++mm) moff += (int)xi.dims[mm];
        for (int mm = 0; mm < xi.order; ++mm) nsg += (int)xi.dims[mm];
        for (int e = tid; e < L; e += NT) lsign[e] = (float)signs[moff + e];
        if (nsg <= kSignLds)
            for (int e = tid; e < nsg; e += NT) sgl[e] = signs[e];
    }
    const int8_t *sgp = (FIRST && nsg <= kSignLds) ? sgl : signs;
    __syncthreads();  // the staged signs are read by the first tile's offsets below
    // 32-bit index arithmetic when the fiber count fits
    const bool small = ncols < (int64_t)INT32_MAX;
    // fiber offsets (and FIRST: sign products over the other modes) of tile t
    auto tile_info = [&](int64_t t, int slot) {
        for (int c = tid; c < FC; c += NT) {
            const int64_t q = t * FC + c;
            if (q >= ncols) {
                cbase[slot][c] = 0;
                csign[slot][c] = 0.f;
                continue;
            }
            if (small) {
                uint32_t j = (uint32_t)q % (uint32_t)J, k = (uint32_t)q / (uint32_t)J;
                cbase[slot][c] = (int64_t)j + J * L * (int64_t)k;
                if (FIRST) {
                    float sg = 1.0f;
                    int off = 0;
                    for (int mm = 0; mm < xi.order; ++mm) {
                        if (mm != m) {
                            const uint32_t d = (uint32_t)xi.dims[mm];
                            uint32_t im;
                            if (mm < m) {
                                im = j % d;
                                j /= d;
                            } else {
                                im = k % d;
                                k /= d;
                            }
                            sg *= (float)sgp[off + (int)im];
                        }
                        off += (int)xi.dims[mm];
                    }
                    csign[slot][c] = sg;
                }
            } else {
                int64_t j = q % J, k = q / J;
                cbase[slot][c] = j + J * L * k;
                if (FIRST) {
                    float sg = 1.0f;
                    int off = 0;
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
                            sg *= (float)sgp[off + im];
                        }
                        off += (int)xi.dims[mm];
                    }
                    csign[slot][c] = sg;
                }
            }
        }
    };
    auto tile_nc = [&](int64_t t) { return (int)min((int64_t)FC, ncols - t * FC); };
    float4 r[PF];
    auto issue_loads = [&](int slot, int nc) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int e = tid + u * NT;
            r[u] = float4{0.f, 0.f, 0.f, 0.f};
            if (e < NV) {
                if (FIRST) {  // fiber fastest: conflict-free LDS writes
                    const int c = e % FC, l4 = (e / FC) * 4;
                    if (c < nc) r[u] = *(const float4 *)(X + cbase[slot][c] + l4);
                } else {
                    const int l = e / (TC / 2), c = (e - l * (TC / 2)) * 2;
                    if (c < nc) r[u] = *(const float4 *)(Xh + cbase[slot][c] + J * (int64_t)l);
                }
            }
        }
    };
    int64_t t = blockIdx.x;
    if (t >= ntiles) {
        if (FIRST && normsq_part && tid == 0) normsq_part[blockIdx.x] = 0.0;
        return;
    }
    double nacc = 0.0;  // FIRST: sum of squares of the raw input (signs do not change it)
    tile_info(t, 0);
    __syncthreads();
    issue_loads(0, tile_nc(t));
    const float scale = (float)(1.0 / sqrt((double)L));
    for (int it = 0; t < ntiles; ++it, t += gridDim.x) {
        const int cur = it % 3, nxt = (it + 1) % 3;
        const int nc = tile_nc(t);
        const int64_t tn = t + gridDim.x;
        if (tn < ntiles) tile_info(tn, nxt);
        __syncthreads();  // the previous tile's output reads are done; tile_info(tn) is visible
        // registers (tile t) -> LDS
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int e = tid + u * NT;
            if (e >= NV) continue;
            const float4 v = r[u];
            if (FIRST) {
                // fiber c goes to the real (even c) or imaginary (odd c) part of column c / 2;
                // fibers past the end write zeros
                const int c = e % FC, l4 = (e / FC) * 4;
                const float sc = c < nc ? csign[cur][c] : 0.f;
                nacc += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
                float *bf = (float *)buf + 2 * (l4 * LDT + (c >> 1)) + (c & 1);
                bf[0] = v.x * sc * lsign[l4 + 0];
                bf[2 * LDT] = v.y * sc * lsign[l4 + 1];
                bf[4 * LDT] = v.z * sc * lsign[l4 + 2];
                bf[6 * LDT] = v.w * sc * lsign[l4 + 3];
            } else {
                const int l = e / (TC / 2), c = (e - l * (TC / 2)) * 2;
                buf[l * LDT + c] = {v.x, v.y};
                buf[l * LDT + c + 1] = {v.z, v.w};
            }
        }
        // the next tile's loads stay in flight through this tile's FFT
        if (tn < ntiles) issue_loads(nxt, tile_nc(tn));
        __syncthreads();
        fft_ct<float, L, TC, NT, -1>(buf, tw);
        __syncthreads();
        if (FIRST) {
            const float hs = 0.5f * scale;
            for (int e = tid; e < L * FC / 2; e += NT) {
                const int c = e / (L / 2), l2 = (e - c * (L / 2)) * 2;
                if (c < nc) {
                    const int cc = c >> 1, m0 = l2 == 0 ? 0 : L - l2, m1 = L - l2 - 1;
                    const cx<float> z0 = buf[l2 * LDT + cc], z1 = buf[(l2 + 1) * LDT + cc];
                    const cx<float> w0 = buf[m0 * LDT + cc], w1 = buf[m1 * LDT + cc];
                    float4 o;
                    if (c & 1)  // (Z(k) - conj Z(L-k)) / (2 i)
                        o = {(z0.im + w0.im) * hs, (w0.re - z0.re) * hs, (z1.im + w1.im) * hs, (w1.re - z1.re) * hs};
                    else        // (Z(k) + conj Z(L-k)) / 2
                        o = {(z0.re + w0.re) * hs, (z0.im - w0.im) * hs, (z1.re + w1.re) * hs, (z1.im - w1.im) * hs};
                    *(float4 *)(Xh + cbase[cur][c] + l2) = o;
                }
            }
        } else {
            for (int e = tid; e < L * TC / 2; e += NT) {
                const int l = e / (TC / 2), c = (e - l * (TC / 2)) * 2;
                if (c < nc) {
                    const cx<float> a = buf[l * LDT + c], b = buf[l * LDT + c + 1];
                    store_nt(Xh + cbase[cur][c] + J * (int64_t)l, float4{a.re * scale, a.im * scale, b.re * scale,
                                                                       b.im * scale});
                }
            }
            if (copy) {  // the same fibers again, each stored contiguously (fiber q at copy + q * L)
                for (int e = tid; e < L * TC / 2; e += NT) {
                    const int c = e / (L / 2), l2 = (e - c * (L / 2)) * 2;
                    if (c < nc) {
                        const cx<float> a = buf[l2 * LDT + c], b = buf[(l2 + 1) * LDT + c];
                        store_nt(copy + (t * TC + c) * (int64_t)L + l2, float4{a.re * scale, a.im * scale,
                                                                             b.re * scale, b.im * scale});
                    }
                }
            }
        }
    }
    if (FIRST && normsq_part) {
        __shared__ double sh[NT / kWave];
        nacc = block_sum<NT>(nacc, sh);
        if (tid == 0) normsq_part[blockIdx.x] = nacc;
    }
}

// Generic tensor pass (any {2,3,5,7}-smooth length, float or double).
template <typename T, typename Tin>
__global__ __launch_bounds__(256) void mix_pass_rt(FftPlan fp, const Tin *X, cx<T> *Xh, int64_t J, int64_t K,
                                                   int tc, int first, ModeInfo xi, int m, const int8_t *signs) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int L = (int)fp.L;
    // tc = 0: a long fiber, one per workgroup, unpadded, twiddles read from
    // global memory (L2) so the two tiles alone fill the LDS
    const bool glong = tc == 0;
    if (glong) tc = 1;
    const int ldt = glong ? 1 : tc + 1;
    cx<T> *b0 = (cx<T> *)lds, *b1 = b0 + L * ldt;
    cx<T> *twl = b1 + L * ldt;
    const cx<T> *tw = glong ? (const cx<T> *)fp.tw : twl;
    __shared__ int64_t cbase[16];
    __shared__ double csign[16];
    const int64_t ncols = J * K;
    const int64_t q0 = (int64_t)blockIdx.x * tc;
    const int nc = (int)min((int64_t)tc, ncols - q0);
    if (!glong)
        for (int e = threadIdx.x; e < L; e += blockDim.x) twl[e] = ((const cx<T> *)fp.tw)[e];
    int moff = 0;
    for (int mm = 0; mm < m; ++mm) moff += (int)xi.dims[mm];
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const int64_t q = q0 + c;
        int64_t j = q % J, k = q / J;
        cbase[c] = j + J * L * k;
        if (first) {
            double sg = 1.0;
            int off = 0;
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
                off += (int)xi.dims[mm];
            }
            csign[c] = sg;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < L * tc; e += blockDim.x) {
        int l, c;
        if (J == 1) {
            c = e / L;
            l = e - c * L;
        } else {
            l = e / tc;
            c = e - l * tc;
        }
        cx<T> v = {(T)0, (T)0};
        if (c < nc) {
            const int64_t o = cbase[c] + J * (int64_t)l;
            if (first)
                v.re = (T)((double)X[o] * csign[c] * (double)signs[moff + l]);
            else
                v = Xh[o];
        }
        b0[l * ldt + c] = v;
    }
    __syncthreads();
    cx<T> *res = fft_tile_rt<T, -1>(b0, b1, fp, ldt, tc, tw);
    const T scale = (T)(1.0 / sqrt((double)L));
    for (int e = threadIdx.x; e < L * tc; e += blockDim.x) {
        int l, c;
        if (J == 1) {
            c = e / L;
            l = e - c * L;
        } else {
            l = e / tc;
            c = e - l * tc;
        }
        if (c < nc) Xh[cbase[c] + J * (int64_t)l] = cscale(res[l * ldt + c], scale);
    }
}

// Columns per tile of the generic path: two tiles + twiddles within ~64 KB;
// 0 (one unpadded fiber, twiddles from global memory) when even one padded
// column and its twiddles would not fit in the 160 KB of LDS.
constexpr size_t kLdsMax = 160 * 1024;
static int tile_cols(int64_t L, int esz) {
    if ((2 * (size_t)L * 2 + (size_t)L) * (size_t)esz > kLdsMax) return 0;
    int64_t tc = (int64_t)(65536 / esz - L) / (2 * L) - 1;
    if (tc > 16) tc = 16;
    if (tc < 1) tc = 1;
    return (int)tc;
}
// Columns per workgroup for the R columns of a factor or mode-step product:
// at most what fits in LDS, and few enough that about eight workgroups share
// the R columns (one workgroup per launch would run the FFT stages serially).
static int tile_cols_for(int64_t L, int esz, int R) {
    const int per = (R + 7) / 8;
    const int tc = tile_cols(L, esz);
    return tc == 0 ? 0 : std::max(1, std::min(tc, per));
}
static size_t tile_lds(int64_t L, int tc, size_t esz) {
    return tc == 0 ? 2 * (size_t)L * esz : (2 * (size_t)L * (tc + 1) + (size_t)L) * esz;
}

// ---------------------------------------------------------------------------
// Factor mix (A-hat = F D A), inverse factor mix (A = Re(D F^* A-hat)) and
// the unmix of a mode step (W = D Re(F^* Y)).  Columns of an I x R
// row-major matrix are the transformed fibers.
template <typename T>
__global__ __launch_bounds__(256) void factor_mix_kernel(FftPlan fp, const T *in, const int8_t *sign, T *out, int R,
                                                         int tc, int inverse) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int L = (int)fp.L;
    const bool glong = tc == 0;  // long fibers: see mix_pass_rt
    if (glong) tc = 1;
    const int ldt = glong ? 1 : tc + 1;
    cx<T> *b0 = (cx<T> *)lds, *b1 = b0 + L * ldt;
    cx<T> *twl = b1 + L * ldt;
    const cx<T> *tw = glong ? (const cx<T> *)fp.tw : twl;
    if (!glong)
        for (int e = threadIdx.x; e < L; e += blockDim.x) twl[e] = ((const cx<T> *)fp.tw)[e];
    const int r0 = blockIdx.x * tc;
    const int nc = min(tc, R - r0);
    for (int e = threadIdx.x; e < L * tc; e += blockDim.x) {
        const int l = e / tc;
        const int c = e - l * tc;
        cx<T> v = {(T)0, (T)0};
        if (c < nc) {
            const int64_t o = (int64_t)l * R + r0 + c;
            if (!inverse)
                v.re = (T)sign[l] * in[o];
            else
                v = {in[2 * o], in[2 * o + 1]};
        }
        b0[l * ldt + c] = v;
    }
    __syncthreads();
    cx<T> *res = inverse ? fft_tile_rt<T, 1>(b0, b1, fp, ldt, tc, tw) : fft_tile_rt<T, -1>(b0, b1, fp, ldt, tc, tw);
    const T scale = (T)(1.0 / sqrt((double)L));
    for (int e = threadIdx.x; e < L * tc; e += blockDim.x) {
        const int l = e / tc;
        const int c = e - l * tc;
        if (c >= nc) continue;
        const int64_t o = (int64_t)l * R + r0 + c;
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
__global__ __launch_bounds__(256) void unmix_kernel(FftPlan fp, const T *ypart, int chunks, int R, const int8_t *sign,
                                                    T *W, int rowmajor, int tc) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int L = (int)fp.L;
    const bool glong = tc == 0;  // long fibers: see mix_pass_rt
    if (glong) tc = 1;
    const int ldt = glong ? 1 : tc + 1;
    cx<T> *b0 = (cx<T> *)lds, *b1 = b0 + L * ldt;
    cx<T> *twl = b1 + L * ldt;
    const cx<T> *tw = glong ? (const cx<T> *)fp.tw : twl;
    if (!glong)
        for (int e = threadIdx.x; e < L; e += blockDim.x) twl[e] = ((const cx<T> *)fp.tw)[e];
    const int r0 = blockIdx.x * tc;
    const int nc = min(tc, R - r0);
    const size_t cstride = (size_t)2 * R * L;
    for (int e = threadIdx.x; e < L * tc; e += blockDim.x) {
        const int c = e / L;
        const int l = e - c * L;
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
    cx<T> *res = fft_tile_rt<T, 1>(b0, b1, fp, ldt, tc, tw);
    const T scale = (T)(1.0 / sqrt((double)L));
    for (int e = threadIdx.x; e < L * tc; e += blockDim.x) {
        const int l = e / tc;
        const int c = e - l * tc;
        if (c >= nc) continue;
        const int r = r0 + c;
        const T v = (T)sign[l] * res[l * ldt + c].re * scale;
        if (rowmajor)
            W[(int64_t)l * R + r] = v;
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
    // the generic tile (two buffers of L x 2 plus twiddles) must fit in LDS
    // the long-fiber layout holds two unpadded tiles of L in LDS
    if (L < 1 || (size_t)L * (dbl ? 16 : 8) * 2 > kLdsMax) {
        *err = hipErrorInvalidValue;
        return nullptr;
    }
    FftPlan p{};
    p.L = L;
    int64_t rem = L;
    while (rem % 4 == 0 && p.nrad < 24) {
        p.rad[p.nrad++] = 4;
        rem /= 4;
    }
    const int primes[4] = {2, 3, 5, 7};
    for (int pi = 0; pi < 4; ++pi)
        while (rem % primes[pi] == 0 && p.nrad < 24) {
            p.rad[p.nrad++] = primes[pi];
            rem /= primes[pi];
        }
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

// Compute units of the current device (cached per device).
static int device_cus() {
    static std::mutex mu;
    static std::map<int, int> cus;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> g(mu);
    auto it = cus.find(dev);
    if (it != cus.end()) return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
    cus[dev] = n;
    return n;
}

template <int L, int TC, int NT>
static hipError_t launch_ct_pass(const FftPlan *fp, const ModeInfo &xi, const void *X, int xkind, void *Xhat, int m,
                                 bool first, const int8_t *signs, int64_t J, int64_t K, MixExtras *ex, hipStream_t st) {
    const unsigned nb = (unsigned)ceil_div(J * K, TC);
    const cx<float> *tw = (const cx<float> *)fp->tw;
    const bool xa = (((uintptr_t)X) & 15) == 0, ha = (((uintptr_t)Xhat) & 15) == 0;
    // the pipelined kernel holds the next tile in registers: long fibers
    // (more than 8 vectors per thread) would spill, they use mix_pass_ct
    constexpr bool kPipe = (L * TC / 2 + NT - 1) / NT <= 8;
    // persistent grid for the pipelined kernel: the workgroups that are
    // resident at once (registers and LDS, as the runtime reports them), one
    // pass over the CUs; a larger grid would run its tail as a second round
    auto persistent_grid = [&](auto kernel, unsigned &cache) -> unsigned {
        if (cache == 0) {
            int n = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, NT, 0) != hipSuccess || n < 1) n = 1;
            cache = (unsigned)n;
        }
        return (unsigned)std::min<int64_t>((int64_t)nb, (int64_t)device_cus() * cache);
    };
    if (first) {
        if (xkind != K_F32) return hipErrorInvalidValue;
        if constexpr (L % 4 == 0) {
            if (J == 1 && xa && ha && !kPipe) {
                hipLaunchKernelGGL((mix_pass_ct<float, L, TC, NT, true, true>), dim3(nb), dim3(NT), 0, st,
                                   (const float *)X, (cx<float> *)Xhat, J, K, xi, m, signs, tw);
                return hipGetLastError();
            }
        }
        if constexpr (L % 4 == 0 && kPipe) {
            if (J == 1 && xa && ha) {
                static unsigned per_cu = 0;
                const unsigned np = persistent_grid(mix_pass_pipe<L, TC, NT, true>, per_cu);
                double *nsp = (ex && np <= 4096) ? ex->normsq_part : nullptr;  // partial buffer: 4096 doubles
                hipLaunchKernelGGL((mix_pass_pipe<L, TC, NT, true>), dim3(np), dim3(NT), 0, st, (const float *)X,
                                   (cx<float> *)Xhat, J, K, xi, m, signs, tw, nsp, (cx<float> *)nullptr);
                if (nsp) ex->nparts = (int32_t)np;
                return hipGetLastError();
            }
        }
        {
            hipLaunchKernelGGL((mix_pass_ct<float, L, TC, NT, true, false>), dim3(nb), dim3(NT), 0, st,
                               (const float *)X, (cx<float> *)Xhat, J, K, xi, m, signs, tw);
        }
    } else {
        if constexpr (kPipe) {
            if (J > 1 && J % TC == 0 && ha) {
                static unsigned per_cu = 0;
                const unsigned np = persistent_grid(mix_pass_pipe<L, TC, NT, false>, per_cu);
                const bool cp = ex && ex->copy && ex->copy_ld == L && (((uintptr_t)ex->copy) & 15) == 0;
                hipLaunchKernelGGL((mix_pass_pipe<L, TC, NT, false>), dim3(np), dim3(NT), 0, st,
                                   (const float *)nullptr, (cx<float> *)Xhat, J, K, xi, m, signs, tw,
                                   (double *)nullptr, cp ? (cx<float> *)ex->copy : (cx<float> *)nullptr);
                if (cp) ex->copied = true;
                return hipGetLastError();
            }
        }
        if (J > 1 && J % TC == 0 && ha)
            hipLaunchKernelGGL((mix_pass_ct<float, L, TC, NT, false, true>), dim3(nb), dim3(NT), 0, st,
                               (const float *)nullptr, (cx<float> *)Xhat, J, K, xi, m, signs, tw);
        else
            hipLaunchKernelGGL((mix_pass_ct<float, L, TC, NT, false, false>), dim3(nb), dim3(NT), 0, st,
                               (const float *)nullptr, (cx<float> *)Xhat, J, K, xi, m, signs, tw);
    }
    return hipGetLastError();
}

// Lengths with a compile-time schedule (single precision).
static bool launch_fixed_length(int64_t L, const FftPlan *fp, const ModeInfo &xi, const void *X, int xkind,
                                void *Xhat, int m, bool first, const int8_t *signs, int64_t J, int64_t K,
                                MixExtras *ex, hipStream_t st, hipError_t *err) {
    switch (L) {
        case 50: *err = launch_ct_pass<50, 16, 512>(fp, xi, X, xkind, Xhat, m, first, signs, J, K, ex, st); return true;
        case 60: *err = launch_ct_pass<60, 16, 512>(fp, xi, X, xkind, Xhat, m, first, signs, J, K, ex, st); return true;
        case 90: *err = launch_ct_pass<90, 16, 512>(fp, xi, X, xkind, Xhat, m, first, signs, J, K, ex, st); return true;
        case 100: *err = launch_ct_pass<100, 16, 512>(fp, xi, X, xkind, Xhat, m, first, signs, J, K, ex, st); return true;
        case 128: *err = launch_ct_pass<128, 16, 512>(fp, xi, X, xkind, Xhat, m, first, signs, J, K, ex, st); return true;
        case 150: *err = launch_ct_pass<150, 16, 512>(fp, xi, X, xkind, Xhat, m, first, signs, J, K, ex, st); return true;
        case 200: *err = launch_ct_pass<200, 16, 512>(fp, xi, X, xkind, Xhat, m, first, signs, J, K, ex, st); return true;
        case 300: *err = launch_ct_pass<300, 16, 512>(fp, xi, X, xkind, Xhat, m, first, signs, J, K, ex, st); return true;
        case 400: *err = launch_ct_pass<400, 16, 1024>(fp, xi, X, xkind, Xhat, m, first, signs, J, K, ex, st); return true;
        case 1000: *err = launch_ct_pass<1000, 16, 512>(fp, xi, X, xkind, Xhat, m, first, signs, J, K, ex, st); return true;
        default: return false;
    }
}

hipError_t launch_mix_pass(const FftPlan *fp, bool dbl, const ModeInfo &xi, const void *X, int xkind, void *Xhat,
                           int32_t m, bool first, const int8_t *signs, MixExtras *ex, hipStream_t st) {
    int64_t J = 1, K = 1;
    for (int i = 0; i < m; ++i) J *= xi.dims[i];
    for (int i = m + 1; i < xi.order; ++i) K *= xi.dims[i];
    if (ex) {
        ex->nparts = 0;
        ex->copied = false;
    }
    if (!dbl && (!first || xkind == K_F32)) {
        hipError_t e;
        if (launch_fixed_length(fp->L, fp, xi, X, xkind, Xhat, m, first, signs, J, K, ex, st, &e)) return e;
    }
    const size_t esz = dbl ? 16 : 8;
    const int tc = tile_cols(fp->L, (int)esz);
    const int64_t nb = ceil_div(J * K, std::max(tc, 1));
    const size_t lds = tile_lds(fp->L, tc, esz);
    if (dbl) {
        hipLaunchKernelGGL((mix_pass_rt<double, double>), dim3((unsigned)nb), dim3(256), lds, st, *fp,
                           (const double *)X, (cx<double> *)Xhat, J, K, tc, first ? 1 : 0, xi, m, signs);
    } else if (first && xkind == K_F64) {
        hipLaunchKernelGGL((mix_pass_rt<float, double>), dim3((unsigned)nb), dim3(256), lds, st, *fp,
                           (const double *)X, (cx<float> *)Xhat, J, K, tc, 1, xi, m, signs);
    } else {
        hipLaunchKernelGGL((mix_pass_rt<float, float>), dim3((unsigned)nb), dim3(256), lds, st, *fp,
                           (const float *)X, (cx<float> *)Xhat, J, K, tc, first ? 1 : 0, xi, m, signs);
    }
    return hipGetLastError();
}

hipError_t launch_factor_mix(const FftPlan *fp, bool dbl, int32_t I, int32_t R, const void *in, const int8_t *sign,
                             void *out, bool inverse, hipStream_t st) {
    const size_t esz = dbl ? 16 : 8;
    const int tc = tile_cols_for(fp->L, (int)esz, (int)R);
    const int nb = (int)ceil_div(R, std::max(tc, 1));
    const size_t lds = tile_lds(fp->L, tc, esz);
    if (dbl)
        hipLaunchKernelGGL(factor_mix_kernel<double>, dim3(nb), dim3(256), lds, st, *fp, (const double *)in, sign,
                           (double *)out, R, tc, inverse ? 1 : 0);
    else
        hipLaunchKernelGGL(factor_mix_kernel<float>, dim3(nb), dim3(256), lds, st, *fp, (const float *)in, sign,
                           (float *)out, R, tc, inverse ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_unmix(const FftPlan *fp, bool dbl, int32_t In, int32_t R, int32_t chunks, const void *ypart,
                        const int8_t *sign, void *W, bool w_rowmajor, hipStream_t st) {
    const size_t esz = dbl ? 16 : 8;
    const int tc = tile_cols_for(fp->L, (int)esz, (int)R);
    const int nb = (int)ceil_div(R, std::max(tc, 1));
    const size_t lds = tile_lds(fp->L, tc, esz);
    if (dbl)
        hipLaunchKernelGGL(unmix_kernel<double>, dim3(nb), dim3(256), lds, st, *fp, (const double *)ypart, chunks, R,
                           sign, (double *)W, w_rowmajor ? 1 : 0, tc);
    else
        hipLaunchKernelGGL(unmix_kernel<float>, dim3(nb), dim3(256), lds, st, *fp, (const float *)ypart, chunks, R,
                           sign, (float *)W, w_rowmajor ? 1 : 0, tc);
    return hipGetLastError();
}

hipError_t launch_signs(const ModeInfo &mi, uint64_t seed, int8_t *signs, hipStream_t st) {
    int64_t total = 0;
    for (int m = 0; m < mi.order; ++m) total += mi.dims[m];
    hipLaunchKernelGGL(signs_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, mi, seed, signs, total);
    return hipGetLastError();
}

}  // namespace cprand
