// Sampled MTTKRP and Gram for one mode step, streaming form for long sample
// sets (Alg. 2 and Alg. 3; complex form for the mixed tensor of Alg. 4 /
// eq. rcLS).
#include <mutex>

#include "mttkrp_device.hpp"

namespace cprand {
// ---------------------------------------------------------------------------
// Streaming form for long sample sets over contiguous fibers.  The grid is
// sized to the workgroups the chip holds at once; workgroup (rb, split) owns
// row block rb and the samples [split * per_split, (split + 1) * per_split).
// Each wave owns up to GW consecutive row groups of the block and keeps their
// accumulators in registers over all of the split's samples, so one partial
// product is written per split rather than per chunk.  A batch of loads is
// KS k-steps (4 samples each) x GW row groups: every wave reads GW * 16 * VE
// consecutive rows (GW * 256 bytes) of each of its fibers per batch, runs of
// fiber bytes long enough for full HBM efficiency under random fiber
// addresses.  The split is processed in chunks of KC samples (indices and
// Khatri-Rao rows in LDS); a chunk's first fiber batch is issued before its
// Khatri-Rao loads, and the other resident workgroups keep HBM busy while
// one forms the rows of its next chunk.  The Gram of the split is
// accumulated by FP64 MFMA in row block 0 (R <= 16: the one 16 x 16 tile,
// the k-steps dealt to the four waves; up to R = 32: three tiles, one per
// wave).  The samples always come drawn (idx); there is no in-kernel draw.

// accumulator registers of one row group
template <typename T, bool CPLX, int CT>
__host__ __device__ constexpr int stream_acc_regs() {
    return CT * Geo<T, CPLX>::VE * (sizeof(T) == 8 ? 8 : 4);
}
// Row groups per wave: kStreamAccRegs accumulator registers at most, four
// at most.  The budget bounds the occupancy: the bytes a CU keeps in flight
// (waves x 8 loads x 16 bytes x 64 lanes) bound the rate.  With a chunk's
// first batch held through its Khatri-Rao phase (below) the real kinds run
// three waves per SIMD, which measured faster than four without it.
constexpr int kStreamAccRegs = 32;
template <typename T, bool CPLX, int CT>
__host__ __device__ constexpr int stream_gw() {
    return stream_acc_regs<T, CPLX, CT>() > kStreamAccRegs ? 0
         : (kStreamAccRegs / stream_acc_regs<T, CPLX, CT>() >= 4 ? 4 : kStreamAccRegs / stream_acc_regs<T, CPLX, CT>());
}

// complex64 at R <= 16 runs held to four waves per SIMD (the _o4 kernel below)
template <typename T, bool CPLX, int CT>
constexpr bool stream_o4() {
    return CPLX && sizeof(T) == 4 && CT <= 2;
}

template <typename T, bool CPLX, int CT, bool WEIGHTED>
__device__ __forceinline__ void gather_stream_body(const KArgs &a) {
    typedef Geo<T, CPLX> G;
    typedef typename AccT<T>::type Acc;
    constexpr int GW = stream_gw<T, CPLX, CT>();
    static_assert(GW >= 1, "accumulators exceed the register budget");
    constexpr int KS = kStreamLoads / GW;
    // each chunk's first fiber batch issued before its Khatri-Rao rows; its
    // registers stay live through them, which the four-wave complex64 form
    // cannot hold without spilling
    constexpr bool PRE = !stream_o4<T, CPLX, CT>();
    constexpr int LDB = ldb_for(CT, (int)sizeof(T));
    extern __shared__ __align__(16) unsigned char lds[];

    const int tid = threadIdx.x;
    const int KC = a.kc;
    const int N = a.mi.order, n = a.mi.n;
    const int R = a.R;
    const int split = blockIdx.y, rb = blockIdx.x;
    const int sa = split * a.per_split, sb = min(a.S, sa + a.per_split);

    int64_t *s_base = (int64_t *)lds;
    double *s_w = (double *)(s_base + KC);
    int32_t *s_idx = (int32_t *)(s_w + KC);
    // Real data: B operand tiles (row stride LDB; weighted: the raw rows in
    // Zr after them).  Complex data: per sample, the B operand pairs of the
    // 2R columns interleaved, then a zero pair (row stride LDZ).
    const int LDZ = CPLX ? stream_ldz(R, (int)sizeof(T)) : LDB;
    T *Bre = (T *)(lds + (((size_t)KC * (16 + 4 * N) + 15) & ~(size_t)15));
    T *Zr = WEIGHTED ? Bre + (size_t)KC * LDB : Bre;
    {
        // padding columns stay zero; sample rows are rewritten per chunk
        const int words = (int)(((size_t)KC * LDZ * sizeof(T) * (WEIGHTED ? 2 : 1)) / 4);
        uint32_t *p = (uint32_t *)Bre;
        for (int e = tid; e < words; e += blockDim.x) p[e] = 0u;
    }

    // wave index as a scalar, so that per-wave conditions branch on SCC
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, li = l & 15, lk = l >> 4;
    const int In = a.In;
    const int row_lo = rb * a.rows_wg, row_end = min(In, row_lo + a.rows_wg);
    const int nrg = (row_end - row_lo + G::RPW - 1) / G::RPW;  // row groups of the block
    const int gpw = (nrg + 3) / 4;                               // <= GW (plan)
    const int g0 = wv * gpw;
    const int gw = max(0, min(gpw, nrg - g0));                   // uniform per wave
    const T *xp = (const T *)a.X;

    Acc acc[GW][CT][G::VE];
#pragma unroll
    for (int g = 0; g < GW; ++g)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int c = 0; c < G::VE; ++c) acc[g][ct][c] = Acc{0, 0, 0, 0};
    // Gram tiles (rt, qt), qt >= rt, of 16 x 16.  R <= 16: the one tile,
    // every wave taking every fourth k-step, the four partial tiles summed in
    // wave order at the end; 16 < R <= 32: tiles (0,0), (0,1), (1,1) on
    // waves 0, 1, 2, each over all k-steps.
    const int nt16 = (R + 15) / 16;
    const bool gram = rb == 0 && (nt16 == 1 || wv < 3);
    const int rt = (nt16 == 1 || wv < nt16) ? 0 : 1;
    const int qt = nt16 == 1 ? 0 : (rt == 0 ? wv : 1);
    const int kk0 = nt16 == 1 ? wv : 0, kkstep = nt16 == 1 ? 4 : 1;
    v4d gacc = {0.0, 0.0, 0.0, 0.0};

    int zoff[CT];  // complex: this lane's B pair of column tile ct (the zero pair past 2R)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const int col = ct * 16 + li;
        zoff[ct] = col < 2 * R ? 2 * col : 4 * R;
    }
    T v[KS][GW][G::NV];
    // The chunk's products: batches of k-steps ks .. ks + 4 KS - 1, lane
    // (li, lk) taking sample ks + 4 k + lk and rows VE li .. VE li + VE - 1
    // of each of the wave's GW row groups.  Every wave runs all GW groups
    // with no branch or mask between the loads, so all stay in flight
    // together.  A lane past the chunk reads the chunk's first fiber: its B
    // operand row is zero, so it adds nothing.  A row past the block reads
    // the block's last vector (a line that is being fetched anyway): each
    // MFMA output row depends only on its own A row, and those rows are never
    // stored.  The plan guarantees I_n % VE == 0, so a row in the block
    // starts a whole vector.
    auto load_batch = [&](const int ks, const int ns) {
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                const int sl = ks + 4 * k + lk;
                const int64_t b = s_base[sl < ns ? sl : 0];
#pragma unroll
                for (int g = 0; g < GW; ++g) {
                    const int row = row_lo + (g0 + g) * G::RPW + G::VE * li;
                    const T *src = xp + (b + (row < row_end ? row : row_end - G::VE)) * (CPLX ? 2 : 1);
                    if (sizeof(T) == 4) {
                        const float4 q = *(const float4 *)src;
                        v[k][g][0] = q.x;
                        v[k][g][1] = q.y;
                        v[k][g][2] = q.z;
                        v[k][g][3] = q.w;
                    } else {
                        const double2 q = *(const double2 *)src;
                        v[k][g][0] = q.x;
                        v[k][g][1] = q.y;
                    }
                }
            }
    };
    // first: the chunk's first batch was issued before its Khatri-Rao rows
    auto run_chunk = [&](const int ns, bool first) {
        for (int ks = 0; ks < ns; ks += 4 * KS) {
            if (!first) load_batch(ks, ns);
            first = false;
            // keep the scheduler from sinking the loads toward their MFMAs
            // (which would leave two in flight): all are issued first
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                if (ks + 4 * k >= ns) break;  // uniform
                const int sl = ks + 4 * k + lk;  // < KC: KC is a multiple of 4 KS
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                    T bre, bim = (T)0;
                    if (!CPLX) {
                        bre = Bre[sl * LDB + ct * 16 + li];
                    } else {
                        // column c < R: (zr, zi) of c; R <= c < 2R: (-zi, zr)
                        // of c - R (the imaginary part of X conj z)
                        bre = Bre[sl * LDZ + zoff[ct]];
                        bim = Bre[sl * LDZ + zoff[ct] + 1];
                    }
#pragma unroll
                    for (int g = 0; g < GW; ++g) {
#pragma unroll
                        for (int c = 0; c < G::VE; ++c) {
                            if (!CPLX) {
                                acc[g][ct][c] = mfma16(v[k][g][c], bre, acc[g][ct][c]);
                            } else {
                                acc[g][ct][c] = mfma16(v[k][g][2 * c], bre, acc[g][ct][c]);
                                acc[g][ct][c] = mfma16(v[k][g][2 * c + 1], bim, acc[g][ct][c]);
                            }
                        }
                    }
                }
            }
        }
    };

    // The indices and weight of sample c0 + tid of the next chunk (KC <= the
    // workgroup size: one sample per thread), loaded into registers a chunk
    // ahead so that their latency hides behind the current chunk's stream.
    int32_t pidx[kMaxOrder];
    double pw;
    auto fetch = [&](int c0n, int tc) {
        const bool in = c0n < sb && tc < min(KC, sb - c0n);
        const int64_t s = in ? (int64_t)c0n + tc : 0;
#pragma unroll
        for (int m = 0; m < kMaxOrder; ++m) pidx[m] = a.idx[s * N + (m < N ? m : 0)];  // no branch between loads
#pragma unroll
        for (int m = 0; m < kMaxOrder; ++m) pidx[m] = (in && m < N && m != n) ? pidx[m] : 0;
        pw = in ? (a.w ? a.w[s] : 1.0) : 0.0;
    };
    fetch(sa, tid);

    for (int c0 = sa; c0 < sb; c0 += KC) {
        const int ns = min(KC, sb - c0);
        // The thread index, opaque to the compiler in each chunk: what the
        // index, Khatri-Rao and Gram phases derive from it is recomputed per
        // chunk rather than hoisted out of the loop, where it would stay live
        // beside the accumulators.
        int tc = tid;
        asm volatile("" : "+v"(tc));
        const int lic = tc & 15, lkc = (tc & 63) >> 4;
        if (tc < KC) {
            int64_t base = 0;
#pragma unroll
            for (int m = 0; m < kMaxOrder; ++m) {
                if (m >= N) break;  // uniform
                s_idx[tc * N + m] = pidx[m];
                base += (int64_t)pidx[m] * a.mi.strides[m];
            }
            s_base[tc] = base;
            s_w[tc] = pw;
        }
        __syncthreads();
        fetch(c0 + KC, tc);
        // the chunk's first fiber batch goes out now: under a loaded memory
        // system the Khatri-Rao loads below take microseconds, and the
        // workgroup keeps streaming through them
        if (PRE && gw > 0) load_batch(0, ns);
        // mode by mode, four elements per pass (the accumulators stay live)
        chunk_krp_by_mode<T, CPLX, WEIGHTED, 4, true>(a, ns, LDZ, s_idx, s_w, Bre, nullptr, Zr, tc);
        if (ns < KC) {
            // B operand rows past the chunk: zero (their lanes read real fibers)
            const int e0 = ns * LDZ, e1 = KC * LDZ;
            for (int e = e0 + tc; e < e1; e += blockDim.x) Bre[e] = (T)0;
        }
        __syncthreads();
        if (gram) {
            const int li = lic, lk = lkc;
            const int r = rt * 16 + li, q = qt * 16 + li;
            const bool rin = r < R, qin = q < R;
            for (int kk = kk0; kk < (ns + 3) / 4; kk += kkstep) {
                const int sl = 4 * kk + lk;
                const bool sin = sl < ns;
                if (!CPLX) {
                    double av = (rin && sin) ? (double)Zr[sl * LDB + r] : 0.0;
                    if (WEIGHTED) av *= s_w[sl];
                    const double bv = (qin && sin) ? (double)Zr[sl * LDB + q] : 0.0;
                    gacc = mfma16(av, bv, gacc);
                } else {
                    gacc = mfma16((rin && sin) ? (double)Bre[sl * LDZ + 2 * r] : 0.0,
                                  (qin && sin) ? (double)Bre[sl * LDZ + 2 * q] : 0.0, gacc);
                    gacc = mfma16((rin && sin) ? (double)Bre[sl * LDZ + 2 * r + 1] : 0.0,
                                  (qin && sin) ? (double)Bre[sl * LDZ + 2 * q + 1] : 0.0, gacc);
                }
            }
        }
        if (gw > 0) run_chunk(ns, PRE);
        __syncthreads();  // the next chunk rewrites the LDS tiles
    }

    // partial product of this split: [split][col][In]; output tile row i' of
    // MFMA c is fiber row base + VE i' + c (see gather_contract)
    T *wp = (T *)a.wpart + (size_t)split * a.ncols * In;
    const bool vec_ok = In % (sizeof(T) == 4 && G::VE == 4 ? 4 : 2) == 0;
#pragma unroll
    for (int g = 0; g < GW; ++g) {
        if (g >= gw) break;
        const int rbase = row_lo + (g0 + g) * G::RPW;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            const int col = ct * 16 + li;
            if (col < a.ncols) store_group<T, G::VE>(wp + (size_t)col * In, acc[g][ct], rbase, row_end, lk, vec_ok);
        }
    }
    if (rb == 0) {
        double *vp = a.vpart + (size_t)split * R * R;
        if (nt16 == 1) {
            // the four waves' partial tiles, summed in wave order (the chunk
            // loop ended on a barrier: the LDS is free)
            double *gt = (double *)lds;
#pragma unroll
            for (int v2 = 0; v2 < 4; ++v2) gt[(wv * 64 + l) * 4 + v2] = gacc[v2];
            __syncthreads();
            if (wv == 0) {
#pragma unroll
                for (int v2 = 0; v2 < 4; ++v2) {
                    double t = gt[l * 4 + v2];
#pragma unroll
                    for (int w2 = 1; w2 < 4; ++w2) t += gt[(w2 * 64 + l) * 4 + v2];
                    gacc[v2] = t;
                }
            }
        }
        if (gram && (nt16 > 1 || wv == 0)) {
#pragma unroll
            for (int v2 = 0; v2 < 4; ++v2) {
                const int rr = rt * 16 + lk + 4 * v2, qq = qt * 16 + li;
                if (rr < R && qq < R) {
                    vp[rr * R + qq] = gacc[v2];
                    if (rt != qt) vp[qq * R + rr] = gacc[v2];
                }
            }
        }
    }
}

template <typename T, bool CPLX, int CT, bool WEIGHTED>
__global__ __launch_bounds__(256) void gather_stream(KArgs a) {
    gather_stream_body<T, CPLX, CT, WEIGHTED>(a);
}

// The same with the registers held to four waves per SIMD: complex64 at
// R <= 16 then runs at occupancy 4 without spilling (its matrix work per
// byte is twice the real case's, and the extra waves hide it).
template <typename T, bool CPLX, int CT, bool WEIGHTED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void gather_stream_o4(KArgs a) {
    gather_stream_body<T, CPLX, CT, WEIGHTED>(a);
}

template <typename T, bool CPLX, int CT, bool WEIGHTED>
static int stream_capacity(size_t lds) {
    // workgroups of this instance the chip holds at once, per device
    static std::mutex mu;
    static int cap[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 768;
    std::lock_guard<std::mutex> lk(mu);
    if (cap[dev] == 0) {
        int nb = 0, cus = 0;
        hipError_t qe;
        if constexpr (stream_o4<T, CPLX, CT>())
            qe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gather_stream_o4<T, CPLX, CT, WEIGHTED>, 256, lds);
        else
            qe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gather_stream<T, CPLX, CT, WEIGHTED>, 256, lds);
        if (qe != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || nb < 1 ||
            cus < 1) {
            (void)hipGetLastError();
            return 768;
        }
        cap[dev] = nb * cus;
    }
    return cap[dev];
}

int stream_gw_host(int kind, int ct) {
    switch (kind) {
        case K_F32: return ct == 1 ? stream_gw<float, false, 1>() : ct == 2 ? stream_gw<float, false, 2>() : 0;
        case K_F64: return ct == 1 ? stream_gw<double, false, 1>() : ct == 2 ? stream_gw<double, false, 2>() : 0;
        case K_C64:
            return ct == 1 ? stream_gw<float, true, 1>() : ct == 2 ? stream_gw<float, true, 2>()
                 : ct == 3 ? stream_gw<float, true, 3>() : ct == 4 ? stream_gw<float, true, 4>() : 0;
        case K_C128:
            return ct == 1 ? stream_gw<double, true, 1>() : ct == 2 ? stream_gw<double, true, 2>()
                 : ct == 3 ? stream_gw<double, true, 3>() : ct == 4 ? stream_gw<double, true, 4>() : 0;
        default: return 0;
    }
}

// resident workgroups of the kernel a plan would launch (the lower of the
// weighted and unweighted forms for real data)
int stream_cap(int kind, int ct, size_t lds) {
    switch (kind) {
        case K_F32:
            return ct == 1 ? std::min(stream_capacity<float, false, 1, false>(lds), stream_capacity<float, false, 1, true>(lds))
                           : std::min(stream_capacity<float, false, 2, false>(lds), stream_capacity<float, false, 2, true>(lds));
        case K_F64:
            return ct == 1 ? std::min(stream_capacity<double, false, 1, false>(lds), stream_capacity<double, false, 1, true>(lds))
                           : std::min(stream_capacity<double, false, 2, false>(lds), stream_capacity<double, false, 2, true>(lds));
        case K_C64:
            return ct == 1 ? stream_capacity<float, true, 1, false>(lds) : ct == 2 ? stream_capacity<float, true, 2, false>(lds)
                 : ct == 3 ? stream_capacity<float, true, 3, false>(lds) : stream_capacity<float, true, 4, false>(lds);
        default:
            return ct == 1 ? stream_capacity<double, true, 1, false>(lds) : ct == 2 ? stream_capacity<double, true, 2, false>(lds)
                 : ct == 3 ? stream_capacity<double, true, 3, false>(lds) : stream_capacity<double, true, 4, false>(lds);
    }
}

template <typename T, bool CPLX, int CT>
static hipError_t launch_stream_ct(const GatherPlan &gp, const KArgs &k, bool weighted, hipStream_t st) {
    dim3 grid(gp.row_blocks, gp.chunks), block(64 * gp.waves);
    if constexpr (stream_o4<T, CPLX, CT>())
        hipLaunchKernelGGL((gather_stream_o4<T, CPLX, CT, false>), grid, block, gp.lds_bytes, st, k);
    else if (weighted && !CPLX)
        hipLaunchKernelGGL((gather_stream<T, CPLX, CT, true>), grid, block, gp.lds_bytes, st, k);
    else
        hipLaunchKernelGGL((gather_stream<T, CPLX, CT, false>), grid, block, gp.lds_bytes, st, k);
    return hipGetLastError();
}

hipError_t launch_gather_stream(const GatherPlan &gp, const KArgs &k, bool weighted, hipStream_t st) {
    switch (gp.kind) {
        case K_F32:
            return gp.ct == 1 ? launch_stream_ct<float, false, 1>(gp, k, weighted, st)
                 : gp.ct == 2 ? launch_stream_ct<float, false, 2>(gp, k, weighted, st) : hipErrorInvalidValue;
        case K_F64:
            return gp.ct == 1 ? launch_stream_ct<double, false, 1>(gp, k, weighted, st)
                 : gp.ct == 2 ? launch_stream_ct<double, false, 2>(gp, k, weighted, st) : hipErrorInvalidValue;
        case K_C64:
            switch (gp.ct) {
                case 1: return launch_stream_ct<float, true, 1>(gp, k, false, st);
                case 2: return launch_stream_ct<float, true, 2>(gp, k, false, st);
                case 3: return launch_stream_ct<float, true, 3>(gp, k, false, st);
                case 4: return launch_stream_ct<float, true, 4>(gp, k, false, st);
                default: return hipErrorInvalidValue;
            }
        case K_C128:
            switch (gp.ct) {
                case 1: return launch_stream_ct<double, true, 1>(gp, k, false, st);
                case 2: return launch_stream_ct<double, true, 2>(gp, k, false, st);
                case 3: return launch_stream_ct<double, true, 3>(gp, k, false, st);
                case 4: return launch_stream_ct<double, true, 4>(gp, k, false, st);
                default: return hipErrorInvalidValue;
            }
        default: return hipErrorInvalidValue;
    }
}

}  // namespace cprand
