// Sampled MTTKRP with BF16 fibers and BF16 Khatri-Rao rows on the gfx950
// MFMA 16x16x32 BF16 instruction with FP32 accumulation; Gram in FP64.
//
// The instruction wants eight consecutive samples of one fiber row per lane,
// while fibers are contiguous along rows, so each 32-sample step is staged
// through LDS: every thread loads 16 bytes (8 rows of one fiber, the eight
// threads of a fiber covering 128 contiguous bytes) and scatters them into a
// [row][sample] tile; each wave then reads its 16-row A operand with 16-byte
// LDS loads.  Z_S is kept transposed ([column][sample]) for the B operand.
#include <mutex>

#include "kernels.hpp"

namespace cprand {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kBfRows = 64;     // fiber rows per workgroup (4 waves x 16)
constexpr int kBfStep = 32;     // samples per MFMA step
constexpr int kBfPadA = 8;      // bf16 padding of an A-tile row

struct BfArgs {
    ModeInfo mi;
    const uint16_t *X;
    FactorPtrs A;         // float factors
    const int32_t *idx;
    const double *w;
    CdfPtrs cdf;
    int use_cdf;
    uint64_t seed, t;
    const uint64_t *t_dev;
    float *wpart;
    double *vpart;
    int32_t R, S, In, kc;
    int32_t rows_wg, per_split;  // streaming form: rows per block, samples per split
};

template <int CT, bool CONTIG>
__global__ __launch_bounds__(256) void gather_contract_bf16(BfArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int tid = threadIdx.x;
    const int KC = a.kc;
    const int N = a.mi.order, n = a.mi.n, R = a.R;
    const int chunk = blockIdx.y;
    const int s0 = chunk * KC;
    const int ns = min(KC, a.S - s0);
    const int ldz = KC + 8;                       // bf16 row stride of Zt
    constexpr int lda = kBfStep + kBfPadA;        // bf16 row stride of the A tile

    int64_t *s_base = (int64_t *)lds;
    double *s_w = (double *)(s_base + KC);
    int32_t *s_idx = (int32_t *)(s_w + KC);
    float *zf = (float *)(lds + (((size_t)KC * (16 + 4 * N) + 15) & ~(size_t)15));  // KC x R (FP32 z_b)
    uint16_t *Zt = (uint16_t *)(zf + (size_t)KC * R);                              // 16*CT x ldz
    uint16_t *At = Zt + (size_t)16 * CT * ldz;                                      // kBfRows x lda

    // given samples never read the device-side iteration counter (its load
    // would be one more round trip ahead of the index loads)
    const uint64_t tt = a.idx ? 0 : (a.t_dev ? *a.t_dev : a.t);
    for (int sl = tid; sl < KC; sl += blockDim.x) {
        int64_t row[kMaxOrder];
        double wv = 0.0;
        int64_t base = 0;
        if (sl < ns) {
            const int64_t s = s0 + sl;
            wv = 1.0;
            if (a.idx) {
                for (int m = 0; m < N; ++m) row[m] = (m == n) ? 0 : a.idx[s * N + m];
                if (a.w) wv = a.w[s];
            } else {
                wv = draw_sample(a.mi, a.seed, tt, s, a.cdf, a.use_cdf != 0, row);
            }
            for (int m = 0; m < N; ++m)
                if (m != n) base += row[m] * a.mi.strides[m];
        } else {
            for (int m = 0; m < N; ++m) row[m] = 0;
        }
        for (int m = 0; m < N; ++m) s_idx[sl * N + m] = (int32_t)row[m];
        s_base[sl] = base;
        s_w[sl] = wv;
    }
    for (int e = tid; e < 16 * CT * ldz; e += blockDim.x) Zt[e] = 0;
    __syncthreads();

    // loader role: sample ls (0..31) of each 32-sample step, rows lg*8 ..
    // lg*8+7 of the block.  The first kBfPre steps' fibers of the lanes whose
    // 8 rows are one 16-byte load go out now, so that their latency overlaps
    // the Khatri-Rao loads and the Gram instead of one round trip per step.
    const int ls = tid >> 3, lg = tid & 7;
    const int rb = blockIdx.x * kBfRows;
    const int r0 = rb + lg * 8;
    const bool vec = CONTIG && r0 + 8 <= a.In;  // uniform per 8 lanes
    constexpr int kBfPre = 4;
    uint4 pre[kBfPre];
#pragma unroll
    for (int j = 0; j < kBfPre; ++j) {
        const int sl = j * kBfStep + ls;
        pre[j] = uint4{0u, 0u, 0u, 0u};
        if (vec && sl < ns) pre[j] = *(const uint4 *)(a.X + s_base[sl] + r0);
    }

    // Z_S rounded to BF16; the B operand carries the weights
    for (int e = tid; e < ns * R; e += blockDim.x) {
        const int sl = e / R, r = e - sl * R;
        float z = 1.0f;
        for (int m = 0; m < N; ++m) {
            if (m == n) continue;
            z *= ((const float *)a.A.p[m])[(int64_t)s_idx[sl * N + m] * R + r];
        }
        const float zb = bf16_to_f32(f32_to_bf16_rne(z));
        zf[sl * R + r] = zb;
        Zt[r * ldz + sl] = f32_to_bf16_rne((float)(s_w[sl] * (double)zb));
    }
    __syncthreads();

    if (blockIdx.x == 0) {
        double *vp = a.vpart + (size_t)chunk * R * R;
        for (int p = tid; p < R * R; p += blockDim.x) {
            const int r = p / R, q = p - r * R;
            if (q < r) continue;
            double acc = 0.0;
            for (int sl = 0; sl < ns; ++sl)
                acc += (double)bf16_to_f32(Zt[r * ldz + sl]) * (double)zf[sl * R + q];
            vp[r * R + q] = acc;
            vp[q * R + r] = acc;
        }
    }

    const int wv = tid >> 6, l = tid & 63, li = l & 15, lq = l >> 4;
    const int In = a.In;
    const int64_t sn = a.mi.strides[n];
    v4f acc[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct] = v4f{0, 0, 0, 0};

    // steps in groups of kBfPre (unrolled, so the preloaded registers are
    // indexed at compile time)
    for (int ks0 = 0; ks0 < ns; ks0 += kBfPre * kBfStep) {
#pragma unroll
        for (int j = 0; j < kBfPre; ++j) {
            const int ks = ks0 + j * kBfStep;
            if (ks >= ns) break;  // uniform
            uint16_t vals[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) vals[e] = 0;
            const int sl = ks + ls;
            if (ks0 == 0 && vec) {  // loaded above (zero past the chunk)
                const uint4 q = pre[j];
                vals[0] = q.x & 0xffff; vals[1] = q.x >> 16;
                vals[2] = q.y & 0xffff; vals[3] = q.y >> 16;
                vals[4] = q.z & 0xffff; vals[5] = q.z >> 16;
                vals[6] = q.w & 0xffff; vals[7] = q.w >> 16;
            } else if (sl < ns && r0 < In) {
                const int64_t b = s_base[sl];
                if (vec) {
                    const uint4 q = *(const uint4 *)(a.X + b + r0);
                    vals[0] = q.x & 0xffff; vals[1] = q.x >> 16;
                    vals[2] = q.y & 0xffff; vals[3] = q.y >> 16;
                    vals[4] = q.z & 0xffff; vals[5] = q.z >> 16;
                    vals[6] = q.w & 0xffff; vals[7] = q.w >> 16;
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        if (r0 + e < In) vals[e] = a.X[b + (int64_t)(r0 + e) * sn];
                }
            }
            __syncthreads();  // previous step's A tile fully consumed
#pragma unroll
            for (int e = 0; e < 8; ++e) At[(lg * 8 + e) * lda + ls] = vals[e];
            __syncthreads();
            const v8bf av = *(const v8bf *)(At + (wv * 16 + li) * lda + lq * 8);
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const v8bf bv = *(const v8bf *)(Zt + (ct * 16 + li) * ldz + ks + lq * 8);
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[ct], 0, 0, 0);
            }
        }
    }

    float *wp = a.wpart + (size_t)chunk * R * In;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const int col = ct * 16 + li;
        if (col >= R) continue;
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) {
            const int row = rb + wv * 16 + 4 * lq + vv;
            if (row < In) wp[(size_t)col * In + row] = acc[ct][vv];
        }
    }
}

// ---------------------------------------------------------------------------
// Streaming form for long sample sets over contiguous fibers (drawn indices,
// I_n % 8 == 0, R <= 32).  The grid is sized to the workgroups the chip holds
// at once; workgroup (rb, split) owns row block rb and the samples [split *
// per_split, (split + 1) * per_split), and each wave keeps the accumulators
// of its GW row groups of 128 rows in registers over the whole split, so one
// partial product is written per split.
//
// A batch is 32 samples.  Lane (li, kq) loads rows 8 li .. 8 li + 7 of each
// of its row groups for the samples ks + 8 kq + u, u < 8: it then holds an
// 8 x 8 block (rows x samples) of BF16 values, and the block's transpose,
// formed in registers by byte permutes, gives the A operands of eight MFMAs.
// MFMA j takes the group's rows 8 i + j (A row i < 16) and, at k = 8 kq + u,
// the sample ks + 8 kq + u, so all eight share one B operand: columns
// 16 ct + li of bf16(w z) for the samples ks + 8 kq .. ks + 8 kq + 7, one
// 16-byte LDS read from Zt.  Lane (li, kq) of MFMA j holds the group's rows
// 8 (4 kq + v) + j, v < 4: eight consecutive rows per v over the eight MFMAs.
// Each wave reads 256 consecutive bytes of every fiber of the batch per row
// group, and the four waves of a workgroup the adjacent ones.
//
// The chunk's rows z (FP32 products in increasing mode order, rounded to
// BF16) and the B operand are formed as in the chunked form; the Gram
// V(r, q) = sum_s bf16(w z)_r bf16(z)_q runs on FP64 MFMA in row block 0:
// R <= 16, the one 16 x 16 tile with the four waves taking every fourth
// k-step and the partial tiles summed in wave order; 16 < R <= 32, the four
// tiles (r, q) on the four waves.

constexpr int kBfStreamMaxR = 32;
constexpr int kBfStreamMinS = 4096;  // sample sets from this size on stream
constexpr int kBfStreamAccRegs = 64;  // accumulator registers per lane

// row groups per wave: whole groups within the accumulator budget, two at most
__host__ __device__ constexpr int bf_stream_gw(int ct) {
    return 32 * ct > kBfStreamAccRegs ? 0 : (kBfStreamAccRegs / (32 * ct) >= 2 ? 2 : 1);
}

typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <int CT, int GW>
__global__ __launch_bounds__(256) void gather_stream_bf16(BfArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int tid = threadIdx.x;
    const int KC = a.kc;  // a multiple of 32, at most the workgroup size
    const int N = a.mi.order, n = a.mi.n, R = a.R;
    const int split = blockIdx.y, rb = blockIdx.x;
    const int sa = split * a.per_split, sb = min(a.S, sa + a.per_split);
    const int ldz = KC + 8;  // bf16 row stride of Zt (16-byte rows)

    int64_t *s_base = (int64_t *)lds;
    double *s_w = (double *)(s_base + KC);
    int32_t *s_idx = (int32_t *)(s_w + KC);
    float *zf = (float *)(lds + (((size_t)KC * (16 + 4 * N) + 15) & ~(size_t)15));  // KC x R, bf16(z) as FP32
    uint16_t *Zt = (uint16_t *)(zf + (size_t)KC * R);                              // 16 CT x ldz, bf16(w z)
    // columns at or past R stay zero; sample columns are rewritten per chunk
    for (int e = tid; e < 8 * CT * ldz; e += blockDim.x) ((uint32_t *)Zt)[e] = 0u;

    // wave index as a scalar, so that per-wave conditions branch on SCC
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, li = l & 15, kq = l >> 4;
    const int In = a.In;
    const int row_lo = rb * a.rows_wg, row_end = min(In, row_lo + a.rows_wg);
    const int nrg = (row_end - row_lo + 127) / 128;  // row groups of the block
    const int gpw = (nrg + 3) / 4;                   // <= GW (plan)
    const int g0 = wv * gpw;
    const int gw = max(0, min(gpw, nrg - g0));       // uniform per wave
    const uint16_t *xp = a.X;

    v4f acc[GW][CT][8];
#pragma unroll
    for (int g = 0; g < GW; ++g)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[g][ct][j] = v4f{0, 0, 0, 0};

    const int nt16 = (R + 15) / 16;
    const bool gram = rb == 0;
    const int rt = nt16 == 1 ? 0 : wv >> 1, qt = nt16 == 1 ? 0 : wv & 1;
    const int kk0 = nt16 == 1 ? wv : 0, kkstep = nt16 == 1 ? 4 : 1;
    v4d gacc = {0.0, 0.0, 0.0, 0.0};

    auto run_chunk = [&](const int ns) {
        for (int ks = 0; ks < ns; ks += 32) {
            v4u q[GW][8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int sl = ks + 8 * kq + u;
                const int64_t b = s_base[sl < ns ? sl : 0];  // past the chunk: zero B rows
#pragma unroll
                for (int g = 0; g < GW; ++g) {
                    // a row past the block reads the block's last 8 rows:
                    // their outputs are never stored
                    const int row = row_lo + (g0 + g) * 128 + 8 * li;
                    q[g][u] = *(const v4u *)(xp + b + (row < row_end ? row : row_end - 8));
                }
            }
            // all loads issued before the first MFMA waits on them
            __builtin_amdgcn_sched_barrier(0);
            v8bf bv[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) bv[ct] = *(const v8bf *)(Zt + (ct * 16 + li) * ldz + ks + 8 * kq);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                // rows j of the lane's blocks: the low (j even) or high half
                // of dword j / 2 of each sample's load, two samples a dword
                const uint32_t sel = (j & 1) ? 0x07060302u : 0x05040100u;
#pragma unroll
                for (int g = 0; g < GW; ++g) {
                    v4u av;
#pragma unroll
                    for (int p = 0; p < 4; ++p)
                        av[p] = __builtin_amdgcn_perm(q[g][2 * p + 1][j >> 1], q[g][2 * p][j >> 1], sel);
                    const v8bf ab = __builtin_bit_cast(v8bf, av);
#pragma unroll
                    for (int ct = 0; ct < CT; ++ct)
                        acc[g][ct][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bv[ct], acc[g][ct][j], 0, 0, 0);
                }
            }
        }
    };

    // indices and weight of sample c0 + tid of the next chunk (one sample
    // per thread), loaded a chunk ahead
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
        // the thread index, opaque per chunk: what the phases below derive
        // from it is recomputed here rather than kept live beside the
        // accumulators
        int tc = tid;
        asm volatile("" : "+v"(tc));
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
        // sampled Khatri-Rao rows: FP32 products in increasing mode order
        for (int e = tc; e < ns * R; e += blockDim.x) {
            const int sl = e / R, r = e - sl * R;
            float z = 1.0f;
#pragma unroll
            for (int m = 0; m < kMaxOrder; ++m) {
                if (m >= N) break;
                if (m == n) continue;
                z *= ((const float *)a.A.p[m])[(int64_t)s_idx[sl * N + m] * R + r];
            }
            const float zb = bf16_to_f32(f32_to_bf16_rne(z));
            zf[sl * R + r] = zb;
            Zt[r * ldz + sl] = f32_to_bf16_rne((float)(s_w[sl] * (double)zb));
        }
        for (int e = tc; e < R * (KC - ns); e += blockDim.x) {  // B rows past the chunk
            const int r = e / (KC - ns), sl = ns + (e - r * (KC - ns));
            Zt[r * ldz + sl] = 0;
        }
        __syncthreads();
        if (gram) {
            const int lic = tc & 15, lkc = (tc & 63) >> 4;
            const int r = rt * 16 + lic, qq = qt * 16 + lic;
            const bool rin = r < R, qin = qq < R;
            for (int kk = kk0; kk < (ns + 3) / 4; kk += kkstep) {
                const int sl = 4 * kk + lkc;
                const bool sin = sl < ns;
                const double av = (rin && sin) ? (double)bf16_to_f32(Zt[r * ldz + sl]) : 0.0;
                const double bq = (qin && sin) ? (double)zf[sl * R + qq] : 0.0;
                gacc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bq, gacc, 0, 0, 0);
            }
        }
        if (gw > 0) run_chunk(ns);
        __syncthreads();  // the next chunk rewrites the LDS tiles
    }

    // partial product of this split, [split][col][In]: for each v, the lane's
    // eight MFMAs hold eight consecutive rows (I_n % 8 == 0 keeps a run of
    // eight wholly inside or outside the block)
    float *wp = a.wpart + (size_t)split * R * In;
#pragma unroll
    for (int g = 0; g < GW; ++g) {
        if (g >= gw) break;
        const int rbase = row_lo + (g0 + g) * 128 + 32 * kq;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            const int col = ct * 16 + li;
            if (col >= R) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r8 = rbase + 8 * v;
                if (r8 >= row_end) continue;
                float *dst = wp + (size_t)col * In + r8;
                *(float4 *)dst = float4{acc[g][ct][0][v], acc[g][ct][1][v], acc[g][ct][2][v], acc[g][ct][3][v]};
                *(float4 *)(dst + 4) = float4{acc[g][ct][4][v], acc[g][ct][5][v], acc[g][ct][6][v], acc[g][ct][7][v]};
            }
        }
    }
    if (gram) {
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
        if (nt16 > 1 || wv == 0) {
#pragma unroll
            for (int v2 = 0; v2 < 4; ++v2) {
                const int rr = rt * 16 + kq + 4 * v2, qc = qt * 16 + li;
                if (rr < R && qc < R) vp[rr * R + qc] = gacc[v2];
            }
        }
    }
}

template <int CT>
static int bf_stream_capacity(size_t lds) {
    // workgroups of this instance the chip holds at once, per device
    static std::mutex mu;
    static int cap[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 768;
    std::lock_guard<std::mutex> lk(mu);
    if (cap[dev] == 0) {
        int nb = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gather_stream_bf16<CT, bf_stream_gw(CT)>, 256, lds) !=
                hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || nb < 1 ||
            cus < 1) {
            (void)hipGetLastError();
            return 768;
        }
        cap[dev] = nb * cus;
    }
    return cap[dev];
}

hipError_t launch_bf16_gather(const GatherPlan &gp, const GatherArgs &g, hipStream_t st) {
    BfArgs a{};
    a.mi = g.mi;
    a.X = (const uint16_t *)g.X;
    a.A = g.A;
    a.idx = g.idx;
    a.w = g.w;
    if (g.cdf) {
        a.cdf = *g.cdf;
        a.use_cdf = 1;
    }
    a.seed = g.seed;
    a.t = g.t;
    a.t_dev = g.t_dev;
    a.wpart = (float *)g.wpart;
    a.vpart = g.vpart;
    a.R = gp.R;
    a.S = gp.S;
    a.In = gp.In;
    a.kc = gp.kc;
    a.rows_wg = gp.rows_wg;
    a.per_split = gp.per_split;
    dim3 grid(gp.row_blocks, gp.chunks), block(256);
    if (gp.stream) {
        if (!g.idx) return hipErrorInvalidValue;  // the streaming form takes drawn samples
        switch (gp.ct) {
            case 1: hipLaunchKernelGGL((gather_stream_bf16<1, bf_stream_gw(1)>), grid, block, gp.lds_bytes, st, a); break;
            case 2: hipLaunchKernelGGL((gather_stream_bf16<2, bf_stream_gw(2)>), grid, block, gp.lds_bytes, st, a); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
#define BF_LAUNCH(CT)                                                                               \
    do {                                                                                            \
        if (gp.contig)                                                                              \
            hipLaunchKernelGGL((gather_contract_bf16<CT, true>), grid, block, gp.lds_bytes, st, a);  \
        else                                                                                        \
            hipLaunchKernelGGL((gather_contract_bf16<CT, false>), grid, block, gp.lds_bytes, st, a); \
    } while (0)
    switch (gp.ct) {
        case 1: BF_LAUNCH(1); break;
        case 2: BF_LAUNCH(2); break;
        case 3: BF_LAUNCH(3); break;
        case 4: BF_LAUNCH(4); break;
        default: return hipErrorInvalidValue;
    }
#undef BF_LAUNCH
    return hipGetLastError();
}

GatherPlan plan_gather_bf16(int32_t R, int32_t S, int64_t In, bool contig_ok, int max_chunks, int order) {
    GatherPlan g{};
    g.kind = K_BF16;
    g.R = R;
    g.S = S;
    g.In = (int32_t)In;
    g.ncols = R;
    g.ct = (R + 15) / 16;
    g.waves = 4;
    g.rows_wg = kBfRows;
    g.row_blocks = (int)ceil_div(In, kBfRows);
    if (max_chunks == 0 && S >= kBfStreamMinS && contig_ok && R <= kBfStreamMaxR && In % 8 == 0) {
        // streaming form: row groups of 128 dealt evenly to the fewest
        // blocks of at most 4 GW groups, one split per resident workgroup
        // and row block
        const int gw = bf_stream_gw(g.ct);
        g.stream = true;
        const int64_t nrg = ceil_div(In, (int64_t)128);
        g.row_blocks = (int)ceil_div(nrg, (int64_t)4 * gw);
        g.rows_wg = (int)(ceil_div(nrg, (int64_t)g.row_blocks) * 128);
        auto lds_stream = [&](int k) {
            const size_t head = (((size_t)k * (16 + 4 * order)) + 15) & ~(size_t)15;
            return head + (size_t)k * R * 4 + (size_t)16 * g.ct * (k + 8) * 2;
        };
        int kc = 256;
        while (kc > 32 && lds_stream(kc) > 40 * 1024) kc -= 32;  // four workgroups per CU
        const size_t lds = std::max(lds_stream(kc), (size_t)256 * 4 * 8);  // room for the Gram tiles at the end
        const int cap = g.ct == 1 ? bf_stream_capacity<1>(lds) : bf_stream_capacity<2>(lds);
        int splits = std::max(1, cap / g.row_blocks);
        splits = (int)std::min<int64_t>(splits, std::max<int64_t>(1, S / 64));
        g.per_split = (int32_t)ceil_div(S, splits);
        g.chunks = (int)ceil_div(S, g.per_split);
        g.kc = kc;
        g.contig = true;
        g.lds_bytes = lds;
        return g;
    }
    int kc = 128;
    if (max_chunks > 0)
        kc = (int)std::min<int64_t>(512, ceil_div(ceil_div(S, max_chunks), kBfStep) * kBfStep);
    else
        while (kc > kBfStep && (int64_t)g.row_blocks * ceil_div(S, kc) < 256) kc /= 2;
    auto lds_for = [&](int k) {
        const size_t head = (((size_t)k * (16 + 4 * kMaxOrder)) + 15) & ~(size_t)15;
        return head + (size_t)k * R * 4 + (size_t)16 * g.ct * (k + 8) * 2 + (size_t)kBfRows * (kBfStep + kBfPadA) * 2 +
               16;
    };
    while (kc > kBfStep && lds_for(kc) > 150 * 1024) kc -= kBfStep;
    g.kc = kc;
    g.chunks = (int)ceil_div(S, kc);
    g.contig = contig_ok;
    g.lds_bytes = lds_for(kc);
    return g;
}

}  // namespace cprand
