// Sampled MTTKRP with BF16 fibers and BF16 Khatri-Rao rows on the gfx950
// MFMA 16x16x32 BF16 instruction with FP32 accumulation; Gram in FP64.
//
// The instruction wants eight consecutive samples of one fiber row per lane,
// while fibers are contiguous along rows, so each 32-sample step is staged
// through LDS: every thread loads 16 bytes (8 rows of one fiber, the eight
// threads of a fiber covering 128 contiguous bytes) and scatters them into a
// [row][sample] tile; each wave then reads its 16-row A operand with 16-byte
// LDS loads.  Z_S is kept transposed ([column][sample]) for the B operand.
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

    const uint64_t tt = a.t_dev ? *a.t_dev : a.t;
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
    const int rb = blockIdx.x * kBfRows;
    const int In = a.In;
    const int64_t sn = a.mi.strides[n];
    // loader role: sample ls (0..31), rows lg*8 .. lg*8+7 of the block
    const int ls = tid >> 3, lg = tid & 7;
    v4f acc[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct] = v4f{0, 0, 0, 0};

    for (int ks = 0; ks < ns; ks += kBfStep) {
        uint16_t vals[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) vals[e] = 0;
        const int sl = ks + ls;
        const int r0 = rb + lg * 8;
        if (sl < ns && r0 < In) {
            const int64_t b = s_base[sl];
            if (CONTIG && r0 + 8 <= In) {
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
    dim3 grid(gp.row_blocks, gp.chunks), block(256);
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

GatherPlan plan_gather_bf16(int32_t R, int32_t S, int64_t In, bool contig_ok, int max_chunks) {
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
