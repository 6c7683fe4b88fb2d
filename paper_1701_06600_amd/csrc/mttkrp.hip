// Sampled MTTKRP and Gram for one mode step (Alg. 2 and Alg. 3; complex
// form for the mixed tensor of Alg. 4 / eq. rcLS).
//
// One workgroup owns a chunk of KC samples and a block of fiber rows.  It
// (1) draws or loads the chunk's multi-indices and fiber base offsets,
// (2) forms the sampled Khatri-Rao rows Z_S in LDS as Hadamard products of
//     factor rows (the factors are small and stay in L2),
// (3) for the first row block only, accumulates the chunk's Gram
//     Z^T diag(w) Z in FP64,
// (4) streams the chunk's fibers straight from HBM with 16-byte loads (one
//     wave covers 16*VE consecutive rows of four fibers per step) into MFMA
//     16x16x4 products against Z_S, FP32 or FP64 accumulation.
// Each lane's 16-byte vector holds VE consecutive fiber rows; MFMA number c
// takes component c, so the A operand needs no shuffle and the output rows
// are a fixed permutation that the store undoes.  Partial products of every
// chunk go to a workspace and are summed by the consumer in a fixed order
// (deterministic results).
#include "mttkrp_device.hpp"

namespace cprand {

template <typename T, bool CPLX, int CT, bool CONTIG, bool WEIGHTED>
__global__ __launch_bounds__(256) void gather_contract(KArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    // the chunk's Gram entries dealt to its row blocks
    gather_chunk<T, CPLX, CT, CONTIG, WEIGHTED>(a, lds, a.vpart + (size_t)blockIdx.y * a.R * a.R, (int)blockIdx.x,
                                                (int)gridDim.x);
}

// ---------------------------------------------------------------------------
GatherPlan plan_gather_bf16(int32_t R, int32_t S, int64_t In, bool contig_ok, int max_chunks, int order);

GatherPlan plan_gather(int kind, int32_t R, int32_t S, int64_t In, bool contig_ok, int max_chunks, int order) {
    if (kind == K_BF16) return plan_gather_bf16(R, S, In, contig_ok, max_chunks, order);
    GatherPlan g{};
    g.kind = kind;
    g.R = R;
    g.S = S;
    g.In = (int32_t)In;
    const bool cplx = (kind == K_C64 || kind == K_C128);
    const int tsize = (kind == K_F64 || kind == K_C128) ? 8 : 4;
    g.ncols = cplx ? 2 * R : R;
    g.ct = (g.ncols + 15) / 16;
    const int nv = 16 / tsize, ve = cplx ? nv / 2 : nv, rpw = 16 * ve;
    g.waves = 4;  // small I_n: the extra waves still share the sampling, Khatri-Rao and Gram phases
    g.rows_wg = g.waves * rpw;
    g.row_blocks = (int)ceil_div(In, g.rows_wg);
    // Samples per chunk: grow while the grid keeps >= 2048 workgroups and the
    // LDS tiles stay within 64 KB (fewer partial products to reduce); shrink
    // while the grid has < 256 workgroups, never below 16 (the MFMA loop
    // consumes 16 samples per iteration).
    const size_t ldb = (size_t)ldb_for(g.ct, tsize);
    auto lds_for = [&](int k) {
        const size_t head = (((size_t)k * (16 + 4 * order)) + 15) & ~(size_t)15;
        return head + (size_t)k * ldb * tsize * 2;  // room for Bre + (Bim or Zraw)
    };
    int kc = 64;
    const int sgw = stream_gw_host(kind, g.ct);
    if (max_chunks == 0 && S >= kWholeFiberS && contig_ok && R <= kStreamMaxR && sgw >= 1 && In % ve == 0) {
        // streaming form: accumulators over whole splits, one split per
        // resident workgroup (per row block)
        const int ks = kStreamLoads / sgw;
        g.stream = true;
        // row groups dealt evenly to the fewest blocks of at most
        // waves * sgw groups
        const int64_t nrg = ceil_div(In, (int64_t)rpw);
        g.row_blocks = (int)ceil_div(nrg, (int64_t)g.waves * sgw);
        g.rows_wg = (int)(ceil_div(nrg, (int64_t)g.row_blocks) * rpw);
        // LDS: indices, then real B tiles (two with weights) or the
        // interleaved complex rows
        auto lds_stream = [&](int k) {
            const size_t head = (((size_t)k * (16 + 4 * order)) + 15) & ~(size_t)15;
            return cplx ? head + (size_t)k * stream_ldz(R, tsize) * tsize : head + (size_t)k * ldb * tsize * 2;
        };
        const int step = std::max(16, 4 * ks);  // KC a multiple of the batch
        kc = 256;
        while (kc > step && lds_stream(kc) > 40 * 1024) kc -= step;  // four workgroups per CU
        const size_t lds = lds_stream(kc);
        int splits = std::max(1, stream_cap(kind, g.ct, lds) / g.row_blocks);
        splits = (int)std::min<int64_t>(splits, std::max<int64_t>(1, S / 64));
        g.per_split = (int32_t)ceil_div(S, splits);
        g.chunks = (int)ceil_div(S, g.per_split);
        g.kc = kc;
        g.contig = true;
        g.lds_bytes = lds;
        return g;
    } else if (max_chunks == 0 && S >= kWholeFiberS) {
        // long sample sets: every workgroup reads whole fibers (all row groups)
        // of its chunk, about a thousand chunks
        g.row_blocks = 1;
        g.rows_wg = (int)(ceil_div(In, (int64_t)g.waves * rpw) * g.waves * rpw);
        kc = (int)std::min<int64_t>(128, std::max<int64_t>(16, ceil_div(ceil_div(S, 1024), 16) * 16));
        while (kc > 16 && lds_for(kc) > 65536) kc -= 16;
    } else if (max_chunks > 0) {
        kc = (int)ceil_div(ceil_div(S, max_chunks), 16) * 16;
        while (kc > 16 && lds_for(kc) > 150 * 1024) kc -= 16;
    } else {
        while (kc < 512 && (int64_t)g.row_blocks * ceil_div(S, 2 * kc) >= 2048 && lds_for(2 * kc) <= 65536) kc *= 2;
        while (kc > 16 && ((int64_t)g.row_blocks * ceil_div(S, kc) < 256 || lds_for(kc) > 65536)) kc /= 2;
    }
    g.kc = kc;
    g.chunks = (int)ceil_div(S, kc);
    g.contig = contig_ok;
    // R <= 16: room for the four partial Gram tiles summed at the end
    g.lds_bytes = std::max(lds_for(kc), (size_t)(R <= 16 ? 4 * 64 * 4 * 8 : 0));
    return g;
}

template <typename T, bool CPLX, int CT>
static hipError_t launch_ct(const GatherPlan &gp, const KArgs &k, bool weighted, hipStream_t st) {
    dim3 grid(gp.row_blocks, gp.chunks), block(64 * gp.waves);
    if (gp.contig) {
        if (weighted && !CPLX)
            hipLaunchKernelGGL((gather_contract<T, CPLX, CT, true, true>), grid, block, gp.lds_bytes, st, k);
        else
            hipLaunchKernelGGL((gather_contract<T, CPLX, CT, true, false>), grid, block, gp.lds_bytes, st, k);
    } else {
        if (weighted && !CPLX)
            hipLaunchKernelGGL((gather_contract<T, CPLX, CT, false, true>), grid, block, gp.lds_bytes, st, k);
        else
            hipLaunchKernelGGL((gather_contract<T, CPLX, CT, false, false>), grid, block, gp.lds_bytes, st, k);
    }
    return hipGetLastError();
}

template <typename T, bool CPLX>
static hipError_t launch_t(const GatherPlan &gp, const KArgs &k, bool weighted, hipStream_t st) {
    switch (gp.ct) {
        case 1: return launch_ct<T, CPLX, 1>(gp, k, weighted, st);
        case 2: return launch_ct<T, CPLX, 2>(gp, k, weighted, st);
        case 3: return launch_ct<T, CPLX, 3>(gp, k, weighted, st);
        case 4: return launch_ct<T, CPLX, 4>(gp, k, weighted, st);
        case 5: return launch_ct<T, CPLX, 5>(gp, k, weighted, st);
        case 6: return launch_ct<T, CPLX, 6>(gp, k, weighted, st);
        case 7: return launch_ct<T, CPLX, 7>(gp, k, weighted, st);
        case 8: return launch_ct<T, CPLX, 8>(gp, k, weighted, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bf16_gather(const GatherPlan &gp, const GatherArgs &a, hipStream_t st);

KArgs make_kargs(const GatherPlan &gp, const GatherArgs &a) {
    KArgs k{};
    k.mi = a.mi;
    k.X = a.X;
    k.A = a.A;
    k.idx = a.idx;
    k.w = a.w;
    if (a.cdf) {
        k.cdf = *a.cdf;
        k.use_cdf = 1;
    }
    k.seed = a.seed;
    k.t = a.t;
    k.t_dev = a.t_dev;
    k.wpart = a.wpart;
    k.vpart = a.vpart;
    k.R = gp.R;
    k.S = gp.S;
    k.In = gp.In;
    k.ncols = gp.ncols;
    k.kc = gp.kc;
    k.rows_wg = gp.rows_wg;
    k.per_split = gp.per_split;
    return k;
}

hipError_t launch_gather(const GatherPlan &gp, const GatherArgs &a, hipStream_t st) {
    if (gp.kind == K_BF16) return launch_bf16_gather(gp, a, st);
    const KArgs k = make_kargs(gp, a);
    const bool weighted = (a.idx && a.w) || (!a.idx && a.cdf);
    if (gp.stream) return launch_gather_stream(gp, k, weighted, st);
    switch (gp.kind) {
        case K_F32: return launch_t<float, false>(gp, k, weighted, st);
        case K_F64: return launch_t<double, false>(gp, k, weighted, st);
        case K_C64: return launch_t<float, true>(gp, k, false, st);
        case K_C128: return launch_t<double, true>(gp, k, false, st);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Partial-product reductions.  Every sum runs in partial order; when there
// are many partials, groups of kGroup consecutive partials are first summed
// in place (group g written over its first partial, in parallel over groups
// and elements), and the group sums are then added in group order.

constexpr int kGroup = 32;

template <typename T>
__global__ __launch_bounds__(256) void group_sum_kernel(T *parts, int32_t np, int64_t count) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const int p0 = blockIdx.y * kGroup, p1 = min(np, p0 + kGroup);
    double acc = 0.0;
    int p = p0;
    for (; p + 8 <= p1; p += 8) {
        T v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = parts[(size_t)(p + k) * count + e];
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += (double)v[k];
    }
    for (; p < p1; ++p) acc += (double)parts[(size_t)p * count + e];
    parts[(size_t)p0 * count + e] = (T)acc;
}

// Sums groups of partials in place when np > kGroup; on return the partials
// to add are parts[p * pstride] for p < np.
static hipError_t group_presum(void *parts, bool dbl, int32_t &np, int64_t count, int64_t &pstride,
                               hipStream_t st) {
    pstride = count;
    if (np <= kGroup) return hipSuccess;
    const int ng = (int)ceil_div(np, kGroup);
    dim3 grid((unsigned)ceil_div(count, 256), (unsigned)ng);
    if (dbl)
        hipLaunchKernelGGL(group_sum_kernel<double>, grid, dim3(256), 0, st, (double *)parts, np, count);
    else
        hipLaunchKernelGGL(group_sum_kernel<float>, grid, dim3(256), 0, st, (float *)parts, np, count);
    np = ng;
    pstride = count * kGroup;
    return hipGetLastError();
}

// Reduce partials into row-major W and V (real kinds).
template <typename T>
__global__ __launch_bounds__(256) void reduce_wv_kernel(const T *wpart, int64_t wstride, const double *vpart,
                                                        int64_t vstride, int32_t wchunks, int32_t vchunks,
                                                        int32_t In, int32_t R, T *W, double *V) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nw = (int64_t)In * R;
    if (e < nw) {
        if (!W) return;
        const int64_t i = e / R, r = e - i * R;
        double acc = 0.0;
        for (int c = 0; c < wchunks; ++c) acc += (double)wpart[(size_t)c * wstride + r * In + i];
        W[e] = (T)acc;
    } else if (e < nw + (int64_t)R * R) {
        const int64_t p = e - nw;
        double acc = 0.0;
        for (int c = 0; c < vchunks; ++c) acc += vpart[(size_t)c * vstride + p];
        V[p] = acc;
    }
}

// out[e] = sum over p of parts[p * pstride + e], in order.
template <typename T>
__global__ __launch_bounds__(256) void sum_parts_kernel(const T *parts, int32_t np, int64_t count, int64_t pstride,
                                                        T *out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    double acc = 0.0;
    for (int p = 0; p < np; ++p) acc += (double)parts[(size_t)p * pstride + e];
    out[e] = (T)acc;
}

// out[e] (FP64) = sum over p of parts[p * pstride + e], in order.
template <typename T>
__global__ __launch_bounds__(256) void sum_parts_f64_kernel(const T *parts, int32_t np, int64_t count,
                                                            int64_t pstride, double *out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    double acc = 0.0;
    for (int p = 0; p < np; ++p) acc += (double)parts[(size_t)p * pstride + e];
    out[e] = acc;
}

hipError_t launch_sum_parts_f64(const void *parts, int32_t np, int64_t count, bool in_double, double *out,
                                hipStream_t st) {
    int64_t ps = count;
    hipError_t e = group_presum(const_cast<void *>(parts), in_double, np, count, ps, st);
    if (e != hipSuccess) return e;
    const int nb = (int)ceil_div(count, 256);
    if (in_double)
        hipLaunchKernelGGL(sum_parts_f64_kernel<double>, dim3(nb), dim3(256), 0, st, (const double *)parts, np, count,
                           ps, out);
    else
        hipLaunchKernelGGL(sum_parts_f64_kernel<float>, dim3(nb), dim3(256), 0, st, (const float *)parts, np, count,
                           ps, out);
    return hipGetLastError();
}

hipError_t launch_sum_parts(const void *parts, int32_t np, int64_t count, bool dbl, void *out, hipStream_t st) {
    int64_t ps = count;
    hipError_t e = group_presum(const_cast<void *>(parts), dbl, np, count, ps, st);
    if (e != hipSuccess) return e;
    const int nb = (int)ceil_div(count, 256);
    if (dbl)
        hipLaunchKernelGGL(sum_parts_kernel<double>, dim3(nb), dim3(256), 0, st, (const double *)parts, np, count, ps,
                           (double *)out);
    else
        hipLaunchKernelGGL(sum_parts_kernel<float>, dim3(nb), dim3(256), 0, st, (const float *)parts, np, count, ps,
                           (float *)out);
    return hipGetLastError();
}

hipError_t launch_reduce_wv(const GatherPlan &gp, const void *wpart, const double *vpart,
                            void *W, double *V, hipStream_t st) {
    const bool dbl = gp.kind == K_F64 || gp.kind == K_C128;
    int32_t wc = gp.chunks, vc = gp.chunks;
    int64_t ws = (int64_t)gp.ncols * gp.In, vs = (int64_t)gp.R * gp.R;
    hipError_t e = hipSuccess;
    if (W && wpart) {
        // the chunk partials are [chunk][ncols][In]; presum over whole chunk slabs
        e = group_presum(const_cast<void *>(wpart), dbl, wc, ws, ws, st);
    }
    if (e == hipSuccess) e = group_presum(const_cast<double *>(vpart), true, vc, vs, vs, st);
    if (e != hipSuccess) return e;
    const int64_t tot = (int64_t)gp.In * gp.R + (int64_t)gp.R * gp.R;
    const int nb = (int)ceil_div(tot, 256);
    if (dbl)
        hipLaunchKernelGGL(reduce_wv_kernel<double>, dim3(nb), dim3(256), 0, st, (const double *)wpart, ws, vpart, vs,
                           wc, vc, gp.In, gp.R, (double *)W, V);
    else
        hipLaunchKernelGGL(reduce_wv_kernel<float>, dim3(nb), dim3(256), 0, st, (const float *)wpart, ws, vpart, vs,
                           wc, vc, gp.In, gp.R, (float *)W, V);
    return hipGetLastError();
}

}  // namespace cprand
