// The whole decomposition: CPRAND (Alg. 3) and CPRAND-MIX (Alg. 4) with the
// sampled fit estimate and the stopping rules of Section 3.4 / Section 4.2,
// plus the BF16 precision form.  A plan owns every device buffer, so a run
// allocates nothing; each outer iteration is a fixed kernel sequence
// (optionally replayed as a HIP graph) whose only host synchronisation is
// the 8-byte read of the fit estimate that the stopping rule needs.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <vector>

#include "api_internal.hpp"

namespace cprand {

int mix_tensor_impl(const cprand_tensor *X, const cprand_tensor *Xhat, uint64_t seed, int8_t *signs,
                    double *normX_out, void *workspace, size_t workspace_bytes, hipStream_t st) {
    if (!workspace || workspace_bytes < 4096 * 8)
        return set_error(CPRAND_EINVAL, "workspace of 32768 bytes needed");
    const int xk = kind_of(X->dtype);
    const bool dbl = kind_of(Xhat->dtype) == K_C128;
    const ModeInfo mi = mode_info(X, 0);
    hipError_t e = hipSuccess;
    FftPlan *fps[CPRAND_MAX_ORDER] = {};
    for (int m = 0; m < X->order; ++m) {
        fps[m] = fft_plan_get(X->dims[m], dbl, &e);
        if (!fps[m]) return set_error(CPRAND_EUNSUPPORTED, "mode %d length %lld does not factor into 2,3,5,7", m,
                                      (long long)X->dims[m]);
    }
    e = launch_signs(mi, seed, signs, st);
    if (e != hipSuccess) return hip_fail(e, "sign kernel");
    // ||X|| from the first pass when its kernel supports it, else its own pass
    int32_t np = 0;
    for (int m = 0; m < X->order; ++m) {
        MixExtras ex{};
        if (m == 0) ex.normsq_part = (double *)workspace;
        e = launch_mix_pass(fps[m], dbl, mi, X->data, xk, Xhat->data, m, m == 0, signs, &ex, st);
        if (e != hipSuccess) return hip_fail(e, "mix pass");
        if (m == 0) np = ex.nparts;
    }
    if (np == 0) e = launch_normsq_partial(mi, X->data, xk, (double *)workspace, &np, st);
    if (e == hipSuccess) e = launch_sqrt_sum((double *)workspace, np, normX_out, st);
    if (e != hipSuccess) return hip_fail(e, "norm kernels");
    return CPRAND_OK;
}

}  // namespace cprand

using namespace cprand;

struct View {
    void *data = nullptr;   // NULL: the caller's X (or the plan's X-hat) at run time
    bool own = false;
    bool from_xhat = false;
    int kind = 0;
    int64_t strides[CPRAND_MAX_ORDER] = {};
    int64_t ld = 0;
    bool contig = true;     // with data: fibers along the view's mode are unit-stride
};

struct cprand_plan {
    cprand_opts o{};
    int N = 0;
    int64_t dims[CPRAND_MAX_ORDER] = {};
    int64_t xstrides[CPRAND_MAX_ORDER] = {};
    int xkind = 0;
    int64_t P = 1;
    bool dbl = false, mix = false, bf16 = false, refine = false;
    // CPRAND-PREMIX: the loop runs plain CPRAND on xdct, the real DCT-mixed
    // tensor (column-major); istrides are the strides of the tensor the loop
    // iterates on (X's own, or xdct's)
    bool premix = false;
    void *xdct = nullptr;
    int64_t istrides[CPRAND_MAX_ORDER] = {};
    // BF16 form with refinement: whether the current iterations refine (all
    // of them with refine_every; else from the first stop-rule hit on)
    bool ref_now = true;
    int gkind = 0;
    View gview[CPRAND_MAX_ORDER], rview[CPRAND_MAX_ORDER];
    void *xhat = nullptr;
    int8_t *signs = nullptr;
    void *fac[CPRAND_MAX_ORDER] = {};
    void *fhat[CPRAND_MAX_ORDER] = {};
    double *lambda = nullptr;
    void *wpart = nullptr;
    void *rpart = nullptr;
    double *vpart = nullptr;
    double *vrpart = nullptr;
    double *colsq = nullptr;
    double *fitpart = nullptr;
    double *normpart = nullptr;
    double *normX = nullptr;
    double *hist_dev = nullptr;
    double *hist_host = nullptr;
    void *wtmp = nullptr;   // maxdim x R doubles: summed (or unmixed) MTTKRP of the split path
    double *vsum = nullptr; // R x R: summed Gram of the split path
    void *snapbuf[2] = {};   // factors + lambda after even / odd iterations (run-ahead loop)
    // samples of every mode step of the run, drawn at setup (direct-launch,
    // non-adaptive plans, when they fit in kPreSampleBytes)
    int32_t *pre_idx = nullptr;
    double *pre_w = nullptr;
    size_t snapbytes = 0;
    int32_t *frow = nullptr; // the fixed fit set: rows [P_hat][N] and tensor values [P_hat][2]
    double *fx = nullptr;
    // importance-weighted fit set (fit_beta > 0): entry weights, slice-energy
    // proposal tables and their fixed-point bins
    double *fw = nullptr;
    uint64_t *fcdf[CPRAND_MAX_ORDER] = {};
    unsigned long long *fbins = nullptr;
    void *ysum = nullptr;
    uint64_t *t_dev = nullptr;
    unsigned *counter = nullptr;
    double *hist_mapped = nullptr;  // device address of hist_host
    int32_t *info = nullptr;
    int64_t *seg_off = nullptr;
    // importance proposals recomputed every mode step (LEARNED / MARGINAL)
    bool adaptive = false;
    double *pstats = nullptr, *pH = nullptr, *pgpart = nullptr, *alpha_dev = nullptr;
    float *pscore[CPRAND_MAX_ORDER] = {};
    uint64_t *pcdf[CPRAND_MAX_ORDER] = {};
    // saved (factors, lambda) states for the proposal fallback: the iterate
    // with the best fit estimate, the start of a duel, the current proposal's
    // result in a duel
    void *snap_fac[3][CPRAND_MAX_ORDER] = {};
    double *snap_lambda[3] = {};
    std::vector<void *> allocs;
    hipStream_t cap = nullptr;
    hipStream_t fst = nullptr;       // the fit estimates of the direct-launch loop
    hipStream_t rst = nullptr;       // the FP32 refinement gathers, beside the BF16 gathers
    hipEvent_t ev_ref[2] = {};       // refinement gather: fork, join
    hipEvent_t ev_state[2] = {};     // iteration state complete (parity of t)
    hipEvent_t ev[4] = {};
    // setup timing: [0,1] norm, [2+2m, 3+2m] mix pass m, [2+2N+2m, 3+2N+2m] layout copy m
    hipEvent_t tev[2 + 4 * CPRAND_MAX_ORDER] = {};
    ~cprand_plan() {
        for (void *p : allocs) (void)hipFree(p);
        if (hist_host) (void)hipHostFree(hist_host);
        if (cap) (void)hipStreamDestroy(cap);
        if (fst) (void)hipStreamDestroy(fst);
        if (rst) (void)hipStreamDestroy(rst);
        for (auto &e : ev_ref)
            if (e) (void)hipEventDestroy(e);
        for (auto &e : ev_state)
            if (e) (void)hipEventDestroy(e);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto &e : tev)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace {

constexpr size_t kPreSampleBytes = (size_t)64 << 20;

hipError_t dalloc(cprand_plan *p, void **ptr, size_t bytes) {
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(ptr, bytes);
    if (e == hipSuccess) p->allocs.push_back(*ptr);
    return e;
}

int vec_elems(int kind) { return (int)(16 / elem_size(kind)); }

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// host stopping rule (Section 3.4 and the rules of Section 4.2): stop after
// iteration t (0-based) when t+1 >= max_iters, |F_t - F_{t-1}| <= tol,
// F_t >= fit_target, or the best F has not improved for `patience` steps.
struct Stop {
    const cprand_opts &o;
    bool have_prev = false;
    double prev = 0, best = -INFINITY;
    int since = 0;
    explicit Stop(const cprand_opts &oo) : o(oo) {}
    bool operator()(int t, double F) {
        bool stop = t + 1 >= o.max_iters;
        if (o.tol > 0 && have_prev && fabs(F - prev) <= o.tol) stop = true;
        if (o.fit_target <= 1.0 && F >= o.fit_target) stop = true;
        if (F > best) {
            best = F;
            since = 0;
        } else {
            ++since;
            if (o.patience > 0 && since >= o.patience) stop = true;
        }
        prev = F;
        have_prev = true;
        return stop;
    }
};

// Sample chunks of the in-loop gathers: the fused step sums at most
// kChunksFused partial products inside its workgroup; the split path sums
// up to kChunksSplit with separate coalesced kernels.
constexpr int kChunksFused = 8, kChunksSplit = 32;

const void *view_ptr(const cprand_plan *p, const View &v, const void *xdata) {
    if (v.data) return v.data;
    return v.from_xhat ? p->xhat : xdata;
}

// The sampled fit estimate of the current model: against X-hat and the mixed
// factors under mixing, else against X (Section 3.4).
FitArgs fit_args(const cprand_plan *p, const void *xdata) {
    const int N = p->N;
    FitArgs fa{};
    fa.mi.order = N;
    for (int m = 0; m < N; ++m) {
        fa.mi.dims[m] = p->dims[m];
        fa.mi.strides[m] = p->istrides[m];
        fa.A.p[m] = p->mix ? p->fhat[m] : p->fac[m];
    }
    if (p->mix) {
        int64_t s = 1;
        for (int m = 0; m < N; ++m) {
            fa.mi.strides[m] = s;
            s *= p->dims[m];
        }
        fa.X = p->xhat;
        fa.kind = p->dbl ? K_C128 : K_C64;
        fa.cplx = true;
    } else {
        fa.X = xdata;
        fa.kind = p->xkind;
        fa.cplx = false;
    }
    fa.fdouble = p->dbl;
    fa.lambda = p->lambda;
    fa.R = p->o.R;
    fa.P_hat = p->o.P_hat;
    fa.seed = p->o.seed;
    fa.part = p->fitpart;
    fa.counter = p->counter;
    fa.P = (double)p->P;
    fa.normX = p->normX;
    fa.hist = p->hist_dev;
    fa.hist_host = p->hist_mapped;
    fa.t_dev = p->t_dev;
    return fa;
}

// One outer iteration on `st`.
// Direct launches of a non-adaptive loop: iteration t passed by value; the
// steps also write the factors and lambda into snapshot buffer t mod 2, and
// the fit estimate of iteration t runs on fit_st from that copy, so the next
// iteration's gathers need not wait for it.
struct IterCtl {
    uint64_t t;
    hipStream_t fit_st;
    hipEvent_t ev_state;
};

// Segment m of snapshot buffer b: the factors (A-hat under mixing) in order,
// then lambda.
static char *snap_segment(const cprand_plan *p, int b, int m) {
    const size_t tsz = p->dbl ? 8 : 4;
    size_t off = 0;
    for (int k = 0; k < m; ++k) off += (size_t)p->dims[k] * p->o.R * tsz * (p->mix ? 2 : 1);
    return (char *)p->snapbuf[b] + off;
}

hipError_t enqueue_iteration(cprand_plan *p, const void *xdata, bool contig_x[CPRAND_MAX_ORDER], hipStream_t st,
                             const IterCtl *ic = nullptr) {
    hipError_t e = hipSuccess;
    const int N = p->N, R = p->o.R;
    const int sb = ic ? (int)(ic->t & 1) : 0;
    // the FP32 refinement gather and step run only in the refined phase
    const bool refine = p->refine && p->ref_now;
    for (int n = 0; n < N && e == hipSuccess; ++n) {
        const View &v = p->gview[n];
        const void *vd = view_ptr(p, v, xdata);
        const int64_t In = p->dims[n];
        // the whole post-gather step in one workgroup when it fits in LDS
        bool fused = step_finish_lds((int32_t)In, R, p->mix) <= 156 * 1024;
        const bool rcontig = refine && (p->rview[n].data ? true : contig_x[n]);
        GatherPlan gp = plan_gather(p->gkind, R, p->o.S, In, v.data ? v.contig : contig_x[n],
                                    fused ? kChunksFused : kChunksSplit);
        GatherPlan gr = refine ? plan_gather(K_F32, R, p->o.S, In, rcontig, fused ? kChunksFused : kChunksSplit)
                                  : GatherPlan{};
        if (fused && (gp.chunks > kChunksFused || (refine && gr.chunks > kChunksFused))) {
            // the LDS limit shrank the chunks: too many partials for the fused step
            fused = false;
            gp = plan_gather(p->gkind, R, p->o.S, In, v.data ? v.contig : contig_x[n], kChunksSplit);
            if (refine) gr = plan_gather(K_F32, R, p->o.S, In, rcontig, kChunksSplit);
        }
        GatherArgs ga{};
        ga.mi.order = N;
        ga.mi.n = n;
        for (int m = 0; m < N; ++m) {
            ga.mi.dims[m] = p->dims[m];
            ga.mi.strides[m] = v.strides[m];
            ga.A.p[m] = (m == n) ? nullptr : (p->mix ? p->fhat[m] : p->fac[m]);
        }
        ga.X = vd;
        CdfPtrs cdf{};
        if (p->o.proposal == CPRAND_PROPOSAL_TABLE) {
            for (int m = 0; m < N; ++m) cdf.p[m] = p->o.proposal_cdf[m];
            ga.cdf = &cdf;
        } else if (p->adaptive) {
            // proposals for the factors of this step from their current values
            const bool learned = p->o.proposal == CPRAND_PROPOSAL_LEARNED;
            const bool marginal = p->o.proposal == CPRAND_PROPOSAL_MARGINAL;
            ModeInfo pm{};
            pm.order = N;
            pm.n = n;
            FactorPtrs fp{};
            for (int m = 0; m < N; ++m) {
                pm.dims[m] = p->dims[m];
                pm.strides[m] = 1;
                fp.p[m] = (m == n) ? nullptr : p->fac[m];
            }
            e = launch_mode_stats(fp, pm, R, p->pstats, p->pgpart, marginal ? p->pH : nullptr, st);
            if (e == hipSuccess)
                e = launch_row_scores(fp, pm, R, p->pstats, marginal ? p->pH : nullptr, p->o.mlp_params, learned,
                                      p->pscore, nullptr, nullptr, nullptr, st);
            uint64_t *cd[CPRAND_MAX_ORDER] = {};
            for (int m = 0; m < N; ++m) cd[m] = (m == n) ? nullptr : p->pcdf[m];
            if (e == hipSuccess) e = launch_cdf(pm, p->pscore, 0.0, p->alpha_dev, cd, st);
            if (e != hipSuccess) break;
            for (int m = 0; m < N; ++m) cdf.p[m] = p->pcdf[m];
            ga.cdf = &cdf;
        }
        ga.seed = p->o.seed;
        if (ic) {
            ga.t = ic->t;
            ga.t_dev = nullptr;
            if (p->pre_idx) {  // drawn at setup
                const size_t y = (size_t)ic->t * N + n;
                ga.idx = p->pre_idx + y * p->o.S * N;
                ga.w = p->pre_w ? p->pre_w + y * p->o.S : nullptr;
            }
        } else {
            ga.t_dev = p->t_dev;
        }
        ga.wpart = p->wpart;
        ga.vpart = p->vpart;
        if (refine) {
            // the FP32 refinement gather (same samples, its own partials) on a
            // second stream, forked before and joined after the BF16 gather
            const View &rv = p->rview[n];
            GatherArgs g2 = ga;
            for (int m = 0; m < N; ++m) g2.mi.strides[m] = rv.strides[m];
            g2.X = view_ptr(p, rv, xdata);
            g2.wpart = p->rpart;
            g2.vpart = p->vrpart;
            e = hipEventRecord(p->ev_ref[0], st);
            if (e == hipSuccess) e = hipStreamWaitEvent(p->rst, p->ev_ref[0], 0);
            if (e == hipSuccess) e = launch_gather(gr, g2, p->rst);
            if (e == hipSuccess) e = hipEventRecord(p->ev_ref[1], p->rst);
        }
        if (e == hipSuccess) e = launch_gather(gp, ga, st);
        if (e == hipSuccess && refine) e = hipStreamWaitEvent(st, p->ev_ref[1], 0);
        if (e != hipSuccess) break;
        if (fused) {
            StepArgs sa{};
            sa.In = (int32_t)In;
            sa.R = R;
            sa.vpart = p->vpart;
            sa.vparts = gp.chunks;
            sa.W = p->wpart;
            sa.wparts = gp.chunks;
            sa.wps = (int64_t)gp.ncols * In;
            sa.wsi = 1;
            sa.wsr = In;
            sa.wdouble = p->dbl;
            sa.mix = p->mix;
            sa.sign = p->mix ? p->signs + p->seg_off[n] : nullptr;
            if (refine) {
                sa.Wref = (const float *)p->rpart;
                sa.wrefparts = gr.chunks;
                sa.rps = (int64_t)R * In;
                sa.rsi = 1;
                sa.rsr = In;
                sa.vref = p->vrpart;
                sa.vrefparts = gr.chunks;
            }
            sa.A = p->fac[n];
            sa.Ahat = p->mix ? p->fhat[n] : nullptr;
            sa.lambda = p->lambda;
            sa.info = p->info;
            if (ic) {
                sa.snapA = snap_segment(p, sb, n);
                sa.snap_lambda = (double *)snap_segment(p, sb, N);
            }
            e = launch_step_finish(sa, p->dbl, st);
            continue;
        }
        // the split path: partial products summed by coalesced FP64 kernels first
        SolveArgs sa{};
        sa.In = (int32_t)In;
        sa.R = R;
        sa.vpart = p->vpart;
        sa.vparts = gp.chunks;
        if (gp.chunks > 1) {
            e = launch_sum_parts_f64(p->vpart, gp.chunks, (int64_t)R * R, true, p->vsum, st);
            sa.vpart = p->vsum;
            sa.vparts = 1;
        }
        if (e == hipSuccess && p->mix) {
            const void *y = p->wpart;
            int32_t np = gp.chunks;
            if (np > 8) {
                e = launch_sum_parts(p->wpart, np, (int64_t)2 * R * In, p->dbl, p->ysum, st);
                y = p->ysum;
                np = 1;
            }
            if (e == hipSuccess) {
                FftPlan *fp = fft_plan_get(In, p->dbl, &e);
                if (fp) e = launch_unmix(fp, p->dbl, (int32_t)In, R, np, y, p->signs + p->seg_off[n], p->wtmp, false, st);
            }
            sa.W = p->wtmp;
            sa.wparts = 1;
            sa.wps = 0;
            sa.wdouble = p->dbl;
        } else if (e == hipSuccess) {
            e = launch_sum_parts_f64(p->wpart, gp.chunks, (int64_t)R * In, p->dbl, (double *)p->wtmp, st);
            sa.W = p->wtmp;
            sa.wparts = 1;
            sa.wps = 0;
            sa.wdouble = true;
        }
        sa.wsi = 1;
        sa.wsr = In;
        if (refine) {
            sa.Wref = (const float *)p->rpart;
            sa.wrefparts = gr.chunks;
            sa.rps = (int64_t)R * In;
            sa.rsi = 1;
            sa.rsr = In;
            sa.vref = p->vrpart;
            sa.vrefparts = gr.chunks;
        }
        sa.A = p->fac[n];
        sa.adouble = p->dbl;
        sa.colsq_part = p->colsq;
        sa.info = p->info;
        sa.info_sticky = 1;
        int32_t nb = 0;
        if (e == hipSuccess) e = launch_solve(sa, &nb, st);
        if (e == hipSuccess) e = launch_normalize((int32_t)In, R, p->fac[n], p->dbl, p->colsq, nb, p->lambda, st);
        if (e == hipSuccess && p->mix) {
            FftPlan *fp = fft_plan_get(In, p->dbl, &e);
            if (fp) e = launch_factor_mix(fp, p->dbl, (int32_t)In, R, p->fac[n], p->signs + p->seg_off[n], p->fhat[n],
                                          false, st);
        }
        if (e == hipSuccess && ic) {
            const size_t b = (size_t)In * R * (p->dbl ? 8 : 4) * (p->mix ? 2 : 1);
            e = hipMemcpyAsync(snap_segment(p, sb, n), p->mix ? p->fhat[n] : p->fac[n], b, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(snap_segment(p, sb, N), p->lambda, (size_t)R * 8, hipMemcpyDeviceToDevice, st);
        }
    }
    if (e != hipSuccess) return e;
    FitArgs fa = fit_args(p, xdata);
    fa.frow = p->frow;
    fa.fx = p->fx;
    fa.fw = p->fw;
    if (ic) {
        // iteration t's state is in snapshot buffer t mod 2: estimate from it on the fit stream
        for (int m = 0; m < N; ++m) fa.A.p[m] = snap_segment(p, sb, m);
        fa.lambda = (const double *)snap_segment(p, sb, N);
        fa.t_dev = nullptr;
        fa.t = ic->t;
        e = hipEventRecord(ic->ev_state, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(ic->fit_st, ic->ev_state, 0);
        int32_t nb = 0;
        if (e == hipSuccess) e = launch_fit_partial(fa, &nb, ic->fit_st);
        return e;
    }
    if (!p->adaptive) {
        const size_t tsz = p->dbl ? 8 : 4;
        for (int m = 0; m < N; ++m) {  // under mixing the state is A-hat (A is formed at the end)
            fa.snap.src[m] = p->mix ? p->fhat[m] : p->fac[m];
            fa.snap.words[m] = (int64_t)(p->dims[m] * R * tsz * (p->mix ? 2 : 1) / 4);
        }
        fa.snap.nsrc = N;
        fa.snap.lambda = p->lambda;
        fa.snap.R = R;
        fa.snap.dst0 = p->snapbuf[0];
        fa.snap.dst1 = p->snapbuf[1];
    }
    int32_t nb = 0;
    e = launch_fit_partial(fa, &nb, st);
    return e;
}

}  // namespace

extern "C" {

int cprand_plan_create(const cprand_tensor *X, const cprand_opts *opts, cprand_plan **plan_out) {
    g_last_error.clear();
    if (!plan_out) return set_error(CPRAND_EINVAL, "plan is NULL");
    *plan_out = nullptr;
    if (!X || !opts) return set_error(CPRAND_EINVAL, "X and opts must be non-NULL");
    if (X->order < 2 || X->order > CPRAND_MAX_ORDER) return set_error(CPRAND_EINVAL, "order outside [2, 8]");
    const int xk = kind_of(X->dtype);
    if (xk != K_F32 && xk != K_F64) return set_error(CPRAND_EINVAL, "X must be F32 or F64");
    for (int m = 0; m < X->order; ++m) {
        if (X->dims[m] < 1 || X->dims[m] > (int64_t)INT32_MAX) return set_error(CPRAND_EINVAL, "dims[%d] invalid", m);
        if (X->strides[m] < 1) return set_error(CPRAND_EINVAL, "strides[%d] < 1", m);
    }
    const cprand_opts &o = *opts;
    if (o.R < 1 || o.R > CPRAND_MAX_RANK) return set_error(CPRAND_EINVAL, "R = %d outside [1, %d]", o.R, CPRAND_MAX_RANK);
    if (o.S < 1) return set_error(CPRAND_EINVAL, "S = %d < 1", o.S);
    if (o.P_hat < 1) return set_error(CPRAND_EINVAL, "P_hat = %d < 1", o.P_hat);
    if (o.max_iters < 1) return set_error(CPRAND_EINVAL, "max_iters = %d < 1", o.max_iters);
    if (o.mix != CPRAND_MIX_NONE && o.mix != CPRAND_MIX_FFT && o.mix != CPRAND_MIX_DCT)
        return set_error(CPRAND_EINVAL, "mix = %d", o.mix);
    const bool cmix = o.mix == CPRAND_MIX_FFT;  // complex mixing (CPRAND-MIX)
    if (o.precision < 0 || o.precision > 2) return set_error(CPRAND_EINVAL, "precision = %d", o.precision);
    if (o.precision != CPRAND_PREC_NATIVE && xk != K_F32)
        return set_error(CPRAND_EINVAL, "the BF16 form reads an F32 tensor");
    if (o.precision != CPRAND_PREC_NATIVE && cmix) return set_error(CPRAND_EUNSUPPORTED, "BF16 with FFT mixing");
    if (!(o.fit_beta >= 0.0 && o.fit_beta < 1.0)) return set_error(CPRAND_EINVAL, "fit_beta outside [0, 1)");
    if (o.fit_beta > 0.0 && !(o.fit_alpha > 0.0 && o.fit_alpha <= 1.0))
        return set_error(CPRAND_EINVAL, "fit_alpha outside (0, 1]");
    if (o.fit_beta > 0.0 && cmix) return set_error(CPRAND_EUNSUPPORTED, "a weighted fit set with FFT mixing");
    if (o.proposal == CPRAND_PROPOSAL_TABLE) {
        if (!o.proposal_cdf) return set_error(CPRAND_EINVAL, "PROPOSAL_TABLE needs proposal_cdf");
        for (int m = 0; m < X->order; ++m)
            if (!o.proposal_cdf[m]) return set_error(CPRAND_EINVAL, "proposal_cdf[%d] is NULL", m);
        if (cmix) return set_error(CPRAND_EUNSUPPORTED, "importance sampling with FFT mixing");
    } else if (o.proposal == CPRAND_PROPOSAL_LEARNED || o.proposal == CPRAND_PROPOSAL_MARGINAL ||
               o.proposal == CPRAND_PROPOSAL_LEVERAGE) {
        if (o.proposal == CPRAND_PROPOSAL_LEARNED && !o.mlp_params)
            return set_error(CPRAND_EINVAL, "PROPOSAL_LEARNED needs mlp_params");
        if (xk != K_F32) return set_error(CPRAND_EUNSUPPORTED, "adaptive proposals read FP32 factors");
        if (cmix) return set_error(CPRAND_EUNSUPPORTED, "importance sampling with FFT mixing");
        if (!(o.alpha >= 0.0 && o.alpha <= 1.0)) return set_error(CPRAND_EINVAL, "alpha outside [0, 1]");
    } else if (o.proposal != CPRAND_PROPOSAL_UNIFORM) {
        return set_error(CPRAND_EINVAL, "proposal %d", o.proposal);
    }
    if (cmix && !is_colmajor(X)) return set_error(CPRAND_EUNSUPPORTED, "FFT mixing needs a column-major X");
    cprand_plan *p = new cprand_plan();
    p->o = o;
    p->N = X->order;
    p->xkind = xk;
    p->dbl = xk == K_F64;
    p->mix = cmix;
    p->premix = o.mix == CPRAND_MIX_DCT;
    p->bf16 = o.precision != CPRAND_PREC_NATIVE;
    p->refine = o.precision == CPRAND_PREC_BF16_REFINE;
    for (int m = 0; m < p->N; ++m) {
        p->dims[m] = X->dims[m];
        p->xstrides[m] = X->strides[m];
        p->istrides[m] = p->premix ? p->P : X->strides[m];
        p->P *= X->dims[m];
    }
    const int N = p->N, R = o.R;
    if (p->premix) {
        // the DCT pass keeps one tile of two real fibers, the complex FFT tiles
        // and the post-rotation table in LDS
        const int64_t dct_max = p->dbl ? 1706 : 3413;
        for (int m = 0; m < N; ++m)
            if (p->dims[m] > dct_max && p->dims[m] != 400 && p->dims[m] != 150 && p->dims[m] != 60) {
                delete p;
                return set_error(CPRAND_EUNSUPPORTED, "mode %d length %lld is too long for the DCT pass", m,
                                 (long long)X->dims[m]);
            }
    }
    if (p->mix || p->premix) {
        for (int m = 0; m < N; ++m) {
            hipError_t fe;
            if (!fft_plan_get(p->dims[m], p->dbl, &fe)) {
                delete p;
                return set_error(CPRAND_EUNSUPPORTED, "mode %d length %lld does not factor into 2,3,5,7", m,
                                 (long long)X->dims[m]);
            }
        }
    }
    p->gkind = p->mix ? (p->dbl ? K_C128 : K_C64) : (p->bf16 ? K_BF16 : xk);
    hipError_t e = hipSuccess;
    const size_t tsz = p->dbl ? 8 : 4;
    auto alloc_copy = [&](View &v, int kind, int n) -> hipError_t {
        v.own = true;
        v.kind = kind;
        v.ld = round_up(p->dims[n], vec_elems(kind));
        cprand_mode_major_strides(N, p->dims, n, v.ld, v.strides);
        return dalloc(p, &v.data, (size_t)(p->P / p->dims[n]) * v.ld * elem_size(kind));
    };
    if (p->mix) {
        e = dalloc(p, &p->xhat, (size_t)p->P * elem_size(p->gkind));
        int64_t s = 1;
        for (int n = 0; n < N && e == hipSuccess; ++n) {
            View &v = p->gview[n];
            const bool use_xhat = o.layout == 1 || (n == 0 && p->dims[0] % vec_elems(p->gkind) == 0);
            if (use_xhat) {
                v.from_xhat = true;
                v.kind = p->gkind;
                int64_t st = 1;
                for (int m = 0; m < N; ++m) {
                    v.strides[m] = st;
                    st *= p->dims[m];
                }
            } else {
                e = alloc_copy(v, p->gkind, n);
            }
        }
        (void)s;
    } else {
        for (int n = 0; n < N && e == hipSuccess; ++n) {
            if (p->bf16) {
                if (o.layout == 1 && n > 0) {
                    // strided BF16 gathers from the mode-0 copy: one conversion of X
                    // instead of a mode-major copy per mode
                    View &v = p->gview[n];
                    v = p->gview[0];
                    v.own = false;
                    v.contig = false;
                } else {
                    e = alloc_copy(p->gview[n], K_BF16, n);
                    if (e != hipSuccess) break;
                }
            }
            View &v = p->bf16 ? p->rview[n] : p->gview[n];
            if (p->bf16 && !p->refine) continue;
            const int ve = vec_elems(xk);
            bool ok = o.layout == 1 || p->istrides[n] == 1;
            for (int m = 0; m < N && ok && o.layout != 1; ++m)
                if (m != n && p->istrides[m] % ve) ok = false;
            if (ok) {
                v.kind = xk;
                for (int m = 0; m < N; ++m) v.strides[m] = p->istrides[m];
            } else {
                if (!p->premix && !is_colmajor(X)) {
                    delete p;
                    return set_error(CPRAND_EUNSUPPORTED, "layout copies read a column-major X");
                }
                e = alloc_copy(v, xk, n);
            }
        }
    }
    if (e == hipSuccess && p->premix) e = dalloc(p, &p->xdct, (size_t)p->P * tsz);
    if (e == hipSuccess) {
        int64_t tot = 0;
        for (int m = 0; m < N; ++m) tot += p->dims[m];
        e = dalloc(p, (void **)&p->signs, (size_t)tot);
        p->seg_off = new int64_t[N];
        int64_t off = 0;
        for (int m = 0; m < N; ++m) {
            p->seg_off[m] = off;
            off += p->dims[m];
        }
    }
    size_t wpart = 0, vpart = 0, rpart = 0;
    int64_t maxdim = 1;
    for (int n = 0; n < N; ++n) {
        for (int maxc : {kChunksSplit, kChunksFused}) {  // the split path and the fused path
            GatherPlan gp = plan_gather(p->gkind, R, o.S, p->dims[n], true, maxc);
            const size_t gts = (p->gkind == K_F64 || p->gkind == K_C128) ? 8 : 4;
            wpart = std::max(wpart, gp.wpart_elems() * gts);
            vpart = std::max(vpart, gp.vpart_elems() * 8);
            if (p->refine) {
                GatherPlan gr = plan_gather(K_F32, R, o.S, p->dims[n], true, maxc);
                rpart = std::max(rpart, gr.wpart_elems() * 4);
                vpart = std::max(vpart, gr.vpart_elems() * 8);
            }
        }
        maxdim = std::max(maxdim, p->dims[n]);
    }
    for (int m = 0; m < N && e == hipSuccess; ++m) {
        e = dalloc(p, &p->fac[m], (size_t)p->dims[m] * R * tsz);
        if (e == hipSuccess && p->mix) e = dalloc(p, &p->fhat[m], (size_t)p->dims[m] * R * tsz * 2);
    }
    if (e == hipSuccess) e = dalloc(p, (void **)&p->lambda, (size_t)R * 8);
    if (e == hipSuccess) e = dalloc(p, &p->wpart, wpart);
    if (e == hipSuccess) e = dalloc(p, (void **)&p->vpart, vpart);
    if (e == hipSuccess && p->refine) e = dalloc(p, &p->rpart, rpart);
    if (e == hipSuccess && p->refine) e = dalloc(p, (void **)&p->vrpart, vpart * 2 + 256);
    if (e == hipSuccess) e = dalloc(p, (void **)&p->colsq, (size_t)ceil_div(maxdim, 32) * R * 8);
    if (e == hipSuccess) e = dalloc(p, (void **)&p->fitpart, (size_t)fit_partials(o.P_hat) * 8);
    if (e == hipSuccess) e = dalloc(p, (void **)&p->normpart, 4096 * 8);
    if (e == hipSuccess) e = dalloc(p, (void **)&p->normX, 8);
    if (e == hipSuccess) e = dalloc(p, (void **)&p->hist_dev, (size_t)o.max_iters * 8);
    if (e == hipSuccess) e = dalloc(p, &p->wtmp, (size_t)maxdim * R * 8);
    if (e == hipSuccess) e = dalloc(p, (void **)&p->vsum, (size_t)R * R * 8);
    if (e == hipSuccess) e = dalloc(p, (void **)&p->frow, (size_t)o.P_hat * N * 4);
    if (e == hipSuccess) {
        p->snapbytes = (size_t)R * 8;
        for (int m = 0; m < N; ++m) p->snapbytes += (size_t)p->dims[m] * R * tsz * (p->mix ? 2 : 1);
        e = dalloc(p, &p->snapbuf[0], p->snapbytes);
        if (e == hipSuccess) e = dalloc(p, &p->snapbuf[1], p->snapbytes);
    }
    if (e == hipSuccess) e = dalloc(p, (void **)&p->fx, (size_t)o.P_hat * 16);
    if (e == hipSuccess && o.fit_beta > 0.0) {
        e = dalloc(p, (void **)&p->fw, (size_t)o.P_hat * 8);
        int64_t tot = 0;
        for (int m = 0; m < N && e == hipSuccess; ++m) {
            e = dalloc(p, (void **)&p->fcdf[m], (size_t)(p->dims[m] + 1) * 8);
            tot += p->dims[m];
        }
        if (e == hipSuccess) e = dalloc(p, (void **)&p->fbins, (size_t)tot * 8);
    }
    if (e == hipSuccess && p->mix) e = dalloc(p, &p->ysum, (size_t)maxdim * 2 * R * tsz);
    p->adaptive = o.proposal == CPRAND_PROPOSAL_LEARNED || o.proposal == CPRAND_PROPOSAL_MARGINAL ||
                  o.proposal == CPRAND_PROPOSAL_LEVERAGE;
    {
        // the samples depend only on (seed, t, n) unless the proposal adapts:
        // draw them all at setup for direct-launch loops
        const size_t steps = (size_t)o.max_iters * N;
        const size_t bytes = steps * o.S * N * 4 + (o.proposal == CPRAND_PROPOSAL_TABLE ? steps * o.S * 8 : 0);
        if (e == hipSuccess && !p->adaptive && !o.use_graph && bytes <= kPreSampleBytes && steps <= 65535) {
            e = dalloc(p, (void **)&p->pre_idx, steps * o.S * N * 4);
            if (e == hipSuccess && o.proposal == CPRAND_PROPOSAL_TABLE)
                e = dalloc(p, (void **)&p->pre_w, steps * o.S * 8);
        }
    }
    if (e == hipSuccess && p->adaptive) {
        e = dalloc(p, (void **)&p->pstats, (size_t)N * mode_stats_doubles(R) * 8);
        if (e == hipSuccess) e = dalloc(p, (void **)&p->pH, (size_t)R * R * 8);
        if (e == hipSuccess) e = dalloc(p, (void **)&p->pgpart, gram_part_doubles(N, R) * 8);
        for (int m = 0; m < N && e == hipSuccess; ++m) {
            e = dalloc(p, (void **)&p->pscore[m], (size_t)p->dims[m] * 4);
            if (e == hipSuccess) e = dalloc(p, (void **)&p->pcdf[m], (size_t)(p->dims[m] + 1) * 8);
        }
        if (e == hipSuccess) e = dalloc(p, (void **)&p->alpha_dev, 8);
        for (int k = 0; k < 3 && e == hipSuccess; ++k) {
            for (int m = 0; m < N && e == hipSuccess; ++m)
                e = dalloc(p, &p->snap_fac[k][m], (size_t)p->dims[m] * R * tsz);
            if (e == hipSuccess) e = dalloc(p, (void **)&p->snap_lambda[k], (size_t)R * 8);
        }
    }
    if (e == hipSuccess) e = dalloc(p, (void **)&p->t_dev, 8);
    if (e == hipSuccess) e = dalloc(p, (void **)&p->counter, 8);
    if (e == hipSuccess) e = dalloc(p, (void **)&p->info, 8);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&p->hist_host, (size_t)o.max_iters * 8, hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&p->hist_mapped, p->hist_host, 0);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->fst, hipStreamNonBlocking);
    if (e == hipSuccess && p->refine) e = hipStreamCreateWithFlags(&p->rst, hipStreamNonBlocking);
    for (int i = 0; i < 2 && e == hipSuccess && p->refine; ++i)
        e = hipEventCreateWithFlags(&p->ev_ref[i], hipEventDisableTiming);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&p->ev_state[i], hipEventDisableTiming);
    for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreate(&p->ev[i]);
    for (int i = 0; i < 2 + 4 * CPRAND_MAX_ORDER && e == hipSuccess; ++i) e = hipEventCreate(&p->tev[i]);
    if (e != hipSuccess) {
        delete p;
        if (e == hipErrorOutOfMemory) return set_error(CPRAND_ENOMEM, "device allocation failed");
        return hip_fail(e, "plan allocation");
    }
    *plan_out = p;
    return CPRAND_OK;
}

void cprand_plan_destroy(cprand_plan *plan) {
    if (!plan) return;
    delete[] plan->seg_off;
    delete plan;
}

int cprand_plan_run(cprand_plan *p, const cprand_tensor *X, void *const *A_inout, double *lambda_out,
                    cprand_report *rep, void *stream) {
    g_last_error.clear();
    if (!p) return set_error(CPRAND_EINVAL, "plan is NULL");
    int rc = check_tensor(X, "X");
    if (rc) return rc;
    if (X->order != p->N || kind_of(X->dtype) != p->xkind) return set_error(CPRAND_EINVAL, "X differs from the plan");
    for (int m = 0; m < p->N; ++m)
        if (X->dims[m] != p->dims[m] || X->strides[m] != p->xstrides[m])
            return set_error(CPRAND_EINVAL, "X shape or strides differ from the plan");
    if (!A_inout || !lambda_out) return set_error(CPRAND_EINVAL, "A_inout and lambda_out must be non-NULL");
    for (int m = 0; m < p->N; ++m)
        if (!A_inout[m]) return set_error(CPRAND_EINVAL, "A_inout[%d] is NULL", m);
    hipStream_t st = (hipStream_t)stream;
    const int N = p->N, R = p->o.R;
    const size_t tsz = p->dbl ? 8 : 4;
    hipError_t e = hipSuccess;
    // the real tensor the loop iterates on: X, or its DCT-mixed copy
    const void *xit = p->premix ? p->xdct : X->data;
    ModeInfo xit_i = mode_info(X, 0);
    for (int m = 0; m < N; ++m) xit_i.strides[m] = p->istrides[m];
    bool contig_x[CPRAND_MAX_ORDER];
    for (int n = 0; n < N; ++n) {
        const View &v = p->mix ? p->gview[n] : (p->bf16 ? p->rview[n] : p->gview[n]);
        contig_x[n] = fibers_vectorizable(p->mix ? p->xhat : xit, p->mix ? p->gkind : p->xkind, v.strides, N, n);
    }

    e = hipEventRecord(p->ev[0], st);
    for (int m = 1; m < N && e == hipSuccess && !p->premix; ++m)
        e = hipMemcpyAsync(p->fac[m], A_inout[m], (size_t)p->dims[m] * R * tsz, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = launch_fill_u64(p->t_dev, 0, st);
    if (e == hipSuccess) e = launch_fill_u64((uint64_t *)p->info, 0, st);
    if (e == hipSuccess) e = launch_fill_u64((uint64_t *)p->counter, 0, st);
    if (e == hipSuccess && p->adaptive) {
        uint64_t bits;
        memcpy(&bits, &p->o.alpha, 8);
        e = launch_fill_u64((uint64_t *)p->alpha_dev, bits, st);
    }
    ModeInfo xi = mode_info(X, 0);
    bool timed_mix[CPRAND_MAX_ORDER] = {}, timed_lay[CPRAND_MAX_ORDER] = {};
    hipEvent_t *tev = p->tev;
    // ||X||: folded into the first mixing pass when its kernel supports it
    // (it reads all of X anyway), else a pass of its own
    bool norm_done = false, copied_last = false;
    if (e == hipSuccess && p->mix) {
        e = launch_signs(xi, p->o.seed, p->signs, st);
        for (int m = 0; m < N && e == hipSuccess; ++m) {
            FftPlan *fp = fft_plan_get(p->dims[m], p->dbl, &e);
            MixExtras ex{};
            if (m == 0) ex.normsq_part = p->normpart;
            if (m == N - 1 && p->gview[m].own) {  // the last pass can also write mode m's mode-major copy
                ex.copy = p->gview[m].data;
                ex.copy_ld = p->gview[m].ld;
            }
            if (fp) e = hipEventRecord(tev[2 + 2 * m], st);
            if (fp && e == hipSuccess)
                e = launch_mix_pass(fp, p->dbl, xi, X->data, p->xkind, p->xhat, m, m == 0, p->signs, &ex, st);
            if (fp && e == hipSuccess) e = hipEventRecord(tev[3 + 2 * m], st);
            timed_mix[m] = e == hipSuccess;
            if (e == hipSuccess && m == 0 && ex.nparts > 0) {
                e = hipEventRecord(tev[0], st);
                if (e == hipSuccess) e = launch_sqrt_sum(p->normpart, ex.nparts, p->normX, st);
                if (e == hipSuccess) e = hipEventRecord(tev[1], st);
                norm_done = e == hipSuccess;
            }
            if (m == N - 1) copied_last = ex.copied;
        }
        cprand_tensor xh{};
        xh.order = N;
        xh.dtype = p->dbl ? CPRAND_C128 : CPRAND_C64;
        int64_t s = 1;
        for (int m = 0; m < N; ++m) {
            xh.dims[m] = p->dims[m];
            xh.strides[m] = s;
            s *= p->dims[m];
        }
        xh.data = p->xhat;
        ModeInfo hi = mode_info(&xh, 0);
        for (int n = 0; n < N && e == hipSuccess; ++n)
            if (p->gview[n].own && !(n == N - 1 && copied_last)) {
                e = hipEventRecord(tev[2 + 2 * N + 2 * n], st);
                if (e == hipSuccess)
                    e = launch_layout_copy(hi, p->xhat, p->gkind, n, p->gview[n].ld, p->gview[n].data, p->gkind, st);
                if (e == hipSuccess) e = hipEventRecord(tev[3 + 2 * N + 2 * n], st);
                timed_lay[n] = e == hipSuccess;
            }
        for (int m = 1; m < N && e == hipSuccess; ++m) {
            FftPlan *fp = fft_plan_get(p->dims[m], p->dbl, &e);
            if (fp) e = launch_factor_mix(fp, p->dbl, (int32_t)p->dims[m], R, p->fac[m], p->signs + p->seg_off[m],
                                          p->fhat[m], false, st);
        }
    } else if (e == hipSuccess) {
        if (p->premix) {
            // CPRAND-PREMIX (Alg. 5): mix X once with the real DCT, and the
            // initial factors with it, then iterate on the mixed tensor
            e = launch_signs(xi, p->o.seed, p->signs, st);
            for (int m = 0; m < N && e == hipSuccess; ++m) {
                MixExtras ex{};
                if (m == 0) ex.normsq_part = p->normpart;  // ||X|| folded into the first pass
                e = hipEventRecord(tev[2 + 2 * m], st);
                if (e == hipSuccess)
                    e = launch_dct_pass(m == 0 ? xi : xit_i, X->data, p->xkind, p->xdct, p->dbl, m, m == 0, p->signs,
                                        st, m == 0 ? &ex : nullptr);
                if (e == hipSuccess) e = hipEventRecord(tev[3 + 2 * m], st);
                timed_mix[m] = e == hipSuccess;
                if (e == hipSuccess && m == 0 && ex.nparts > 0) {
                    e = hipEventRecord(tev[0], st);
                    if (e == hipSuccess) e = launch_sqrt_sum(p->normpart, ex.nparts, p->normX, st);
                    if (e == hipSuccess) e = hipEventRecord(tev[1], st);
                    norm_done = e == hipSuccess;
                }
            }
            for (int m = 1; m < N && e == hipSuccess; ++m)
                e = launch_factor_dct((int32_t)p->dims[m], R, A_inout[m], p->signs + p->seg_off[m], p->fac[m], p->dbl,
                                      false, st);
        }
        for (int n = 0; n < N && e == hipSuccess; ++n) {
            const bool any = p->gview[n].own || (p->refine && p->rview[n].own);
            if (any) e = hipEventRecord(tev[2 + 2 * N + 2 * n], st);
            if (e == hipSuccess && p->gview[n].own)
                e = launch_layout_copy(xit_i, xit, p->xkind, n, p->gview[n].ld, p->gview[n].data, p->gview[n].kind, st);
            if (e == hipSuccess && p->refine && p->rview[n].own)
                e = launch_layout_copy(xit_i, xit, p->xkind, n, p->rview[n].ld, p->rview[n].data, p->rview[n].kind, st);
            if (any && e == hipSuccess) e = hipEventRecord(tev[3 + 2 * N + 2 * n], st);
            timed_lay[n] = any && e == hipSuccess;
        }
    }
    if (e == hipSuccess && !norm_done) {
        int32_t np = 0;
        e = hipEventRecord(tev[0], st);
        if (e == hipSuccess) e = launch_normsq_partial(xi, X->data, p->xkind, p->normpart, &np, st);
        if (e == hipSuccess) e = launch_sqrt_sum(p->normpart, np, p->normX, st);
        if (e == hipSuccess) e = hipEventRecord(tev[1], st);
    }
    if (e == hipSuccess && p->pre_idx) {
        ModeInfo mi{};
        mi.order = N;
        for (int m = 0; m < N; ++m) {
            mi.dims[m] = p->dims[m];
            mi.strides[m] = 1;
        }
        CdfPtrs cdf{};
        if (p->o.proposal == CPRAND_PROPOSAL_TABLE)
            for (int m = 0; m < N; ++m) cdf.p[m] = p->o.proposal_cdf[m];
        e = launch_sample_all(mi, p->o.S, p->o.max_iters, p->o.seed,
                              p->o.proposal == CPRAND_PROPOSAL_TABLE ? &cdf : nullptr, p->pre_idx, p->pre_w, st);
    }
    // the fixed fit set: rows and tensor values drawn once per run
    if (e == hipSuccess && p->fw) {
        // the weighted fit set: slice-energy tables of the iterated tensor, then the draw
        CdfPtrs c{};
        for (int m = 0; m < N; ++m) c.p[m] = p->fcdf[m];
        e = launch_energy_tables(xit_i, xit, p->xkind, p->normX, p->fbins, p->o.fit_alpha, c, nullptr, st);
        if (e == hipSuccess)
            e = launch_fit_set_weighted(xit_i, xit, p->xkind, p->o.P_hat, p->o.seed, c, p->o.fit_beta, p->frow, p->fx,
                                        p->fw, st);
    } else if (e == hipSuccess) {
        e = launch_fit_set(fit_args(p, xit), p->frow, p->fx, st);
    }
    if (e == hipSuccess) e = hipEventRecord(p->ev[1], st);
    if (e != hipSuccess) return hip_fail(e, "setup");

    // The BF16 form with refinement follows a schedule unless refine_every
    // is set: BF16 solves only, until the stop rule first holds (or one
    // iteration before the cap), then refined solves until it holds again,
    // so at least the last iteration is refined.
    const bool sched = p->refine && !p->o.refine_every && p->o.max_iters > 1;
    p->ref_now = !sched;
    int refined_from = p->refine ? (sched ? -1 : 0) : -1;

    // the ALS loop: one graph per iteration kind (BF16-only and refined)
    hipGraphExec_t execs[2] = {nullptr, nullptr};
    hipGraph_t graphs[2] = {nullptr, nullptr};
    auto destroy_graphs = [&]() {
        for (int k = 0; k < 2; ++k) {
            if (execs[k]) (void)hipGraphExecDestroy(execs[k]);
            if (graphs[k]) (void)hipGraphDestroy(graphs[k]);
            execs[k] = nullptr;
            graphs[k] = nullptr;
        }
    };
    if (p->o.use_graph) {
        for (int k = sched ? 0 : 1; k < 2 && e == hipSuccess; ++k) {
            p->ref_now = k == 1;
            e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed);
            if (e == hipSuccess) {
                hipError_t e2 = enqueue_iteration(p, xit, contig_x, p->cap);
                e = hipStreamEndCapture(p->cap, &graphs[k]);
                if (e2 != hipSuccess) e = e2;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&execs[k], graphs[k], nullptr, nullptr, 0);
        }
        p->ref_now = !sched;
        if (e != hipSuccess) {
            destroy_graphs();
            return hip_fail(e, "graph capture");
        }
    }
    auto cur_exec = [&]() { return execs[p->ref_now ? 1 : 0]; };
    const bool graphed = p->o.use_graph != 0;
    Stop stop(p->o);
    int it = 0;
    double F = 0.0;
    // Adaptive proposals fall back learned -> mixture (alpha 0.5) -> uniform
    // (alpha 1, which reproduces uniform sampling exactly) when the sampled
    // fit estimate judges the current proposal worse, by either of two tests.
    //  - Duel: at t = 1, 3, 7, 15, ... one outer iteration is run with the
    //    current proposal and, from the same factors and with the same random
    //    counters, with uniform sampling; uniform sampling wins when its F-hat
    //    is higher by three standard deviations of the estimate,
    //    (1 - F)/sqrt(2 P-hat), and its residual 1 - F-hat is less than half.
    //    The winner's iterate is kept.
    //  - Decline: F-hat below the best so far by more than both three standard
    //    deviations and half the best residual, twice in a row; the proposal
    //    steps down one level and the run resumes from the factors of the best
    //    iterate.
    // The margins are wide because sampled ALS is not monotone: a good
    // proposal moves F-hat by up to about a third of the residual between
    // iterations.
    enum { SNAP_BEST = 0, SNAP_PRE = 1, SNAP_CUR = 2 };
    auto save = [&](int k) {
        hipError_t r = hipSuccess;
        for (int m = 0; m < N && r == hipSuccess; ++m)
            r = hipMemcpyAsync(p->snap_fac[k][m], p->fac[m], (size_t)p->dims[m] * R * tsz, hipMemcpyDeviceToDevice,
                               st);
        if (r == hipSuccess) r = hipMemcpyAsync(p->snap_lambda[k], p->lambda, (size_t)R * 8, hipMemcpyDeviceToDevice, st);
        return r;
    };
    auto load = [&](int k) {
        hipError_t r = hipSuccess;
        for (int m = 0; m < N && r == hipSuccess; ++m)
            r = hipMemcpyAsync(p->fac[m], p->snap_fac[k][m], (size_t)p->dims[m] * R * tsz, hipMemcpyDeviceToDevice,
                               st);
        if (r == hipSuccess) r = hipMemcpyAsync(p->lambda, p->snap_lambda[k], (size_t)R * 8, hipMemcpyDeviceToDevice, st);
        return r;
    };
    auto level_alpha = [&](int l) { return l == 0 ? p->o.alpha : (l == 1 ? 0.5 : 1.0); };
    auto set_alpha = [&](double a) {
        uint64_t bits;
        memcpy(&bits, &a, 8);
        return launch_fill_u64((uint64_t *)p->alpha_dev, bits, st);
    };
    auto run_iteration = [&]() {
        hipError_t r = graphed ? hipGraphLaunch(cur_exec(), st) : enqueue_iteration(p, xit, contig_x, st);
        if (r == hipSuccess) r = hipEventRecord(p->ev[2], st);
        if (r == hipSuccess) r = hipEventSynchronize(p->ev[2]);
        return r;
    };
    int level = 0, worse = 0, fell_back = 0;
    double best = -INFINITY;
    std::vector<int> levels;
    if (!p->adaptive) {
        // One iteration ahead: iteration t+1 is launched before the host reads
        // F-hat of iteration t; every iteration saves the factors and lambda
        // (buffer t mod 2), so a stop at t restores exactly that state.  With
        // direct launches the fit estimate of t runs on its own stream from
        // that copy while iteration t+1 proceeds; snapshot buffer t mod 2 is
        // written again only by iteration t+2, launched after the host has
        // waited for the fit of t.
        auto launch_one = [&](int t) {
            hipError_t r;
            if (graphed) {
                r = hipGraphLaunch(cur_exec(), st);
                if (r == hipSuccess) r = hipEventRecord(p->ev[t & 1 ? 3 : 2], st);
            } else {
                const IterCtl ic{(uint64_t)t, p->fst, p->ev_state[t & 1]};
                r = enqueue_iteration(p, xit, contig_x, st, &ic);
                if (r == hipSuccess) r = hipEventRecord(p->ev[t & 1 ? 3 : 2], p->fst);
            }
            return r;
        };
        // the state after iteration t back into the live factors and lambda
        auto restore = [&](int t) {
            const char *sb = (const char *)p->snapbuf[t & 1];
            size_t off = 0;
            hipError_t r = hipSuccess;
            for (int m = 0; m < N && r == hipSuccess; ++m) {
                const size_t b = (size_t)p->dims[m] * R * tsz * (p->mix ? 2 : 1);
                r = hipMemcpyAsync(p->mix ? p->fhat[m] : p->fac[m], sb + off, b, hipMemcpyDeviceToDevice, st);
                off += b;
            }
            if (r == hipSuccess) r = hipMemcpyAsync(p->lambda, sb + off, (size_t)R * 8, hipMemcpyDeviceToDevice, st);
            return r;
        };
        bool ahead = false;
        e = launch_one(0);
        for (; e == hipSuccess && it < p->o.max_iters; ++it) {
            ahead = it + 1 < p->o.max_iters;
            if (ahead) e = launch_one(it + 1);
            if (e == hipSuccess) e = hipEventSynchronize(p->ev[it & 1 ? 3 : 2]);
            if (e != hipSuccess) break;
            F = p->hist_host[it];
            if (!isfinite(F)) {
                e = hipErrorUnknown;
                break;
            }
            levels.push_back(0);
            const bool s = stop(it, F);
            if (sched && !p->ref_now && (s || it + 2 >= p->o.max_iters)) {
                // switch to refined solves from iteration it + 1: drop the
                // BF16 iteration already launched and restart it refined
                e = hipStreamSynchronize(st);
                if (e == hipSuccess) e = hipStreamSynchronize(p->fst);
                if (e == hipSuccess && ahead) e = restore(it);
                // graphs read the iteration number from the device counter
                // that the dropped iteration has already advanced
                if (e == hipSuccess && graphed) e = launch_fill_u64(p->t_dev, (uint64_t)(it + 1), st);
                p->ref_now = true;
                refined_from = it + 1;
                if (e == hipSuccess) e = launch_one(it + 1);
                continue;
            }
            if (s) {
                ++it;
                break;
            }
            ahead = false;
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = hipStreamSynchronize(p->fst);
        if (e == hipSuccess && ahead) e = restore(it - 1);  // undo the iteration launched past the stop
    }
    for (; p->adaptive && it < p->o.max_iters; ++it) {
        const bool duel = p->adaptive && level < 2 && it > 0 && ((it + 1) & it) == 0;
        if (duel) e = save(SNAP_PRE);
        if (e == hipSuccess) e = run_iteration();
        if (e != hipSuccess) break;
        F = p->hist_host[it];
        if (duel && isfinite(F)) {
            const double F1 = F;
            e = save(SNAP_CUR);
            if (e == hipSuccess) e = load(SNAP_PRE);
            if (e == hipSuccess) e = set_alpha(level_alpha(2));
            if (e == hipSuccess) e = launch_fill_u64(p->t_dev, (uint64_t)it, st);
            if (e == hipSuccess) e = run_iteration();
            if (e != hipSuccess) break;
            const double F2 = p->hist_host[it];
            const double sigma = (1.0 - F1) / sqrt(2.0 * p->o.P_hat);
            if (isfinite(F2) && F2 > F1 + 3.0 * sigma && (1.0 - F2) < 0.5 * (1.0 - F1)) {
                level = 2;
                worse = 0;
                fell_back = 1;
                F = F2;
            } else {
                e = load(SNAP_CUR);
                if (e == hipSuccess) e = set_alpha(level_alpha(level));
                p->hist_host[it] = F1;
                F = F1;
            }
        }
        if (!isfinite(F)) {
            e = hipErrorUnknown;
            break;
        }
        levels.push_back(level);
        if (p->adaptive && e == hipSuccess) {
            const double sigma = (1.0 - F) / sqrt(2.0 * p->o.P_hat);
            worse = (F < best - fmax(3.0 * sigma, 0.5 * (1.0 - best))) ? worse + 1 : 0;
            if (F > best) {
                best = F;
                e = save(SNAP_BEST);
            }
            if (e == hipSuccess && worse >= 2 && level < 2) {
                ++level;
                worse = 0;
                fell_back = 1;
                e = set_alpha(level_alpha(level));
                if (e == hipSuccess) e = load(SNAP_BEST);
            }
        }
        if (e != hipSuccess) break;
        const bool s = stop(it, F);
        if (sched && !p->ref_now && (s || it + 2 >= p->o.max_iters)) {
            p->ref_now = true;  // refined solves from the next iteration on
            refined_from = it + 1;
            continue;
        }
        if (s) {
            ++it;
            break;
        }
    }
    destroy_graphs();
    if (e != hipSuccess && isfinite(F)) return hip_fail(e, "ALS loop");
    if (!isfinite(F)) return set_error(CPRAND_ENAN, "non-finite fit estimate at iteration %d", it);
    // under mixing the loop keeps only A-hat: A = D_n F_n^* A-hat (Alg. 4, final unmix)
    for (int m = 0; p->mix && m < N && e == hipSuccess; ++m) {
        FftPlan *fp = fft_plan_get(p->dims[m], p->dbl, &e);
        if (fp) e = launch_factor_mix(fp, p->dbl, (int32_t)p->dims[m], R, p->fhat[m], p->signs + p->seg_off[m],
                                      p->fac[m], true, st);
    }
    if (e != hipSuccess) return hip_fail(e, "final unmix");
    hipEventRecord(p->ev[3], st);
    // CPRAND-PREMIX: A = D_m F_m^T A-hat (Alg. 5, final unmix)
    for (int m = 0; m < N && e == hipSuccess; ++m)
        e = p->premix ? launch_factor_dct((int32_t)p->dims[m], R, p->fac[m], p->signs + p->seg_off[m], A_inout[m], p->dbl,
                                          true, st)
                      : hipMemcpyAsync(A_inout[m], p->fac[m], (size_t)p->dims[m] * R * tsz, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(lambda_out, p->lambda, (size_t)R * 8, hipMemcpyDeviceToDevice, st);
    int32_t info = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&info, p->info, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "results");
    int flags = info ? CPRAND_W_PINV : 0;
    if (fell_back) flags |= CPRAND_W_FALLBACK;
    if (it >= p->o.max_iters) flags |= CPRAND_W_MAXIT;
    if (rep) {
        rep->iters = it;
        rep->flags = flags;
        rep->fit_est = F;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, p->ev[0], p->ev[1]);
        rep->setup_ms = ms;
        (void)hipEventElapsedTime(&ms, p->ev[1], p->ev[3]);
        rep->loop_ms = ms;
        (void)hipEventElapsedTime(&ms, tev[0], tev[1]);
        rep->norm_ms = ms;
        rep->fused = (p->mix && norm_done ? 1 : 0) | (copied_last ? 2 : 0);
        rep->refined_from = refined_from < it ? refined_from : -1;
        for (int m = 0; m < CPRAND_MAX_ORDER; ++m) {
            rep->mix_ms[m] = 0.0;
            rep->layout_ms[m] = 0.0;
            if (m < N && timed_mix[m] && hipEventElapsedTime(&ms, tev[2 + 2 * m], tev[3 + 2 * m]) == hipSuccess)
                rep->mix_ms[m] = ms;
            if (m < N && timed_lay[m] &&
                hipEventElapsedTime(&ms, tev[2 + 2 * N + 2 * m], tev[3 + 2 * N + 2 * m]) == hipSuccess)
                rep->layout_ms[m] = ms;
        }
        if (rep->fit_history) memcpy(rep->fit_history, p->hist_host, (size_t)it * 8);
        if (rep->proposal_history)
            for (int i = 0; i < it; ++i) {
                const int lv = i < (int)levels.size() ? levels[i] : 0;
                rep->proposal_history[i] =
                    lv == 0 ? p->o.proposal : (lv == 1 ? CPRAND_PROPOSAL_MIXTURE : CPRAND_PROPOSAL_UNIFORM);
            }
    }
    return flags;
}

int cprand_als(const cprand_tensor *X, const cprand_opts *opts, void *const *A_inout, double *lambda_out,
               cprand_report *report, void *stream) {
    cprand_plan *p = nullptr;
    int rc = cprand_plan_create(X, opts, &p);
    if (rc < 0) return rc;
    rc = cprand_plan_run(p, X, A_inout, lambda_out, report, stream);
    cprand_plan_destroy(p);
    return rc;
}

}  // extern "C"
