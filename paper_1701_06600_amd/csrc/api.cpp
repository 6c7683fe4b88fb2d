// The C ABI: argument validation, workspace carving and kernel sequencing
// for the per-step calls of include/cprand.h.  The whole-decomposition plan
// lives in als.cpp.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "api_internal.hpp"

namespace cprand {

thread_local std::string g_last_error;

int set_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return set_error(CPRAND_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int kind_of(int dtype) {
    switch (dtype) {
        case CPRAND_F64: return K_F64;
        case CPRAND_F32: return K_F32;
        case CPRAND_BF16: return K_BF16;
        case CPRAND_C64: return K_C64;
        case CPRAND_C128: return K_C128;
        default: return -1;
    }
}

size_t elem_size(int kind) {
    switch (kind) {
        case K_F64: return 8;
        case K_F32: return 4;
        case K_BF16: return 2;
        case K_C64: return 8;
        case K_C128: return 16;
        default: return 0;
    }
}

int check_tensor(const cprand_tensor *X, const char *name) {
    if (!X) return set_error(CPRAND_EINVAL, "%s is NULL", name);
    if (X->order < 2 || X->order > CPRAND_MAX_ORDER)
        return set_error(CPRAND_EINVAL, "%s: order %d outside [2, %d]", name, X->order, CPRAND_MAX_ORDER);
    if (kind_of(X->dtype) < 0) return set_error(CPRAND_EINVAL, "%s: unknown dtype %d", name, X->dtype);
    for (int m = 0; m < X->order; ++m) {
        if (X->dims[m] < 1 || X->dims[m] > (int64_t)INT32_MAX)
            return set_error(CPRAND_EINVAL, "%s: dims[%d] = %lld invalid", name, m, (long long)X->dims[m]);
        if (X->strides[m] < 1) return set_error(CPRAND_EINVAL, "%s: strides[%d] < 1", name, m);
    }
    if (!X->data) return set_error(CPRAND_EINVAL, "%s->data is NULL", name);
    return CPRAND_OK;
}

ModeInfo mode_info(const cprand_tensor *X, int n) {
    ModeInfo mi{};
    mi.order = X->order;
    mi.n = n;
    for (int m = 0; m < X->order; ++m) {
        mi.dims[m] = X->dims[m];
        mi.strides[m] = X->strides[m];
    }
    return mi;
}

bool is_colmajor(const cprand_tensor *X) {
    int64_t e = 1;
    for (int m = 0; m < X->order; ++m) {
        if (X->strides[m] != e) return false;
        e *= X->dims[m];
    }
    return true;
}

// 16-byte vector loads along mode-n fibers are legal when the fiber stride
// is 1 and every fiber start is 16-byte aligned.
bool fibers_vectorizable(const void *data, int kind, const int64_t *strides, int order, int n) {
    const size_t esz = elem_size(kind);
    const int64_t ve = (int64_t)(16 / esz);
    if (strides[n] != 1) return false;
    if (((uintptr_t)data) & 15) return false;
    for (int m = 0; m < order; ++m)
        if (m != n && strides[m] % ve != 0) return false;
    return true;
}

int64_t numel(const cprand_tensor *X) {
    int64_t p = 1;
    for (int m = 0; m < X->order; ++m) p *= X->dims[m];
    return p;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

WsLayout ws_layout(const cprand_tensor *X, int32_t R, int32_t S, int32_t P_hat) {
    WsLayout w{};
    const int kind = kind_of(X->dtype);
    size_t wpart = 0, vpart = 0;
    for (int n = 0; n < X->order; ++n) {
        // the vector-load (streaming for long sample sets) and the strided plans
        for (bool contig : {true, false}) {
            GatherPlan gp = plan_gather(kind, R, S, X->dims[n], contig, 0, X->order);
            const size_t tsz = (kind == K_F64 || kind == K_C128) ? 8 : 4;
            wpart = std::max(wpart, gp.wpart_elems() * tsz);
            vpart = std::max(vpart, gp.vpart_elems() * 8);
        }
    }
    int64_t maxdim = 1;
    for (int n = 0; n < X->order; ++n) maxdim = std::max(maxdim, X->dims[n]);
    const size_t colsq = (size_t)ceil_div(maxdim, 32) * R * 8;
    const size_t fit = (size_t)fit_partials(P_hat) * 8;
    const size_t norm = (size_t)4096 * 8;
    const size_t wtmp = (size_t)maxdim * R * 16;
    w.wpart = 0;
    w.vpart = align256(w.wpart + wpart);
    w.colsq = align256(w.vpart + vpart);
    w.fit = align256(w.colsq + colsq);
    w.norm = align256(w.fit + fit);
    w.wtmp = align256(w.norm + norm);
    w.total = align256(w.wtmp + wtmp);
    return w;
}

int check_mttkrp_args(const cprand_tensor *X, int32_t n, const void *const *A, int32_t R, int32_t S,
                      const int32_t *idx, const double *w, const int8_t *unmix_signs, const void *W, const double *V) {
    int rc = check_tensor(X, "X");
    if (rc) return rc;
    if (n < 0 || n >= X->order) return set_error(CPRAND_EINVAL, "mode %d outside [0, %d)", n, X->order);
    if (R < 1 || R > CPRAND_MAX_RANK) return set_error(CPRAND_EINVAL, "R = %d outside [1, %d]", R, CPRAND_MAX_RANK);
    if (S < 1) return set_error(CPRAND_EINVAL, "S = %d < 1", S);
    if (!A) return set_error(CPRAND_EINVAL, "A is NULL");
    for (int m = 0; m < X->order; ++m)
        if (m != n && !A[m]) return set_error(CPRAND_EINVAL, "A[%d] is NULL", m);
    if (!idx || !W || !V) return set_error(CPRAND_EINVAL, "idx, W and V must be non-NULL");
    const int kind = kind_of(X->dtype);
    const bool cplx = kind == K_C64 || kind == K_C128;
    if (cplx && !unmix_signs) return set_error(CPRAND_EINVAL, "a mixed tensor needs unmix_signs");
    if (cplx && w) return set_error(CPRAND_EUNSUPPORTED, "importance weights with a mixed tensor");
    return CPRAND_OK;
}

void mttkrp_scratch_bytes(const cprand_tensor *X, int32_t n, int32_t R, int32_t S, size_t *wpart, size_t *vpart) {
    const int kind = kind_of(X->dtype);
    const bool contig = fibers_vectorizable(X->data, kind, X->strides, X->order, n);
    GatherPlan gp = plan_gather(kind, R, S, X->dims[n], contig, 0, X->order);
    const size_t tsz = (kind == K_F64 || kind == K_C128) ? 8 : 4;
    *wpart = gp.wpart_elems() * tsz;
    *vpart = gp.vpart_elems() * 8;
}

int mttkrp_sampled_run(const cprand_tensor *X, int32_t n, const void *const *A, int32_t R, int32_t S,
                       const int32_t *idx, const double *w, const int8_t *unmix_signs, void *W, double *V,
                       void *wpart, double *vpart, void *wtmp, hipStream_t st) {
    const int kind = kind_of(X->dtype);
    const bool cplx = kind == K_C64 || kind == K_C128;
    const bool contig = fibers_vectorizable(X->data, kind, X->strides, X->order, n);
    GatherPlan gp = plan_gather(kind, R, S, X->dims[n], contig, 0, X->order);
    GatherArgs ga{};
    ga.mi = mode_info(X, n);
    ga.X = X->data;
    for (int m = 0; m < X->order; ++m) ga.A.p[m] = (m == n) ? nullptr : A[m];
    ga.idx = idx;
    ga.w = w;
    ga.wpart = wpart;
    ga.vpart = vpart;
    hipError_t e = launch_gather(gp, ga, st);
    if (e != hipSuccess) return hip_fail(e, "gather kernel");
    if (!cplx) {
        e = launch_reduce_wv(gp, ga.wpart, ga.vpart, W, V, st);
    } else {
        const bool dbl = kind == K_C128;
        FftPlan *fp = fft_plan_get(X->dims[n], dbl, &e);
        if (!fp) return set_error(CPRAND_EUNSUPPORTED, "mode length %lld does not factor into 2,3,5,7",
                                  (long long)X->dims[n]);
        const void *y = ga.wpart;
        int32_t np = gp.chunks;
        if (np > 8) {  // many partials: sum them in parallel before the per-column transforms
            e = launch_sum_parts(ga.wpart, np, (int64_t)2 * R * X->dims[n], dbl, wtmp, st);
            if (e != hipSuccess) return hip_fail(e, "partial sums");
            y = wtmp;
            np = 1;
        }
        e = launch_unmix(fp, dbl, (int32_t)X->dims[n], R, np, y, unmix_signs, W, true, st);
        if (e == hipSuccess) e = launch_reduce_wv(gp, nullptr, ga.vpart, nullptr, V, st);
    }
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "mttkrp reduction");
}

}  // namespace cprand

using namespace cprand;

extern "C" {

const char *cprand_version(void) { return "cprand-gfx950 0.1.0"; }

const char *cprand_strerror(int status) {
    switch (status) {
        case CPRAND_OK: return "ok";
        case CPRAND_W_PINV: return "warning: pseudo-inverse used for a singular normal matrix";
        case CPRAND_W_MAXIT: return "warning: iteration cap reached";
        case CPRAND_W_FALLBACK: return "warning: learned proposal fell back";
        case CPRAND_EINVAL: return "invalid argument";
        case CPRAND_ENAN: return "non-finite value";
        case CPRAND_EHIP: return "HIP runtime error";
        case CPRAND_ENOMEM: return "out of device memory";
        case CPRAND_EUNSUPPORTED: return "unsupported configuration";
        default: return status > 0 ? "warning" : "unknown error";
    }
}

const char *cprand_last_error(void) { return g_last_error.c_str(); }

size_t cprand_workspace_size(const cprand_tensor *X, int32_t R, int32_t S, int32_t P_hat) {
    if (!X || X->order < 2 || X->order > CPRAND_MAX_ORDER || kind_of(X->dtype) < 0) return 0;
    if (R < 1 || R > CPRAND_MAX_RANK || S < 1 || P_hat < 0) return 0;
    for (int m = 0; m < X->order; ++m)
        if (X->dims[m] < 1) return 0;
    return ws_layout(X, R, S, P_hat).total;
}

int cprand_sample(int32_t order, const int64_t *dims, int32_t n, int32_t S, uint64_t seed, uint64_t t,
                  const uint64_t *const *cdf, int32_t *idx, double *w, void *stream) {
    g_last_error.clear();
    if (order < 2 || order > CPRAND_MAX_ORDER) return set_error(CPRAND_EINVAL, "order %d outside [2, 8]", order);
    if (!dims) return set_error(CPRAND_EINVAL, "dims is NULL");
    if (n < 0 || n >= order) return set_error(CPRAND_EINVAL, "mode %d outside [0, %d)", n, order);
    if (S < 1) return set_error(CPRAND_EINVAL, "S = %d < 1", S);
    if (!idx) return set_error(CPRAND_EINVAL, "idx is NULL");
    ModeInfo mi{};
    mi.order = order;
    mi.n = n;
    CdfPtrs c{};
    for (int m = 0; m < order; ++m) {
        if (dims[m] < 1 || dims[m] > (int64_t)INT32_MAX)
            return set_error(CPRAND_EINVAL, "dims[%d] = %lld invalid", m, (long long)dims[m]);
        mi.dims[m] = dims[m];
        mi.strides[m] = 1;
        if (cdf && m != n) {
            if (!cdf[m]) return set_error(CPRAND_EINVAL, "cdf[%d] is NULL", m);
            c.p[m] = cdf[m];
        }
    }
    hipError_t e = launch_sample(mi, S, seed, t, nullptr, cdf ? &c : nullptr, idx, w, (hipStream_t)stream);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_sample");
}

int cprand_mttkrp_sampled(const cprand_tensor *X, int32_t n, const void *const *A, int32_t R, int32_t S,
                          const int32_t *idx, const double *w, const int8_t *unmix_signs, void *W, double *V,
                          void *workspace, size_t workspace_bytes, void *stream) {
    g_last_error.clear();
    int rc = check_mttkrp_args(X, n, A, R, S, idx, w, unmix_signs, W, V);
    if (rc) return rc;
    const WsLayout L = ws_layout(X, R, S, 0);
    if (!workspace || workspace_bytes < L.total)
        return set_error(CPRAND_EINVAL, "workspace of %zu bytes needed", L.total);
    return mttkrp_sampled_run(X, n, A, R, S, idx, w, unmix_signs, W, V, (char *)workspace + L.wpart,
                              (double *)((char *)workspace + L.vpart), (char *)workspace + L.wtmp,
                              (hipStream_t)stream);
}

int cprand_solve(int32_t I_n, int32_t R, const double *V, const void *W, int32_t dtype, const float *W_refine,
                 const double *V_refine, void *A_out, double *lambda_out, int32_t *info, void *workspace,
                 size_t workspace_bytes, void *stream) {
    g_last_error.clear();
    if (I_n < 1) return set_error(CPRAND_EINVAL, "I_n = %d < 1", I_n);
    if (R < 1 || R > CPRAND_MAX_RANK) return set_error(CPRAND_EINVAL, "R = %d outside [1, %d]", R, CPRAND_MAX_RANK);
    if (dtype != CPRAND_F64 && dtype != CPRAND_F32) return set_error(CPRAND_EINVAL, "dtype must be F64 or F32");
    if (!V || !W || !A_out || !lambda_out) return set_error(CPRAND_EINVAL, "V, W, A_out, lambda_out must be non-NULL");
    if ((W_refine == nullptr) != (V_refine == nullptr))
        return set_error(CPRAND_EINVAL, "W_refine and V_refine must both be given or both be NULL");
    const size_t need = (size_t)ceil_div(I_n, 32) * R * 8;
    if (!workspace || workspace_bytes < need) return set_error(CPRAND_EINVAL, "workspace of %zu bytes needed", need);
    hipStream_t st = (hipStream_t)stream;
    SolveArgs a{};
    a.In = I_n;
    a.R = R;
    a.vpart = V;
    a.vparts = 1;
    a.W = W;
    a.wparts = 1;
    a.wps = 0;
    a.wsi = R;
    a.wsr = 1;
    a.wdouble = dtype == CPRAND_F64;
    a.Wref = W_refine;
    a.wrefparts = 1;
    a.rps = 0;
    a.rsi = R;
    a.rsr = 1;
    a.vref = V_refine;
    a.vrefparts = 1;
    a.A = A_out;
    a.adouble = dtype == CPRAND_F64;
    a.colsq_part = (double *)workspace;
    a.info = info;
    a.info_sticky = 0;
    int32_t nb = 0;
    hipError_t e = launch_solve(a, &nb, st);
    if (e == hipSuccess) e = launch_normalize(I_n, R, A_out, a.adouble, a.colsq_part, nb, lambda_out, st);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_solve");
}

int cprand_fit_est(const cprand_tensor *X, const double *normX, const void *const *A, const double *lambda,
                   int32_t R, int32_t P_hat, uint64_t seed, double *fit_out, void *workspace,
                   size_t workspace_bytes, void *stream) {
    g_last_error.clear();
    int rc = check_tensor(X, "X");
    if (rc) return rc;
    if (R < 1 || R > CPRAND_MAX_RANK) return set_error(CPRAND_EINVAL, "R = %d outside [1, %d]", R, CPRAND_MAX_RANK);
    if (P_hat < 1) return set_error(CPRAND_EINVAL, "P_hat = %d < 1", P_hat);
    if (!normX || !A || !lambda || !fit_out) return set_error(CPRAND_EINVAL, "NULL pointer argument");
    for (int m = 0; m < X->order; ++m)
        if (!A[m]) return set_error(CPRAND_EINVAL, "A[%d] is NULL", m);
    const size_t need = (size_t)fit_partials(P_hat) * 8;
    if (!workspace || workspace_bytes < need) return set_error(CPRAND_EINVAL, "workspace of %zu bytes needed", need);
    const int kind = kind_of(X->dtype);
    FitArgs fa{};
    fa.mi = mode_info(X, 0);
    fa.X = X->data;
    fa.kind = kind;
    for (int m = 0; m < X->order; ++m) fa.A.p[m] = A[m];
    fa.fdouble = kind == K_F64 || kind == K_C128;
    fa.cplx = kind == K_C64 || kind == K_C128;
    fa.lambda = lambda;
    fa.R = R;
    fa.P_hat = P_hat;
    fa.seed = seed;
    fa.part = (double *)workspace;
    hipStream_t st = (hipStream_t)stream;
    int32_t nb = 0;
    hipError_t e = launch_fit_partial(fa, &nb, st);
    if (e == hipSuccess)
        e = launch_fit_final(fa.part, nb, P_hat, (double)numel(X), normX, fit_out, nullptr, nullptr, st);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_fit_est");
}

size_t cprand_fit_weighted_workspace_size(int32_t order, int32_t P_hat) {
    if (order < 2 || order > CPRAND_MAX_ORDER || P_hat < 1) return 0;
    return align256((size_t)fit_partials(P_hat) * 8) + align256((size_t)P_hat * order * 4) +
           align256((size_t)P_hat * 16) + align256((size_t)P_hat * 8);
}

int cprand_energy_proposals(const cprand_tensor *X, const double *normX, double alpha, uint64_t *const *cdf_out,
                            double *energy_out, void *workspace, size_t workspace_bytes, void *stream) {
    g_last_error.clear();
    int rc = check_tensor(X, "X");
    if (rc) return rc;
    const int kind = kind_of(X->dtype);
    if (kind != K_F64 && kind != K_F32 && kind != K_BF16) return set_error(CPRAND_EINVAL, "X must be real");
    if (!normX || !cdf_out) return set_error(CPRAND_EINVAL, "normX and cdf_out must be non-NULL");
    if (!(alpha > 0.0 && alpha <= 1.0)) return set_error(CPRAND_EINVAL, "alpha outside (0, 1]");
    CdfPtrs c{};
    size_t bins = 0;
    for (int m = 0; m < X->order; ++m) {
        if (!cdf_out[m]) return set_error(CPRAND_EINVAL, "cdf_out[%d] is NULL", m);
        c.p[m] = cdf_out[m];
        bins += (size_t)X->dims[m];
    }
    if (!workspace || workspace_bytes < bins * 8)
        return set_error(CPRAND_EINVAL, "workspace of %zu bytes needed", bins * 8);
    hipError_t e = launch_energy_tables(mode_info(X, 0), X->data, kind, normX, (unsigned long long *)workspace, alpha,
                                        c, energy_out, (hipStream_t)stream);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_energy_proposals");
}

static int check_weighted_set(int32_t order, const int64_t *dims, int32_t P_hat, const uint64_t *const *cdf,
                              double beta, CdfPtrs *c) {
    if (order < 2 || order > CPRAND_MAX_ORDER || !dims) return set_error(CPRAND_EINVAL, "bad order or dims");
    if (P_hat < 1) return set_error(CPRAND_EINVAL, "P_hat = %d < 1", P_hat);
    if (!(beta >= 0.0 && beta < 1.0)) return set_error(CPRAND_EINVAL, "beta outside [0, 1)");
    if (!cdf) return set_error(CPRAND_EINVAL, "cdf is NULL");
    for (int m = 0; m < order; ++m) {
        if (dims[m] < 1 || dims[m] > (int64_t)INT32_MAX) return set_error(CPRAND_EINVAL, "dims[%d] invalid", m);
        if (!cdf[m]) return set_error(CPRAND_EINVAL, "cdf[%d] is NULL", m);
        c->p[m] = cdf[m];
    }
    return CPRAND_OK;
}

int cprand_fit_set_weighted(int32_t order, const int64_t *dims, int32_t P_hat, uint64_t seed,
                            const uint64_t *const *cdf, double beta, int32_t *idx, double *w, void *stream) {
    g_last_error.clear();
    CdfPtrs c{};
    int rc = check_weighted_set(order, dims, P_hat, cdf, beta, &c);
    if (rc) return rc;
    if (!idx || !w) return set_error(CPRAND_EINVAL, "idx and w must be non-NULL");
    ModeInfo mi{};
    mi.order = order;
    for (int m = 0; m < order; ++m) {
        mi.dims[m] = dims[m];
        mi.strides[m] = 1;
    }
    hipError_t e = launch_fit_set_weighted(mi, nullptr, K_F32, P_hat, seed, c, beta, idx, nullptr, w,
                                           (hipStream_t)stream);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_fit_set_weighted");
}

int cprand_fit_est_weighted(const cprand_tensor *X, const double *normX, const void *const *A, const double *lambda,
                            int32_t R, int32_t P_hat, uint64_t seed, const uint64_t *const *cdf, double beta,
                            double *fit_out, void *workspace, size_t workspace_bytes, void *stream) {
    g_last_error.clear();
    int rc = check_tensor(X, "X");
    if (rc) return rc;
    const int kind = kind_of(X->dtype);
    if (kind != K_F64 && kind != K_F32 && kind != K_BF16) return set_error(CPRAND_EINVAL, "X must be real");
    if (R < 1 || R > CPRAND_MAX_RANK) return set_error(CPRAND_EINVAL, "R = %d outside [1, %d]", R, CPRAND_MAX_RANK);
    CdfPtrs c{};
    rc = check_weighted_set(X->order, X->dims, P_hat, cdf, beta, &c);
    if (rc) return rc;
    if (!normX || !A || !lambda || !fit_out) return set_error(CPRAND_EINVAL, "NULL pointer argument");
    for (int m = 0; m < X->order; ++m)
        if (!A[m]) return set_error(CPRAND_EINVAL, "A[%d] is NULL", m);
    const size_t need = cprand_fit_weighted_workspace_size(X->order, P_hat);
    if (!workspace || workspace_bytes < need) return set_error(CPRAND_EINVAL, "workspace of %zu bytes needed", need);
    char *ws = (char *)workspace;
    double *part = (double *)ws;
    int32_t *frow = (int32_t *)(ws + align256((size_t)fit_partials(P_hat) * 8));
    double *fx = (double *)((char *)frow + align256((size_t)P_hat * X->order * 4));
    double *fw = (double *)((char *)fx + align256((size_t)P_hat * 16));
    hipStream_t st = (hipStream_t)stream;
    const ModeInfo mi = mode_info(X, 0);
    hipError_t e = launch_fit_set_weighted(mi, X->data, kind, P_hat, seed, c, beta, frow, fx, fw, st);
    FitArgs fa{};
    fa.mi = mi;
    fa.X = X->data;
    fa.kind = kind;
    for (int m = 0; m < X->order; ++m) fa.A.p[m] = A[m];
    fa.fdouble = kind == K_F64;
    fa.cplx = false;
    fa.lambda = lambda;
    fa.R = R;
    fa.P_hat = P_hat;
    fa.seed = seed;
    fa.part = part;
    fa.frow = frow;
    fa.fx = fx;
    fa.fw = fw;
    int32_t nb = 0;
    if (e == hipSuccess) e = launch_fit_partial(fa, &nb, st);
    if (e == hipSuccess)
        e = launch_fit_final(part, nb, P_hat, (double)numel(X), normX, fit_out, nullptr, nullptr, st);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_fit_est_weighted");
}

int cprand_norm(const cprand_tensor *X, double *normX_out, void *workspace, size_t workspace_bytes, void *stream) {
    g_last_error.clear();
    int rc = check_tensor(X, "X");
    if (rc) return rc;
    if (!normX_out) return set_error(CPRAND_EINVAL, "normX_out is NULL");
    if (!workspace || workspace_bytes < 4096 * 8) return set_error(CPRAND_EINVAL, "workspace of 32768 bytes needed");
    hipStream_t st = (hipStream_t)stream;
    int32_t np = 0;
    hipError_t e = launch_normsq_partial(mode_info(X, 0), X->data, kind_of(X->dtype), (double *)workspace, &np, st);
    if (e == hipSuccess) e = launch_sqrt_sum((double *)workspace, np, normX_out, st);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_norm");
}

int cprand_mix(const cprand_tensor *X, uint64_t seed, const cprand_tensor *Xhat, int8_t *signs, double *normX_out,
               void *workspace, size_t workspace_bytes, void *stream) {
    g_last_error.clear();
    int rc = check_tensor(X, "X");
    if (rc) return rc;
    rc = check_tensor(Xhat, "Xhat");
    if (rc) return rc;
    const int xk = kind_of(X->dtype), hk = kind_of(Xhat->dtype);
    if (xk != K_F32 && xk != K_F64) return set_error(CPRAND_EINVAL, "X must be F32 or F64");
    if (!(hk == K_C64 || hk == K_C128)) return set_error(CPRAND_EINVAL, "Xhat must be C64 or C128");
    if (xk == K_F64 && hk != K_C128) return set_error(CPRAND_EINVAL, "an F64 tensor mixes into C128");
    if (xk == K_F32 && hk != K_C64) return set_error(CPRAND_EINVAL, "an F32 tensor mixes into C64");
    if (Xhat->order != X->order) return set_error(CPRAND_EINVAL, "Xhat order differs");
    for (int m = 0; m < X->order; ++m)
        if (Xhat->dims[m] != X->dims[m]) return set_error(CPRAND_EINVAL, "Xhat dims differ");
    if (!is_colmajor(X) || !is_colmajor(Xhat))
        return set_error(CPRAND_EUNSUPPORTED, "mixing needs column-major X and Xhat");
    if (!signs || !normX_out) return set_error(CPRAND_EINVAL, "signs and normX_out must be non-NULL");
    hipStream_t st = (hipStream_t)stream;
    return mix_tensor_impl(X, Xhat, seed, signs, normX_out, workspace, workspace_bytes, st);
}

int cprand_mix_factor(int32_t I, int32_t R, const void *A, int32_t dtype, const int8_t *signs, void *Ahat,
                      int32_t inverse, void *stream) {
    g_last_error.clear();
    if (I < 1 || R < 1 || R > CPRAND_MAX_RANK) return set_error(CPRAND_EINVAL, "bad sizes I=%d R=%d", I, R);
    if (dtype != CPRAND_F32 && dtype != CPRAND_F64) return set_error(CPRAND_EINVAL, "dtype must be F32 or F64");
    if (!A || !signs || !Ahat) return set_error(CPRAND_EINVAL, "NULL pointer argument");
    hipError_t e;
    const bool dbl = dtype == CPRAND_F64;
    FftPlan *fp = fft_plan_get(I, dbl, &e);
    if (!fp) return set_error(CPRAND_EUNSUPPORTED, "length %d does not factor into 2,3,5,7", I);
    e = launch_factor_mix(fp, dbl, I, R, A, signs, Ahat, inverse != 0, (hipStream_t)stream);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_mix_factor");
}

int cprand_mix_dct(const cprand_tensor *X, uint64_t seed, const cprand_tensor *Xhat, int8_t *signs,
                   double *normX_out, void *workspace, size_t workspace_bytes, void *stream) {
    g_last_error.clear();
    int rc = check_tensor(X, "X");
    if (rc) return rc;
    rc = check_tensor(Xhat, "Xhat");
    if (rc) return rc;
    const int xk = kind_of(X->dtype);
    if (xk != K_F32 && xk != K_F64) return set_error(CPRAND_EINVAL, "X must be F32 or F64");
    if (Xhat->dtype != X->dtype) return set_error(CPRAND_EINVAL, "Xhat must have the dtype of X");
    if (Xhat->order != X->order) return set_error(CPRAND_EINVAL, "Xhat order differs");
    for (int m = 0; m < X->order; ++m)
        if (Xhat->dims[m] != X->dims[m]) return set_error(CPRAND_EINVAL, "Xhat dims differ");
    if (!is_colmajor(Xhat)) return set_error(CPRAND_EUNSUPPORTED, "Xhat must be column-major");
    if (!signs || !normX_out) return set_error(CPRAND_EINVAL, "signs and normX_out must be non-NULL");
    if (!workspace || workspace_bytes < 4096 * 8) return set_error(CPRAND_EINVAL, "workspace of 32768 bytes needed");
    const bool dbl = xk == K_F64;
    for (int m = 0; m < X->order; ++m) {
        hipError_t fe;
        if (!fft_plan_get(X->dims[m], dbl, &fe))
            return set_error(CPRAND_EUNSUPPORTED, "mode %d length %lld: not {2,3,5,7}-smooth or too long", m,
                             (long long)X->dims[m]);
    }
    hipStream_t st = (hipStream_t)stream;
    const ModeInfo xi = mode_info(X, 0), hi = mode_info(Xhat, 0);
    hipError_t e = launch_signs(xi, seed, signs, st);
    // ||X|| from the first pass when its kernel supports it, else its own pass
    MixExtras ex{};
    ex.normsq_part = (double *)workspace;
    for (int m = 0; m < X->order && e == hipSuccess; ++m)
        e = launch_dct_pass(m == 0 ? xi : hi, X->data, xk, Xhat->data, dbl, m, m == 0, signs, st,
                            m == 0 ? &ex : nullptr);
    if (e == hipErrorInvalidValue) return set_error(CPRAND_EUNSUPPORTED, "a mode is too long for the DCT tile");
    int32_t np = ex.nparts;
    if (e == hipSuccess && np == 0) e = launch_normsq_partial(xi, X->data, xk, (double *)workspace, &np, st);
    if (e == hipSuccess) e = launch_sqrt_sum((double *)workspace, np, normX_out, st);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_mix_dct");
}

int cprand_mix_factor_dct(int32_t I, int32_t R, const void *A, int32_t dtype, const int8_t *signs, void *out,
                          int32_t inverse, void *stream) {
    g_last_error.clear();
    if (I < 1 || R < 1 || R > CPRAND_MAX_RANK) return set_error(CPRAND_EINVAL, "bad sizes I=%d R=%d", I, R);
    if (dtype != CPRAND_F32 && dtype != CPRAND_F64) return set_error(CPRAND_EINVAL, "dtype must be F32 or F64");
    if (!A || !signs || !out) return set_error(CPRAND_EINVAL, "NULL pointer argument");
    if (A == out) return set_error(CPRAND_EINVAL, "A and out must not overlap");
    hipError_t e = launch_factor_dct(I, R, A, signs, out, dtype == CPRAND_F64, inverse != 0, (hipStream_t)stream);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_mix_factor_dct");
}

int cprand_mode_major_strides(int32_t order, const int64_t *dims, int32_t n, int64_t ld, int64_t *strides_out) {
    g_last_error.clear();
    if (order < 2 || order > CPRAND_MAX_ORDER || !dims || !strides_out || n < 0 || n >= order)
        return set_error(CPRAND_EINVAL, "bad arguments");
    if (ld < dims[n]) return set_error(CPRAND_EINVAL, "ld %lld < dims[n] %lld", (long long)ld, (long long)dims[n]);
    int64_t s = ld;
    for (int m = 0; m < order; ++m) {
        if (m == n) {
            strides_out[m] = 1;
            continue;
        }
        strides_out[m] = s;
        s *= dims[m];
    }
    return CPRAND_OK;
}

int cprand_layout_copy(const cprand_tensor *X, int32_t n, const cprand_tensor *Y, void *stream) {
    g_last_error.clear();
    int rc = check_tensor(X, "X");
    if (rc) return rc;
    rc = check_tensor(Y, "Y");
    if (rc) return rc;
    if (n < 0 || n >= X->order) return set_error(CPRAND_EINVAL, "mode %d outside [0, %d)", n, X->order);
    if (!is_colmajor(X)) return set_error(CPRAND_EUNSUPPORTED, "layout copies read a column-major X");
    if (Y->order != X->order) return set_error(CPRAND_EINVAL, "Y order differs");
    for (int m = 0; m < X->order; ++m)
        if (Y->dims[m] != X->dims[m]) return set_error(CPRAND_EINVAL, "Y dims differ");
    int64_t ld = 1;
    for (int m = 0; m < X->order; ++m)
        if (m != n) {
            ld = Y->strides[m];
            break;
        }
    // ld = stride of the first mode other than n
    int64_t want[CPRAND_MAX_ORDER];
    rc = cprand_mode_major_strides(X->order, X->dims, n, ld, want);
    if (rc) return rc;
    for (int m = 0; m < X->order; ++m)
        if (Y->strides[m] != want[m]) return set_error(CPRAND_EINVAL, "Y strides are not mode-major for mode %d", n);
    hipError_t e = launch_layout_copy(mode_info(X, n), X->data, kind_of(X->dtype), n, ld, Y->data,
                                      kind_of(Y->dtype), (hipStream_t)stream);
    if (e == hipErrorInvalidValue) return set_error(CPRAND_EUNSUPPORTED, "dtype conversion not supported");
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_layout_copy");
}

}  // extern "C"
