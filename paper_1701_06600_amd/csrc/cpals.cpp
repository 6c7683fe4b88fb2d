// The dense comparison path of the C ABI: the full MTTKRP, the exact fit
// (Section 3.4) and dense CP-ALS (Alg. 1), built on mttkrp_full.hip and the
// FP64 solve of solve.hip.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <vector>

#include "api_internal.hpp"

namespace cprand {
namespace {

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

// Scratch of the dense calls: partial products (the largest over modes), Gram
// partials, the Grams of every mode, V, W and the solve's column sums.
struct FullWs {
    size_t wpart, gpart, G, V, W, colsq, total;
};

FullWs full_ws(const cprand_tensor *X, int32_t R) {
    const int kind = kind_of(X->dtype);
    size_t wp = 0;
    int64_t maxdim = 1;
    for (int n = 0; n < X->order; ++n) {
        ModeInfo mi = mode_info(X, n);
        wp = std::max(wp, plan_full(mi, kind, R, true).wpart_bytes());
        wp = std::max(wp, plan_full(mi, kind, R, false).wpart_bytes());
        maxdim = std::max(maxdim, X->dims[n]);
    }
    FullWs w{};
    w.wpart = 0;
    w.gpart = a256(w.wpart + wp);
    w.G = a256(w.gpart + (size_t)ceil_div(maxdim, 64) * R * R * 8);
    w.V = a256(w.G + (size_t)X->order * R * R * 8);
    w.W = a256(w.V + (size_t)R * R * 8);
    w.colsq = a256(w.W + (size_t)maxdim * R * 8);
    w.total = a256(w.colsq + (size_t)ceil_div(maxdim, 32) * R * 8);
    return w;
}

int check_full(const cprand_tensor *X, int32_t R) {
    int rc = check_tensor(X, "X");
    if (rc) return rc;
    const int kind = kind_of(X->dtype);
    if (kind != K_F32 && kind != K_F64) return set_error(CPRAND_EINVAL, "X must be F32 or F64");
    if (!is_colmajor(X)) return set_error(CPRAND_EUNSUPPORTED, "the full MTTKRP reads a column-major X");
    if (R < 1 || R > CPRAND_MAX_RANK) return set_error(CPRAND_EINVAL, "R = %d outside [1, %d]", R, CPRAND_MAX_RANK);
    return CPRAND_OK;
}

hipError_t full_mttkrp(const cprand_tensor *X, int n, const void *const *A, int32_t R, void *wpart, double *W,
                       hipStream_t st) {
    const int kind = kind_of(X->dtype);
    ModeInfo mi = mode_info(X, n);
    FullPlan f = plan_full(mi, kind, R, (((uintptr_t)X->data) & 15) == 0);
    FactorPtrs fp{};
    for (int m = 0; m < X->order; ++m) fp.p[m] = (m == n) ? nullptr : A[m];
    return launch_mttkrp_full(f, mi, X->data, fp, wpart, W, st);
}

}  // namespace
}  // namespace cprand

using namespace cprand;

extern "C" {

size_t cprand_full_workspace_size(const cprand_tensor *X, int32_t R) {
    if (!X || X->order < 2 || X->order > CPRAND_MAX_ORDER || R < 1 || R > CPRAND_MAX_RANK) return 0;
    const int kind = kind_of(X->dtype);
    if (kind != K_F32 && kind != K_F64) return 0;
    for (int m = 0; m < X->order; ++m)
        if (X->dims[m] < 1) return 0;
    return full_ws(X, R).total;
}

int cprand_mttkrp_full(const cprand_tensor *X, int32_t n, const void *const *A, int32_t R, double *W,
                       void *workspace, size_t workspace_bytes, void *stream) {
    g_last_error.clear();
    int rc = check_full(X, R);
    if (rc) return rc;
    if (n < 0 || n >= X->order) return set_error(CPRAND_EINVAL, "mode %d outside [0, %d)", n, X->order);
    if (!A || !W) return set_error(CPRAND_EINVAL, "A and W must be non-NULL");
    for (int m = 0; m < X->order; ++m)
        if (m != n && !A[m]) return set_error(CPRAND_EINVAL, "A[%d] is NULL", m);
    const FullWs L = full_ws(X, R);
    if (!workspace || workspace_bytes < L.total) return set_error(CPRAND_EINVAL, "workspace of %zu bytes needed", L.total);
    hipError_t e = full_mttkrp(X, n, A, R, (char *)workspace + L.wpart, W, (hipStream_t)stream);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_mttkrp_full");
}

int cprand_fit_exact(const cprand_tensor *X, const double *normX, const void *const *A, const double *lambda,
                     int32_t R, double *fit_out, void *workspace, size_t workspace_bytes, void *stream) {
    g_last_error.clear();
    int rc = check_full(X, R);
    if (rc) return rc;
    if (!normX || !A || !lambda || !fit_out) return set_error(CPRAND_EINVAL, "NULL pointer argument");
    for (int m = 0; m < X->order; ++m)
        if (!A[m]) return set_error(CPRAND_EINVAL, "A[%d] is NULL", m);
    const FullWs L = full_ws(X, R);
    if (!workspace || workspace_bytes < L.total) return set_error(CPRAND_EINVAL, "workspace of %zu bytes needed", L.total);
    char *ws = (char *)workspace;
    hipStream_t st = (hipStream_t)stream;
    const bool dbl = kind_of(X->dtype) == K_F64;
    double *G = (double *)(ws + L.G), *V = (double *)(ws + L.V), *W = (double *)(ws + L.W);
    hipError_t e = full_mttkrp(X, 0, A, R, ws + L.wpart, W, st);
    for (int m = 0; m < X->order && e == hipSuccess; ++m)
        e = launch_gram_full(A[m], dbl, (int32_t)X->dims[m], R, (double *)(ws + L.gpart), G + (size_t)m * R * R, st);
    if (e == hipSuccess) e = launch_gram_hadamard(G, X->order, R, -1, V, st);
    if (e == hipSuccess) e = launch_fit_exact(W, A[0], dbl, (int32_t)X->dims[0], R, lambda, V, normX, fit_out, st);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_fit_exact");
}

int cprand_cpals(const cprand_tensor *X, int32_t R, int32_t max_iters, double tol, void *const *A_inout,
                 double *lambda_out, double *fit_history, int32_t *iters_out, void *stream) {
    g_last_error.clear();
    int rc = check_full(X, R);
    if (rc) return rc;
    if (max_iters < 1) return set_error(CPRAND_EINVAL, "max_iters = %d < 1", max_iters);
    if (!A_inout || !lambda_out) return set_error(CPRAND_EINVAL, "A_inout and lambda_out must be non-NULL");
    for (int m = 0; m < X->order; ++m)
        if (!A_inout[m]) return set_error(CPRAND_EINVAL, "A_inout[%d] is NULL", m);
    const int N = X->order;
    const bool dbl = kind_of(X->dtype) == K_F64;
    const FullWs L = full_ws(X, R);
    hipStream_t st = (hipStream_t)stream;
    char *ws = nullptr;
    hipError_t e = hipMalloc((void **)&ws, L.total + 4 * 4096 * 8 + 256);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? set_error(CPRAND_ENOMEM, "device allocation failed")
                                                          : hip_fail(e, "cprand_cpals workspace");
    double *G = (double *)(ws + L.G), *V = (double *)(ws + L.V), *W = (double *)(ws + L.W);
    double *colsq = (double *)(ws + L.colsq);
    double *normpart = (double *)(ws + L.total);
    double *normX = normpart + 4096, *fit = normX + 1;
    int32_t *info = (int32_t *)(fit + 1);
    double *fit_host = nullptr;
    e = hipHostMalloc((void **)&fit_host, 8, hipHostMallocDefault);
    int32_t np = 0;
    if (e == hipSuccess) e = launch_normsq_partial(mode_info(X, 0), X->data, kind_of(X->dtype), normpart, &np, st);
    if (e == hipSuccess) e = launch_sqrt_sum(normpart, np, normX, st);
    if (e == hipSuccess) e = launch_fill_u64((uint64_t *)info, 0, st);
    for (int m = 1; m < N && e == hipSuccess; ++m)
        e = launch_gram_full(A_inout[m], dbl, (int32_t)X->dims[m], R, (double *)(ws + L.gpart), G + (size_t)m * R * R,
                             st);
    int it = 0;
    double prev = 0.0;
    for (; it < max_iters && e == hipSuccess; ++it) {
        for (int n = 0; n < N && e == hipSuccess; ++n) {
            // Alg. 1: W = X_(n) Z^(n), V = * of the other Grams, A^(n) = W V^+, normalise
            const int32_t In = (int32_t)X->dims[n];
            e = launch_gram_hadamard(G, N, R, n, V, st);
            if (e == hipSuccess) e = full_mttkrp(X, n, A_inout, R, ws + L.wpart, W, st);
            if (e != hipSuccess) break;
            SolveArgs a{};
            a.In = In;
            a.R = R;
            a.vpart = V;
            a.vparts = 1;
            a.W = W;
            a.wparts = 1;
            a.wps = 0;
            a.wsi = R;
            a.wsr = 1;
            a.wdouble = true;
            a.A = A_inout[n];
            a.adouble = dbl;
            a.colsq_part = colsq;
            a.info = info;
            a.info_sticky = 1;
            int32_t nb = 0;
            e = launch_solve(a, &nb, st);
            if (e == hipSuccess) e = launch_normalize(In, R, A_inout[n], dbl, colsq, nb, lambda_out, st);
            if (e == hipSuccess)
                e = launch_gram_full(A_inout[n], dbl, In, R, (double *)(ws + L.gpart), G + (size_t)n * R * R, st);
        }
        // exact fit from the last mode's MTTKRP (no extra pass over X)
        if (e == hipSuccess) e = launch_gram_hadamard(G, N, R, -1, V, st);
        if (e == hipSuccess)
            e = launch_fit_exact(W, A_inout[N - 1], dbl, (int32_t)X->dims[N - 1], R, lambda_out, V, normX, fit, st);
        if (e == hipSuccess) e = hipMemcpyAsync(fit_host, fit, 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) break;
        const double F = *fit_host;
        if (fit_history) fit_history[it] = F;
        if (!isfinite(F)) {
            rc = set_error(CPRAND_ENAN, "non-finite fit at iteration %d", it);
            ++it;
            break;
        }
        if (tol > 0 && it > 0 && fabs(F - prev) <= tol) {
            ++it;
            break;
        }
        prev = F;
    }
    int32_t info_h = 0;
    if (e == hipSuccess && rc == CPRAND_OK) e = hipMemcpy(&info_h, info, 4, hipMemcpyDeviceToHost);
    if (fit_host) (void)hipHostFree(fit_host);
    (void)hipFree(ws);
    if (iters_out) *iters_out = it;
    if (e != hipSuccess) return hip_fail(e, "cprand_cpals");
    if (rc != CPRAND_OK) return rc;
    int flags = info_h ? CPRAND_W_PINV : 0;
    if (it >= max_iters) flags |= CPRAND_W_MAXIT;
    return flags;
}

}  // extern "C"
