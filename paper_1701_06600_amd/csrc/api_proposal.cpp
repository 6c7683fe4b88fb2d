// C ABI of the importance proposals and the proposal network (a project
// addition; see include/cprand.h): validation, workspace carving, launches.
#include <hip/hip_runtime.h>
#include <string.h>

#include <vector>

#include "api_internal.hpp"

namespace cprand {

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct PropWs {
    size_t stats, H, gpart, score, total;
};

static PropWs prop_layout(int32_t order, const int64_t *dims, int32_t R) {
    PropWs w{};
    w.stats = 0;
    w.H = align256(w.stats + (size_t)order * mode_stats_doubles(R) * 8);
    w.gpart = align256(w.H + (size_t)R * R * 8);
    w.score = align256(w.gpart + gram_part_doubles(order, R) * 8);
    size_t rows = 0;
    for (int m = 0; m < order; ++m) rows += (size_t)align256((size_t)dims[m] * 4);
    w.total = align256(w.score + rows);
    return w;
}

static int check_dims(int32_t order, const int64_t *dims, int32_t n, int32_t R) {
    if (order < 2 || order > CPRAND_MAX_ORDER) return set_error(CPRAND_EINVAL, "order %d outside [2, 8]", order);
    if (!dims) return set_error(CPRAND_EINVAL, "dims is NULL");
    if (n < 0 || n >= order) return set_error(CPRAND_EINVAL, "mode %d outside [0, %d)", n, order);
    if (R < 1 || R > CPRAND_MAX_RANK) return set_error(CPRAND_EINVAL, "R = %d outside [1, %d]", R, CPRAND_MAX_RANK);
    for (int m = 0; m < order; ++m)
        if (dims[m] < 1 || dims[m] > (int64_t)INT32_MAX)
            return set_error(CPRAND_EINVAL, "dims[%d] = %lld invalid", m, (long long)dims[m]);
    return CPRAND_OK;
}

// stats (+ H) for mode step n; scores per mode into the workspace
static hipError_t prop_common(int32_t order, const int64_t *dims, int32_t n, int32_t R, const void *const *A,
                              bool learned, bool need_h, const float *params, const PropWs &L, void *ws,
                              float *const *score, float *feat, float *target, const int64_t *row_off,
                              hipStream_t st) {
    ModeInfo mi{};
    mi.order = order;
    mi.n = n;
    FactorPtrs fp{};
    for (int m = 0; m < order; ++m) {
        mi.dims[m] = dims[m];
        mi.strides[m] = 1;
        fp.p[m] = (m == n) ? nullptr : A[m];
    }
    double *stats = (double *)((char *)ws + L.stats);
    double *H = (double *)((char *)ws + L.H);
    double *gpart = (double *)((char *)ws + L.gpart);
    hipError_t e = launch_mode_stats(fp, mi, R, stats, gpart, need_h ? H : nullptr, st);
    if (e == hipSuccess)
        e = launch_row_scores(fp, mi, R, stats, need_h ? H : nullptr, params, learned, score, feat, target, row_off,
                              st);
    return e;
}

}  // namespace cprand

using namespace cprand;

extern "C" {

int32_t cprand_mlp_param_count(void) { return kMlpParams; }

size_t cprand_proposal_workspace_size(int32_t order, const int64_t *dims, int32_t R) {
    if (order < 2 || order > CPRAND_MAX_ORDER || !dims || R < 1 || R > CPRAND_MAX_RANK) return 0;
    for (int m = 0; m < order; ++m)
        if (dims[m] < 1) return 0;
    return prop_layout(order, dims, R).total;
}

int cprand_proposal(int32_t order, const int64_t *dims, int32_t n, int32_t R, const void *const *A, int32_t kind,
                    const float *params, double alpha, uint64_t *const *cdf_out, void *workspace,
                    size_t workspace_bytes, void *stream) {
    g_last_error.clear();
    int rc = check_dims(order, dims, n, R);
    if (rc) return rc;
    if (kind != CPRAND_PROPOSAL_LEARNED && kind != CPRAND_PROPOSAL_MARGINAL && kind != CPRAND_PROPOSAL_LEVERAGE)
        return set_error(CPRAND_EINVAL, "kind must be PROPOSAL_LEARNED, PROPOSAL_MARGINAL or PROPOSAL_LEVERAGE");
    if (kind == CPRAND_PROPOSAL_LEARNED && !params) return set_error(CPRAND_EINVAL, "params is NULL");
    if (!(alpha >= 0.0 && alpha <= 1.0)) return set_error(CPRAND_EINVAL, "alpha outside [0, 1]");
    if (!A || !cdf_out) return set_error(CPRAND_EINVAL, "A and cdf_out must be non-NULL");
    for (int m = 0; m < order; ++m)
        if (m != n && (!A[m] || !cdf_out[m])) return set_error(CPRAND_EINVAL, "A[%d] or cdf_out[%d] is NULL", m, m);
    const PropWs L = prop_layout(order, dims, R);
    if (!workspace || workspace_bytes < L.total)
        return set_error(CPRAND_EINVAL, "workspace of %zu bytes needed", L.total);
    hipStream_t st = (hipStream_t)stream;
    float *score[CPRAND_MAX_ORDER] = {};
    uint64_t *cdf[CPRAND_MAX_ORDER] = {};
    size_t off = L.score;
    for (int m = 0; m < order; ++m) {
        score[m] = (float *)((char *)workspace + off);
        off += align256((size_t)dims[m] * 4);
        cdf[m] = (m == n) ? nullptr : cdf_out[m];
    }
    hipError_t e = prop_common(order, dims, n, R, A, kind == CPRAND_PROPOSAL_LEARNED, kind == CPRAND_PROPOSAL_MARGINAL,
                               params, L, workspace, score, nullptr, nullptr, nullptr, st);
    ModeInfo mi{};
    mi.order = order;
    mi.n = n;
    for (int m = 0; m < order; ++m) mi.dims[m] = dims[m];
    if (e == hipSuccess) e = launch_cdf(mi, score, alpha, nullptr, cdf, st);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_proposal");
}

int cprand_mlp_features(int32_t order, const int64_t *dims, int32_t n, int32_t R, const void *const *A, float *X_out,
                        float *t_out, void *workspace, size_t workspace_bytes, void *stream) {
    g_last_error.clear();
    int rc = check_dims(order, dims, n, R);
    if (rc) return rc;
    if (!A || !X_out) return set_error(CPRAND_EINVAL, "A and X_out must be non-NULL");
    for (int m = 0; m < order; ++m)
        if (m != n && !A[m]) return set_error(CPRAND_EINVAL, "A[%d] is NULL", m);
    const PropWs L = prop_layout(order, dims, R);
    if (!workspace || workspace_bytes < L.total)
        return set_error(CPRAND_EINVAL, "workspace of %zu bytes needed", L.total);
    int64_t row_off[CPRAND_MAX_ORDER] = {};
    int64_t r = 0;
    for (int m = 0; m < order; ++m) {
        row_off[m] = r;
        if (m != n) r += dims[m];
    }
    hipError_t e = prop_common(order, dims, n, R, A, false, true, nullptr, L, workspace, nullptr, X_out, t_out,
                               row_off, (hipStream_t)stream);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_mlp_features");
}

int cprand_mlp_forward(const float *params, const float *X, int64_t rows, float *logits, void *stream) {
    g_last_error.clear();
    if (!params || !X || !logits || rows < 1) return set_error(CPRAND_EINVAL, "bad arguments");
    hipError_t e = launch_mlp_logits(params, X, rows, logits, (hipStream_t)stream);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_mlp_forward");
}

size_t cprand_mlp_workspace_size(int64_t rows, int32_t ngroups) {
    if (rows < 1 || ngroups < 1) return 0;
    return align256((size_t)rows * 4) * 2 + align256((size_t)ngroups * 8) +
           align256((size_t)mlp_grad_blocks(rows) * kMlpParams * 4) + 256;
}

int cprand_mlp_grad(const float *params, const float *X, const float *t, const int64_t *group_off, int32_t ngroups,
                    int64_t rows, float *grad, double *loss, void *workspace, size_t workspace_bytes, void *stream) {
    g_last_error.clear();
    if (!params || !X || !t || !group_off || !grad || rows < 1 || ngroups < 1)
        return set_error(CPRAND_EINVAL, "bad arguments");
    const size_t need = cprand_mlp_workspace_size(rows, ngroups);
    if (!workspace || workspace_bytes < need) return set_error(CPRAND_EINVAL, "workspace of %zu bytes needed", need);
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)workspace;
    float *z = (float *)w;
    float *dz = (float *)(w + align256((size_t)rows * 4));
    double *gloss = (double *)(w + 2 * align256((size_t)rows * 4));
    float *gpart = (float *)((char *)gloss + align256((size_t)ngroups * 8));
    hipError_t e = launch_mlp_logits(params, X, rows, z, st);
    if (e == hipSuccess) e = launch_group_ce(z, t, group_off, ngroups, dz, gloss, st);
    if (e == hipSuccess) e = launch_mlp_grad(params, X, dz, rows, gpart, grad, st);
    if (e == hipSuccess && loss) e = launch_sum_parts(gloss, ngroups, 1, true, loss, st);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_mlp_grad");
}

int cprand_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t step, float lr, void *stream) {
    g_last_error.clear();
    if (!params || !grad || !m || !v || step < 1 || !(lr > 0.f)) return set_error(CPRAND_EINVAL, "bad arguments");
    hipError_t e = launch_adam(params, grad, m, v, step, lr, (hipStream_t)stream);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_mlp_adam");
}

int cprand_mlp_train(float *params, const float *X, const float *t, const int64_t *group_off, int32_t ngroups,
                     int64_t rows, int32_t epochs, float lr, double *loss_history, void *stream) {
    g_last_error.clear();
    if (!params || !X || !t || !group_off || rows < 1 || ngroups < 1 || epochs < 1 || !(lr > 0.f))
        return set_error(CPRAND_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    const size_t ws = cprand_mlp_workspace_size(rows, ngroups);
    void *buf = nullptr;
    const size_t pbytes = align256((size_t)3 * kMlpParams * 4);
    hipError_t e = hipMalloc(&buf, ws + pbytes + (size_t)epochs * 8);
    if (e != hipSuccess) return set_error(CPRAND_ENOMEM, "training buffers");
    char *b = (char *)buf;
    float *grad = (float *)(b + ws);
    float *mom = grad + kMlpParams;
    float *vel = mom + kMlpParams;
    double *losses = (double *)(b + ws + pbytes);
    e = hipMemsetAsync(mom, 0, (size_t)2 * kMlpParams * 4, st);
    for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
        int rc = cprand_mlp_grad(params, X, t, group_off, ngroups, rows, grad, losses + ep, buf, ws, stream);
        if (rc) {
            (void)hipFree(buf);
            return rc;
        }
        e = launch_adam(params, grad, mom, vel, ep + 1, lr, st);
    }
    if (e == hipSuccess && loss_history)
        e = hipMemcpyAsync(loss_history, losses, (size_t)epochs * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(buf);
    return e == hipSuccess ? CPRAND_OK : hip_fail(e, "cprand_mlp_train");
}

}  // extern "C"
