// Helpers shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "../../include/cprand.h"
#include "kernels.hpp"

namespace cprand {

extern thread_local std::string g_last_error;
int set_error(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int kind_of(int dtype);
size_t elem_size(int kind);
int check_tensor(const cprand_tensor *X, const char *name);
ModeInfo mode_info(const cprand_tensor *X, int n);
bool is_colmajor(const cprand_tensor *X);
bool fibers_vectorizable(const void *data, int kind, const int64_t *strides, int order, int n);
int64_t numel(const cprand_tensor *X);

// Byte offsets of the per-step scratch regions in a caller workspace.
struct WsLayout {
    size_t wpart, vpart, colsq, fit, norm, wtmp, total;
};
WsLayout ws_layout(const cprand_tensor *X, int32_t R, int32_t S, int32_t P_hat);

// The sampled MTTKRP behind cprand_mttkrp_sampled: argument checks, the
// scratch it needs for mode n (partial products, Gram partials), and the
// kernel sequence on caller-given scratch (wtmp: I_n x 2R reals, used by
// mixed tensors only).
int check_mttkrp_args(const cprand_tensor *X, int32_t n, const void *const *A, int32_t R, int32_t S,
                      const int32_t *idx, const double *w, const int8_t *unmix_signs, const void *W, const double *V);
void mttkrp_scratch_bytes(const cprand_tensor *X, int32_t n, int32_t R, int32_t S, size_t *wpart, size_t *vpart);
int mttkrp_sampled_run(const cprand_tensor *X, int32_t n, const void *const *A, int32_t R, int32_t S,
                       const int32_t *idx, const double *w, const int8_t *unmix_signs, void *W, double *V,
                       void *wpart, double *vpart, void *wtmp, hipStream_t st);

// The tensor mix: signs, N FFT passes, ||X||.  Arguments already validated.
int mix_tensor_impl(const cprand_tensor *X, const cprand_tensor *Xhat, uint64_t seed, int8_t *signs,
                    double *normX_out, void *workspace, size_t workspace_bytes, hipStream_t st);

}  // namespace cprand
