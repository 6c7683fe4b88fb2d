/*
 * cprand.h -- C ABI of a gfx950 (MI355X) library for randomized CP-ALS:
 * CPRAND and CPRAND-MIX of Battaglino, Ballard and Kolda, "A Practical
 * Randomized CP Tensor Decomposition" (SIAM J. Matrix Anal. Appl., 2018).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Indices are 0-based (the paper is 1-based).  Modes are 0 .. order-1.
 *  - A tensor is a device buffer described by cprand_tensor: dims and
 *    per-mode strides in elements.  The usual layout is column-major (mode 0
 *    fastest), the element order of the unfolding map of Section 2.1; any
 *    strides are accepted by the calls that gather fibers, so a copy with
 *    mode n innermost (cprand_layout_copy) serves mode-n steps.
 *  - Factor matrices A^(m) are row-major I_m x R device buffers (the R
 *    entries of a row are contiguous).  Their element type is the "real
 *    type" of the tensor: double for F64/C128 tensors, float for F32, C64
 *    and BF16 tensors.  Mixed (complex) factors are interleaved (re, im)
 *    pairs of that real type.
 *  - Every pointer named "device" must point to memory the GPU can read or
 *    write; "host" pointers are read on the calling thread before the call
 *    returns.  The caller owns every buffer; the library never frees or
 *    retains caller memory.  Scratch memory comes from a caller-provided
 *    workspace whose size cprand_workspace_size() returns (the plan API
 *    allocates its own).
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *    and is stream-ordered; calls return once the work is enqueued, without
 *    synchronising, except where stated.
 *  - Return value: 0 on success, a negative CPRAND_E* code on error (outputs
 *    then unspecified; cprand_last_error() holds a message).  Argument
 *    validation happens before any HIP call.
 */
#ifndef CPRAND_H
#define CPRAND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPRAND_MAX_ORDER 8
#define CPRAND_MAX_RANK 64

/* status codes */
#define CPRAND_OK 0
#define CPRAND_W_PINV 1          /* a normal matrix was not positive definite: pseudo-inverse used */
#define CPRAND_W_MAXIT 2         /* the iteration cap ended the run */
#define CPRAND_W_FALLBACK 4      /* the learned proposal fell back to mixture/uniform sampling */
#define CPRAND_EINVAL (-1)
#define CPRAND_ENAN (-2)
#define CPRAND_EHIP (-3)
#define CPRAND_ENOMEM (-4)
#define CPRAND_EUNSUPPORTED (-5)

/* element types */
#define CPRAND_F64 0
#define CPRAND_F32 1
#define CPRAND_BF16 2
#define CPRAND_C64 3   /* complex float, interleaved */
#define CPRAND_C128 4  /* complex double, interleaved */

typedef struct cprand_tensor {
    int32_t order;                       /* 2 .. CPRAND_MAX_ORDER */
    int32_t dtype;                       /* CPRAND_F64 .. CPRAND_C128 */
    int64_t dims[CPRAND_MAX_ORDER];      /* I_m >= 1 */
    int64_t strides[CPRAND_MAX_ORDER];   /* in elements, >= 1 */
    void *data;                          /* device */
} cprand_tensor;

/* ---------------------------------------------------------------------------
 * Version, errors, workspace.
 */
const char *cprand_version(void);
const char *cprand_strerror(int status);
/* Message of the last failing call on this thread ("" if none). */
const char *cprand_last_error(void);

/* Bytes of workspace that cprand_mttkrp_sampled, cprand_solve,
 * cprand_fit_est, cprand_norm and cprand_mix need for a tensor X (its dims),
 * rank R, S samples and P_hat fit entries.  0 on invalid arguments. */
size_t cprand_workspace_size(const cprand_tensor *X, int32_t R, int32_t S, int32_t P_hat);

/* ---------------------------------------------------------------------------
 * Sampling (Section 3.2; Alg. 3 "define sampling operator").
 *
 * Draws S multi-indices over the modes other than n, independently and with
 * replacement.  Sample s of outer iteration t uses Philox4x64-10 with key
 * (seed, 5) and counter (s, t, n, b); the k-th mode other than n takes word
 * k % 4 of block b = k / 4.  Uniform sampling maps a word u to
 * floor(u * I_m / 2^64).  With cdf != NULL, cdf[m] (device, I_m + 1 uint64
 * values, cdf[m][0] = 0, strictly increasing) is the integer proposal table
 * of mode m: the row drawn is the first i with cdf[m][i+1] > floor(u * Q /
 * 2^64), Q = cdf[m][I_m]; w[s] = prod_m Q_m / (I_m q_i) (FP64, modes in
 * increasing order) is the importance weight (1 for uniform sampling).
 *
 *   dims  host, `order` entries        cdf   host array of `order` device
 *   idx   device, S x order int32,           pointers (entry n ignored), or NULL
 *         row-major, column n = -1     w     device, S doubles, or NULL
 */
int cprand_sample(int32_t order, const int64_t *dims, int32_t n, int32_t S,
                  uint64_t seed, uint64_t t, const uint64_t *const *cdf,
                  int32_t *idx, double *w, void *stream);

/* ---------------------------------------------------------------------------
 * Sampled MTTKRP and Gram (Alg. 2 and Alg. 3; for mixed tensors Alg. 4 and
 * eq. rcLS).
 *
 * With Z_S the sampled Khatri-Rao rows (row s = Hadamard product of rows
 * idx[s, m] of A^(m), m != n) and X_S the I_n x S sampled mode-n fibers:
 *   W = X_S diag(w) Z_S   (I_n x R, row-major, real type of X)
 *   V = Z_S^T diag(w) Z_S (R x R, row-major, FP64)
 * For a mixed tensor (dtype C64/C128) A holds the mixed factors, the fibers
 * are unmixed in mode n by D_n F_n^* (unmix_signs = D_n, device int8, I_n
 * entries of +-1) and W, V are the normal-equation blocks of the stacked
 * real problem: W = Re(M) Re(Z) + Im(M) Im(Z), V = Re(Z^H Z) with M the
 * unmixed fibers.  For BF16 tensors the fibers and Z_S enter the product in
 * BF16 with FP32 accumulation; W is then float.
 *
 *   A     host array of `order` device pointers (entry n ignored)
 *   idx   device S x order int32 from cprand_sample
 *   w     device S doubles or NULL (all ones)
 *   W, V  device outputs
 */
int cprand_mttkrp_sampled(const cprand_tensor *X, int32_t n, const void *const *A,
                          int32_t R, int32_t S, const int32_t *idx, const double *w,
                          const int8_t *unmix_signs, void *W, double *V,
                          void *workspace, size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * cprand_mttkrp_sampled without a workspace.  Same arguments, results and
 * kernels as cprand_mttkrp_sampled for real tensors (F64, F32, BF16; a
 * mixed C64/C128 tensor returns CPRAND_EUNSUPPORTED).  The partial products
 * and Gram partials go to a fixed device array of
 * CPRAND_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held until
 * the process ends; a shape whose partials do not fit returns CPRAND_EINVAL
 * (the message names the bytes needed).  The call allocates nothing and
 * clears nothing: the gather overwrites every partial it later reads.  All
 * calls on one GPU share that GPU's array, so calls that overlap on one GPU
 * (unordered streams, or threads) race; calls ordered on one stream do not. */
#define CPRAND_NOALLOC_SCRATCH_BYTES 33554432  /* 32 MiB */
int cprand_mttkrp_sampled_noalloc(const cprand_tensor *X, int32_t n, const void *const *A,
                                  int32_t R, int32_t S, const int32_t *idx, const double *w,
                                  void *W, double *V, void *stream);

/* ---------------------------------------------------------------------------
 * Least-squares solve and normalisation (Alg. 3 solve and normalise steps).
 *
 * A = W V^{-1} through the normal equations, in FP64: V is inverted by
 * Gauss-Jordan elimination without pivoting (V is symmetric positive
 * definite when Z_S has full column rank; its pivots are then the squared
 * diagonal of its Cholesky factor).  If a pivot falls below 1e-12 of the
 * largest diagonal entry, V is diagonalised by cyclic Jacobi rotations and
 * its pseudo-inverse (eigenvalues below 1e-12 of the largest dropped) is
 * used instead, which gives the minimum-norm solution, and *info =
 * CPRAND_W_PINV.  With W_refine and V_refine (the MTTKRP, float, I_n x R
 * row-major, and the Gram, FP64 R x R, of the same samples from FP32 data
 * and FP32 Khatri-Rao rows) one step of iterative refinement follows: the
 * residual of the FP32 normal equations is corrected with the inverse of V,
 * A += (W_refine - A V_refine) V^{-1}.  The columns of A are then scaled to
 * unit 2-norm and lambda_out receives the norms (a zero column stays zero
 * with lambda 0).
 *
 *   V        device R x R FP64          dtype   CPRAND_F64 or CPRAND_F32, the
 *   W        device I_n x R row-major            type of W and A_out
 *   A_out    device I_n x R row-major   info    device int32 or NULL
 *   lambda_out device R doubles         W_refine, V_refine  device, both or neither
 *   workspace  ceil(I_n / 32) * R * 8 bytes
 */
int cprand_solve(int32_t I_n, int32_t R, const double *V, const void *W, int32_t dtype,
                 const float *W_refine, const double *V_refine, void *A_out, double *lambda_out,
                 int32_t *info, void *workspace, size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Sampled fit estimate (Section 3.4).
 *
 * Draws P_hat multi-indices once per seed (Philox key (seed, 6), counter
 * (p, 0, 0, b), mode k from word k % 4 of block k / 4) and writes
 *   *fit_out = 1 - sqrt(P * mean_p |x_p - model_p|^2) / normX,
 * model_p = sum_r lambda_r prod_m A^(m)(i_m, r), P = prod I_m; all sums in
 * FP64.  For a mixed tensor pass the mixed factors: the estimate is then of
 * the mixed residual, whose norm equals the unmixed one.
 *
 *   normX   device scalar (||X||)     fit_out  device scalar
 *   A       host array of `order` device pointers; lambda device R doubles
 */
int cprand_fit_est(const cprand_tensor *X, const double *normX, const void *const *A,
                   const double *lambda, int32_t R, int32_t P_hat, uint64_t seed,
                   double *fit_out, void *workspace, size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Importance-weighted fit estimate (a project addition to Section 3.4 for
 * unmixed tensors whose energy sits in few slices, where few uniformly
 * drawn entries see the residual).  Entries come from a defensive mixture:
 * with probability beta from the product over modes of the proposal tables
 * cdf[m] (as cprand_sample reads them), else uniformly.  Entry p uses
 * Philox4x64-10 with key (seed, 6) and counter (p, 1, 0, b); word j of the
 * sequence (block j / 4, word j % 4) serves as: j = 0, the component (the
 * product when (u >> 11) < floor(beta 2^53)); j = k + 1, the row of mode k
 * (the table search of cprand_sample for the product, floor(u I_k / 2^64)
 * otherwise).  The weight of entry i is
 *   w = 1 / (beta P prod_k (q_k(i_k) / Q_k) + (1 - beta)),
 * in FP64 with the operations in that order (no fused multiply-add), so
 * P mean(w e^2) estimates ||X - X~||^2 without bias and w <= 1 / (1 - beta);
 * beta = 0 gives the paper's estimate on a uniform set.
 *
 * cprand_energy_proposals: the tables of the slice energies of X, s_m(i) =
 * sum of x^2 over the entries with index i in mode m, mixed with uniform by
 * alpha and quantised like cprand_proposal: cdf_out[m] (device, I_m + 1
 * uint64).  The energies are summed in 64-bit fixed point (x^2 scaled by
 * 2^62 / (||X||^2 (1 + 1e-6))), so the tables are the same at every call;
 * energy_out (device, sum I_m doubles, mode 0 first, or NULL) receives
 * them.  normX: device ||X||.  workspace: 8 sum I_m bytes.
 * cprand_fit_set_weighted: the rows (idx, device P_hat x order int32) and
 * weights (w, device P_hat doubles) of the set.
 * cprand_fit_est_weighted: *fit_out = 1 - sqrt(P mean(w |x - model|^2)) /
 * normX over that set.  workspace: cprand_fit_weighted_workspace_size(order,
 * P_hat) bytes. */
size_t cprand_fit_weighted_workspace_size(int32_t order, int32_t P_hat);
int cprand_energy_proposals(const cprand_tensor *X, const double *normX, double alpha, uint64_t *const *cdf_out,
                            double *energy_out, void *workspace, size_t workspace_bytes, void *stream);
int cprand_fit_set_weighted(int32_t order, const int64_t *dims, int32_t P_hat, uint64_t seed,
                            const uint64_t *const *cdf, double beta, int32_t *idx, double *w, void *stream);
int cprand_fit_est_weighted(const cprand_tensor *X, const double *normX, const void *const *A,
                            const double *lambda, int32_t R, int32_t P_hat, uint64_t seed,
                            const uint64_t *const *cdf, double beta, double *fit_out, void *workspace,
                            size_t workspace_bytes, void *stream);

/* ||X|| (Frobenius, FP64 sums over all elements) into device *normX_out. */
int cprand_norm(const cprand_tensor *X, double *normX_out, void *workspace,
                size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Mixing (Section 2.2 and Section 3.3, Alg. 4).
 *
 * signs: D_m entry i is -1 when bit 63 of word 0 of Philox4x64-10 with key
 * (seed, 3) and counter (i, m, 0, 0) is set, else +1; written to `signs`
 * (device int8, sum I_m entries, mode 0 first).
 * Xhat = X x_0 F_0 D_0 ... x_{N-1} F_{N-1} D_{N-1}, F_m the unitary DFT
 * (scaled by 1/sqrt(I_m)).  X is real (F32 or F64, any strides); Xhat is a
 * caller-allocated complex tensor (C64 for F32 input, C128 for F64) with
 * column-major strides.  ||X|| is written to device *normX_out.  Every I_m
 * must factor into 2, 3, 5 and 7 and be at most 10240 (C64) or 5120 (C128).
 */
int cprand_mix(const cprand_tensor *X, uint64_t seed, const cprand_tensor *Xhat,
               int8_t *signs, double *normX_out, void *workspace, size_t workspace_bytes,
               void *stream);

/* A-hat = F D A for one I x R row-major real factor (dtype F32 or F64) into
 * the complex row-major Ahat; with inverse != 0, A = Re(D F^* A-hat) instead
 * (A complex input, Ahat real output). */
int cprand_mix_factor(int32_t I, int32_t R, const void *A, int32_t dtype,
                      const int8_t *signs, void *Ahat, int32_t inverse, void *stream);

/* ---------------------------------------------------------------------------
 * Real mixing for CPRAND-PREMIX (Section 3.3, Alg. 5): with a real orthogonal
 * F_m the mixed problem stays real, so plain CPRAND runs on the mixed tensor
 * and its factors are unmixed once at the end.  F_m is the orthonormal
 * DCT-II, (F_m)[k][i] = s_k cos(pi k (2i + 1) / (2 I_m)), s_0 = sqrt(1/I_m),
 * s_k = sqrt(2/I_m) for k > 0; the signs D_m are those of cprand_mix.
 *
 * cprand_mix_dct: Xhat = X x_0 F_0 D_0 ... x_{N-1} F_{N-1} D_{N-1}.  X is
 * F32 or F64 with any strides; Xhat is a caller-allocated column-major
 * tensor of the same dtype and dims that does not overlap X.  signs and
 * normX_out as for cprand_mix (||Xhat|| = ||X||).  Every I_m must factor
 * into 2, 3, 5 and 7 and be at most 3413 (F32) or 1706 (F64), the lengths
 * whose transform tile fits in LDS; otherwise CPRAND_EUNSUPPORTED.  workspace: 32768 bytes.
 *
 * cprand_mix_factor_dct: A-hat = F D A for one I x R row-major real factor
 * (dtype F32 or F64; A and out do not overlap); with inverse != 0, A =
 * D F^T A-hat (the unmix of Alg. 5).  Sums in FP64. */
int cprand_mix_dct(const cprand_tensor *X, uint64_t seed, const cprand_tensor *Xhat, int8_t *signs,
                   double *normX_out, void *workspace, size_t workspace_bytes, void *stream);
int cprand_mix_factor_dct(int32_t I, int32_t R, const void *A, int32_t dtype, const int8_t *signs, void *out,
                          int32_t inverse, void *stream);

/* ---------------------------------------------------------------------------
 * Layout: a copy of X with mode n innermost (its mode-n fibers contiguous,
 * each padded to ld elements), optionally converted to BF16 (round to
 * nearest even) or between real types.  Y->dims must equal X->dims;
 * Y->strides must be the ones cprand_mode_major_strides() returns for
 * (dims, n, ld).  A one-time pass that makes fiber gathers contiguous. */
int cprand_mode_major_strides(int32_t order, const int64_t *dims, int32_t n, int64_t ld,
                              int64_t *strides_out);
int cprand_layout_copy(const cprand_tensor *X, int32_t n, const cprand_tensor *Y,
                       void *stream);

/* ---------------------------------------------------------------------------
 * The dense method the paper compares against: CP-ALS (Alg. 1) with the
 * full MTTKRP, and the exact fit of Section 3.4.  X is a column-major F32 or
 * F64 tensor; factors are row-major I_m x R of its type.
 *
 * cprand_mttkrp_full: W = X_(n) Z^(n) (I_n x R, row-major, FP64), Z^(n) the
 * Khatri-Rao product of every factor but the n-th in the column order of the
 * mode-n unfolding (eq. Zn).  Products on MFMA with FP32 accumulation (FP64
 * for F64 data) over ranges of unfolding columns, the ranges summed in FP64.
 *
 * cprand_fit_exact: *fit_out = 1 - ||X - X~|| / ||X|| for X~ = [[lambda;
 * A^(0), ..., A^(N-1)]], through ||X||^2 - 2 <X, X~> + ||X~||^2 with
 * <X, X~> from the full MTTKRP of mode 0 and ||X~||^2 = lambda^T (*_m A^(m)T
 * A^(m)) lambda (FP64).  normX: device ||X||.  lambda: device R doubles.
 *
 *   workspace: cprand_full_workspace_size(X, R) bytes.
 *
 * cprand_cpals: CP-ALS from A_inout[1..N-1] (A_inout[0] is written before it
 * is read): per mode, V = Hadamard product of the other factors' Grams, W =
 * the full MTTKRP, A^(n) = W V^{-1} by the FP64 solve of cprand_solve
 * (pseudo-inverse when V is not positive definite, CPRAND_W_PINV), columns
 * normalised into lambda_out.  After every outer iteration the exact fit is
 * formed from the last mode's MTTKRP (no extra pass over X); the run stops
 * after max_iters iterations or when the fit changes by at most tol (tol > 0).
 * fit_history: host, max_iters doubles, or NULL.  Allocates its own scratch;
 * synchronises the stream once per iteration.  Returns 0, warning bits
 * (CPRAND_W_PINV, CPRAND_W_MAXIT) or a negative error. */
size_t cprand_full_workspace_size(const cprand_tensor *X, int32_t R);
int cprand_mttkrp_full(const cprand_tensor *X, int32_t n, const void *const *A, int32_t R, double *W,
                       void *workspace, size_t workspace_bytes, void *stream);
int cprand_fit_exact(const cprand_tensor *X, const double *normX, const void *const *A, const double *lambda,
                     int32_t R, double *fit_out, void *workspace, size_t workspace_bytes, void *stream);
int cprand_cpals(const cprand_tensor *X, int32_t R, int32_t max_iters, double tol, void *const *A_inout,
                 double *lambda_out, double *fit_history, int32_t *iters_out, void *stream);

/* ---------------------------------------------------------------------------
 * Importance proposals for the Khatri-Rao rows of a mode step (a project
 * addition to the paper's uniform sampling of Section 3.2; the leverage
 * definitions are those of Section 2.2).
 *
 * For the mode step of mode n, with K the other modes, each factor m in K
 * gets a distribution over its rows: CPRAND_PROPOSAL_MARGINAL uses the exact
 * marginal of Khatri-Rao leverage, L(i) = a_i^T (G_K^{-1} * prod_{k in K,
 * k != m} G_k) a_i (G_k = A^(k)T A^(k), G_K their Hadamard product, * =
 * Hadamard); CPRAND_PROPOSAL_LEVERAGE uses the row's leverage in its own
 * factor, a_i^T G_m^{-1} a_i; CPRAND_PROPOSAL_LEARNED uses softmax over rows of a 4-64-64-1
 * ReLU network (params, cprand_mlp_param_count() floats) applied to the row
 * features (log f1, log f2, log f3, f4): f1 = I|a_i|^2/|A|_F^2, f2 = (I/R)
 * a_i^T G_m^{-1} a_i, f3 = (I/R) sum_r a_ir^2/(G_m)_rr, f4 = mean |cosine|
 * between distinct columns of the other factors in K.  Either is mixed with
 * uniform, (1-alpha) p + alpha/I, quantised to q_i = max(1, floor(p 2^32))
 * and written as the table cdf_out[m] (device, I_m + 1 uint64) that
 * cprand_sample reads.  A: host array of `order` device pointers to float
 * factors.  workspace: cprand_proposal_workspace_size() bytes.
 */
#define CPRAND_PROPOSAL_MARGINAL 3
#define CPRAND_PROPOSAL_MIXTURE 4  /* reported in proposal_history: fallback, alpha = 0.5 */
#define CPRAND_PROPOSAL_LEVERAGE 5 /* each factor's rows by their leverage in that factor alone,
                                      a_i^T G_m^{-1} a_i (the product of factor leverages over the
                                      other modes, a non-learned reference proposal) */

int32_t cprand_mlp_param_count(void);
size_t cprand_proposal_workspace_size(int32_t order, const int64_t *dims, int32_t R);
int cprand_proposal(int32_t order, const int64_t *dims, int32_t n, int32_t R, const void *const *A,
                    int32_t kind, const float *params, double alpha, uint64_t *const *cdf_out,
                    void *workspace, size_t workspace_bytes, void *stream);

/* Training data for the proposal network from one set of factors: for mode
 * step n, the feature rows (4 floats each) of every factor m != n in
 * increasing m, and the target distribution of each factor (its exact
 * Khatri-Rao leverage marginal divided by R).  X_out: device, rows x 4;
 * t_out: device, rows; rows = sum_{m != n} I_m. */
int cprand_mlp_features(int32_t order, const int64_t *dims, int32_t n, int32_t R, const void *const *A,
                        float *X_out, float *t_out, void *workspace, size_t workspace_bytes, void *stream);
/* logits[i] = network(X[i]) for `rows` feature rows (device). */
int cprand_mlp_forward(const float *params, const float *X, int64_t rows, float *logits, void *stream);
/* Gradient (grad, device, param_count floats) of the mean over groups of
 * the cross-entropy -sum_i t_i log softmax(logits)_i, a group being the rows
 * group_off[g] .. group_off[g+1]-1 (device int64, ngroups+1 entries, t sums
 * to 1 within each group); *loss (device) gets the loss, if non-NULL.
 * workspace: cprand_mlp_workspace_size(rows, ngroups) bytes. */
size_t cprand_mlp_workspace_size(int64_t rows, int32_t ngroups);
int cprand_mlp_grad(const float *params, const float *X, const float *t, const int64_t *group_off,
                    int32_t ngroups, int64_t rows, float *grad, double *loss, void *workspace,
                    size_t workspace_bytes, void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step counts from 1) on
 * params with moment buffers m, v (device, param_count floats each). */
int cprand_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t step, float lr, void *stream);
/* epochs x (gradient + Adam) over a fixed training set; loss_history: host,
 * epochs doubles, or NULL.  Synchronises the stream at the end. */
int cprand_mlp_train(float *params, const float *X, const float *t, const int64_t *group_off, int32_t ngroups,
                     int64_t rows, int32_t epochs, float lr, double *loss_history, void *stream);

/* ---------------------------------------------------------------------------
 * The whole decomposition (Alg. 3 / Alg. 4 with the stopping rules of
 * Section 3.4 and Section 4.2).
 */
#define CPRAND_MIX_NONE 0
#define CPRAND_MIX_FFT 1
#define CPRAND_MIX_DCT 2   /* CPRAND-PREMIX: real DCT-II mixing, plain CPRAND on the mixed tensor */

#define CPRAND_PREC_NATIVE 0       /* arithmetic in the tensor's own type (F64 or F32) */
#define CPRAND_PREC_BF16_REFINE 1  /* BF16 products, FP64 solve, FP32 refinement (see refine_every) */
#define CPRAND_PREC_BF16 2         /* BF16 products, FP64 solve, no refinement */

#define CPRAND_PROPOSAL_UNIFORM 0
#define CPRAND_PROPOSAL_TABLE 1    /* caller-provided integer proposals, fixed */
#define CPRAND_PROPOSAL_LEARNED 2  /* MLP proposal recomputed each mode step */

typedef struct cprand_opts {
    int32_t R;            /* rank, 1 .. CPRAND_MAX_RANK */
    int32_t S;            /* samples per least-squares solve */
    int32_t P_hat;        /* entries of the fit estimate */
    int32_t max_iters;    /* outer iterations at most */
    uint64_t seed;
    double tol;           /* stop when |F_t - F_{t-1}| <= tol (0 = off) */
    double fit_target;    /* stop when F_t >= fit_target (> 1 = off) */
    int32_t patience;     /* stop when the best F has not improved for this many iterations (0 = off) */
    int32_t mix;          /* CPRAND_MIX_* */
    int32_t precision;    /* CPRAND_PREC_* */
    int32_t proposal;     /* CPRAND_PROPOSAL_*: UNIFORM; TABLE (fixed caller tables); LEARNED,
                             MARGINAL or LEVERAGE (recomputed from the current factors at every mode step,
                             FP32 tensors without mixing; falls back to a half-uniform mixture and
                             then to uniform sampling when the fit estimate drops by more than
                             three of its standard deviations below the best, twice in a row) */
    int32_t layout;       /* 0 = mode-major copies where fibers are strided or misaligned, 1 = never copy */
    int32_t use_graph;    /* 1 = replay each outer iteration as a HIP graph */
    double alpha;         /* uniform share of importance proposals */
    const uint64_t *const *proposal_cdf; /* PROPOSAL_TABLE: host array of `order` device CDFs */
    const float *mlp_params;            /* PROPOSAL_LEARNED: device, cprand_mlp_param_count() floats */
    int32_t refine_every; /* PREC_BF16_REFINE: 1 = refine every solve; 0 = BF16 solves until the stop
                             rule first holds (or one iteration before max_iters), then refined
                             solves until it holds again */
    double fit_beta;      /* 0 = the uniform fit set of Section 3.4; in (0, 1): the importance-weighted
                             fit set of cprand_fit_est_weighted with this beta (not with MIX_FFT) */
    double fit_alpha;     /* with fit_beta > 0: uniform share of the slice-energy proposals, (0, 1] */
} cprand_opts;

typedef struct cprand_report {
    int32_t iters;          /* outer iterations run */
    int32_t flags;          /* OR of CPRAND_W_* warnings */
    double fit_est;         /* last sampled fit estimate */
    double setup_ms;        /* norm / mixing / layout copies / conversions */
    double loop_ms;         /* the ALS loop */
    double *fit_history;    /* host, max_iters entries, or NULL */
    int32_t *proposal_history; /* host, max_iters entries (proposal in use), or NULL */
    double norm_ms;                      /* ||X|| pass (HIP events) */
    double mix_ms[CPRAND_MAX_ORDER];     /* mixing pass along each mode, 0 when not mixed */
    double layout_ms[CPRAND_MAX_ORDER];  /* mode-major copy for each mode, 0 when none or fused */
    int32_t fused;          /* setup work folded into the mixing passes: bit 0, ||X|| in the first
                               pass; bit 1, the last mode's mode-major copy written by the last pass */
    int32_t refined_from;   /* first iteration (0-based) with refined solves, -1 if none */
} cprand_report;

typedef struct cprand_plan cprand_plan;

/* Allocate the device buffers for decomposing tensors shaped like X under
 * opts (X->data is not read).  X: F64 or F32, any strides. */
int cprand_plan_create(const cprand_tensor *X, const cprand_opts *opts, cprand_plan **plan);
/* Decompose X (same shape and strides as at creation).  A_inout: host array
 * of `order` device pointers to row-major I_m x R factors of the real type;
 * A^(1..N-1) on entry are the initial factors (A^(0) is not read); on return
 * all hold the final unit-column factors and lambda_out (device, R doubles)
 * the weights.  Synchronises `stream` once per outer iteration to read the
 * fit estimate.  Returns 0 or a warning bit set, or a negative error. */
int cprand_plan_run(cprand_plan *plan, const cprand_tensor *X, void *const *A_inout,
                    double *lambda_out, cprand_report *report, void *stream);
void cprand_plan_destroy(cprand_plan *plan);

/* cprand_plan_create + cprand_plan_run + cprand_plan_destroy. */
int cprand_als(const cprand_tensor *X, const cprand_opts *opts, void *const *A_inout,
               double *lambda_out, cprand_report *report, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CPRAND_H */
