// Host-side launchers of the HIP kernels (one .hip file per family).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace cprand {

// ---- sampling ---------------------------------------------------------------
hipError_t launch_sample(const ModeInfo &mi, int32_t S, uint64_t seed, uint64_t t,
                         const uint64_t *t_dev, const CdfPtrs *cdf, int32_t *idx, double *w,
                         hipStream_t st);
// The samples of every mode step of iterations 0 .. T-1 (uniform or fixed
// tables): step (t, n) at idx + (t * order + n) * S * order, weights (when w)
// at w + (t * order + n) * S; the same draws as launch_sample.
hipError_t launch_sample_all(const ModeInfo &mi, int32_t S, int32_t T, uint64_t seed, const CdfPtrs *cdf,
                             int32_t *idx, double *w, hipStream_t st);

// ---- sampled MTTKRP -----------------------------------------------------------
// Element kinds of the gathered tensor.
enum Kind { K_F64 = 0, K_F32 = 1, K_BF16 = 2, K_C64 = 3, K_C128 = 4 };

struct GatherPlan {
    int kind;
    int32_t R, S, In;
    int32_t ncols;      // R (real) or 2R (complex)
    int32_t ct;         // column tiles of 16
    int32_t kc;         // samples per chunk
    int32_t chunks;     // gridDim.y
    int32_t rows_wg;    // rows per workgroup
    int32_t waves;      // waves per workgroup
    int32_t row_blocks; // gridDim.x
    bool contig;        // vector loads along the fiber
    bool stream;        // streaming form: chunks = sample splits of per_split samples
    int32_t per_split;
    size_t lds_bytes;
    size_t wpart_elems() const { return (size_t)chunks * (size_t)ncols * (size_t)In; }
    size_t vpart_elems() const { return (size_t)chunks * (size_t)R * (size_t)R; }
};

// Choose tiling for one mode step.  elem_align: true when the data pointer
// and every stride other than mode n allow 16-byte vector loads along fibers.
// max_chunks > 0 caps the number of sample chunks (partial products) for
// consumers that sum them inside one workgroup.
// order: the tensor's order (sizes the per-sample index slots in LDS).
GatherPlan plan_gather(int kind, int32_t R, int32_t S, int64_t In, bool contig_ok, int max_chunks = 0,
                       int order = kMaxOrder);

struct GatherArgs {
    ModeInfo mi;
    const void *X;
    FactorPtrs A;        // row-major I_m x R, real type (complex interleaved for mixed)
    const int32_t *idx;  // S x order, or NULL: draw in-kernel
    const double *w;     // S weights or NULL (only with idx)
    const CdfPtrs *cdf;  // NULL or proposal tables for in-kernel draws (host struct, copied)
    uint64_t seed, t;
    const uint64_t *t_dev;
    void *wpart;         // [chunks][ncols][In] real type (float for BF16)
    double *vpart;       // [chunks][R][R]
};

hipError_t launch_gather(const GatherPlan &gp, const GatherArgs &a, hipStream_t st);

// out[e] = sum_p parts[p*count + e] (fixed order), float or double.
hipError_t launch_sum_parts(const void *parts, int32_t np, int64_t count, bool dbl, void *out, hipStream_t st);
// the same sums written as FP64 (inputs FP32 or FP64)
hipError_t launch_sum_parts_f64(const void *parts, int32_t np, int64_t count, bool in_double, double *out,
                                hipStream_t st);

// Sum partials into row-major W (In x R, real type) and V (R x R).  For real
// kinds only (complex ones go through launch_unmix).
hipError_t launch_reduce_wv(const GatherPlan &gp, const void *wpart, const double *vpart,
                            void *W, double *V, hipStream_t st);

// ---- FFT-based mixing -------------------------------------------------------------
struct FftPlan;  // per-length twiddles and radix schedule on the device
FftPlan *fft_plan_get(int64_t L, bool dbl, hipError_t *err);  // cached per (L, precision, device)

// Unmix the complex partial sums Y (chunks x 2R x In) of one mode step:
// W[i][r] = sign[i] Re( (F^* y_r)[i] ), y_r = sum over chunks.  W row-major
// (In x R) when w_rowmajor, else column-major [R][In].
hipError_t launch_unmix(const FftPlan *fp, bool dbl, int32_t In, int32_t R, int32_t chunks,
                        const void *ypart, const int8_t *sign, void *W, bool w_rowmajor,
                        hipStream_t st);
// A-hat = F D A (inverse = false) or A = Re(D F^* A-hat) (inverse = true).
hipError_t launch_factor_mix(const FftPlan *fp, bool dbl, int32_t I, int32_t R, const void *in,
                             const int8_t *sign, void *out, bool inverse, hipStream_t st);
// One pass of the tensor mix along mode m.  first: read the real input X
// (any strides), apply all sign vectors and write column-major complex
// Xhat; otherwise transform Xhat in place.  normsq_part: per-block partial
// sums of x^2 (first pass only) or NULL.
// Optional work folded into a mixing pass.  In: normsq_part (first pass:
// per-workgroup sums of squares of the input, at least 4096 doubles) and
// copy / copy_ld (a later pass: the pass's output fibers also stored
// contiguously, fiber q at copy + q * copy_ld, the layout of a mode-major
// copy).  Out: nparts (partials written, 0 if none) and copied.  Kernels
// that do not support an item leave it undone and report so.
struct MixExtras {
    double *normsq_part;
    int32_t nparts;
    void *copy;
    int64_t copy_ld;
    bool copied;
};
hipError_t launch_mix_pass(const FftPlan *fp, bool dbl, const ModeInfo &xi, const void *X,
                           int xkind, void *Xhat, int32_t m, bool first, const int8_t *signs,
                           MixExtras *ex, hipStream_t st);
hipError_t launch_signs(const ModeInfo &mi, uint64_t seed, int8_t *signs, hipStream_t st);

// ---- importance-weighted fit set (fitset.hip) ------------------------------------------
// Slice-energy proposal tables of every mode (cdf.p[m]: I_m + 1 uint64) from
// one pass over X; bins: sum I_m uint64 of scratch; energy_out (sum I_m
// doubles, mode 0 first) receives the slice energies when non-NULL.
hipError_t launch_energy_tables(const ModeInfo &mi, const void *X, int kind, const double *normX,
                                unsigned long long *bins, double alpha, const CdfPtrs &cdf, double *energy_out,
                                hipStream_t st);
// The P_hat entries of the weighted fit set: rows [P_hat][order], values
// [P_hat][2] (fx may be NULL) and weights [P_hat].
hipError_t launch_fit_set_weighted(const ModeInfo &mi, const void *X, int kind, int32_t P_hat, uint64_t seed,
                                   const CdfPtrs &cdf, double beta, int32_t *frow, double *fx, double *fw,
                                   hipStream_t st);

// ---- full MTTKRP, Gram matrices, exact fit (mttkrp_full.hip) ----------------------------
// Launch shape of the full MTTKRP of mode n of a column-major tensor.
struct FullPlan {
    int kind;             // K_F32 or K_F64
    int32_t In, R, ct;
    int64_t J, K, Q;      // dims before n, after n, columns of the unfolding
    bool iv, vec;         // vectors along the fiber (J == 1) / 16-byte vector loads
    int32_t rows_wg, row_blocks;
    int64_t qchunk;
    int32_t chunks;
    size_t wpart_bytes() const { return (size_t)chunks * R * In * (kind == K_F64 ? 8 : 4); }
};
// aligned: X is 16-byte aligned
FullPlan plan_full(const ModeInfo &mi, int kind, int32_t R, bool aligned);
// W (row-major I_n x R, FP64) = X_(n) Z^(n); wpart: f.wpart_bytes() of scratch.
hipError_t launch_mttkrp_full(const FullPlan &f, const ModeInfo &mi, const void *X, const FactorPtrs &A, void *wpart,
                              double *W, hipStream_t st);
// G = A^T A (FP64, R x R) of one I x R row-major factor; part: ceil(I/64) R^2 doubles.
hipError_t launch_gram_full(const void *A, bool dbl, int32_t I, int32_t R, double *part, double *G, hipStream_t st);
// V = Hadamard product of G[m] (order x R x R), m != skip (skip = -1: all).
hipError_t launch_gram_hadamard(const double *G, int32_t order, int32_t R, int32_t skip, double *V, hipStream_t st);
// Exact fit from the mode-n MTTKRP W, the mode-n factor An, lambda and the
// Hadamard product Gall of every factor's Gram.
hipError_t launch_fit_exact(const double *W, const void *An, bool dbl, int32_t In, int32_t R, const double *lambda,
                            const double *Gall, const double *normX, double *fit_out, hipStream_t st);

// ---- real orthogonal mixing (CPRAND-PREMIX) ------------------------------------------
// One orthonormal DCT-II pass along mode m of a real tensor (dct.hip).  first
// (m = 0 only): read X (kind xkind, any strides), apply every mode's signs and
// write the column-major real tensor Y (double when dbl, else float);
// otherwise transform Y in place.  hipErrorInvalidValue when the length is
// not {2,3,5,7}-smooth or its tile does not fit in LDS.  ex (first pass):
// per-block partial sums of ||X||^2 into ex->normsq_part when the pass's
// kernel supports it (ex->nparts partials written, else 0).
hipError_t launch_dct_pass(const ModeInfo &xi, const void *X, int xkind, void *Y, bool dbl, int32_t m, bool first,
                           const int8_t *signs, hipStream_t st, MixExtras *ex = nullptr);
// A-hat = C D A (inverse: A = D C^T A-hat) for one I x R row-major factor; in != out.
hipError_t launch_factor_dct(int32_t I, int32_t R, const void *in, const int8_t *sign, void *out, bool dbl,
                             bool inverse, hipStream_t st);

// ---- solve / normalise -------------------------------------------------------------
struct SolveArgs {
    int32_t In, R;
    const double *vpart;   // parts x R x R
    int32_t vparts;
    const void *W;         // element (p, i, r) at W[p*wps + i*wsi + r*wsr]
    int32_t wparts;
    int64_t wps, wsi, wsr;
    bool wdouble;          // W element type double (else float)
    const float *Wref;     // refinement MTTKRP (p, i, r) at Wref[p*rps + i*rsi + r*rsr], or NULL
    int32_t wrefparts;
    int64_t rps, rsi, rsr;
    const double *vref;    // with Wref: Gram of the FP32 rows, parts x R x R
    int32_t vrefparts;
    void *A;               // row-major In x R, unnormalised on output of solve
    bool adouble;
    double *colsq_part;    // [blocks][R]
    int32_t *info;         // device flag or NULL
    int32_t info_sticky;   // 1: only ever set the flag; 0: also clear it on success
};
hipError_t launch_solve(const SolveArgs &a, int32_t *nblocks, hipStream_t st);

// The whole post-gather part of a mode step in one workgroup (step.hip).
struct StepArgs {
    int32_t In, R;
    const double *vpart;
    int32_t vparts;
    const void *W;          // real: (p, i, r) at W[p*wps + i*wsi + r*wsr]; MIX: [wparts][2R][In]
    int32_t wparts;
    int64_t wps, wsi, wsr;
    bool wdouble;
    bool mix;
    const int8_t *sign;     // D_n (MIX)
    const float *Wref;      // refinement partials or NULL
    int32_t wrefparts;
    int64_t rps, rsi, rsr;
    const double *vref;     // with Wref: Gram partials of the FP32 rows
    int32_t vrefparts;
    void *A;                // row-major In x R, real type (not written under mixing)
    void *Ahat;             // MIX: row-major In x R complex
    double *lambda;
    void *snapA;            // optional second copy of the factor written (A, or A-hat under mixing)
    double *snap_lambda;    // optional second copy of lambda
    int32_t *info;          // set to CPRAND_W_PINV when the pseudo-inverse was used
};
size_t step_finish_lds(int32_t In, int32_t R, bool mix);
constexpr int kMaxParts = 8;  // partial products the one-workgroup finish sums (the fused gathers' chunk cap)

// Under mixing only A-hat and lambda are written (A is left untouched).
hipError_t launch_step_finish(const StepArgs &a, bool dbl, hipStream_t st);
hipError_t launch_normalize(int32_t In, int32_t R, void *A, bool adouble,
                            const double *colsq_part, int32_t nblocks, double *lambda,
                            hipStream_t st);

// ---- fit ------------------------------------------------------------------------------
// The state after an outer iteration, copied into one of two buffers chosen
// by the parity of the iteration: the loop can launch the next iteration
// before it reads this one's fit estimate, and undo it from the copy.
struct SnapArgs {
    const void *src[kMaxOrder];   // factors (4-byte words each: words[m])
    int64_t words[kMaxOrder];
    int32_t nsrc;                 // 0: no copy
    const double *lambda;         // R doubles, stored after the factors
    int32_t R;
    void *dst0, *dst1;            // by the parity of the iteration (even / odd)
};
struct FitArgs {
    ModeInfo mi;          // dims/strides of X (n unused)
    const void *X;
    int kind;             // K_*
    FactorPtrs A;         // real or complex (interleaved) factors
    bool fdouble;         // factor real type
    bool cplx;            // factors complex
    const double *lambda;
    int32_t R;
    int32_t P_hat;
    uint64_t seed;
    double *part;         // per-block partial sums
    // Optional single-launch finish: the last block to finish sums the
    // partials, writes F-hat to fit_out / hist[t] / hist_host[t], advances
    // *t_dev and clears *counter (which must start at zero).
    unsigned *counter;
    double P;
    const double *normX;
    double *fit_out;
    double *hist;
    double *hist_host;
    uint64_t *t_dev;
    uint64_t t;           // the iteration when t_dev is NULL
    // Optional cached fit set (the same P-hat entries are used at every
    // iteration): rows [P_hat][order] and tensor values [P_hat][2] (re, im)
    // written once by launch_fit_set; when NULL the entries are regenerated
    // from Philox and loaded from X.
    const int32_t *frow;
    const double *fx;
    const double *fw;     // with frow: per-entry weights of a weighted fit set, or NULL (all 1)
    // Optional copy of the iteration's state (iteration *t_dev, before the
    // advance), spread over all blocks.
    SnapArgs snap;
};
// Draw the fit set once (rows and tensor values) for FitArgs::frow / fx.
hipError_t launch_fit_set(const FitArgs &a, int32_t *frow, double *fx, hipStream_t st);
// Block partials of the fit estimate: one per kFitSamplesPerBlock entries.
constexpr int kFitSamplesPerBlock = 256;
inline int64_t fit_partials(int64_t P_hat) { return (P_hat < 1 ? 1 : P_hat + kFitSamplesPerBlock - 1) / kFitSamplesPerBlock; }
hipError_t launch_fit_partial(const FitArgs &a, int32_t *nblocks, hipStream_t st);
// fit_out = 1 - sqrt(P * sum(part)/P_hat) / *normX; also hist[t] (t from t_dev) if hist.
hipError_t launch_fit_final(const double *part, int32_t nparts, int32_t P_hat, double P,
                            const double *normX, double *fit_out, double *hist,
                            const uint64_t *t_dev, hipStream_t st);
hipError_t launch_normsq_partial(const ModeInfo &mi, const void *X, int kind, double *part,
                                 int32_t *nparts, hipStream_t st);
hipError_t launch_sqrt_sum(const double *part, int32_t nparts, double *out, hipStream_t st);

// ---- proposals and the proposal network (proposal.hip) ------------------------------
constexpr int kMlpParams = 4545;
// per-mode stats (doubles): G [R*R], G^{-1} [R*R], |A|_F^2, mean |cosine|
__host__ __device__ inline size_t mode_stats_doubles(int R) { return 2 * (size_t)R * R + 2; }
// Partial Grams (gpart, gram_part_doubles(order, R) doubles), then per mode
// m != n: G, G^{-1}, trace and mean |cosine| into stats; with Hinv non-NULL
// also the inverse of the Hadamard product of the Grams of all modes but n.
size_t gram_part_doubles(int order, int R);
hipError_t launch_mode_stats(const FactorPtrs &A, const ModeInfo &mi, int32_t R, double *stats, double *gpart,
                             double *Hinv, hipStream_t st);
hipError_t launch_row_scores(const FactorPtrs &A, const ModeInfo &mi, int32_t R, const double *stats, const double *Hinv,
                             const float *params, bool learned, float *const *score, float *feat, float *target,
                             const int64_t *row_off, hipStream_t st);
// alpha_dev (device) overrides alpha when non-NULL
hipError_t launch_cdf(const ModeInfo &mi, float *const *score, double alpha, const double *alpha_dev,
                      uint64_t *const *cdf, hipStream_t st);
hipError_t launch_mlp_logits(const float *params, const float *X, int64_t rows, float *z, hipStream_t st);
hipError_t launch_group_ce(const float *z, const float *t, const int64_t *goff, int32_t ngroups, float *dz,
                           double *gloss, hipStream_t st);
int32_t mlp_grad_blocks(int64_t rows);
hipError_t launch_mlp_grad(const float *params, const float *X, const float *dz, int64_t rows, float *gpart,
                           float *grad, hipStream_t st);
hipError_t launch_adam(float *params, const float *grad, float *m, float *v, int32_t step, float lr, hipStream_t st);

// ---- layout --------------------------------------------------------------------------
hipError_t launch_layout_copy(const ModeInfo &xi, const void *X, int xkind, int32_t n,
                              int64_t ld, void *Y, int ykind, hipStream_t st);

// ---- small helpers ---------------------------------------------------------------------
hipError_t launch_fill_u64(uint64_t *p, uint64_t v, hipStream_t st);
hipError_t launch_inc_u64(uint64_t *p, hipStream_t st);

}  // namespace cprand
