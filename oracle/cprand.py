"""FP64 reference of CPRAND (Alg. 3) and CPRAND-MIX (Alg. 4), step by step.

Test infrastructure (see oracle/__init__.py).  Every function takes the
paper's steps in the paper's order; numpy's least squares (LAPACK gelsd, SVD
based; the same minimiser as the paper's QR for full-rank Z_S), FFT and
matrix products serve as library steps.

Conventions: X is a numpy array of shape dims (FP64, or complex128 once
mixed); A is a list of N factor matrices (I_m, R); indices are 0-based; a
sample index array idx is (S, N) with column n unused.
"""
import math

import numpy as np

from . import philox
from .tensor import fnorm, cp_full


# ----------------------------------------------------------------------------
# Sample size rule (Section 3.2): S = 10 R log R, natural log, rounded to the
# nearest integer (this reproduces S=80 at R=5 and S=108 at R=6, Section 4.2).
def sample_size(R):
    return int(math.floor(10 * R * math.log(R) + 0.5))


def sample_size_ceil_log(R):
    """The variant 10 R ceil(ln R) used for the larger workloads."""
    return int(10 * R * math.ceil(math.log(R)))


# ----------------------------------------------------------------------------
# Sampled Khatri-Rao product and fiber sampling (Section 3.2, Alg. 2).
def skr(idx, A, n):
    """Z_S: row s is the Hadamard product of rows idx[s, m] of A^(m), m != n
    (Alg. 2).  Works for real or complex (mixed) factors."""
    S = idx.shape[0]
    R = A[(n + 1) % len(A)].shape[1]
    dt = np.result_type(*[A[m] for m in range(len(A)) if m != n])
    Z = np.ones((S, R), dtype=dt)
    for m in range(len(A)):
        if m == n:
            continue
        Z = Z * A[m][idx[:, m], :]
    return Z


def sample_fibers(X, idx, n):
    """X_S (I_n x S): column s is the mode-n fiber x_{i_1..i_{n-1} : i_{n+1}..i_N}
    at the sampled indices, pulled straight from the tensor (Section 3.2)."""
    S = idx.shape[0]
    out = np.empty((X.shape[n], S), dtype=X.dtype)
    for s in range(S):
        key = tuple(slice(None) if m == n else int(idx[s, m]) for m in range(X.ndim))
        out[:, s] = X[key]
    return out


def sampled_normal_blocks(X, idx, A, n, w=None):
    """The sampled MTTKRP and Gram: W = X_S diag(w) Z_S (I_n x R) and
    V = Z_S^T diag(w) Z_S (R x R), the normal-equation blocks of the sampled
    least-squares problem of Alg. 3 (weights w = 1 for uniform sampling)."""
    Z = skr(idx, A, n)
    Xs = sample_fibers(X, idx, n)
    wz = Z if w is None else Z * np.asarray(w)[:, None]
    return Xs @ wz, Z.T @ wz


def sampled_ls(X, idx, A, n, w=None):
    """A^(n) = argmin_A || Z_S A^T - X_S^T ||_F (Alg. 3), solved by LAPACK's
    SVD-based least squares (the paper uses QR; both give the minimiser when
    Z_S has full column rank).  Importance weights scale the rows by sqrt(w)."""
    Z = skr(idx, A, n)
    Xs = sample_fibers(X, idx, n)
    if w is not None:
        sw = np.sqrt(np.asarray(w, dtype=np.float64))[:, None]
        Z = Z * sw
        Xs = Xs * sw.T
    sol, *_ = np.linalg.lstsq(Z, Xs.T, rcond=None)
    return sol.T


def normalize(An):
    """Normalise columns to unit 2-norm; lambda_r is the norm (a zero column
    keeps lambda_r = 0 and stays zero)."""
    lam = np.sqrt(np.sum(np.abs(An) ** 2, axis=0))
    safe = np.where(lam > 0, lam, 1.0)
    return An / safe, lam


# ----------------------------------------------------------------------------
# Mixing (Section 2.2 and Section 3.3): D_m random signs, F_m the unitary DFT.
def mix_tensor(X, signs):
    """X-hat = X x_1 F_1 D_1 ... x_N F_N D_N with unitary (orthonormal) FFTs."""
    Xh = np.asarray(X, dtype=np.complex128)
    for m, d in enumerate(signs):
        shape = [1] * Xh.ndim
        shape[m] = -1
        Xh = np.fft.fft(Xh * d.reshape(shape), axis=m, norm="ortho")
    return Xh


def mix_factor(Am, sign):
    """A-hat^(m) = F_m D_m A^(m) (Alg. 4)."""
    return np.fft.fft(sign[:, None].astype(np.float64) * Am, axis=0, norm="ortho")


def unmix_factor(Ahm, sign):
    """Inverse of mix_factor: D_m F_m^* A-hat^(m)."""
    return sign[:, None] * np.fft.ifft(Ahm, axis=0, norm="ortho")


def unmix_fibers(Xs_hat, sign_n):
    """D_n F_n^* applied along each sampled fiber (eq. unmixX; Alg. 4)."""
    return sign_n[:, None] * np.fft.ifft(Xs_hat, axis=0, norm="ortho")


def mixed_sampled_ls(Xh, idx, Ah, n, sign_n):
    """The real-constrained sampled LS of CPRAND-MIX (Alg. 4 and eq. rcLS):
    Z-hat_S from the mixed factors, right-hand side from the unmixed sampled
    fibers, rows stacked as [Re; Im]."""
    Zh = skr(idx, Ah, n)
    M = unmix_fibers(sample_fibers(Xh, idx, n), sign_n)   # I_n x S
    lhs = np.vstack([Zh.real, Zh.imag])
    rhs = np.vstack([M.T.real, M.T.imag])
    sol, *_ = np.linalg.lstsq(lhs, rhs, rcond=None)
    return sol.T


def mixed_normal_blocks(Xh, idx, Ah, n, sign_n):
    """Normal-equation blocks of the stacked real LS of eq. rcLS:
    W = Re(M) Re(Z) + Im(M) Im(Z), V = Re(Z)^T Re(Z) + Im(Z)^T Im(Z), with M
    the unmixed sampled fibers."""
    Zh = skr(idx, Ah, n)
    M = unmix_fibers(sample_fibers(Xh, idx, n), sign_n)
    W = M.real @ Zh.real + M.imag @ Zh.imag
    V = Zh.real.T @ Zh.real + Zh.imag.T @ Zh.imag
    return W, V


# ----------------------------------------------------------------------------
# Fit (Section 3.4 and Section 4.2).
def exact_fit(X, lam, A):
    """F = 1 - ||X - X~|| / ||X|| with X~ reconstructed in full."""
    return 1.0 - fnorm(X - cp_full(lam, A)) / fnorm(X)


def model_entries(lam, A, idx):
    """x~_i = sum_r lam_r prod_m A^(m)(i_m, r) at each multi-index row of idx."""
    P = idx.shape[0]
    R = A[0].shape[1]
    dt = np.result_type(*A, np.asarray(lam))
    prod = np.ones((P, R), dtype=dt)
    for m, Am in enumerate(A):
        prod = prod * Am[idx[:, m], :]
    return prod @ np.asarray(lam)


def sampled_fit(X, normX, lam, A, fidx):
    """F-hat = 1 - sqrt(P mu-hat) / ||X||, mu-hat the mean squared error over
    the sampled entries (Section 3.4).  Complex data use |e|^2."""
    P = X.size
    x = X[tuple(fidx[:, m] for m in range(X.ndim))]
    e = x - model_entries(lam, A, fidx)
    mu_hat = float(np.mean(np.abs(e) ** 2))
    return 1.0 - math.sqrt(P * mu_hat) / normX


# ----------------------------------------------------------------------------
# Stopping rules (Section 3.4 and Section 4.2).
class StopRule:
    """Stop when any enabled rule holds after outer iteration t (0-based):
    t+1 >= max_iters; |F_t - F_{t-1}| <= tol; F_t >= fit_target;
    best F not improved for `patience` iterations."""

    def __init__(self, max_iters, tol=0.0, fit_target=None, patience=0):
        self.max_iters = max_iters
        self.tol = tol
        self.fit_target = fit_target
        self.patience = patience
        self.prev = None
        self.best = -np.inf
        self.since_best = 0

    def __call__(self, t, F):
        stop = t + 1 >= self.max_iters
        if self.tol > 0 and self.prev is not None and abs(F - self.prev) <= self.tol:
            stop = True
        if self.fit_target is not None and F >= self.fit_target:
            stop = True
        if F > self.best:
            self.best = F
            self.since_best = 0
        else:
            self.since_best += 1
            if self.patience > 0 and self.since_best >= self.patience:
                stop = True
        self.prev = F
        return stop


# ----------------------------------------------------------------------------
# The ALS drivers.
def cprand(X, R, S, A_init, seed, max_iters, tol=0.0, fit_target=None,
           patience=0, P_hat=2 ** 14, sampler=None):
    """CPRAND (Alg. 3).  A_init supplies A^(2..N) (A_init[0] is unused).
    `sampler(t, n, A)` may replace uniform sampling; it returns (idx, w).
    Returns (lam, A, history of F-hat)."""
    N = X.ndim
    dims = X.shape
    A = [np.array(M, dtype=np.float64) for M in A_init]
    lam = np.ones(R)
    normX = fnorm(X)
    fidx = philox.fit_indices(dims, P_hat, seed)
    rule = StopRule(max_iters, tol, fit_target, patience)
    hist = []
    for t in range(max_iters):
        for n in range(N):
            if sampler is None:
                idx, w = philox.sample_indices(dims, n, S, seed, t), None
            else:
                idx, w = sampler(t, n, A)
            A[n], lam = normalize(sampled_ls(X, idx, A, n, w))
        F = sampled_fit(X, normX, lam, A, fidx)
        hist.append(F)
        if rule(t, F):
            break
    return lam, A, hist


def cprand_mix(X, R, S, A_init, seed, max_iters, tol=0.0, fit_target=None,
               patience=0, P_hat=2 ** 14):
    """CPRAND-MIX (Alg. 4): one upfront mix of X and of A^(2..N); each mode
    step samples the mixed problem, unmixes the sampled fibers in mode n,
    solves the real-constrained LS, normalises and remixes A^(n).  F-hat is
    estimated in the mixed domain (unitary mixing keeps ||E|| unchanged).
    Returns (lam, A (real, unmixed), history of F-hat)."""
    N = X.ndim
    dims = X.shape
    signs = philox.sign_vectors(dims, seed)
    A = [np.array(M, dtype=np.float64) for M in A_init]
    Ah = [mix_factor(A[m], signs[m]) if m > 0 else None for m in range(N)]
    Xh = mix_tensor(X, signs)
    normX = fnorm(X)
    lam = np.ones(R)
    fidx = philox.fit_indices(dims, P_hat, seed)
    rule = StopRule(max_iters, tol, fit_target, patience)
    hist = []
    for t in range(max_iters):
        for n in range(N):
            idx = philox.sample_indices(dims, n, S, seed, t)
            A[n], lam = normalize(mixed_sampled_ls(Xh, idx, Ah, n, signs[n]))
            Ah[n] = mix_factor(A[n], signs[n])
        F = sampled_fit(Xh, normX, lam, Ah, fidx)
        hist.append(F)
        if rule(t, F):
            break
    return lam, A, hist
