"""Dense CP-ALS (Alg. 1) and the exact fit, the method the paper measures
CPRAND against (per-iteration times and fit-check times, Section 4.1).

Test infrastructure (see oracle/__init__.py).

The exact fit 1 - ||X - X~|| / ||X|| (Section 3.4) is evaluated without
forming X~ through ||X - X~||^2 = ||X||^2 - 2 <X, X~> + ||X~||^2, where
<X, X~> = sum_r lam_r sum_i A^(n)(i, r) W(i, r) for W the MTTKRP of any
mode n (the factors of the other modes in Z^(n)), and ||X~||^2 =
lam^T (G_1 * ... * G_N) lam with G_m = A^(m)T A^(m) (eq. KRGram).
"""
import math

import numpy as np

from .cprand import StopRule, normalize
from .tensor import fnorm, krp_except, unfold


def mttkrp(X, A, n):
    """W = X_(n) Z^(n) with Z^(n) the Khatri-Rao product of all factors but
    the n-th (Alg. 1, KR and MTTKRP lines), from the explicit unfolding."""
    return unfold(X, n) @ krp_except(A, n)


def gram_hadamard(A, n):
    """V = Hadamard product of A^(m)T A^(m) over m != n (Alg. 1, Gram line),
    which equals Z^(n)T Z^(n) (eq. KRGram)."""
    R = A[(n + 1) % len(A)].shape[1]
    V = np.ones((R, R))
    for m, M in enumerate(A):
        if m != n:
            V = V * (M.T @ M)
    return V


def cpals_update(X, A, n):
    """Alg. 1's solve: A^(n) V = W for A^(n) (through V's pseudo-inverse, so
    a rank-deficient V gives the minimum-norm solution); returns the
    unnormalised A^(n) and the W it used."""
    W = mttkrp(X, A, n)
    V = gram_hadamard(A, n)
    return W @ np.linalg.pinv(V), W


def fit_from_mttkrp(normX, lam, A, n, W):
    """Exact fit from the MTTKRP W of mode n for the model (lam, A) whose
    factors other than A^(n) are those W was formed with."""
    lam = np.asarray(lam, dtype=np.float64)
    inner = float(np.sum(lam * np.sum(A[n] * W, axis=0)))
    G = np.ones((lam.size, lam.size))
    for M in A:
        G = G * (M.T @ M)
    model_sq = float(lam @ G @ lam)
    res_sq = max(normX ** 2 - 2.0 * inner + model_sq, 0.0)
    return 1.0 - math.sqrt(res_sq) / normX


def exact_fit_inner(X, lam, A, n=0):
    """The exact fit through one MTTKRP (mode n), as a fit check costs."""
    return fit_from_mttkrp(fnorm(X), lam, A, n, mttkrp(X, A, n))


def cp_als(X, R, A_init, max_iters, tol=0.0, fit_target=None, patience=0):
    """CP-ALS (Alg. 1) from A^(2..N) = A_init[1:], with the exact fit after
    every outer iteration (from the last mode's MTTKRP) and the stop rules
    of Section 4.2.  Returns (lam, A, fit history)."""
    N = X.ndim
    A = [np.array(M, dtype=np.float64) for M in A_init]
    lam = np.ones(R)
    normX = fnorm(X)
    rule = StopRule(max_iters, tol, fit_target, patience)
    hist = []
    for t in range(max_iters):
        for n in range(N):
            An, W = cpals_update(X, A, n)
            A[n], lam = normalize(An)
        F = fit_from_mttkrp(normX, lam, A, N - 1, W)
        hist.append(F)
        if rule(t, F):
            break
    return lam, A, hist
