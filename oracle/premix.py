"""CPRAND-PREMIX (Section 3.3, Alg. 5) with a real orthogonal transform: the
orthonormal DCT-II.

Test infrastructure (see oracle/__init__.py).

With F_m real and orthogonal the mixed problem needs no real-constrained
solve (Section 3.3): mix X once, X-hat = X x_1 F_1 D_1 ... x_N F_N D_N, run
plain CPRAND (Alg. 3) on X-hat, and unmix the factors, A^(n) = D_n F_n^T
A-hat^(n).  The random signs D_m come from the same Philox stream as
CPRAND-MIX's; the initial factors given for A^(2..N) are mixed the same way
before the run, and the sampled fit estimate is taken on X-hat (an
orthogonal transform keeps the residual norm).  scipy's DCT serves as the
library step; dct_matrix is the definition it is pinned against.
"""
import numpy as np
import scipy.fft

from . import philox
from .cprand import cprand


def dct_matrix(I):
    """Orthonormal DCT-II: C[k, i] = s_k cos(pi k (2 i + 1) / (2 I)), s_0 =
    sqrt(1/I), s_k = sqrt(2/I) for k > 0."""
    k = np.arange(I)[:, None]
    i = np.arange(I)[None, :]
    C = np.cos(np.pi * k * (2 * i + 1) / (2.0 * I))
    C[0, :] *= np.sqrt(1.0 / I)
    C[1:, :] *= np.sqrt(2.0 / I)
    return C


def dct_along(Y, axis):
    """C applied along one axis (every fiber of that mode)."""
    return scipy.fft.dct(Y, type=2, norm="ortho", axis=axis)


def mix_tensor_dct(X, signs):
    """X-hat = X x_1 C_1 D_1 ... x_N C_N D_N."""
    Xh = np.asarray(X, dtype=np.float64)
    for m, d in enumerate(signs):
        shape = [1] * Xh.ndim
        shape[m] = -1
        Xh = dct_along(Xh * d.reshape(shape).astype(np.float64), m)
    return Xh


def mix_factor_dct(Am, sign):
    """A-hat^(m) = C_m D_m A^(m)."""
    return dct_along(sign[:, None].astype(np.float64) * Am, 0)


def unmix_factor_dct(Ahm, sign):
    """A^(m) = D_m C_m^T A-hat^(m) (Alg. 5's unmix line; C^T is the DCT-III)."""
    return sign[:, None].astype(np.float64) * scipy.fft.idct(Ahm, type=2, norm="ortho", axis=0)


def cprand_premix(X, R, S, A_init, seed, max_iters, tol=0.0, fit_target=None, patience=0, P_hat=2 ** 14):
    """Alg. 5: mix, CPRAND on the mixed tensor from the mixed initial factors,
    unmix.  Returns (lam, A (unmixed), history of F-hat on X-hat)."""
    dims = X.shape
    signs = philox.sign_vectors(dims, seed)
    Xh = mix_tensor_dct(X, signs)
    Ah0 = [mix_factor_dct(np.asarray(A_init[m], dtype=np.float64), signs[m]) for m in range(len(dims))]
    lam, Ah, hist = cprand(Xh, R, S, Ah0, seed, max_iters, tol=tol, fit_target=fit_target, patience=patience,
                           P_hat=P_hat)
    A = [unmix_factor_dct(Ah[m], signs[m]) for m in range(len(dims))]
    return lam, A, hist
