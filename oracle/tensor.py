"""Plain FP64 definitions of the tensor algebra of Section 2.1.

Test infrastructure (see oracle/__init__.py).

A tensor is a numpy array of shape (I_1, ..., I_N) indexed X[i_1, ..., i_N]
(0-based).  Its memory image on the GPU is column-major (mode 1 fastest);
`to_colmajor` / `from_colmajor` convert.  Factor matrices are (I_m, R).
"""
import numpy as np


def to_colmajor(X):
    """Flat column-major (mode 1 fastest) image of X."""
    return np.asarray(X).ravel(order="F")


def from_colmajor(flat, dims):
    return np.asarray(flat).reshape(tuple(dims), order="F")


def unfold(X, n):
    """Mode-n unfolding X_(n) (eq. unfoldmapping): entry (i_1..i_N) goes to
    row i_n and column j = sum_{k != n} i_k J_k with J_k the product of the
    dimensions of the modes m < k, m != n (0-based form of the 1-based map).
    So among the remaining modes the lowest one varies fastest."""
    N = X.ndim
    order = [n] + [m for m in range(N) if m != n]
    return np.reshape(np.transpose(X, order), (X.shape[n], -1), order="F")


def column_index(i, dims, n):
    """Column j of X_(n) that holds the multi-index i (eq. unfoldmapping)."""
    j, J = 0, 1
    for k in range(len(dims)):
        if k == n:
            continue
        j += int(i[k]) * J
        J *= dims[k]
    return j


def kron(A, B):
    """Kronecker product by its block definition (Section 2.1)."""
    I, J = A.shape
    K, L = B.shape
    out = np.empty((I * K, J * L), dtype=np.result_type(A, B))
    for i in range(I):
        for j in range(J):
            out[i * K:(i + 1) * K, j * L:(j + 1) * L] = A[i, j] * B
    return out


def khatri_rao(mats):
    """Khatri-Rao product mats[0] (.) mats[1] (.) ... : column r is the
    Kronecker product of the r-th columns (Section 2.1)."""
    R = mats[0].shape[1]
    cols = []
    for r in range(R):
        v = mats[0][:, r:r + 1]
        for M in mats[1:]:
            v = kron(v, M[:, r:r + 1])
        cols.append(v[:, 0])
    return np.stack(cols, axis=1)


def krp_except(A, n):
    """Z^(n) = A^(N) (.) ... (.) A^(n+1) (.) A^(n-1) (.) ... (.) A^(1)
    (eq. Zn): the lowest remaining mode varies fastest, matching the column
    order of unfold()."""
    mats = [A[m] for m in reversed(range(len(A))) if m != n]
    return khatri_rao(mats)


def cp_full(lam, A):
    """Dense tensor sum_r lam_r a_r^(1) o ... o a_r^(N) (eq. cpform+lambda)."""
    dims = tuple(M.shape[0] for M in A)
    R = A[0].shape[1]
    dt = np.result_type(*A, np.asarray(lam))
    X = np.zeros(dims, dtype=dt)
    for r in range(R):
        term = lam[r] * A[0][:, r]
        for M in A[1:]:
            term = np.multiply.outer(term, M[:, r])
        X = X + term
    return X


def ttm(X, U, n):
    """Mode-n tensor-times-matrix product: Y_(n) = U X_(n) (Section 2.1)."""
    Xn = np.moveaxis(X, n, 0)
    Y = np.tensordot(U, Xn, axes=(1, 0))
    return np.moveaxis(Y, 0, n)


def fnorm(X):
    return float(np.sqrt(np.sum(np.abs(X) ** 2)))
