"""Leverage scores and coherence (Section 2.2 definitions; Section 3.2
lemmas), and the per-mode marginals of Khatri-Rao leverage used as targets
of the learned sampling proposal.

Test infrastructure (see oracle/__init__.py).
"""
import numpy as np

from .tensor import khatri_rao


def leverage_scores(A, rtol=1e-12):
    """l_i = ||U(i,:)||^2 with U the left singular vectors of A (definition
    in Section 2.2); numerically zero singular values are dropped."""
    U, s, _ = np.linalg.svd(np.asarray(A), full_matrices=False)
    if s.size == 0 or s[0] == 0:
        return np.zeros(A.shape[0])
    r = int(np.sum(s > rtol * s[0]))
    return np.sum(np.abs(U[:, :r]) ** 2, axis=1)


def coherence(A):
    """mu(A) = max_i l_i (definition in Section 2.2)."""
    return float(np.max(leverage_scores(A)))


def krp_leverage_exact(mats):
    """Leverage of every row of mats[0] (.) mats[1] (.) ..., formed in full."""
    return leverage_scores(khatri_rao(mats))


def krp_leverage_gram(mats):
    """Same scores without an SVD of the product: for full column rank,
    l_j = z_j^T (Z^T Z)^{-1} z_j with Z^T Z the Hadamard product of the factor
    Grams (eq. KRGram)."""
    Z = khatri_rao(mats)
    G = np.ones((Z.shape[1], Z.shape[1]))
    for M in mats:
        G = G * (M.T @ M)
    Ginv = np.linalg.inv(G)
    return np.einsum("jr,rs,js->j", Z, Ginv, Z)


def krp_marginals(mats):
    """Per-factor marginals of Khatri-Rao leverage: for factor k, entry i sums
    the leverage of every row of the product whose index in factor k is i.

    Summing z_j^T G^{-1} z_j over the indices of the other factors replaces
    each of their outer products by its Gram, so
        L_k(i) = a_i^T (G^{-1} * prod_{l != k} G_l) a_i   (* = Hadamard),
    with G = prod_l G_l (eq. KRGram).  sum_i L_k(i) = R for full rank."""
    Gs = [M.T @ M for M in mats]
    G = np.ones_like(Gs[0])
    for Gl in Gs:
        G = G * Gl
    Ginv = np.linalg.inv(G)
    out = []
    for k, M in enumerate(mats):
        H = Ginv.copy()
        for l, Gl in enumerate(Gs):
            if l != k:
                H = H * Gl
        out.append(np.einsum("ir,rs,is->i", M, H, M))
    return out


def krp_marginals_bruteforce(mats):
    """The same marginals by summing the exact leverage of the full product
    (small inputs only).  Row j of the product has index j // prod(I_l, l>k)
    mod I_k in factor k (first factor varies slowest, Kronecker order)."""
    lev = krp_leverage_exact(mats)
    dims = [M.shape[0] for M in mats]
    grid = lev.reshape(dims)   # C order: first factor slowest
    out = []
    for k in range(len(mats)):
        axes = tuple(a for a in range(len(mats)) if a != k)
        out.append(grid.sum(axis=axes))
    return out
