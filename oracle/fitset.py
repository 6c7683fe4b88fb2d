"""Importance-weighted fit estimate for unmixed tensors whose energy and
residual sit in few slices (a project addition to the sampled fit estimate
of Section 3.4).

Test infrastructure (see oracle/__init__.py).

The paper estimates ||X - X~||^2 as P times the mean squared residual over
P-hat uniformly drawn entries, and relies on the residual being spread over
the tensor, which its mixing provides (Section 3.3).  Without mixing, on a
tensor with a few heavy slices, few uniform draws land where the residual is
and the estimate overstates the fit.  Here the entries come from a defensive
mixture (Hesterberg, "Weighted average importance sampling and defensive
mixture distributions", Technometrics 1995): with probability beta from the
product of per-mode proposals built from the mode slice energies of X,
s_m(i) = sum of x^2 over the entries with index i in mode m (each mixed with
uniform by alpha and quantised to integers like the Khatri-Rao proposals),
and with probability 1 - beta uniformly.  Entry i gets the weight

    w(i) = 1 / (P q(i)),  q(i) = beta prod_m q_m(i_m) / Q_m + (1 - beta) / P,

so that P * mean_p w e^2 is an unbiased estimate of ||E||^2 for any residual
and w <= 1 / (1 - beta).  With beta = 0 every weight is 1 and the estimate is
the paper's.

Random words: entry p uses counter (p, 1, 0, b) under key (seed, FIT); word j
of the sequence (block j // 4, word j % 4) serves as: j = 0, the component
(the product when (u >> 11) < floor(beta 2^53)); j = k + 1, the row of mode
k (integer table search for the product, floor(u I_k / 2^64) otherwise).
"""
import math

import numpy as np

from . import philox
from .cprand import model_entries
from .proposal import cdf, draw_rows, quantize


def slice_energies(X):
    """s_m(i) = sum over the entries with index i in mode m of |x|^2, every m."""
    X2 = np.abs(np.asarray(X)) ** 2
    N = X2.ndim
    return [X2.sum(axis=tuple(k for k in range(N) if k != m)) for m in range(N)]


def energy_proposals(X, alpha):
    """Integer proposals q_m from the normalised slice energies of X."""
    out = []
    for s in slice_energies(X):
        tot = float(s.sum())
        p = s / tot if tot > 0 else np.full(s.size, 1.0 / s.size)
        out.append(quantize(p, alpha))
    return out


def _words(N, P_hat, seed):
    """(P_hat, N + 1) raw words: column 0 the component, column k + 1 mode k."""
    p = np.arange(P_hat, dtype=np.uint64)
    out = np.zeros((P_hat, N + 1), dtype=np.uint64)
    for b in range((N + 1 + 3) // 4):
        w = philox.philox4x64_10((p, 1, 0, b), (seed, philox.TAG_FIT))
        for j in range(4):
            if 4 * b + j < N + 1:
                out[:, 4 * b + j] = w[:, j]
    return out


def beta_threshold(beta):
    """The product component is drawn when (u >> 11) < floor(beta 2^53)."""
    return np.uint64(int(math.floor(beta * 2.0 ** 53)))


def weights(idx, qs, beta, dims):
    """w(i) = 1 / (beta P prod_m q_m(i_m)/Q_m + (1 - beta)), FP64, modes in order."""
    P = float(np.prod([float(I) for I in dims]))
    prod = np.ones(idx.shape[0], dtype=np.float64)
    for m, q in enumerate(qs):
        Q = float(np.sum(q.astype(np.uint64)))
        prod = prod * (q[idx[:, m]].astype(np.float64) / Q)
    return 1.0 / (beta * P * prod + (1.0 - beta))


def weighted_fit_indices(dims, P_hat, seed, qs, beta):
    """(idx, w): the P_hat entries of the weighted fit set and their weights."""
    N = len(dims)
    u = _words(N, P_hat, seed)
    prod_comp = (u[:, 0] >> np.uint64(11)) < beta_threshold(beta)
    idx = np.zeros((P_hat, N), dtype=np.int64)
    for m in range(N):
        uni = philox.bounded(u[:, m + 1], dims[m])
        imp = draw_rows(u[:, m + 1], cdf(qs[m]))
        idx[:, m] = np.where(prod_comp, imp, uni)
    return idx, weights(idx, qs, beta, dims)


def weighted_sampled_fit(X, normX, lam, A, idx, w):
    """F-hat = 1 - sqrt(P mean_p w_p |e_p|^2) / ||X||."""
    P = X.size
    x = X[tuple(idx[:, m] for m in range(X.ndim))]
    e = x - model_entries(lam, A, idx)
    mu_hat = float(np.mean(w * np.abs(e) ** 2))
    return 1.0 - math.sqrt(P * mu_hat) / normX
