"""The learned sampling proposal (a project addition, not in the paper), in
FP64: per-row features of a factor matrix, the 4-64-64-1 ReLU network,
its hand-written backward pass, the per-mode softmax cross-entropy against
exact Khatri-Rao leverage marginals, and Adam (Kingma and Ba, ICLR 2015).

Test infrastructure (see oracle/__init__.py).

Features of row i of A = A^(m) (I x R), for the Khatri-Rao product Z of the
factors in a set K (the modes other than the one being updated, m in K):
  f1 = I ||a_i||^2 / ||A||_F^2                        (row energy, mean 1)
  f2 = (I/R) a_i^T G^{-1} a_i,  G = A^T A             (factor leverage, mean 1)
  f3 = (I/R) sum_r a_ir^2 / G_rr                      (column-normalised energy, mean 1)
  f4 = mean over k in K, k != m, of the mean |cosine| between distinct
       columns of A^(k)                               (one value per mode)
The network sees x = (log f1, log f2, log f3, f4).  When the other factors
have orthogonal columns the exact marginal is proportional to f3; when they
are collinear it approaches f2; f4 says which regime applies.

Parity status: the network and Adam are pinned by finite differences and a
closed-form first Adam step; the features by their means and limiting
cases; the targets by the brute-force leverage of the explicit product.
What the trained network gains over uniform sampling has no paper value
(parity unpinned beyond the relative comparison).
"""
import numpy as np

from .leverage import krp_marginals

H1 = 64
H2 = 64
N_IN = 4
FEAT_EPS = 1e-6

# flat parameter layout: W1 (H1 x N_IN), b1, W2 (H2 x H1), b2, w3 (H2), b3
SHAPES = [("W1", (H1, N_IN)), ("b1", (H1,)), ("W2", (H2, H1)), ("b2", (H2,)), ("w3", (H2,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def congruence(A):
    """Mean |cosine| between distinct columns of A (0 for one column)."""
    R = A.shape[1]
    if R < 2:
        return 0.0
    G = A.T @ A
    d = np.sqrt(np.diag(G))
    C = np.abs(G) / np.outer(d, d)
    return float((C.sum() - np.trace(C)) / (R * (R - 1)))


def row_features(A, others):
    """(I, 4) features of the rows of A given the other factors in K."""
    I, R = A.shape
    G = A.T @ A
    rn = np.sum(A * A, axis=1)
    f1 = I * rn / rn.sum()
    f2 = (I / R) * np.einsum("ir,rs,is->i", A, np.linalg.inv(G), A)
    f3 = (I / R) * np.sum(A * A / np.diag(G)[None, :], axis=1)
    f4 = np.mean([congruence(B) for B in others]) if others else 0.0
    return np.stack([np.log(f1 + FEAT_EPS), np.log(f2 + FEAT_EPS), np.log(f3 + FEAT_EPS),
                     np.full(I, f4)], axis=1)


def targets(mats, k):
    """Training target for factor k of the product of `mats`: the exact
    marginal of Khatri-Rao leverage over the rows of mats[k], normalised to
    a distribution (it sums to R)."""
    L = krp_marginals(mats)[k]
    return L / L.sum()


def forward(theta, X):
    """Logits (n,) and the activations needed by backward."""
    P = unpack(theta)
    a1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ P["w3"] + P["b3"][0]
    return z, (X, a1, h1, a2, h2)


def backward(theta, cache, dz):
    """Gradient of sum_i dz_i * z_i with respect to the flat parameters."""
    P = unpack(theta)
    X, a1, h1, a2, h2 = cache
    g = {}
    g["w3"] = h2.T @ dz
    g["b3"] = np.array([dz.sum()])
    dh2 = np.outer(dz, P["w3"])
    da2 = dh2 * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ P["W2"]
    da1 = dh1 * (a1 > 0)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(axis=0)
    return pack(g)


def group_softmax(z, groups):
    """Softmax of z within each group (groups: list of index arrays)."""
    p = np.empty_like(z)
    for idx in groups:
        zz = z[idx] - z[idx].max()
        e = np.exp(zz)
        p[idx] = e / e.sum()
    return p


def loss_and_dz(z, t, groups):
    """Mean over groups of the cross-entropy -sum t log softmax(z), and its
    gradient with respect to z (p - t within a group, over the group count)."""
    p = group_softmax(z, groups)
    G = len(groups)
    loss = 0.0
    for idx in groups:
        loss -= float(np.sum(t[idx] * np.log(p[idx])))
    return loss / G, (p - t) / G


def loss_fn(theta, X, t, groups):
    z, _ = forward(theta, X)
    return loss_and_dz(z, t, groups)[0]


def grad_fn(theta, X, t, groups):
    z, cache = forward(theta, X)
    loss, dz = loss_and_dz(z, t, groups)
    return loss, backward(theta, cache, dz)


class Adam:
    """Adam with bias correction (Kingma and Ba)."""

    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)


def proposal_probs(theta, A, others, alpha):
    """Mixture (1-alpha) softmax(MLP(features)) + alpha/I over the rows of A."""
    z, _ = forward(theta, row_features(A, others))
    p = group_softmax(z, [np.arange(A.shape[0])])
    return (1 - alpha) * p + alpha / A.shape[0]
