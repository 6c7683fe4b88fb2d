"""Importance sampling of Khatri-Rao rows from per-mode proposals.

Test infrastructure (see oracle/__init__.py).

A proposal for mode m is a vector of positive integers q (one per row of
A^(m)), so that both the GPU and this reference search the same integer
cumulative table and draw identical indices.  Row i of mode m is drawn with
probability q_i / Q_m, Q_m = sum q.  A multi-index is drawn mode by mode from
the same Philox words as uniform sampling; the least-squares rows are then
weighted by w_s = prod_m (1/I_m) / (q_{i_m}/Q_m), the ratio of the uniform
probability to the proposal probability, so that the sampled normal equations
stay unbiased estimates of the full ones (with uniform proposals w_s = 1 and
the method reduces to CPRAND, Section 3.2).
"""
import numpy as np

from . import philox

Q_SCALE = 2.0 ** 32


def quantize(p, alpha):
    """Mix a probability vector with uniform, (1-alpha) p + alpha/I, and
    quantise to integers q_i = max(1, floor(p_i 2^32)), at most 2^32 - 1."""
    p = np.asarray(p, dtype=np.float64)
    I = p.size
    pm = (1.0 - alpha) * p + alpha / I
    q = np.floor(pm * Q_SCALE)
    q = np.clip(q, 1, Q_SCALE - 1)
    return q.astype(np.uint64)


def cdf(q):
    """Inclusive prefix table with a leading zero: c[0] = 0, c[i+1] = c[i] + q_i."""
    c = np.zeros(q.size + 1, dtype=np.uint64)
    c[1:] = np.cumsum(q.astype(np.uint64))
    return c


def draw_rows(words, c):
    """First i with c[i+1] > target, target = floor(u * Q / 2^64)."""
    Q = c[-1]
    target, _ = philox.mulhilo64(words, np.uint64(Q))
    return np.searchsorted(c[1:], target, side="right").astype(np.int64)


def importance_indices(dims, n, S, seed, t, qs):
    """(idx, w): S multi-indices drawn from the per-mode proposals qs[m]
    (m != n) with the Philox words of uniform sampling, and their weights."""
    N = len(dims)
    words = philox.sample_words(N, n, S, seed, t)
    idx = np.full((S, N), -1, dtype=np.int64)
    w = np.ones(S, dtype=np.float64)
    for m in range(N):
        if m == n:
            continue
        c = cdf(qs[m])
        idx[:, m] = draw_rows(words[:, m], c)
        Q = float(c[-1])
        qi = qs[m][idx[:, m]].astype(np.float64)
        w = w * (Q / (float(dims[m]) * qi))
    return idx, w
