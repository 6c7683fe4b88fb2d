"""Pins of the importance-weighted fit estimate (oracle/fitset.py): slice
energies by brute force, the estimator's expectation by enumerating every
entry with its probability, draw frequencies, the weight bound, the beta = 0
reduction to the paper's estimate (Section 3.4), and its accuracy against
the exact fit on a tensor with heavy slices."""
import itertools

import numpy as np
import pytest

from oracle import cprand as C
from oracle import fitset as FS
from oracle import philox
from oracle.tensor import fnorm
import synth


def test_slice_energies_brute_force():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((3, 4, 5))
    s = FS.slice_energies(X)
    for m in range(3):
        assert np.isclose(s[m].sum(), (X ** 2).sum())
        for i in range(X.shape[m]):
            tot = 0.0
            for idx in itertools.product(*[range(d) for d in X.shape]):
                if idx[m] == i:
                    tot += X[idx] ** 2
            assert np.isclose(s[m][i], tot, rtol=1e-13)


def _probabilities(dims, qs, beta):
    """q(i) for every multi-index (row-major over dims), from the integer tables."""
    P = int(np.prod(dims))
    out = np.empty(P)
    for k, idx in enumerate(itertools.product(*[range(d) for d in dims])):
        prod = 1.0
        for m, q in enumerate(qs):
            prod *= float(q[idx[m]]) / float(q.sum())
        out[k] = beta * prod + (1.0 - beta) / P
    return out


@pytest.mark.parametrize("beta", [0.0, 0.3, 0.5, 0.9])
def test_expectation_is_the_residual_norm(beta):
    """sum_i q(i) * P w(i) e_i^2 = sum_i e_i^2: the estimate is unbiased."""
    dims = (3, 4, 5)
    rng = np.random.default_rng(2)
    X = rng.standard_normal(dims) * np.linspace(0.1, 3.0, 3)[:, None, None]
    qs = FS.energy_proposals(X, 0.1)
    prob = _probabilities(dims, qs, beta)
    assert np.isclose(prob.sum(), 1.0, atol=1e-14)
    E = rng.standard_normal(dims)
    allidx = np.array(list(itertools.product(*[range(d) for d in dims])))
    w = FS.weights(allidx, qs, beta, dims)
    P = np.prod(dims)
    e2 = E[tuple(allidx.T)] ** 2
    assert np.isclose(np.sum(prob * P * w * e2), np.sum(E ** 2), rtol=1e-13)
    assert np.all(w <= 1.0 / (1.0 - beta) * (1 + 1e-15)) if beta < 1 else True


def test_draw_frequencies_follow_the_mixture():
    dims = (3, 2, 4)
    rng = np.random.default_rng(3)
    X = rng.standard_normal(dims) * np.array([1.0, 5.0, 0.2])[:, None, None]
    qs = FS.energy_proposals(X, 0.1)
    beta = 0.6
    P_hat = 200000
    idx, w = FS.weighted_fit_indices(dims, P_hat, 17, qs, beta)
    prob = _probabilities(dims, qs, beta)
    flat = np.ravel_multi_index(tuple(idx.T), dims)
    counts = np.bincount(flat, minlength=int(np.prod(dims)))
    expected = prob * P_hat
    z = (counts - expected) / np.sqrt(expected)
    assert np.max(np.abs(z)) < 5.0, z
    assert np.all(w <= 1.0 / (1.0 - beta) + 1e-12)
    # the weights are those of the entries drawn
    assert np.allclose(w, FS.weights(idx, qs, beta, dims), rtol=0, atol=0)


def test_beta_zero_is_the_papers_estimate():
    p = synth.make_problem((20, 15, 10), 3, congruence=0.5, noise=0.05, seed=4)
    X = synth.dense_tensor(p)
    qs = FS.energy_proposals(X, 0.1)
    idx, w = FS.weighted_fit_indices(X.shape, 4096, 9, qs, 0.0)
    assert np.all(w == 1.0)
    # uniform draws: every row of every mode appears about equally often
    for m in range(3):
        c = np.bincount(idx[:, m], minlength=X.shape[m])
        assert c.min() > 0.6 * 4096 / X.shape[m]
    nx = fnorm(X)
    F1 = FS.weighted_sampled_fit(X, nx, p.lam, p.factors, idx, w)
    F2 = C.sampled_fit(X, nx, p.lam, p.factors, idx)
    assert F1 == F2


def test_beats_uniform_on_a_tensor_with_heavy_slices():
    """Spiky factors (10% of rows x20) and a model that misses them: the
    uniform estimate overstates the exact fit; the weighted one, from the
    slice energies of X, stays close (median over seeds)."""
    p = synth.make_problem((30, 30, 30, 30), 4, congruence=0.5, noise=0.05, seed=5, spiky=0.1, spike=20.0)
    X = synth.dense_tensor(p)
    nx = fnorm(X)
    rng = np.random.default_rng(6)
    # a model with the right structure but the spiky rows damped
    A = []
    for M, sp in zip(p.factors, p.spike_rows):
        M = M.copy()
        M[sp] *= 0.6
        A.append(M + 0.02 * rng.standard_normal(M.shape))
    F = C.exact_fit(X, p.lam, A)
    qs = FS.energy_proposals(X, 0.1)
    err_u, err_w = [], []
    for seed in range(20):
        fidx = philox.fit_indices(X.shape, 2 ** 14, seed)
        err_u.append(C.sampled_fit(X, nx, p.lam, A, fidx) - F)
        idx, w = FS.weighted_fit_indices(X.shape, 2 ** 14, seed, qs, 0.5)
        err_w.append(FS.weighted_sampled_fit(X, nx, p.lam, A, idx, w) - F)
    mu, mw = np.median(np.abs(err_u)), np.median(np.abs(err_w))
    assert mw < 0.2 * mu, (mu, mw, F)
    assert mw < 5e-3, (mw, F)
