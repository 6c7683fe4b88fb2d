"""Pins of the oracle's importance-weighted least-squares branch (sampling
with weights, Section 2.2's sketching view of the sampled LS of Alg. 3).

A weight w_s on a sampled row means the row counts w_s times: for integer
weights the weighted problem is exactly the unweighted problem on a sample
that lists row s w_s times.  That fixes both the normal-equation blocks
(rows scaled by w) and the least-squares rows (scaled by sqrt(w)), and a
slip of w for sqrt(w) in either fails here."""
import numpy as np
import pytest

from oracle import cprand as C
from oracle import philox
import synth


def _problem(dims, R, seed):
    p = synth.make_problem(dims, R, congruence=None, noise=0.05, seed=seed)
    return synth.dense_tensor(p), [np.asarray(M) for M in p.init]


@pytest.mark.parametrize("dims,n", [((7, 6, 5), 0), ((7, 6, 5), 2), ((4, 3, 5, 3), 1)])
def test_integer_weights_equal_repeated_rows(dims, n):
    R, S = 3, 11
    X, A = _problem(dims, R, 1701066101)
    A[n] = np.zeros((dims[n], R))
    idx = philox.sample_indices(dims, n, S, 1701066101, 3)
    w = np.random.default_rng(5).integers(1, 5, S).astype(np.float64)
    rep = np.repeat(idx, w.astype(int), axis=0)
    # least-squares solution
    ls_w = C.sampled_ls(X, idx, A, n, w)
    ls_rep = C.sampled_ls(X, rep, A, n)
    assert np.allclose(ls_w, ls_rep, rtol=1e-11, atol=1e-12)
    # normal-equation blocks
    Ww, Vw = C.sampled_normal_blocks(X, idx, A, n, w)
    Wr, Vr = C.sampled_normal_blocks(X, rep, A, n)
    assert np.allclose(Ww, Wr, rtol=1e-12, atol=1e-12)
    assert np.allclose(Vw, Vr, rtol=1e-12, atol=1e-12)


def test_weighted_ls_solves_weighted_normal_equations():
    dims, n, R, S = (8, 7, 6), 1, 4, 40
    X, A = _problem(dims, R, 1701066102)
    idx = philox.sample_indices(dims, n, S, 1701066102, 0)
    w = np.random.default_rng(6).uniform(0.1, 3.0, S)
    W, V = C.sampled_normal_blocks(X, idx, A, n, w)
    assert np.allclose(C.sampled_ls(X, idx, A, n, w), np.linalg.solve(V, W.T).T, rtol=1e-9, atol=1e-11)


def test_unit_and_constant_weights():
    dims, n, R, S = (6, 5, 7), 2, 3, 25
    X, A = _problem(dims, R, 1701066103)
    idx = philox.sample_indices(dims, n, S, 1701066103, 1)
    one = np.ones(S)
    assert np.array_equal(C.sampled_ls(X, idx, A, n, one), C.sampled_ls(X, idx, A, n))
    W0, V0 = C.sampled_normal_blocks(X, idx, A, n)
    W1, V1 = C.sampled_normal_blocks(X, idx, A, n, one)
    assert np.array_equal(W0, W1) and np.array_equal(V0, V1)
    # a constant weight scales both blocks and leaves the minimiser alone
    Wc, Vc = C.sampled_normal_blocks(X, idx, A, n, 2.5 * one)
    assert np.allclose(Wc, 2.5 * W0, rtol=1e-14) and np.allclose(Vc, 2.5 * V0, rtol=1e-14)
    assert np.allclose(C.sampled_ls(X, idx, A, n, 2.5 * one), C.sampled_ls(X, idx, A, n), rtol=1e-10)
