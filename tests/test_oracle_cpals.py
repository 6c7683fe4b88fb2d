"""Pins of the dense CP-ALS oracle (Alg. 1) and of the exact fit through
inner products: the MTTKRP against an element-by-element sum, the update
against the least-squares problem it solves (lstsq on the explicit
Khatri-Rao product), the inner-product fit against the fit of the
reconstructed tensor, and exact recovery of a noise-free tensor."""
import numpy as np
import pytest

from oracle import cpals as CA
from oracle import cprand as C
from oracle import score as SC
from oracle.tensor import cp_full, fnorm, krp_except, unfold
import synth


@pytest.mark.parametrize("dims,n", [((4, 3, 5), 0), ((4, 3, 5), 1), ((3, 4, 2, 3), 2), ((3, 4, 2, 3), 3)])
def test_mttkrp_matches_elementwise_sum(dims, n):
    rng = np.random.default_rng(31)
    R = 3
    X = rng.standard_normal(dims)
    A = [rng.standard_normal((I, R)) for I in dims]
    W = CA.mttkrp(X, A, n)
    want = np.zeros((dims[n], R))
    for idx in np.ndindex(*dims):
        for r in range(R):
            z = np.prod([A[m][idx[m], r] for m in range(len(dims)) if m != n])
            want[idx[n], r] += X[idx] * z
    assert np.allclose(W, want, rtol=1e-12, atol=1e-12)


def test_update_solves_the_full_least_squares_problem():
    rng = np.random.default_rng(32)
    dims, R = (6, 5, 7), 3
    X = rng.standard_normal(dims)
    A = [rng.standard_normal((I, R)) for I in dims]
    for n in range(3):
        An, _ = CA.cpals_update(X, A, n)
        Z = krp_except(A, n)
        sol, *_ = np.linalg.lstsq(Z, unfold(X, n).T, rcond=None)
        assert np.allclose(An, sol.T, rtol=1e-9, atol=1e-10)
        assert np.allclose(CA.gram_hadamard(A, n), Z.T @ Z, rtol=1e-12)


@pytest.mark.parametrize("n", [0, 1, 2])
def test_inner_product_fit_equals_reconstructed_fit(n):
    p = synth.make_problem((9, 8, 7), 3, congruence=0.5, noise=0.1, seed=1701066121)
    X = synth.dense_tensor(p)
    rng = np.random.default_rng(33)
    A = [M + 0.05 * rng.standard_normal(M.shape) for M in p.factors]
    A, lam = [normalize_cols(M)[0] for M in A], rng.uniform(0.5, 1.5, 3)
    F = CA.exact_fit_inner(X, lam, A, n)
    assert abs(F - C.exact_fit(X, lam, A)) < 1e-12
    assert abs(F - (1 - fnorm(X - cp_full(lam, A)) / fnorm(X))) < 1e-12


def normalize_cols(M):
    return C.normalize(M)


def test_cp_als_recovers_noise_free_tensor_and_fit_is_monotone():
    p = synth.make_problem((12, 10, 11), 3, congruence=0.5, noise=0.0, seed=1701066122)
    X = synth.dense_tensor(p)
    lam, A, hist = CA.cp_als(X, 3, p.init, 200, tol=1e-10)
    assert hist[-1] > 1 - 1e-6
    # near a perfect fit the expansion cancels: its error is ~ sqrt(eps)
    assert abs(hist[-1] - C.exact_fit(X, lam, A)) < 1e-7
    assert SC.score(p.factors, A) > 0.99
    # ALS never increases the residual of the exact problem
    assert all(b >= a - 1e-12 for a, b in zip(hist, hist[1:]))
