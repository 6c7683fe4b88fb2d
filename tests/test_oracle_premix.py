"""Pins of the CPRAND-PREMIX oracle: scipy's DCT against the DCT-II matrix
written from its definition and its orthogonality, the tensor mix against
explicit mode products, the exact-step identity (the unsampled least
squares on the mixed tensor, unmixed, is the unmixed least squares), the
unmix as the inverse of the mix, and recovery of a coherent tensor."""
import numpy as np
import pytest

from oracle import cpals as CA
from oracle import cprand as C
from oracle import philox
from oracle import premix as PM
from oracle import score as SC
from oracle.tensor import fnorm, ttm
import synth


@pytest.mark.parametrize("I", [1, 2, 3, 5, 8, 13, 60])
def test_dct_matches_definition_and_is_orthogonal(I):
    Cm = PM.dct_matrix(I)
    assert np.allclose(Cm @ Cm.T, np.eye(I), atol=1e-13)
    rng = np.random.default_rng(51)
    Y = rng.standard_normal((I, 4))
    assert np.allclose(PM.dct_along(Y, 0), Cm @ Y, atol=1e-13)
    # spot values of the definition: row 0 constant 1/sqrt(I), row 1 a half-cosine
    assert np.allclose(Cm[0], np.full(I, 1 / np.sqrt(I)))
    if I > 1:
        assert abs(Cm[1, 0] - np.sqrt(2.0 / I) * np.cos(np.pi / (2 * I))) < 1e-15


def test_mix_matches_mode_products_and_keeps_the_norm():
    rng = np.random.default_rng(52)
    dims = (5, 4, 6)
    X = rng.standard_normal(dims)
    signs = philox.sign_vectors(dims, 9)
    Xh = PM.mix_tensor_dct(X, signs)
    want = X
    for m, I in enumerate(dims):
        want = ttm(want, PM.dct_matrix(I) @ np.diag(signs[m].astype(np.float64)), m)
    assert np.allclose(Xh, want, atol=1e-12)
    assert abs(fnorm(Xh) - fnorm(X)) < 1e-12
    A = rng.standard_normal((6, 3))
    assert np.allclose(PM.unmix_factor_dct(PM.mix_factor_dct(A, signs[2]), signs[2]), A, atol=1e-13)


@pytest.mark.parametrize("n", [0, 1, 2])
def test_exact_step_on_mixed_tensor_unmixes_to_the_plain_step(n):
    """Section 3.3: the LS update in the mixed basis is the mixed LS update."""
    rng = np.random.default_rng(53)
    dims, R = (7, 6, 5), 3
    X = rng.standard_normal(dims)
    A = [rng.standard_normal((I, R)) for I in dims]
    signs = philox.sign_vectors(dims, 11)
    Xh = PM.mix_tensor_dct(X, signs)
    Ah = [PM.mix_factor_dct(A[m], signs[m]) for m in range(3)]
    got, _ = CA.cpals_update(Xh, Ah, n)
    want, _ = CA.cpals_update(X, A, n)
    assert np.allclose(PM.unmix_factor_dct(got, signs[n]), want, rtol=1e-9, atol=1e-10)


def test_premix_recovers_noise_free_tensor():
    p = synth.make_problem((20, 22, 24), 3, congruence=0.5, noise=0.0, seed=5)
    X = synth.dense_tensor(p)
    lam, A, hist = PM.cprand_premix(X, 3, 60, p.init, 17, 60, fit_target=1 - 1e-9)
    assert C.exact_fit(X, lam, A) > 1 - 1e-6
    assert SC.score(p.factors, A) > 0.99


def test_premix_recovers_coherent_tensor():
    """The coherent problem on which uniform sampling of the unmixed tensor
    fails (Section 3.3): after the DCT mix the same sampling recovers it, and
    the fit estimate on the mixed tensor tracks the exact fit."""
    p = synth.make_problem((24, 24, 24), 3, congruence=0.5, noise=0.01, seed=7, spiky=0.1, spike=20.0)
    X = synth.dense_tensor(p)
    lam, A, hist = PM.cprand_premix(X, 3, 80, p.init, 5, 200)
    F = C.exact_fit(X, lam, A)
    assert abs(F - 0.99) < 3e-3
    assert abs(hist[-1] - F) < 2e-3
    lam0, A0, _ = C.cprand(X, 3, 80, p.init, seed=5, max_iters=60, tol=0.0)
    assert C.exact_fit(X, lam0, A0) < 0.9
