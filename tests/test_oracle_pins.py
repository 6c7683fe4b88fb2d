"""Pins of the FP64 oracle against what the paper and the mathematics fix:
identities, brute force on tiny tensors, exact recovery, the coherence
lemmas and their tight example, the sample-size rule's printed values, the
accuracy of the sampled fit estimate, and unitarity of the mixing."""
import math

import numpy as np
import pytest

from oracle import cprand as C
from oracle import leverage as L
from oracle import philox, proposal, score as SC
from oracle.tensor import (column_index, cp_full, fnorm, khatri_rao, kron,
                           krp_except, ttm, unfold)
import synth


def _rand_factors(rng, dims, R):
    return [rng.standard_normal((I, R)) for I in dims]


def _outer_tensor(lam, A):
    """Brute-force sum of outer products, element by element."""
    dims = [M.shape[0] for M in A]
    X = np.zeros(dims)
    for i in np.ndindex(*dims):
        X[i] = sum(lam[r] * np.prod([A[m][i[m], r] for m in range(len(A))])
                   for r in range(len(lam)))
    return X


# --- identities of Section 2.1 ------------------------------------------------
def test_kron_matches_library():
    rng = np.random.default_rng(1)
    A, B = rng.standard_normal((3, 4)), rng.standard_normal((5, 2))
    assert np.allclose(kron(A, B), np.kron(A, B), rtol=0, atol=1e-15)


def test_krp_gram_and_distributivity():
    rng = np.random.default_rng(2)
    A, B = rng.standard_normal((4, 3)), rng.standard_normal((5, 3))
    Z = khatri_rao([A, B])
    assert np.allclose(Z.T @ Z, (A.T @ A) * (B.T @ B), rtol=1e-13)       # eq. KRGram
    Am, Bm = rng.standard_normal((4, 6)), rng.standard_normal((6, 3))
    Cm, Dm = rng.standard_normal((5, 2)), rng.standard_normal((2, 3))
    assert np.allclose(np.kron(Am @ Bm, Cm @ Dm), np.kron(Am, Cm) @ np.kron(Bm, Dm))
    assert np.allclose(khatri_rao([Am @ Bm, Cm @ Dm]),
                       np.kron(Am, Cm) @ khatri_rao([Bm, Dm]))            # eq. krdist


@pytest.mark.parametrize("dims,R", [((3, 4, 5), 2), ((2, 3, 2, 3), 3)])
def test_unfold_equals_factor_times_krp(dims, R):
    """X~_(n) = A^(n) Z^(n)T (eq. Zn) on a tensor built entry by entry."""
    rng = np.random.default_rng(3)
    A = _rand_factors(rng, dims, R)
    lam = rng.uniform(0.5, 1.5, R)
    X = _outer_tensor(lam, A)
    assert np.allclose(cp_full(lam, A), X, atol=1e-13)
    for n in range(len(dims)):
        Z = krp_except(A, n)
        assert np.allclose(unfold(X, n), (A[n] * lam) @ Z.T, atol=1e-12)
        # Gram of Z is the Hadamard product of the other Grams
        G = np.ones((R, R))
        for m in range(len(dims)):
            if m != n:
                G = G * (A[m].T @ A[m])
        assert np.allclose(Z.T @ Z, G, rtol=1e-12)


@pytest.mark.parametrize("dims,R", [((3, 4, 5), 2), ((2, 3, 2, 3), 3)])
def test_skr_and_fibers_match_explicit_rows(dims, R):
    """Sampled KRP rows equal rows of the explicit product, and sampled fibers
    equal columns of the explicit unfolding, at the column given by the
    unfolding index map (Alg. 2; Section 3.2)."""
    rng = np.random.default_rng(4)
    A = _rand_factors(rng, dims, R)
    X = rng.standard_normal(dims)
    for n in range(len(dims)):
        idx = philox.sample_indices(dims, n, 40, 11, n)
        Zs = C.skr(idx, A, n)
        Xs = C.sample_fibers(X, idx, n)
        Z = krp_except(A, n)
        Xn = unfold(X, n)
        for s in range(idx.shape[0]):
            j = column_index(idx[s], dims, n)
            assert np.array_equal(Zs[s], Z[j]) or np.allclose(Zs[s], Z[j], rtol=1e-15)
            assert np.array_equal(Xs[:, s], Xn[:, j])


def test_ttm_unfolding_identity():
    """Y = X x_1 U1 ... x_N UN  <=>  Y_(n) = Un X_(n) (U_N (x) .. (x) U_1, skip n)^T."""
    rng = np.random.default_rng(5)
    dims = (2, 3, 4)
    X = rng.standard_normal(dims)
    U = [rng.standard_normal((I + 1, I)) for I in dims]
    Y = X
    for m in range(3):
        Y = ttm(Y, U[m], m)
    for n in range(3):
        K = None
        for m in reversed(range(3)):
            if m == n:
                continue
            K = U[m] if K is None else np.kron(K, U[m])
        assert np.allclose(unfold(Y, n), U[n] @ unfold(X, n) @ K.T)


# --- the sampled least-squares step ---------------------------------------------
def test_sample_size_rule_printed_values():
    assert C.sample_size(5) == 80 and C.sample_size(6) == 108
    assert C.sample_size_ceil_log(10) == 300
    assert C.sample_size_ceil_log(25) == 1000
    assert C.sample_size_ceil_log(50) == 2000


def test_exact_recovery_noise_free():
    """Noise-free rank-R tensor, other factors at the truth: the sampled LS
    returns the true factor scaled by lam, with zero residual."""
    rng = np.random.default_rng(6)
    dims, R = (6, 7, 8), 3
    A = _rand_factors(rng, dims, R)
    lam = np.array([1.0, 2.0, 0.5])
    X = cp_full(lam, A)
    for n in range(3):
        idx = philox.sample_indices(dims, n, 12, 3, 0)
        got = C.sampled_ls(X, idx, A, n)
        assert np.allclose(got, A[n] * lam, rtol=1e-10, atol=1e-12)
        W, V = C.sampled_normal_blocks(X, idx, A, n)
        assert np.allclose(np.linalg.solve(V, W.T).T, A[n] * lam, rtol=1e-9, atol=1e-11)


def test_all_rows_once_is_textbook_als():
    """Enumerating every Khatri-Rao row exactly once turns the sampled LS into
    the exact CP-ALS update X_(n) Z (Z^T Z)^{-1} (Alg. 1)."""
    rng = np.random.default_rng(7)
    dims, R = (4, 3, 5), 2
    A = _rand_factors(rng, dims, R)
    X = rng.standard_normal(dims)
    n = 1
    grid = np.array(list(np.ndindex(*[dims[m] if m != n else 1 for m in range(3)])))
    grid[:, n] = -1
    got = C.sampled_ls(X, grid, A, n)
    Z = krp_except(A, n)
    G = (A[0].T @ A[0]) * (A[2].T @ A[2])
    want = unfold(X, n) @ Z @ np.linalg.inv(G)
    assert np.allclose(got, want, rtol=1e-11)


def test_normalize_and_zero_column():
    M = np.array([[3.0, 0.0], [4.0, 0.0]])
    An, lam = C.normalize(M)
    assert np.allclose(lam, [5.0, 0.0])
    assert np.allclose(An, [[0.6, 0.0], [0.8, 0.0]])


# --- mixing ---------------------------------------------------------------------
def _dft(I):
    k = np.arange(I)
    return np.exp(-2j * np.pi * np.outer(k, k) / I) / np.sqrt(I)


def test_fft_ortho_is_unitary_dft():
    for I in (1, 2, 3, 5, 6, 50):
        x = np.random.default_rng(I).standard_normal(I) + 0j
        assert np.allclose(np.fft.fft(x, norm="ortho"), _dft(I) @ x)
        F = _dft(I)
        assert np.allclose(F.conj().T @ F, np.eye(I))


def test_mix_tensor_matches_explicit_ttm_and_unmix_identity():
    rng = np.random.default_rng(8)
    dims = (3, 4, 5)
    X = rng.standard_normal(dims)
    signs = philox.sign_vectors(dims, 21)
    Xh = C.mix_tensor(X, signs)
    Y = X.astype(complex)
    for m in range(3):
        Y = ttm(Y, _dft(dims[m]) @ np.diag(signs[m]), m)
    assert np.allclose(Xh, Y)
    assert math.isclose(fnorm(Xh), fnorm(X), rel_tol=1e-13)      # unitary
    # eq. unmixX: (kron_{m != n} F_m D_m) X_(n)^T = (D_n F_n^* Xh_(n))^T
    for n in range(3):
        K = None
        for m in reversed(range(3)):
            if m == n:
                continue
            Fm = _dft(dims[m]) @ np.diag(signs[m])
            K = Fm if K is None else np.kron(K, Fm)
        lhs = K @ unfold(X, n).T
        rhs = (np.diag(signs[n]) @ _dft(dims[n]).conj().T @ unfold(Xh, n)).T
        assert np.allclose(lhs, rhs)


def test_mixed_unsampled_ls_is_real_and_equals_unmixed():
    """With every row kept, the mixed problem is a unitary change of basis of
    the original one, so its solution is real and equals the unmixed one."""
    rng = np.random.default_rng(9)
    dims, R = (4, 5, 3), 2
    A = _rand_factors(rng, dims, R)
    X = rng.standard_normal(dims)
    signs = philox.sign_vectors(dims, 4)
    Xh = C.mix_tensor(X, signs)
    Ah = [C.mix_factor(A[m], signs[m]) for m in range(3)]
    n = 2
    grid = np.array(list(np.ndindex(*[dims[m] if m != n else 1 for m in range(3)])))
    grid[:, n] = -1
    Zh = C.skr(grid, Ah, n)
    M = C.unmix_fibers(C.sample_fibers(Xh, grid, n), signs[n])
    sol, *_ = np.linalg.lstsq(Zh, M.T, rcond=None)
    assert np.abs(sol.imag).max() < 1e-12
    real = C.mixed_sampled_ls(Xh, grid, Ah, n, signs[n])
    plain = C.sampled_ls(X, grid, A, n)
    assert np.allclose(sol.real.T, plain) and np.allclose(real, plain)
    W, V = C.mixed_normal_blocks(Xh, grid, Ah, n, signs[n])
    assert np.allclose(np.linalg.solve(V, W.T).T, plain)


def test_mixed_step_needs_no_fft():
    """The remixed solution of the real-constrained sampled LS (Alg. 4, eq.
    rcLS) in closed form: with Y = X-hat_S conj(Z-hat_S) and Z = Y V^{-1},
    F D Re(D F^* Z) = (Z + P conj Z) / 2, P the index reversal k -> -k mod I_n
    (the DFT is symmetric and F^2 = P).  Column norms agree across the mix.
    Odd and even I_n (the self-paired rows differ)."""
    rng = np.random.default_rng(21)
    for dims in [(7, 5, 6), (8, 5, 6)]:
        R, n = 3, 0
        A = _rand_factors(rng, dims, R)
        X = rng.standard_normal(dims)
        signs = philox.sign_vectors(dims, 8)
        Xh = C.mix_tensor(X, signs)
        Ah = [C.mix_factor(A[m], signs[m]) for m in range(3)]
        idx = philox.sample_indices(dims, n, 12, 8, 0)
        Wr, V = C.mixed_normal_blocks(Xh, idx, Ah, n, signs[n])
        ref_A, ref_lam = C.normalize(C.mixed_sampled_ls(Xh, idx, Ah, n, signs[n]))
        ref = C.mix_factor(ref_A, signs[n])
        Y = C.sample_fibers(Xh, idx, n) @ np.conj(C.skr(idx, Ah, n))
        assert np.allclose(C.unmix_factor(Y, signs[n]).real, Wr)
        Z = Y @ np.linalg.inv(V)
        rev = (-np.arange(dims[n])) % dims[n]
        Ahat = 0.5 * (Z + np.conj(Z[rev]))
        lam = np.linalg.norm(Ahat, axis=0)
        assert np.allclose(lam, ref_lam, rtol=1e-12)
        assert np.allclose(Ahat / lam, ref, rtol=1e-10, atol=1e-12)
        assert np.abs(Ahat[0].imag).max() < 1e-15


def test_mix_factor_roundtrip():
    rng = np.random.default_rng(10)
    A = rng.standard_normal((50, 4))
    s = philox.sign_vectors((50,), 2)[0]
    assert np.allclose(C.unmix_factor(C.mix_factor(A, s), s).real, A)


# --- coherence (Section 3.2 lemmas) ---------------------------------------------
def test_coherence_tight_example():
    A = np.array([[1.0], [1.0]])
    B = np.array([[1.0], [-1.0]])
    assert math.isclose(L.coherence(A), 0.5)
    assert math.isclose(L.coherence(B), 0.5)
    assert math.isclose(L.coherence(khatri_rao([A, B])), 0.25)


def test_coherence_lemmas_random():
    rng = np.random.default_rng(11)
    for trial in range(20):
        I, K, R = rng.integers(3, 9), rng.integers(3, 9), rng.integers(1, 3)
        A = rng.standard_normal((I, R))
        B = rng.standard_normal((K, R))
        if trial % 3 == 0:
            A[0] *= 30.0               # a coherent factor
        muA, muB = L.coherence(A), L.coherence(B)
        assert math.isclose(L.coherence(np.kron(A, B)), muA * muB, rel_tol=1e-10)
        assert L.coherence(khatri_rao([A, B])) <= muA * muB * (1 + 1e-12)
        lA, lB = L.leverage_scores(A), L.leverage_scores(B)
        lZ = L.leverage_scores(khatri_rao([A, B]))
        assert np.all(lZ <= np.outer(lA, lB).ravel() + 1e-12)          # every row
        for M in (A, B):
            l = L.leverage_scores(M)
            assert math.isclose(l.sum(), np.linalg.matrix_rank(M), rel_tol=1e-10)
            assert M.shape[1] / M.shape[0] - 1e-12 <= l.max() <= 1 + 1e-12


def test_krp_marginal_closed_form_matches_bruteforce():
    rng = np.random.default_rng(12)
    for dims, R in (((5, 6, 7), 3), ((4, 3, 5, 6), 4)):
        mats = [rng.standard_normal((I, R)) for I in dims]
        mats[0][1] *= 10
        cf = L.krp_marginals(mats)
        bf = L.krp_marginals_bruteforce(mats)
        for a, b in zip(cf, bf):
            assert np.allclose(a, b, rtol=1e-9)
            assert math.isclose(a.sum(), R, rel_tol=1e-9)
        assert np.allclose(L.krp_leverage_gram(mats), L.krp_leverage_exact(mats), rtol=1e-9)


# --- the sampled fit estimate (Section 3.4) ----------------------------------------
def test_chernoff_numbers():
    gamma = 1.05 ** 2 - 1
    assert math.isclose(gamma, 0.1025)
    assert round(math.log(1 / 0.02) / gamma ** 2) == 372


def test_sampled_fit_accuracy_at_95_percent():
    """At P-hat = 2^14 and an exact fit of 95%, the sampled estimate is within
    1e-3 relative of the exact fit (Section 4.1), and its spread over seeds
    matches the Gaussian-residual value (1-F)/sqrt(2 P-hat)."""
    rng = np.random.default_rng(13)
    dims, R = (40, 40, 40), 3
    A = _rand_factors(rng, dims, R)
    lam = np.ones(R)
    Xt = cp_full(lam, A)
    Nz = rng.standard_normal(dims)
    X = Xt + (0.05 / math.sqrt(1 - 0.05 ** 2)) * fnorm(Xt) / fnorm(Nz) * Nz  # ||E||/||X|| ~ 0.05
    normX = fnorm(X)
    F = C.exact_fit(X, lam, A)
    assert abs(F - 0.95) < 2e-3
    est = np.array([C.sampled_fit(X, normX, lam, A, philox.fit_indices(dims, 2 ** 14, s))
                    for s in range(100)])
    rel = np.abs(est - F) / F
    assert rel.max() < 1e-3
    sigma = (1 - F) / math.sqrt(2 * 2 ** 14)
    assert 0.7 * sigma < est.std() < 1.3 * sigma


def test_stop_rule():
    r = C.StopRule(max_iters=10, tol=1e-4)
    assert not r(0, 0.5) and not r(1, 0.6) and r(2, 0.60005)
    r = C.StopRule(max_iters=10, fit_target=0.9)
    assert not r(0, 0.8) and r(1, 0.95)
    r = C.StopRule(max_iters=100, patience=2)
    assert not r(0, 0.5) and not r(1, 0.4) and r(2, 0.45)
    r = C.StopRule(max_iters=3)
    assert not r(0, 0.1) and not r(1, 0.1) and r(2, 0.1)


# --- score (eq. score) -----------------------------------------------------------
def test_score_invariances():
    rng = np.random.default_rng(14)
    A = _rand_factors(rng, (6, 7, 8), 4)
    assert math.isclose(SC.score(A, A), 1.0)
    perm = [2, 0, 3, 1]
    B = [M[:, perm] * rng.uniform(0.5, 2, 4) for M in A]
    assert math.isclose(SC.score(A, B), 1.0)
    S = SC.component_scores(A, [M + 0.3 * rng.standard_normal(M.shape) for M in A])
    rows = np.arange(4)
    import itertools
    brute = max(np.mean(S[rows, list(p)]) for p in itertools.permutations(range(4)))
    from scipy.optimize import linear_sum_assignment
    r, c = linear_sum_assignment(-S)
    assert math.isclose(brute, S[r, c].mean())


# --- importance sampling -----------------------------------------------------------
def test_uniform_proposal_reproduces_uniform_sampling():
    dims = (9, 12, 7)
    qs = [np.full(I, 1000, dtype=np.uint64) for I in dims]
    for n in range(3):
        idx, w = proposal.importance_indices(dims, n, 500, 8, 2, qs)
        assert np.array_equal(idx, philox.sample_indices(dims, n, 500, 8, 2))
        assert np.all(w == 1.0)


def test_importance_draws_follow_proposal_and_are_unbiased():
    rng = np.random.default_rng(15)
    dims, R = (6, 5, 4), 3
    A = _rand_factors(rng, dims, R)
    A[1][0] *= 8
    n = 0
    qs = [None] + [proposal.quantize(L.leverage_scores(A[m]) / R, 0.1) for m in (1, 2)]
    S = 40000
    idx, w = proposal.importance_indices(dims, n, S, 9, 0, qs)
    for m in (1, 2):
        p = qs[m].astype(float) / qs[m].sum()
        counts = np.bincount(idx[:, m], minlength=dims[m])
        assert np.allclose(counts / S, p, atol=4 * np.sqrt(p * (1 - p) / S).max())
    Z = C.skr(idx, A, n)
    est = (Z * w[:, None]).T @ Z / S
    full = krp_except(A, n)
    want = full.T @ full / full.shape[0]
    assert np.allclose(est, want, rtol=0.05, atol=0.05 * np.abs(want).max())


def test_quantize_and_cdf():
    p = np.array([0.5, 0.25, 0.25, 0.0])
    q = proposal.quantize(p, 0.0)
    assert list(q) == [2 ** 31, 2 ** 30, 2 ** 30, 1]
    c = proposal.cdf(q)
    assert c[0] == 0 and c[-1] == q.sum()
    words = np.array([0, 2 ** 63, 2 ** 64 - 1], dtype=np.uint64)
    assert list(proposal.draw_rows(words, c)) == [0, 1, 3]


# --- end to end ---------------------------------------------------------------------
def test_cprand_recovers_noise_free_tensor():
    p = synth.make_problem((20, 22, 24), 3, congruence=0.5, noise=0.0, seed=5)
    X = synth.dense_tensor(p)
    lam, A, hist = C.cprand(X, 3, 60, p.init, seed=17, max_iters=60, tol=0.0,
                            fit_target=1 - 1e-9)
    assert C.exact_fit(X, lam, A) > 1 - 1e-6
    assert SC.score(p.factors, A) > 0.99


def test_cprand_noisy_fit_near_one_minus_eta():
    p = synth.make_problem((30, 30, 30), 3, congruence=0.5, noise=0.01, seed=6)
    X = synth.dense_tensor(p)
    lam, A, hist = C.cprand(X, 3, C.sample_size(5), p.init, seed=3, max_iters=60,
                            tol=0.0)
    F = C.exact_fit(X, lam, A)
    assert abs(F - 0.99) < 2e-3
    assert SC.score(p.factors, A) > 0.97


def test_cprand_mix_recovers_coherent_tensor():
    p = synth.make_problem((24, 24, 24), 3, congruence=0.5, noise=0.01, seed=7,
                           spiky=0.1, spike=20.0)
    X = synth.dense_tensor(p)
    lam, A, hist = C.cprand_mix(X, 3, 80, p.init, seed=5, max_iters=200, tol=0.0)
    assert abs(C.exact_fit(X, lam, A) - 0.99) < 3e-3
    # without mixing, uniform sampling of the coherent problem fails (Section 3.3)
    lam0, A0, _ = C.cprand(X, 3, 80, p.init, seed=5, max_iters=60, tol=0.0)
    assert C.exact_fit(X, lam0, A0) < 0.9
    assert all(np.isrealobj(M) for M in A)
    # the mixed-domain fit estimate tracks the exact fit
    assert abs(hist[-1] - C.exact_fit(X, lam, A)) < 2e-3
