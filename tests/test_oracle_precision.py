"""Pins of the oracle's BF16 precision form: the rounding against torch's
own BF16 conversion and hand-built ties, the BF16 normal blocks against
the exact ones on data that BF16 holds exactly, and the refinement step
against the fixed point and contraction of iterative refinement."""
import numpy as np
import torch

from oracle import cprand as C
from oracle import philox
from oracle import precision as PR
import synth


def test_bf16_round_matches_torch_and_ties():
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.standard_normal(20000), rng.standard_normal(2000) * 1e-30,
                        rng.standard_normal(2000) * 1e30]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(PR.bf16_round(x), want)
    # exact ties: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7 -> even (1);
    # 1 + 3 * 2^-8 lies halfway between 1 + 2^-7 and 1 + 2^-6 -> even (1 + 2^-6)
    t = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 0.0], dtype=np.float32)
    assert np.array_equal(PR.bf16_round(t), np.array([1.0, 1 + 2.0 ** -6, -1.0, 0.0], dtype=np.float32))


def test_bf16_blocks_exact_on_bf16_representable_data():
    """Small integers and their products are exact in BF16 and FP32: the
    BF16 blocks then equal the plain sampled blocks exactly."""
    rng = np.random.default_rng(12)
    dims, n, R, S = (6, 5, 4), 1, 3, 17
    X = rng.integers(-8, 9, dims).astype(np.float64)
    A = [rng.integers(-3, 4, (I, R)).astype(np.float64) for I in dims]
    idx = philox.sample_indices(dims, n, S, 77, 0)
    W, V = PR.bf16_normal_blocks(X.astype(np.float32), idx, [M.astype(np.float32) for M in A], n)
    W0, V0 = C.sampled_normal_blocks(X, idx, A, n)
    assert np.array_equal(W, W0) and np.array_equal(V, V0)


def test_bf16_blocks_error_is_bf16_sized():
    p = synth.make_problem((30, 20, 25), 4, congruence=0.5, noise=0.01, seed=1701066111)
    X = synth.dense_tensor(p)
    A = [np.asarray(M) for M in p.init]
    idx = philox.sample_indices(X.shape, 0, 200, 5, 0)
    W, V = PR.bf16_normal_blocks(X.astype(np.float32), idx, [M.astype(np.float32) for M in A], 0)
    W0, V0 = C.sampled_normal_blocks(X, idx, A, 0)
    # two roundings per product term of relative size <= 2^-9 each
    assert np.linalg.norm(W - W0) / np.linalg.norm(W0) < 2 * 2.0 ** -9
    assert np.linalg.norm(V - V0) / np.linalg.norm(V0) < 2 * 2.0 ** -9
    assert np.linalg.norm(W - W0) / np.linalg.norm(W0) > 1e-5        # the rounding is really there


def test_refinement_fixed_point_and_contraction():
    rng = np.random.default_rng(13)
    R, In = 6, 9
    Z = rng.standard_normal((40, R))
    V_hi = Z.T @ Z
    W_hi = rng.standard_normal((In, R))
    A_star = np.linalg.solve(V_hi, W_hi.T).T
    # exact operator: one step lands on the solution from anywhere
    A0 = rng.standard_normal((In, R))
    assert np.allclose(PR.refine_step(A0, V_hi, W_hi, V_hi), A_star, rtol=1e-10, atol=1e-12)
    # the solution is a fixed point for any operator
    V_lo = V_hi + 1e-2 * np.diag(np.diag(V_hi))
    assert np.allclose(PR.refine_step(A_star, V_lo, W_hi, V_hi), A_star, rtol=1e-12, atol=1e-12)
    # a perturbed operator contracts the error by ||I - V_hi V_lo^{-1}||
    A0 = np.linalg.solve(V_lo, (W_hi + 1e-2 * rng.standard_normal((In, R))).T).T
    A1 = PR.refine_step(A0, V_lo, W_hi, V_hi)
    rho = np.linalg.norm(np.eye(R) - V_hi @ np.linalg.inv(V_lo), 2)
    e0, e1 = np.linalg.norm(A0 - A_star), np.linalg.norm(A1 - A_star)
    assert rho < 0.05 and e1 <= rho * e0 * (1 + 1e-9) and e1 < 0.1 * e0
