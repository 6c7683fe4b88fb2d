"""GPU parity: every C-ABI entry point against the FP64 oracle on the same
seeded inputs.  Tolerances: sample indices bit-exact; FP64 arithmetic 1e-12
relative; FP32 sampled MTTKRP 1e-5 relative (Frobenius); BF16 products 1e-2
relative (8-bit mantissa); fit estimates 1e-9 (FP64) / 1e-6 (FP32)."""
import math

import numpy as np
import pytest
import torch

from oracle import cprand as OC
from oracle import philox as OP
from oracle import proposal as OQ
from oracle.tensor import to_colmajor, from_colmajor
from gpu_util import close, cplx_factors_dev, dev, factors_dev, rel, view_of

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1701_06600_amd")


def _rng(s):
    return np.random.default_rng(s)


# --------------------------------------------------------------------------
# sampling
@pytest.mark.parametrize("dims,n,S,seed,t", [
    ((50, 50, 50), 0, 200, 1701066001, 0),
    ((400, 400, 400), 2, 300, 1701066002, 17),
    ((7, 5, 11, 3, 2, 13), 3, 1000, 5, 3),          # two Philox blocks per sample
    ((1, 2, 3), 1, 64, 9, 0),
    ((2 ** 31 - 1, 3, 2 ** 31 - 1), 1, 5000, 123, 99),
])
def test_sample_uniform_bit_exact(dims, n, S, seed, t):
    idx, w = P.cprand_sample(dims, n, S, seed, t)
    torch.cuda.synchronize()
    ref = OP.sample_indices(dims, n, S, seed, t)
    assert np.array_equal(idx.cpu().numpy().astype(np.int64), ref)


def test_sample_importance_bit_exact():
    rng = _rng(1)
    dims, n, S = (40, 55, 33), 1, 4000
    qs = [OQ.quantize(rng.dirichlet(np.ones(I) * 0.3), 0.1) for I in dims]
    cdfs = [dev(OQ.cdf(q).astype(np.uint64)) for q in qs]
    idx, w = P.cprand_sample(dims, n, S, 77, 4, cdf=cdfs)
    ref_idx, ref_w = OQ.importance_indices(dims, n, S, 77, 4, qs)
    assert np.array_equal(idx.cpu().numpy().astype(np.int64), ref_idx)
    assert np.array_equal(w.cpu().numpy(), ref_w)


# --------------------------------------------------------------------------
# sampled MTTKRP
CASES = [  # dims, R, S
    ((50, 50, 50), 5, 200),
    ((130, 70, 9), 20, 333),
    ((64, 37, 23, 5), 10, 97),
    ((400, 13, 11), 64, 300),
]


def _mttkrp_case(dims, R, S, seed, dtype):
    rng = _rng(seed)
    X = rng.standard_normal(dims)
    A = [rng.standard_normal((I, R)) for I in dims]
    return X, A


@pytest.mark.parametrize("dims,R,S", CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_mttkrp_colmajor_matches_oracle(dims, R, S, dtype):
    X, A = _mttkrp_case(dims, R, S, 3, dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    Xv = view_of(X, tdt)
    Ad = factors_dev(A, tdt)
    tol = 1e-12 if dtype == "f64" else 1e-5
    for n in range(len(dims)):
        idx, _ = P.cprand_sample(dims, n, S, 11, n)
        W, V = P.cprand_mttkrp_sampled(Xv, n, Ad, R, S, idx)
        ref_idx = OP.sample_indices(dims, n, S, 11, n)
        Xr = X if dtype == "f64" else X.astype(np.float32).astype(np.float64)
        Ar = A if dtype == "f64" else [M.astype(np.float32).astype(np.float64) for M in A]
        Wr, Vr = OC.sampled_normal_blocks(Xr, ref_idx, Ar, n)
        close(W.cpu().numpy(), Wr, tol)
        close(V.cpu().numpy(), Vr, tol)


@pytest.mark.parametrize("dims,R,S", CASES[:3])
def test_mttkrp_mode_major_copy_matches(dims, R, S):
    X, A = _mttkrp_case(dims, R, S, 4, "f32")
    Xv = view_of(X, torch.float32)
    Ad = factors_dev(A, torch.float32)
    for n in range(len(dims)):
        Y = P.mode_major_copy(Xv, n)
        idx, _ = P.cprand_sample(dims, n, S, 5, 2)
        W1, V1 = P.cprand_mttkrp_sampled(Xv, n, Ad, R, S, idx)
        W2, V2 = P.cprand_mttkrp_sampled(Y, n, Ad, R, S, idx)
        close(W2.cpu().numpy(), W1.cpu().numpy(), 1e-6)
        assert torch.equal(V1, V2)


def test_mttkrp_weighted_matches_oracle():
    rng = _rng(5)
    dims, R, S = (60, 45, 30), 8, 500
    X = rng.standard_normal(dims)
    A = [rng.standard_normal((I, R)) for I in dims]
    qs = [OQ.quantize(rng.dirichlet(np.ones(I)), 0.2) for I in dims]
    cdfs = [dev(OQ.cdf(q).astype(np.uint64)) for q in qs]
    Xv = view_of(X, torch.float64)
    Ad = factors_dev(A, torch.float64)
    for n in range(3):
        idx, w = P.cprand_sample(dims, n, S, 3, 1, cdf=cdfs)
        W, V = P.cprand_mttkrp_sampled(Xv, n, Ad, R, S, idx, w=w)
        ridx, rw = OQ.importance_indices(dims, n, S, 3, 1, qs)
        Wr, Vr = OC.sampled_normal_blocks(X, ridx, A, n, rw)
        close(W.cpu().numpy(), Wr, 1e-12)
        close(V.cpu().numpy(), Vr, 1e-12)


@pytest.mark.parametrize("cdt", ["c64", "c128"])
def test_mttkrp_mixed_matches_oracle(cdt):
    rng = _rng(6)
    dims, R, S = (20, 30, 12), 6, 150
    X = rng.standard_normal(dims)
    A = [rng.standard_normal((I, R)) for I in dims]
    signs = OP.sign_vectors(dims, 42)
    Xh = OC.mix_tensor(X, signs)
    Ah = [OC.mix_factor(A[m], signs[m]) for m in range(3)]
    ct = torch.complex64 if cdt == "c64" else torch.complex128
    Xv = view_of(Xh, ct)
    Ad = cplx_factors_dev(Ah, ct)
    tol = 1e-5 if cdt == "c64" else 1e-11
    for n in range(3):
        idx, _ = P.cprand_sample(dims, n, S, 8, 0)
        sg = dev(signs[n])
        W, V = P.cprand_mttkrp_sampled(Xv, n, Ad, R, S, idx, unmix_signs=sg)
        Wr, Vr = OC.mixed_normal_blocks(Xh, OP.sample_indices(dims, n, S, 8, 0), Ah, n, signs[n])
        close(W.cpu().numpy(), Wr, tol, "W mode %d" % n)
        close(V.cpu().numpy(), Vr, tol, "V mode %d" % n)


def test_mttkrp_bf16_error_bound():
    rng = _rng(7)
    dims, R, S = (150, 40, 24, 9), 20, 1000
    X = rng.standard_normal(dims).astype(np.float32)
    A = [rng.standard_normal((I, R)).astype(np.float32) for I in dims]
    Xv = view_of(X, torch.float32)
    Ad = factors_dev(A, torch.float32)
    for n in range(4):
        Y = P.mode_major_copy(Xv, n, dtype=torch.bfloat16)
        Yv = P.View(Y.data, Y.dims, Y.strides, dtype=P.BF16)
        idx, _ = P.cprand_sample(dims, n, S, 9, 0)
        W, V = P.cprand_mttkrp_sampled(Yv, n, Ad, R, S, idx)
        Wr, Vr = OC.sampled_normal_blocks(X.astype(np.float64), OP.sample_indices(dims, n, S, 9, 0),
                                          [M.astype(np.float64) for M in A], n)
        # inputs rounded to 8-bit mantissas: relative error ~ 2^-9 per factor,
        # a few of them per product term
        close(W.cpu().numpy(), Wr, 1e-2, "BF16 W mode %d" % n)
        close(V.cpu().numpy(), Vr, 1e-2, "BF16 V mode %d" % n)


@pytest.mark.parametrize("dims,R,S", [((150, 40, 24, 9), 20, 1000), ((67, 33, 29), 7, 333)])
def test_mttkrp_bf16_matches_bf16_oracle(dims, R, S):
    """Against the oracle of the BF16 product (the same roundings, sums in
    FP64): only the FP32 accumulation of the MFMA remains."""
    from oracle import precision as OR
    rng = _rng(17)
    X = rng.standard_normal(dims).astype(np.float32)
    A = [rng.standard_normal((I, R)).astype(np.float32) for I in dims]
    Xv = view_of(X, torch.float32)
    Ad = factors_dev(A, torch.float32)
    for n in range(len(dims)):
        Y = P.mode_major_copy(Xv, n, dtype=torch.bfloat16)
        Yv = P.View(Y.data, Y.dims, Y.strides, dtype=P.BF16)
        idx, _ = P.cprand_sample(dims, n, S, 19, 2)
        W, V = P.cprand_mttkrp_sampled(Yv, n, Ad, R, S, idx)
        Wr, Vr = OR.bf16_normal_blocks(X, OP.sample_indices(dims, n, S, 19, 2), A, n)
        close(W.cpu().numpy(), Wr, 1e-5, "BF16 W mode %d" % n)
        close(V.cpu().numpy(), Vr, 1e-12, "BF16 V mode %d" % n)


# --------------------------------------------------------------------------
# solve and normalise
@pytest.mark.parametrize("In,R", [(50, 5), (401, 10), (70, 17), (40, 25), (64, 32), (90, 33), (1000, 50), (33, 64)])
def test_solve_matches_numpy(In, R):
    rng = _rng(In + R)
    Z = rng.standard_normal((3 * R, R))
    V = Z.T @ Z
    W = rng.standard_normal((In, R))
    A, lam, info = P.cprand_solve(dev(V), dev(W))
    ref = np.linalg.solve(V, W.T).T
    rl = np.linalg.norm(ref, axis=0)
    close(lam.cpu().numpy(), rl, 1e-10)
    close(A.cpu().numpy(), ref / rl, 1e-10)
    assert int(info.item()) == 0


@pytest.mark.parametrize("R,rk", [(6, 4), (6, 5), (7, 6), (24, 12), (40, 30)])
def test_solve_singular_uses_pseudoinverse(R, rk):
    rng = _rng(3 + R)
    Z = rng.standard_normal((rk, R))         # rank rk < R
    V = Z.T @ Z
    W = rng.standard_normal((20, rk)) @ Z     # right-hand side in the row space
    A, lam, info = P.cprand_solve(dev(V), dev(W))
    assert int(info.item()) == P.W_PINV
    ref = W @ np.linalg.pinv(V, rcond=1e-10)
    rl = np.linalg.norm(ref, axis=0)
    close(A.cpu().numpy() * lam.cpu().numpy(), ref, 1e-8)


def test_solve_f32_refinement():
    """One refinement step: residual of the FP32 normal equations (W_ref,
    V_ref), corrected with the inverse of the lower-precision V."""
    from oracle import precision as OR
    rng = _rng(9)
    In, R = 150, 20
    Z = rng.standard_normal((200, R))
    V_ref = Z.T @ Z
    V_lo = V_ref + 1e-3 * np.diag(np.diag(V_ref)) + 1e-4 * (lambda E: E + E.T)(rng.standard_normal((R, R)))
    W = rng.standard_normal((In, R)).astype(np.float32).astype(np.float64)
    Wb = (W + 1e-3 * rng.standard_normal((In, R))).astype(np.float32).astype(np.float64)
    A, lam, _ = P.cprand_solve(dev(V_lo), dev(Wb, torch.float32), W_refine=dev(W, torch.float32),
                               V_refine=dev(V_ref))
    A0 = np.linalg.solve(V_lo, Wb.T).T
    want = OR.refine_step(A0, V_lo, W, V_ref)
    close(A.cpu().numpy() * lam.cpu().numpy(), want, 1e-5, "refined A")
    # the step moved A0 most of the way to the FP32 solution
    star = np.linalg.solve(V_ref, W.T).T
    assert np.linalg.norm(want - star) < 0.1 * np.linalg.norm(A0 - star)


def test_solve_refinement_needs_both_blocks():
    V = dev(np.eye(3))
    W = dev(np.ones((4, 3)), torch.float32)
    with pytest.raises(P.CprandError):
        P.cprand_solve(V, W, W_refine=W)


def test_sampled_step_matches_qr_solution():
    """sample -> MTTKRP -> solve equals the oracle's QR least squares."""
    rng = _rng(10)
    dims, R, S = (45, 52, 39), 7, 120
    X = rng.standard_normal(dims)
    A = [rng.standard_normal((I, R)) for I in dims]
    Xv, Ad = view_of(X, torch.float64), factors_dev(A, torch.float64)
    for n in range(3):
        idx, _ = P.cprand_sample(dims, n, S, 1, 0)
        W, V = P.cprand_mttkrp_sampled(Xv, n, Ad, R, S, idx)
        An, lam, _ = P.cprand_solve(V, W)
        ref, rl = OC.normalize(OC.sampled_ls(X, OP.sample_indices(dims, n, S, 1, 0), A, n))
        close(An.cpu().numpy(), ref, 1e-9, "A mode %d" % n)
        close(lam.cpu().numpy(), rl, 1e-9, "lambda mode %d" % n)


# --------------------------------------------------------------------------
# fit estimate and norm
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fit_est_matches_oracle(dtype):
    rng = _rng(11)
    dims, R = (30, 41, 17, 6), 4
    A = [rng.standard_normal((I, R)) for I in dims]
    lam = rng.uniform(0.5, 2.0, R)
    from oracle.tensor import cp_full
    X = cp_full(lam, A) + 0.05 * rng.standard_normal(dims)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        X = X.astype(np.float32).astype(np.float64)
        A = [M.astype(np.float32).astype(np.float64) for M in A]
    Xv = view_of(X, tdt)
    nrm = P.cprand_norm(Xv)
    assert abs(nrm.item() - np.linalg.norm(X)) < 1e-12 * np.linalg.norm(X)
    F = P.cprand_fit_est(Xv, nrm, factors_dev(A, tdt), dev(lam), R, 2 ** 14, 31)
    ref = OC.sampled_fit(X, np.linalg.norm(X), lam, A, OP.fit_indices(dims, 2 ** 14, 31))
    assert abs(F.item() - ref) < (1e-12 if dtype == "f64" else 1e-6)


# --------------------------------------------------------------------------
# mixing
@pytest.mark.parametrize("dims,cdt", [((20, 30, 12), "c64"), ((50, 60, 7), "c64"), ((14, 9, 10, 8), "c128"),
                                      ((100, 90, 16), "c64"), ((400, 6, 150), "c64"), ((3, 1000, 5), "c64"),
                                      ((60, 60, 60, 5), "c64"), ((100, 9, 7), "c64"), ((400, 3, 7), "c64"),
                                      ((128, 5, 5), "c64")])
def test_mix_matches_oracle(dims, cdt):
    rng = _rng(12)
    X = rng.standard_normal(dims)
    rdt = torch.float32 if cdt == "c64" else torch.float64
    if cdt == "c64":
        X = X.astype(np.float32).astype(np.float64)
    Xv = view_of(X, rdt)
    Xh, signs, nrm = P.cprand_mix(Xv, 99)
    ref_signs = np.concatenate(OP.sign_vectors(dims, 99))
    assert np.array_equal(signs.cpu().numpy(), ref_signs)
    ref = OC.mix_tensor(X, OP.sign_vectors(dims, 99))
    got = from_colmajor(Xh.data.cpu().numpy(), dims)
    tol = 2e-6 if cdt == "c64" else 1e-13
    close(got, ref, tol)
    assert abs(nrm.item() - np.linalg.norm(X)) < 1e-10 * np.linalg.norm(X)


@pytest.mark.parametrize("I,R", [(50, 5), (400, 10), (1000, 50), (60, 25), (7, 3), (98, 2)])
def test_mix_factor_matches_oracle(I, R):
    rng = _rng(I)
    A = rng.standard_normal((I, R))
    s = OP.sign_vectors((I,), 5)[0]
    Ah = P.cprand_mix_factor(dev(A), dev(s))
    ref = OC.mix_factor(A, s)
    close(Ah.cpu().numpy(), ref, 1e-12)
    back = P.cprand_mix_factor(Ah, dev(s), inverse=True)
    close(back.cpu().numpy(), A, 1e-12)


# --------------------------------------------------------------------------
# layout copies
def test_layout_copy_exact_and_bf16_rne():
    rng = _rng(13)
    dims = (21, 6, 10, 3)
    X = rng.standard_normal(dims).astype(np.float32)
    Xv = view_of(X, torch.float32)
    for n in range(4):
        Y = P.mode_major_copy(Xv, n)
        flat = Y.data.cpu().numpy()
        for i in np.ndindex(*dims):
            off = sum(ii * s for ii, s in zip(i, Y.strides))
            assert flat[off] == X[i]
        Yb = P.mode_major_copy(Xv, n, dtype=torch.bfloat16)
        want = torch.as_tensor(X).to(torch.bfloat16).view(torch.int16).numpy()
        gotb = Yb.data.cpu().view(torch.int16).numpy()
        for i in list(np.ndindex(*dims))[::7]:
            off = sum(ii * s for ii, s in zip(i, Yb.strides))
            assert gotb[off] == want[i]


@pytest.mark.parametrize("dims", [(66, 70, 3), (21, 16, 9)])
def test_layout_copy_complex_exact(dims):
    """Mode-major copies of a complex64 tensor (the mixed tensor's copies):
    bit-exact for every mode, with even sizes (16-byte pair transpose, edge
    tiles) and odd ones (element transpose)."""
    rng = _rng(17)
    X = (rng.standard_normal(dims) + 1j * rng.standard_normal(dims)).astype(np.complex64)
    Xv = view_of(X, torch.complex64)
    idx = np.indices(dims).reshape(len(dims), -1)
    for n in range(len(dims)):
        Y = P.mode_major_copy(Xv, n)
        flat = Y.data.cpu().numpy()
        off = sum(idx[m] * Y.strides[m] for m in range(len(dims)))
        assert np.array_equal(flat[off], X.reshape(-1)[np.ravel_multi_index(idx, dims)]), n
