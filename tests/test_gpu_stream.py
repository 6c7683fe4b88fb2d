"""GPU parity of the sampled MTTKRP on long sample sets (S >= 4096), where
contiguous fibers take the streaming form: accumulators kept over whole
sample splits, one partial product per split.  Each case is checked against
the FP64 oracle (Alg. 2 / Alg. 3 normal blocks; the mixed form of Alg. 4)
on the same drawn samples, and the shapes cover one full row block, several
row blocks with a ragged last one, waves with no row groups, a last wave with
fewer row groups than the others, importance weights, a sample count that
leaves a ragged last split, and the rank above which the chunked form takes
over.  Tolerances as in the other parity tests: FP32 1e-5, FP64 1e-12,
complex64 1e-5, complex128 1e-11 (relative, Frobenius)."""
import numpy as np
import pytest
import torch

from oracle import cprand as OC
from oracle import philox as OP
from oracle import proposal as OQ
from gpu_util import close, cplx_factors_dev, dev, factors_dev, view_of

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1701_06600_amd")


def _case(dims, R, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal(dims)
    A = [rng.standard_normal((I, R)) for I in dims]
    return X, A


def _r32(a):
    return a.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("dims,R,S,modes", [
    ((1000, 60, 50), 10, 9001, (0, 1)),     # 16 row groups in one block; mode 1: 60 rows, waves 1..3 idle
    ((1000, 30, 20), 32, 6000, (0,)),       # two column tiles: two row groups per wave
    ((4100, 12, 10), 7, 4096, (0,)),        # five row blocks, ragged last block
])
def test_stream_f32_matches_oracle(dims, R, S, modes):
    X, A = _case(dims, R, 21)
    Xv = view_of(X, torch.float32)
    Ad = factors_dev(A, torch.float32)
    for n in modes:
        Y = Xv if n == 0 else P.mode_major_copy(Xv, n)
        idx, _ = P.cprand_sample(dims, n, S, 31, n)
        W, V = P.cprand_mttkrp_sampled(Y, n, Ad, R, S, idx)
        Wr, Vr = OC.sampled_normal_blocks(_r32(X), OP.sample_indices(dims, n, S, 31, n), [_r32(M) for M in A], n)
        close(W.cpu().numpy(), Wr, 1e-5, "W mode %d" % n)
        close(V.cpu().numpy(), Vr, 1e-5, "V mode %d" % n)
        # the same call again: fixed partition, fixed summation order
        W2, V2 = P.cprand_mttkrp_sampled(Y, n, Ad, R, S, idx)
        assert torch.equal(W, W2) and torch.equal(V, V2)


def test_stream_f32_weighted_matches_oracle():
    rng = np.random.default_rng(22)
    dims, R, S = (512, 40, 30), 8, 6000
    X = rng.standard_normal(dims)
    A = [rng.standard_normal((I, R)) for I in dims]
    qs = [OQ.quantize(rng.dirichlet(np.ones(I)), 0.2) for I in dims]
    cdfs = [dev(OQ.cdf(q).astype(np.uint64)) for q in qs]
    Xv = view_of(X, torch.float32)
    Ad = factors_dev(A, torch.float32)
    idx, w = P.cprand_sample(dims, 0, S, 3, 1, cdf=cdfs)
    W, V = P.cprand_mttkrp_sampled(Xv, 0, Ad, R, S, idx, w=w)
    ridx, rw = OQ.importance_indices(dims, 0, S, 3, 1, qs)
    Wr, Vr = OC.sampled_normal_blocks(_r32(X), ridx, [_r32(M) for M in A], 0, rw)
    close(W.cpu().numpy(), Wr, 1e-5, "W")
    close(V.cpu().numpy(), Vr, 1e-5, "V")


def test_stream_f64_row_blocks_match_oracle():
    # R = 20: two column tiles, two row groups (64 rows) per wave, 256 rows
    # per block: ten full blocks and one of 40 rows
    dims, R, S = (2600, 20, 12), 20, 5000
    X, A = _case(dims, R, 23)
    Xv = view_of(X, torch.float64)
    Ad = factors_dev(A, torch.float64)
    idx, _ = P.cprand_sample(dims, 0, S, 41, 0)
    W, V = P.cprand_mttkrp_sampled(Xv, 0, Ad, R, S, idx)
    Wr, Vr = OC.sampled_normal_blocks(X, OP.sample_indices(dims, 0, S, 41, 0), A, 0)
    close(W.cpu().numpy(), Wr, 1e-12, "W")
    close(V.cpu().numpy(), Vr, 1e-12, "V")


@pytest.mark.parametrize("cdt,dims,R,S", [
    ("c64", (400, 30, 20), 10, 8000),     # 13 row groups of 32: the last wave has one
    ("c128", (96, 40, 25), 12, 4500),     # 6 row groups of 16: the last wave has none
])
def test_stream_mixed_matches_oracle(cdt, dims, R, S):
    X, A = _case(dims, R, 24)
    signs = OP.sign_vectors(dims, 43)
    Xh = OC.mix_tensor(X, signs)
    Ah = [OC.mix_factor(A[m], signs[m]) for m in range(3)]
    ct = torch.complex64 if cdt == "c64" else torch.complex128
    Xv = view_of(Xh, ct)
    Ad = cplx_factors_dev(Ah, ct)
    tol = 1e-5 if cdt == "c64" else 1e-11
    idx, _ = P.cprand_sample(dims, 0, S, 9, 0)
    W, V = P.cprand_mttkrp_sampled(Xv, 0, Ad, R, S, idx, unmix_signs=dev(signs[0]))
    Wr, Vr = OC.mixed_normal_blocks(Xh, OP.sample_indices(dims, 0, S, 9, 0), Ah, 0, signs[0])
    close(W.cpu().numpy(), Wr, tol, "W")
    close(V.cpu().numpy(), Vr, tol, "V")


def test_rank_above_stream_limit_matches_oracle():
    # R = 40 > 32: the chunked whole-fiber form on the same long sample set
    dims, R, S = (800, 30, 20), 40, 5000
    X, A = _case(dims, R, 25)
    Xv = view_of(X, torch.float32)
    Ad = factors_dev(A, torch.float32)
    idx, _ = P.cprand_sample(dims, 0, S, 51, 0)
    W, V = P.cprand_mttkrp_sampled(Xv, 0, Ad, R, S, idx)
    Wr, Vr = OC.sampled_normal_blocks(_r32(X), OP.sample_indices(dims, 0, S, 51, 0), [_r32(M) for M in A], 0)
    close(W.cpu().numpy(), Wr, 1e-5, "W")
    close(V.cpu().numpy(), Vr, 1e-5, "V")


@pytest.mark.parametrize("dims,R,S,modes,weighted", [
    ((1000, 40, 30), 10, 9001, (0, 1, 2), False),  # mode 0: 8 row groups of 128, two per wave, the last of 104
                                                   # rows; mode 1: one group of 40 rows; mode 2: I_n % 8 != 0
    ((1288, 30, 20), 20, 6000, (0,), False),       # three row blocks, the last ending in a group of 8 rows;
                                                   # four Gram tiles
    ((512, 40, 30), 12, 5000, (0,), True),         # importance weights: V = bf16(w z)^T bf16(z)
])
def test_stream_bf16_matches_bf16_oracle(dims, R, S, modes, weighted):
    """BF16 fibers on long sample sets (the register-transposed streaming
    form where I_n % 8 == 0) against the oracle of the BF16 product: the same
    roundings, sums in FP64, so only the FP32 accumulation remains."""
    from oracle import precision as OR
    rng = np.random.default_rng(26)
    X = rng.standard_normal(dims).astype(np.float32)
    A = [rng.standard_normal((I, R)).astype(np.float32) for I in dims]
    Xv = view_of(X, torch.float32)
    Ad = factors_dev(A, torch.float32)
    for n in modes:
        Y = P.mode_major_copy(Xv, n, dtype=torch.bfloat16)
        Yv = P.View(Y.data, Y.dims, Y.strides, dtype=P.BF16)
        if weighted:
            qs = [OQ.quantize(rng.dirichlet(np.ones(I)), 0.2) for I in dims]
            cdfs = [dev(OQ.cdf(q).astype(np.uint64)) for q in qs]
            idx, w = P.cprand_sample(dims, n, S, 5, 1, cdf=cdfs)
            ridx, rw = OQ.importance_indices(dims, n, S, 5, 1, qs)
        else:
            idx, w = P.cprand_sample(dims, n, S, 33, n)
            ridx, rw = OP.sample_indices(dims, n, S, 33, n), None
        W, V = P.cprand_mttkrp_sampled(Yv, n, Ad, R, S, idx, w=w)
        Wr, Vr = OR.bf16_normal_blocks(X, ridx, A, n, rw)
        close(W.cpu().numpy(), Wr, 1e-5, "BF16 W mode %d" % n)
        close(V.cpu().numpy(), Vr, 1e-12, "BF16 V mode %d" % n)
        W2, V2 = P.cprand_mttkrp_sampled(Yv, n, Ad, R, S, idx, w=w)
        assert torch.equal(W, W2) and torch.equal(V, V2)
