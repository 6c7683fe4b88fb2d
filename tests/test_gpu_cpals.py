"""GPU parity of the dense comparison path: the full MTTKRP of Alg. 1, the
exact fit of Section 3.4 and CP-ALS, against the oracle's plain
definitions (oracle/cpals.py) on the same inputs.  Tolerances: FP64 1e-12
element-wise (column-scaled); FP32 data 1e-5 (FP32 products summed in FP64
per range of unfolding columns); exact fits 1e-9 (FP64) / 1e-5 (FP32)."""
import numpy as np
import pytest
import torch

import synth
from oracle import cpals as OA
from oracle import cprand as OC
from oracle import score as OS
from oracle.tensor import fnorm
from gpu_util import close, dev, factors_dev, view_of

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1701_06600_amd")

CASES = [  # dims, R
    ((50, 50, 50), 5),
    ((130, 70, 9), 20),       # rows past one workgroup's block, odd last mode
    ((64, 37, 23, 5), 10),    # order 4, J not a multiple of the vector width for mode 1
    ((400, 13, 11), 64),      # four column tiles
    ((3, 257, 5), 17),        # short fibers in mode 0, ragged row blocks in mode 1
    ((1, 40, 2, 6), 3),       # modes of length 1 and 2
]


@pytest.mark.parametrize("dims,R", CASES)
@pytest.mark.parametrize("tdt", [torch.float64, torch.float32])
def test_mttkrp_full_matches_oracle(dims, R, tdt):
    print("mttkrp_full dims=%s R=%d %s" % (dims, R, tdt), flush=True)
    rng = np.random.default_rng(sum(dims) + R)
    X = rng.standard_normal(dims)
    A = [rng.standard_normal((I, R)) for I in dims]
    if tdt == torch.float32:
        X = X.astype(np.float32).astype(np.float64)
        A = [M.astype(np.float32).astype(np.float64) for M in A]
    Xv = view_of(X, tdt)
    Ad = factors_dev(A, tdt)
    tol = 1e-12 if tdt == torch.float64 else 1e-5
    for n in range(len(dims)):
        W = P.cprand_mttkrp_full(Xv, n, Ad, R)
        torch.cuda.synchronize()
        close(W.cpu().numpy(), OA.mttkrp(X, A, n), tol, "full MTTKRP mode %d" % n)


def test_mttkrp_full_unaligned_tensor_start():
    """A tensor that starts 4 bytes past a 16-byte boundary takes the scalar
    loads."""
    dims, R = (36, 20, 12), 7
    rng = np.random.default_rng(5)
    X = rng.standard_normal(dims).astype(np.float32).astype(np.float64)
    A = [rng.standard_normal((I, R)).astype(np.float32).astype(np.float64) for I in dims]
    from oracle.tensor import to_colmajor
    buf = dev(np.concatenate([[0.0], to_colmajor(X)]), torch.float32)
    Xv = P.View(buf[1:], dims)
    Ad = factors_dev(A, torch.float32)
    for n in range(3):
        W = P.cprand_mttkrp_full(Xv, n, Ad, R)
        torch.cuda.synchronize()
        close(W.cpu().numpy(), OA.mttkrp(X, A, n), 1e-5, "unaligned mode %d" % n)


@pytest.mark.parametrize("tdt", [torch.float64, torch.float32])
def test_fit_exact_matches_oracle(tdt):
    p = synth.make_problem((60, 45, 30), 6, congruence=0.5, noise=0.05, seed=11)
    X = synth.dense_tensor(p)
    if tdt == torch.float32:
        X = X.astype(np.float32).astype(np.float64)
    # a model near the truth (a fit around 0.95) and a poor one
    rng = np.random.default_rng(2)
    for scale in (0.0, 0.3):
        A = [(M + scale * rng.standard_normal(M.shape)) for M in p.factors]
        if tdt == torch.float32:
            A = [M.astype(np.float32).astype(np.float64) for M in A]
        lam = p.lam * (1 + 0.1 * rng.standard_normal(p.lam.shape))
        Xv = view_of(X, tdt)
        nX = torch.tensor([fnorm(X)], dtype=torch.float64, device="cuda")
        F = P.cprand_fit_exact(Xv, nX, factors_dev(A, tdt), dev(lam), 6)
        torch.cuda.synchronize()
        ref = OC.exact_fit(X, lam, A)
        assert abs(F.item() - ref) < (1e-9 if tdt == torch.float64 else 1e-5), (F.item(), ref)


def test_cpals_f64_tracks_oracle():
    p = synth.make_problem((40, 35, 30), 4, congruence=0.5, noise=0.01, seed=23)
    X = synth.dense_tensor(p)
    A = factors_dev(p.init, torch.float64)
    out = P.cprand_cpals(view_of(X, torch.float64), A, 4, 15)
    lam_r, A_r, hist_r = OA.cp_als(X, 4, p.init, 15)
    assert out["iters"] == 15
    assert np.max(np.abs(np.array(out["fit_history"]) - np.array(hist_r))) < 1e-9
    Ag = [M.cpu().numpy() for M in A]
    for a, b in zip(Ag, A_r):
        close(a, b, 1e-8, "CP-ALS factor")
    assert np.allclose(out["lambda"].cpu().numpy(), lam_r, rtol=1e-8)


def test_cpals_f32_converges_and_stops():
    p = synth.make_problem((80, 70, 60), 5, congruence=0.5, noise=0.01, seed=21)
    X = synth.dense_tensor(p).astype(np.float32).astype(np.float64)
    A = factors_dev(p.init, torch.float32)
    out = P.cprand_cpals(view_of(X, torch.float32), A, 5, 200, tol=1e-6)
    lam_r, A_r, hist_r = OA.cp_als(X, 5, p.init, 200, tol=1e-6)
    Ag = [M.double().cpu().numpy() for M in A]
    F = OC.exact_fit(X, out["lambda"].cpu().numpy(), Ag)
    assert abs(F - hist_r[-1]) < 1e-4
    assert abs(out["fit_history"][-1] - F) < 1e-4   # the loop's exact fit is the fit of its result
    assert out["iters"] < 200 and abs(out["iters"] - len(hist_r)) <= 2
    assert OS.score(p.factors, Ag) > 0.99
