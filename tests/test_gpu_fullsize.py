"""GPU parity at the benchmarked size: the 400 x 400 x 400 FP32 workload
(rank 10, congruence 0.5, 1% noise, S = 300, P-hat = 2^14), in the launch
configuration the benchmark times (mode-major copies, HIP graph), against the
FP64 oracle on the same tensor copied to the host.  Tolerances as in the
small parity tests: indices and signs bit-exact, FP32 sampled MTTKRP and the
mixing 1e-5 relative, fit estimates 1e-6, the fit history of the whole
decomposition 1e-3."""
import numpy as np
import pytest
import torch

import synth
from oracle import cprand as OC
from oracle import philox as OP
from oracle.tensor import from_colmajor
from gpu_util import close, cplx_factors_dev, factors_dev, rel

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1701_06600_amd")

W = synth.WORKLOADS["cprand-400cube-f32"]


@pytest.fixture(scope="module")
def big():
    prob = synth.problem_for(W)
    X = synth.device_tensor(prob, torch.device("cuda:0"), "f32")
    torch.cuda.synchronize()
    Xh = from_colmajor(X.double().cpu().numpy(), W.dims)       # the same FP32 values, in FP64
    init = [M.astype(np.float32).astype(np.float64) for M in prob.init]
    return {"X": X, "Xv": P.View(X, W.dims), "host": Xh, "init": init, "prob": prob}


@pytest.fixture(scope="module")
def mixed(big):
    Xhat, signs, nrm = P.cprand_mix(big["Xv"], W.seed)
    torch.cuda.synchronize()
    sg = OP.sign_vectors(W.dims, W.seed)
    ref = OC.mix_tensor(big["host"], sg)
    return {"Xhat": Xhat, "signs": signs, "norm": nrm, "sg": sg, "ref": ref}


def test_fullsize_sampled_mttkrp_matches_oracle(big):
    """Mode-major copies (the benchmark's layout): bit-exact indices, W and V
    within 1e-5 of the oracle for every mode."""
    R, S = W.R, W.S
    A = factors_dev(big["init"])
    for n in range(3):
        idx, _ = P.cprand_sample(W.dims, n, S, W.seed, 7)
        ref_idx = OP.sample_indices(W.dims, n, S, W.seed, 7)
        assert np.array_equal(idx.cpu().numpy().astype(np.int64), ref_idx)
        Xn = P.mode_major_copy(big["Xv"], n)
        Wg, Vg = P.cprand_mttkrp_sampled(Xn, n, A, R, S, idx)
        Wr, Vr = OC.sampled_normal_blocks(big["host"], ref_idx, big["init"], n)
        close(Wg.cpu().numpy(), Wr, 1e-5)
        close(Vg.cpu().numpy(), Vr, 1e-5)


def test_fullsize_mix_matches_oracle(big, mixed):
    """The whole mixed tensor (three FFT passes with random signs) against the
    oracle's FFTs; signs bit-exact, the norm to 1e-9."""
    assert np.array_equal(mixed["signs"].cpu().numpy().astype(np.int64),
                          np.concatenate(mixed["sg"]).astype(np.int64))
    got = from_colmajor(mixed["Xhat"].data.cpu().numpy().astype(np.complex128), W.dims)
    close(got, mixed["ref"], 1e-5)
    normX = float(np.linalg.norm(big["host"]))
    assert abs(mixed["norm"].item() - normX) < 1e-9 * normX


def test_fullsize_mixed_mttkrp_matches_oracle(big, mixed):
    """Sampled MTTKRP of the mixed tensor with the unmix (eq. rcLS)."""
    R, S, n = W.R, W.S, 1
    sg = mixed["sg"]
    Ah = [OC.mix_factor(big["init"][m], sg[m]) for m in range(3)]
    offs = np.cumsum([0] + list(W.dims))
    idx, _ = P.cprand_sample(W.dims, n, S, W.seed, 3)
    ref_idx = idx.cpu().numpy().astype(np.int64)
    Ahd = cplx_factors_dev(Ah)
    Wg, Vg = P.cprand_mttkrp_sampled(mixed["Xhat"], n, Ahd, R, S, idx,
                                     unmix_signs=mixed["signs"][offs[n]:offs[n + 1]])
    Wr, Vr = OC.mixed_normal_blocks(mixed["ref"], ref_idx, Ah, n, sg[n])
    close(Wg.cpu().numpy(), Wr, 1e-5)
    close(Vg.cpu().numpy(), Vr, 1e-5)


def test_fullsize_fit_estimate_matches_oracle(big):
    """F-hat over the same P-hat entries as the oracle."""
    lam = np.array([1.0, 0.5, 2.0, 0.25, 1.5, 0.75, 1.25, 0.6, 0.9, 1.1])
    A = big["init"]
    nrm = P.cprand_norm(big["Xv"])
    F = P.cprand_fit_est(big["Xv"], nrm, factors_dev(A), torch.tensor(lam, device="cuda"), W.R, W.P_hat,
                         W.seed).item()
    ref = OC.sampled_fit(big["host"], float(np.linalg.norm(big["host"])), lam, A,
                         OP.fit_indices(W.dims, W.P_hat, W.seed))
    assert abs(F - ref) < 1e-6, (F, ref)


@pytest.mark.parametrize("use_graph", [0, 1])
def test_fullsize_decomposition_tracks_oracle(big, use_graph):
    """The benchmarked decomposition (CPRAND-MIX, mode-major X-hat copies,
    one-iteration run-ahead; direct launches with the fit estimate on its own
    stream, or one HIP graph per iteration) against the oracle's CPRAND-MIX
    for its first iterations: F-hat history within 1e-3."""
    iters = 3
    A = factors_dev(big["init"])
    opts = P.make_opts(W.R, W.S, P_hat=W.P_hat, max_iters=iters, seed=W.seed, tol=0.0, mix=P.MIX_FFT,
                       layout=0, use_graph=use_graph)
    out = P.cprand_als(big["Xv"], A, opts)
    _, _, hist = OC.cprand_mix(big["host"], W.R, W.S, big["init"], W.seed, iters, P_hat=W.P_hat)
    got = np.array(out["fit_history"])
    assert got.shape == (iters,)
    assert np.max(np.abs(got - np.array(hist))) < 1e-3, (got, hist)
