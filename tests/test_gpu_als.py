"""End-to-end parity of the whole decomposition (cprand_plan_run) against
the oracle's ALS loops on the same seeded inputs and sample streams."""
import numpy as np
import pytest
import torch

import synth
from oracle import cprand as OC
from oracle import leverage as OL
from oracle import proposal as OQ
from oracle import score as OS
from gpu_util import dev, factors_dev, view_of

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1701_06600_amd")


def _run_gpu(X, init, R, S, seed, tdt, **kw):
    Xv = view_of(X, tdt)
    A = factors_dev(init, tdt)
    opts = P.make_opts(R, S, seed=seed, **kw)
    out = P.cprand_als(Xv, A, opts)
    return out, [M.double().cpu().numpy() for M in A]


@pytest.mark.parametrize("use_graph", [0, 1])
def test_cprand_50cube_f64_tracks_oracle(use_graph):
    w = synth.WORKLOADS["cprand-50cube-f64"]
    p = synth.problem_for(w)
    X = synth.dense_tensor(p)
    out, A = _run_gpu(X, p.init, w.R, w.S, w.seed, torch.float64, max_iters=w.max_iters, use_graph=use_graph)
    lam_r, A_r, hist_r = OC.cprand(X, w.R, w.S, p.init, w.seed, w.max_iters)
    assert out["iters"] == len(hist_r) == 50
    assert np.max(np.abs(np.array(out["fit_history"]) - np.array(hist_r))) < 1e-8
    lam = out["lambda"].cpu().numpy()
    F = OC.exact_fit(X, lam, A)
    assert abs(F - OC.exact_fit(X, lam_r, A_r)) < 1e-6
    assert OS.score(p.factors, A) > 0.99
    for a, b in zip(A, A_r):
        assert np.allclose(a, b, atol=1e-7)


@pytest.mark.parametrize("use_graph", [0, 1])
@pytest.mark.parametrize("patience", [2, 4])
def test_patience_rule_stops_like_the_oracle(use_graph, patience):
    """Stop when the best F-hat has not improved for `patience` iterations
    (the rule of the paper's real-data runs, Section 4.3 and 4.4): the GPU
    stops at the oracle's iteration, with the same F-hat history (FP64)."""
    w = synth.WORKLOADS["cprand-50cube-f64"]
    p = synth.problem_for(w)
    X = synth.dense_tensor(p)
    out, A = _run_gpu(X, p.init, w.R, w.S, w.seed, torch.float64, max_iters=200, patience=patience,
                      use_graph=use_graph)
    lam_r, A_r, hist_r = OC.cprand(X, w.R, w.S, p.init, w.seed, 200, patience=patience)
    assert len(hist_r) < 200
    assert out["iters"] == len(hist_r)
    assert np.max(np.abs(np.array(out["fit_history"]) - np.array(hist_r))) < 1e-8
    best = int(np.argmax(hist_r))
    assert len(hist_r) - 1 - best == patience   # the stop fired exactly `patience` iterations after the best


@pytest.mark.parametrize("use_graph", [0, 1])
def test_cprand_f32_stop_rules_and_fit(use_graph):
    """Stops before max_iters, so the iteration launched past the stop is
    undone from the saved state (graph: saved by the fit kernel; direct
    launches: saved by the step kernels, fit estimated on its own stream)."""
    p = synth.make_problem((80, 70, 60), 5, congruence=0.5, noise=0.01, seed=21)
    X = synth.dense_tensor(p).astype(np.float32).astype(np.float64)
    S = OC.sample_size(5)
    out, A = _run_gpu(X, p.init, 5, S, 1234, torch.float32, max_iters=200, tol=1e-4,
                      fit_target=1 - 1.2 * 0.01, use_graph=use_graph)
    lam_r, A_r, hist_r = OC.cprand(X, 5, S, p.init, 1234, 200, tol=1e-4, fit_target=1 - 1.2 * 0.01)
    F = OC.exact_fit(X, out["lambda"].cpu().numpy(), A)
    assert abs(F - OC.exact_fit(X, lam_r, A_r)) < 1e-3
    # the same stop rule fired at the same iteration (here the change-in-fit
    # rule fires early, at a local plateau, on both sides)
    assert out["iters"] == len(hist_r)
    sc, sc_r = OS.score(p.factors, A), OS.score(p.factors, A_r)
    assert abs(sc - sc_r) < 1e-3, (sc, sc_r)
    # without the change-in-fit rule the run recovers the factors
    out, A = _run_gpu(X, p.init, 5, S, 1234, torch.float32, max_iters=200, use_graph=use_graph)
    F = OC.exact_fit(X, out["lambda"].cpu().numpy(), A)
    sc = OS.score(p.factors, A)
    assert abs(F - 0.99) < 2e-3 and sc > 0.99, (F, sc)


def test_cprand_mix_f32_on_coherent_tensor():
    p = synth.make_problem((24, 24, 24), 3, congruence=0.5, noise=0.01, seed=7, spiky=0.1, spike=20.0)
    X = synth.dense_tensor(p).astype(np.float32).astype(np.float64)
    out, A = _run_gpu(X, p.init, 3, 80, 5, torch.float32, max_iters=200, mix=P.MIX_FFT)
    lam_r, A_r, hist_r = OC.cprand_mix(X, 3, 80, p.init, 5, 200)
    F = OC.exact_fit(X, out["lambda"].cpu().numpy(), A)
    assert abs(F - OC.exact_fit(X, lam_r, A_r)) < 1e-3
    assert abs(out["fit_history"][-1] - hist_r[-1]) < 1e-3


@pytest.mark.parametrize("use_graph", [0, 1])
def test_cprand_mix_f64_tracks_oracle(use_graph):
    p = synth.make_problem((20, 30, 12), 4, congruence=0.5, noise=0.01, seed=8)
    X = synth.dense_tensor(p)
    out, A = _run_gpu(X, p.init, 4, 60, 9, torch.float64, max_iters=30, mix=P.MIX_FFT, use_graph=use_graph)
    lam_r, A_r, hist_r = OC.cprand_mix(X, 4, 60, p.init, 9, 30)
    assert np.max(np.abs(np.array(out["fit_history"]) - np.array(hist_r))) < 1e-8
    for a, b in zip(A, A_r):
        assert np.allclose(a, b, atol=1e-7)


@pytest.mark.parametrize("layout,use_graph,every", [(0, 0, 0), (1, 1, 0), (0, 1, 1), (1, 0, 1)])
def test_cprand_bf16_refined_reaches_fp64_fit(layout, use_graph, every):
    """layout 0: BF16 and FP32 mode-major copies; layout 1: strided gathers
    from one BF16 conversion of X and from X itself.  every = 0: BF16 solves
    until the stop rule holds, then refined solves; every = 1: refinement in
    every solve."""
    p = synth.make_problem((40, 36, 32, 28), 5, congruence=0.5, noise=0.01, seed=9)
    X = synth.dense_tensor(p).astype(np.float32).astype(np.float64)
    S = 200
    out, A = _run_gpu(X, p.init, 5, S, 4, torch.float32, max_iters=60, tol=1e-4, precision=P.PREC_BF16_REFINE,
                      layout=layout, use_graph=use_graph, refine_every=every)
    lam_r, A_r, hist_r = OC.cprand(X, 5, S, p.init, 4, 60, tol=1e-4)
    F_r = OC.exact_fit(X, lam_r, A_r)
    F = OC.exact_fit(X, out["lambda"].cpu().numpy(), A)
    assert abs(F - F_r) < 1e-3
    if every:
        assert out["refined_from"] == 0
    else:
        assert 0 < out["refined_from"] < out["iters"], (out["refined_from"], out["iters"])
    out2, A2 = _run_gpu(X, p.init, 5, S, 4, torch.float32, max_iters=60, precision=P.PREC_BF16, layout=layout)
    F2 = OC.exact_fit(X, out2["lambda"].cpu().numpy(), A2)
    assert abs(F2 - F_r) < 1e-3
    assert out2["refined_from"] == -1


@pytest.mark.parametrize("mix", [0, 1])
def test_multi_kernel_step_path_tracks_oracle(mix):
    """A 1000-row mode is too large for the one-workgroup step and takes the
    multi-kernel solve path; the other modes take the fused path."""
    p = synth.make_problem((1000, 12, 10), 10, congruence=0.5, noise=0.01, seed=12)
    X = synth.dense_tensor(p)
    R, S, it = 10, 300, 6
    out, A = _run_gpu(X, p.init, R, S, 77, torch.float64, max_iters=it, mix=mix)
    if mix:
        lam_r, A_r, hist_r = OC.cprand_mix(X, R, S, p.init, 77, it)
    else:
        lam_r, A_r, hist_r = OC.cprand(X, R, S, p.init, 77, it)
    assert np.max(np.abs(np.array(out["fit_history"]) - np.array(hist_r))) < 1e-8
    for a, b in zip(A, A_r):
        assert np.allclose(a, b, atol=1e-7)


@pytest.mark.parametrize("use_graph", [0, 1])
def test_cprand_fixed_proposal_tracks_oracle(use_graph):
    """Fixed importance tables; with direct launches the weighted samples of
    every step are drawn at setup, with a graph inside the gathers."""
    p = synth.make_problem((30, 40, 50), 4, congruence=0.5, noise=0.01, seed=10, spiky=0.1)
    X = synth.dense_tensor(p)
    qs = [OQ.quantize(OL.leverage_scores(M) / 4, 0.2) for M in p.factors]
    cdfs = [dev(OQ.cdf(q).astype(np.uint64)) for q in qs]
    S = 150

    def sampler(t, n, A):
        return OQ.importance_indices(X.shape, n, S, 3, t, qs)

    out, A = _run_gpu(X, p.init, 4, S, 3, torch.float64, max_iters=20, proposal=P.PROPOSAL_TABLE,
                      proposal_cdf=cdfs, use_graph=use_graph)
    lam_r, A_r, hist_r = OC.cprand(X, 4, S, p.init, 3, 20, sampler=sampler)
    assert np.max(np.abs(np.array(out["fit_history"]) - np.array(hist_r))) < 1e-8


@pytest.mark.parametrize("dims,R", [((21, 16, 9), 5), ((30, 25, 20), 20), ((12, 10, 9, 8), 3)])
def test_mixed_step_shapes_track_oracle(dims, R):
    """The fused mixed step on odd and even I_n (rows 0 and I_n/2 pair with
    themselves), R <= 16 (one-wave inverse, FP64 MFMA solve) and R = 20
    (blocked inverse, scalar solve), and an order-4 tensor: F-hat history and
    final factors against the oracle's CPRAND-MIX."""
    p = synth.make_problem(dims, R, congruence=0.5, noise=0.01, seed=31)
    X = synth.dense_tensor(p)
    S, it = max(OC.sample_size(R), 2 * R), 8
    out, A = _run_gpu(X, p.init, R, S, 41, torch.float64, max_iters=it, mix=P.MIX_FFT)
    lam_r, A_r, hist_r = OC.cprand_mix(X, R, S, p.init, 41, it)
    assert np.max(np.abs(np.array(out["fit_history"]) - np.array(hist_r))) < 1e-8
    assert np.allclose(out["lambda"].cpu().numpy(), lam_r, rtol=1e-7)
    for a, b in zip(A, A_r):
        assert np.allclose(a, b, atol=1e-7)
