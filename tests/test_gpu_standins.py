"""GPU parity on reduced proxies of the paper's real-data shapes (the
datasets are not available; tensors come from the synthetic generator):
COIL-100's 7200-long image mode under CPRAND-MIX (mixing FFTs longer than a
padded LDS tile, run one unpadded fiber per workgroup), and the hazardous
gas tensor's 25,900 x ... x 899 unmixed shape with its patience stop rule.
Tolerances: mixing and factor mixes 1e-5 (FP32), fit histories 1e-3."""
import numpy as np
import pytest
import torch

import synth
from oracle import cprand as OC
from oracle import philox as OP
from oracle.tensor import from_colmajor
from gpu_util import close, dev, factors_dev

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1701_06600_amd")


def _device_problem(dims, R, noise, seed, congruence=0.5):
    p = synth.make_problem(dims, R, congruence=congruence, noise=noise, seed=seed)
    X = synth.device_tensor(p, torch.device("cuda:0"), "f32")
    torch.cuda.synchronize()
    host = from_colmajor(X.double().cpu().numpy(), dims)
    init = [M.astype(np.float32).astype(np.float64) for M in p.init]
    return p, X, host, init


def test_coil_proxy_long_mode_mixing_and_loop():
    dims, R, S = (8, 8, 3, 7200), 5, 200
    print("COIL proxy %s" % (dims,), flush=True)
    p, X, host, init = _device_problem(dims, R, 0.34, 1701066006, congruence=None)
    Xv = P.View(X, dims)
    Xh, signs, _ = P.cprand_mix(Xv, 77)
    torch.cuda.synchronize()
    sg = OP.sign_vectors(dims, 77)
    ref = OC.mix_tensor(host, sg)
    got = from_colmajor(Xh.data.cpu().numpy().astype(np.complex128), dims)
    close(got.ravel(), ref.ravel(), 1e-5, "mixed tensor")
    # factor mix and unmix along the 7200-long mode
    A3 = init[3]
    Ah = P.cprand_mix_factor(dev(A3, torch.float32), signs[8 + 8 + 3:])
    torch.cuda.synchronize()
    close(Ah.cpu().numpy().astype(np.complex128), OC.mix_factor(A3, sg[3]), 1e-5, "factor mix")
    back = P.cprand_mix_factor(Ah, signs[8 + 8 + 3:], inverse=True)
    torch.cuda.synchronize()
    close(back.double().cpu().numpy(), A3, 1e-5, "factor unmix")
    # CPRAND-MIX loop (the 7200-long mode's steps unmix on the split path)
    A = factors_dev(init)
    out = P.cprand_als(Xv, A, P.make_opts(R, S, max_iters=8, seed=77, mix=P.MIX_FFT, use_graph=0))
    _, _, hist = OC.cprand_mix(host, R, S, init, 77, 8)
    assert np.max(np.abs(np.array(out["fit_history"]) - np.array(hist))) < 1e-3, (out["fit_history"], hist)


@pytest.mark.parametrize("layout", [0, 1])
def test_gas_proxy_unmixed_with_patience(layout):
    dims, R, S = (25900, 6, 899), 5, 1000
    print("gas proxy %s layout %d" % (dims, layout), flush=True)
    p, X, host, init = _device_problem(dims, R, 0.30, 1701066007)
    A = factors_dev(init)
    out = P.cprand_als(P.View(X, dims), A, P.make_opts(R, S, max_iters=40, seed=5, patience=10, layout=layout,
                                                       use_graph=0))
    _, _, hist = OC.cprand(host, R, S, init, 5, 40, patience=10)
    print("GPU %d iterations, oracle %d" % (out["iters"], len(hist)), flush=True)
    n = min(out["iters"], len(hist))
    assert np.max(np.abs(np.array(out["fit_history"][:n]) - np.array(hist[:n]))) < 1e-3
    assert out["iters"] == len(hist)
