"""cprand_mttkrp_sampled_noalloc (the entry point with the library's fixed
scratch array) against cprand_mttkrp_sampled (caller workspace) on the same
inputs: two calls in a row per element type, the second on a smaller
problem, so the second call reads partials the first call left behind in
the shared array only if it fails to overwrite them.  Both run the same
kernels in the same order, so the results must be identical bit for bit."""
import numpy as np
import pytest
import torch

from gpu_util import dev, view_of

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1701_06600_amd")

CALLS = [  # (dims, n, R, S): each problem smaller than the one before
    ((1000, 40, 30), 0, 10, 6000),  # S >= 4096: the streaming forms (FP32, FP64, BF16)
    ((300, 41, 52), 0, 16, 2000),
    ((60, 33, 20), 1, 5, 150),
]


def _inputs(dims, R, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(dims), [rng.standard_normal((I, R)) for I in dims]


def _both(Xv, n, Ad, R, S, idx, w=None):
    W0, V0 = P.cprand_mttkrp_sampled(Xv, n, Ad, R, S, idx, w=w)
    W1, V1 = P.cprand_mttkrp_sampled_noalloc(Xv, n, Ad, R, S, idx, w=w)
    torch.cuda.synchronize()
    return W0.cpu(), V0.cpu(), W1.cpu(), V1.cpu()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_matches_workspace_entry_point(dtype):
    for k, (dims, n, R, S) in enumerate(CALLS):
        print("noalloc %s call %d dims=%s n=%d R=%d S=%d" % (dtype, k, dims, n, R, S), flush=True)
        X, A = _inputs(dims, R, 40 + k)
        Xv = view_of(X, dtype)
        Ad = [dev(M, dtype) for M in A]
        idx, _ = P.cprand_sample(dims, n, S, 1701066000 + k, 3)
        W0, V0, W1, V1 = _both(Xv, n, Ad, R, S, idx)
        assert torch.equal(W0, W1) and torch.equal(V0, V1), "call %d differs" % k
        # importance weights take the weighted kernel variant
        w = dev(np.random.default_rng(k).uniform(0.5, 2.0, S), torch.float64)
        W0, V0, W1, V1 = _both(Xv, n, Ad, R, S, idx, w)
        assert torch.equal(W0, W1) and torch.equal(V0, V1), "weighted call %d differs" % k


def test_noalloc_bf16_matches_workspace_entry_point():
    for k, (dims, n, R, S) in enumerate(CALLS):
        print("noalloc bf16 call %d dims=%s n=%d R=%d S=%d" % (k, dims, n, R, S), flush=True)
        X, A = _inputs(dims, R, 50 + k)
        Xv = view_of(X, torch.float32)
        Y = P.mode_major_copy(Xv, n, dtype=torch.bfloat16)
        Yv = P.View(Y.data, Y.dims, Y.strides, dtype=P.BF16)
        Ad = [dev(M, torch.float32) for M in A]
        idx, _ = P.cprand_sample(dims, n, S, 1701066100 + k, 1)
        W0, V0, W1, V1 = _both(Yv, n, Ad, R, S, idx)
        assert torch.equal(W0, W1) and torch.equal(V0, V1), "BF16 call %d differs" % k


def test_noalloc_rejects_what_it_cannot_do():
    dims, R, S = (50, 40, 30), 4, 100
    X, A = _inputs(dims, R, 7)
    Ad = [dev(M, torch.float32) for M in A]
    idx, _ = P.cprand_sample(dims, 0, S, 5, 0)
    Xc = P.View(dev(np.zeros(int(np.prod(dims)) * 2), torch.float32), dims, dtype=P.C64)
    with pytest.raises(RuntimeError):
        P.cprand_mttkrp_sampled_noalloc(Xc, 0, Ad, R, S, idx)
