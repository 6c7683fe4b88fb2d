"""Seeded synthetic CP problems, shared by the tests, the benchmark and the
oracle as their only common input source.  It holds no step of the method:
it builds ground-truth factors, the observed tensor and random initial
factors, nothing else.

Construction (Section 4.2, eq. synth): X = X_true + eta (||X_true||/||N||) N
with X_true = sum_r lam_r a_r^(1) o ... o a_r^(N) and N standard normal.
Factors with a prescribed column congruence C have Gram matrix
(1-C) I + C 11^T exactly: A = Q L^T with Q the thin-QR Q of a Gaussian
(I x R) matrix and L L^T the Cholesky factorisation of that Gram.  lam is
uniform on [0.2, 0.8].  "Spiky" factors scale a random 10% of their rows by
20 after the congruence construction, which makes them coherent.  Initial
factors are N(0,1).
"""
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 1701066000


@dataclass
class Workload:
    name: str
    dims: tuple
    R: int
    S: int
    congruence: Optional[float]      # None = raw N(0,1) factors, lam = 1
    noise: float
    dtype: str                       # storage of the tensor: f64, f32, bf16
    spiky: float = 0.0               # fraction of rows scaled
    spike: float = 20.0
    max_iters: int = 200
    tol: float = 1e-4
    fit_target: Optional[float] = None
    patience: int = 0
    P_hat: int = 2 ** 14
    seed: int = SEED_BASE


def _ceil_log_rule(R):
    return int(10 * R * math.ceil(math.log(R)))


WORKLOADS = {
    # 50^3 FP64, R=5 raw Gaussian factors, 1% noise, S=200, 50 iterations.
    "cprand-50cube-f64": Workload("cprand-50cube-f64", (50, 50, 50), 5, 200, None,
                                  0.01, "f64", max_iters=50, tol=0.0,
                                  seed=SEED_BASE + 1),
    # 400^3 FP32, R=10, congruence 0.5, 1% noise, S = 10 R ceil(ln R) = 300.
    "cprand-400cube-f32": Workload("cprand-400cube-f32", (400, 400, 400), 10,
                                   _ceil_log_rule(10), 0.5, 0.01, "f32",
                                   max_iters=200, tol=1e-4, fit_target=1 - 1.2 * 0.01,
                                   seed=SEED_BASE + 2),
    # 150^4 BF16 (+FP32 copy), R=20, congruence 0.5, 1% noise, S=1000.
    "cprand-150pow4-bf16": Workload("cprand-150pow4-bf16", (150, 150, 150, 150), 20,
                                    1000, 0.5, 0.01, "bf16", max_iters=200,
                                    tol=1e-4, fit_target=1 - 1.2 * 0.01,
                                    seed=SEED_BASE + 3),
    # 1000^3 FP32, R=50, congruence 0.9, spiky, 1% noise, S=2000.
    "cprand-1000cube-f32-spiky": Workload("cprand-1000cube-f32-spiky",
                                          (1000, 1000, 1000), 50, 2000, 0.9, 0.01,
                                          "f32", spiky=0.1, max_iters=200, tol=1e-4,
                                          fit_target=1 - 1.2 * 0.01,
                                          seed=SEED_BASE + 4),
    # 60^5 BF16, R=25, congruence 0.7, spiky, 5% noise, S=1000, tol 1e-4.
    "cprand-60pow5-bf16-spiky": Workload("cprand-60pow5-bf16-spiky",
                                         (60, 60, 60, 60, 60), 25, 1000, 0.7, 0.05,
                                         "bf16", spiky=0.1, max_iters=200, tol=1e-4,
                                         fit_target=1 - 1.2 * 0.05,
                                         seed=SEED_BASE + 5),
    # Stand-ins at the shapes of the paper's real-data runs (the datasets are
    # not available; values come from the same generator).  COIL-100:
    # 128 x 128 pixels x 3 colours x 7200 images, R = 20, CPRAND-MIX with
    # S = 400 .. 1000, stop after 5 iterations without improvement; noise
    # 0.34 puts the attainable fit near the paper's 0.68.  Raw Gaussian
    # factors: the colour mode (3 rows) cannot hold 20 congruent columns.
    "coil-standin-f32": Workload("coil-standin-f32", (128, 128, 3, 7200), 20, 400, None, 0.34, "f32",
                                 max_iters=200, tol=0.0, patience=5, seed=SEED_BASE + 6),
    # Hazardous gases: 25,900 x 72 x 899, R = 5, S = 1000, no mixing, stop
    # after 10 iterations without improvement; noise 0.30 puts the attainable
    # fit near the paper's 0.72.
    "gas-standin-f32": Workload("gas-standin-f32", (25900, 72, 899), 5, 1000, 0.5, 0.30, "f32",
                                max_iters=200, tol=0.0, patience=10, seed=SEED_BASE + 7),
}


def _rng(seed, stream):
    return np.random.Generator(np.random.Philox(key=[seed & (2**64 - 1), stream]))


def congruent_factor(rng, I, R, C):
    """I x R matrix with unit columns and pairwise cosine C."""
    if I < R:
        raise ValueError("congruent factors need I >= R")
    G = (1.0 - C) * np.eye(R) + C * np.ones((R, R))
    L = np.linalg.cholesky(G)
    Q, _ = np.linalg.qr(rng.standard_normal((I, R)))
    return Q @ L.T


@dataclass
class Problem:
    dims: tuple
    R: int
    lam: np.ndarray
    factors: List[np.ndarray]
    init: List[np.ndarray]
    noise: float
    seed: int
    spike_rows: List[np.ndarray] = field(default_factory=list)


def make_problem(dims, R, congruence=None, noise=0.01, seed=SEED_BASE,
                 spiky=0.0, spike=20.0, R_model=None):
    """Ground truth (lam, factors) and N(0,1) initial factors of rank
    R_model (default R) for a tensor of shape dims."""
    R_model = R if R_model is None else R_model
    fr = _rng(seed, 0)
    factors, spikes = [], []
    for I in dims:
        if congruence is None:
            A = fr.standard_normal((I, R))
        else:
            A = congruent_factor(fr, I, R, congruence)
        rows = np.array([], dtype=np.int64)
        if spiky > 0:
            k = max(1, int(round(spiky * I)))
            rows = fr.permutation(I)[:k]
            A = A.copy()
            A[rows, :] *= spike
        factors.append(A)
        spikes.append(rows)
    if congruence is None:
        lam = np.ones(R)
    else:
        lam = _rng(seed, 1).uniform(0.2, 0.8, size=R)
    ir = _rng(seed, 4)
    init = [ir.standard_normal((I, R_model)) for I in dims]
    return Problem(tuple(dims), R, lam, factors, init, noise, seed, spikes)


def mlp_init(seed=SEED_BASE, n_in=4, h1=64, h2=64):
    """Initial parameters of the 4-64-64-1 proposal network (uniform in
    +-1/sqrt(fan-in), zero biases), flat in the library's layout:
    W1 (h1 x n_in), b1, W2 (h2 x h1), b2, w3 (h2), b3."""
    rng = _rng(seed, 8)
    W1 = rng.uniform(-1, 1, (h1, n_in)) / math.sqrt(n_in)
    W2 = rng.uniform(-1, 1, (h2, h1)) / math.sqrt(h1)
    w3 = rng.uniform(-1, 1, h2) / math.sqrt(h2)
    return np.concatenate([W1.ravel(), np.zeros(h1), W2.ravel(), np.zeros(h2), w3, np.zeros(1)])


def training_problems(n_inst, dims, R, congruence, spiky, noise=0.01, seed=SEED_BASE + 9):
    """Problems for training the proposal network: instance k draws its
    factors, tensor and initial factors like make_problem with seed
    seed + 1000 k.  The training targets come from the true factors, the
    initial factors and ALS iterates computed from them by the caller."""
    return [make_problem(dims, R, congruence, noise, seed + 1000 * k, spiky) for k in range(n_inst)]


def problem_for(workload: Workload, R_model=None):
    w = workload
    return make_problem(w.dims, w.R, w.congruence, w.noise, w.seed, w.spiky,
                        w.spike, R_model)


def dense_truth(p: Problem):
    """X_true as a numpy FP64 array of shape dims (small sizes)."""
    X = np.zeros(p.dims)
    for r in range(p.R):
        t = p.lam[r] * p.factors[0][:, r]
        for A in p.factors[1:]:
            t = np.multiply.outer(t, A[:, r])
        X += t
    return X


def dense_tensor(p: Problem):
    """Observed tensor (numpy FP64, shape dims) by eq. synth."""
    Xt = dense_truth(p)
    if p.noise == 0:
        return Xt
    Nz = _rng(p.seed, 2).standard_normal(p.dims)
    return Xt + p.noise * (np.linalg.norm(Xt) / np.linalg.norm(Nz)) * Nz


def device_tensor(p: Problem, device, dtype):
    """Observed tensor generated with torch on `device` as a flat column-major
    buffer (mode 1 fastest), for sizes where a host build is too slow.  The
    values come from torch's seeded generator, so they differ from
    dense_tensor(); tests that need both sides on identical data copy this
    buffer to the host."""
    import torch
    dims = p.dims
    N = len(dims)
    # X_(1) = A1 diag(lam) (A_N (.) ... (.) A_2)^T, built one slab of the last
    # mode at a time so no (P x R) matrix is held.
    A = [torch.as_tensor(M, dtype=torch.float64, device=device) for M in p.factors]
    lam = torch.as_tensor(p.lam, dtype=torch.float64, device=device)
    P = int(np.prod(dims))
    out = torch.empty(P, dtype=torch.float32 if dtype in ("f32", "bf16") else torch.float64,
                      device=device)
    inner = int(np.prod(dims[:-1]))
    # Khatri-Rao of modes 2..N-1 (mode 2 fastest), shape (prod dims[1:-1], R)
    K = torch.ones(1, p.R, dtype=torch.float64, device=device)
    for m in range(1, N - 1):
        K = (A[m][:, None, :] * K[None, :, :]).reshape(-1, p.R)
    left = A[0] * lam[None, :]
    g = torch.Generator(device=device)
    g.manual_seed(int(p.seed) * 7 + 2)
    sq_true = 0.0
    sq_noise = 0.0
    chunk = max(1, (1 << 26) // inner)
    for k0 in range(0, dims[-1], chunk):
        k1 = min(dims[-1], k0 + chunk)
        # slab[i1, j, k] with j over modes 2..N-1 (mode 2 fastest)
        KK = (A[-1][k0:k1, None, :] * K[None, :, :]).reshape(-1, p.R)   # (k, j) flattened, j fastest
        slab = left @ KK.T          # (I1, (k1-k0)*inner/I1)
        flat = slab.T.reshape(-1)   # column-major: i1 fastest, then j, then k
        sq_true += float(torch.dot(flat, flat))
        out[k0 * inner:k1 * inner] = flat.to(out.dtype)
    if p.noise > 0:
        for k0 in range(0, P, 1 << 26):
            k1 = min(P, k0 + (1 << 26))
            z = torch.randn(k1 - k0, generator=g, dtype=torch.float32, device=device)
            sq_noise += float(torch.dot(z.double(), z.double()))
        scale = p.noise * math.sqrt(sq_true) / math.sqrt(sq_noise)
        g.manual_seed(int(p.seed) * 7 + 2)
        for k0 in range(0, P, 1 << 26):
            k1 = min(P, k0 + (1 << 26))
            z = torch.randn(k1 - k0, generator=g, dtype=torch.float32, device=device)
            out[k0:k1] += (scale * z).to(out.dtype)
    return out
