"""Pins of the oracle's learned-proposal pieces: analytic gradients against
central finite differences, a closed-form first Adam step, feature means
and limiting cases, and targets against brute-force leverage."""
import math

import numpy as np

from oracle import leverage as L
from oracle import mlp as M
from oracle.tensor import khatri_rao


def _theta(seed=0):
    rng = np.random.default_rng(seed)
    d = {}
    for name, shp in M.SHAPES:
        fan = shp[1] if len(shp) == 2 else 8
        d[name] = rng.uniform(-1, 1, shp) / math.sqrt(fan)
    return M.pack(d)


def test_param_count():
    assert M.N_PARAMS == 4545


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((30, 4))
    groups = [np.arange(0, 12), np.arange(12, 30)]
    t = np.concatenate([rng.dirichlet(np.ones(12)), rng.dirichlet(np.ones(18))])
    th = _theta(2)
    loss, g = M.grad_fn(th, X, t, groups)
    h = 1e-6
    idx = rng.choice(M.N_PARAMS, 60, replace=False)
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (M.loss_fn(th + e, X, t, groups) - M.loss_fn(th - e, X, t, groups)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_softmax_ce_gradient_is_p_minus_t():
    z = np.array([0.3, -1.0, 2.0])
    t = np.array([0.2, 0.5, 0.3])
    loss, dz = M.loss_and_dz(z, t, [np.arange(3)])
    p = np.exp(z) / np.exp(z).sum()
    assert np.allclose(dz, p - t)
    assert math.isclose(loss, -float(np.sum(t * np.log(p))))


def test_adam_first_step_closed_form():
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    opt = M.Adam(3, lr=1e-3)
    new = opt.step(th, g)
    # after one step m-hat = g and v-hat = g^2, so the move is lr g/(|g|+eps)
    assert np.allclose(new, th - 1e-3 * g / (np.abs(g) + 1e-8))


def test_feature_means_and_limits():
    rng = np.random.default_rng(3)
    I, R = 80, 6
    A = rng.standard_normal((I, R))
    Q, _ = np.linalg.qr(rng.standard_normal((50, R)))
    F = M.row_features(A, [Q])
    for j in range(3):
        assert math.isclose(np.mean(np.exp(F[:, j]) - M.FEAT_EPS), 1.0, rel_tol=1e-9)
    assert abs(F[0, 3]) < 1e-12                   # orthogonal other factor: congruence 0
    C = 0.9
    Gt = (1 - C) * np.eye(R) + C * np.ones((R, R))
    B = Q @ np.linalg.cholesky(Gt).T
    assert math.isclose(M.congruence(B), C, rel_tol=1e-12)


def test_orthogonal_others_make_marginal_proportional_to_f3():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((40, 5))
    A[3] *= 20
    Q, _ = np.linalg.qr(rng.standard_normal((30, 5)))
    Q = Q * rng.uniform(0.5, 2.0, 5)          # orthogonal columns, unequal norms
    t = M.targets([A, Q], 0)
    f3 = np.exp(M.row_features(A, [Q])[:, 2]) - M.FEAT_EPS
    assert np.allclose(t, f3 / f3.sum(), rtol=1e-9)
    # and the targets are the normalised brute-force leverage marginals
    bf = L.krp_marginals_bruteforce([A, Q])[0]
    assert np.allclose(t, bf / bf.sum(), rtol=1e-9)


def test_training_lowers_the_loss():
    rng = np.random.default_rng(5)
    Xs, ts, groups, off = [], [], [], 0
    for k in range(6):
        A = rng.standard_normal((30, 4))
        A[rng.choice(30, 3, replace=False)] *= 10
        B = rng.standard_normal((25, 4))
        Xs.append(M.row_features(A, [B]))
        ts.append(M.targets([A, B], 0))
        groups.append(np.arange(off, off + 30))
        off += 30
    X, t = np.concatenate(Xs), np.concatenate(ts)
    th = _theta(6)
    opt = M.Adam(M.N_PARAMS, lr=3e-3)
    l0 = M.loss_fn(th, X, t, groups)
    for _ in range(300):
        _, g = M.grad_fn(th, X, t, groups)
        th = opt.step(th, g)
    assert M.loss_fn(th, X, t, groups) < l0 - 0.1
