"""Training set of the learned sampling proposal (a project addition).

Every step runs in the library: the ALS iterates come from cprand_als with
uniform sampling, the features and the exact Khatri-Rao leverage marginals
(the targets) from cprand_mlp_features, the training from cprand_mlp_train.
This module only strings the calls together.
"""
import torch

from . import PROPOSAL_UNIFORM, cprand_als, cprand_mlp_features, make_opts


def proposal_training_set(instances, R, S, iterates=(1, 2, 5), seed=1):
    """Features (rows x 4), targets (rows) and group offsets for a list of
    training instances, each (X view, true factors or None, initial factors)
    with factors as lists of FP32 (I_m x R) device tensors.

    Each instance contributes its true factors, its initial factors and the
    uniform-CPRAND iterates after t outer iterations for t in `iterates`
    (S samples, sampling seed `seed + k` for instance k), so the network sees
    factors like the ones ALS visits.  For every factor set and mode step n,
    the rows of every factor m != n form one softmax group whose target is the
    exact marginal of Khatri-Rao leverage over those rows."""
    sets = []
    dims = None
    for k, (Xv, truth, init) in enumerate(instances):
        dims = tuple(Xv.dims)
        if truth is not None:
            sets.append(truth)
        sets.append(init)
        for t in iterates:
            A = [M.clone() for M in init]
            cprand_als(Xv, A, make_opts(R, S, seed=seed + k, max_iters=t, proposal=PROPOSAL_UNIFORM))
            sets.append(A)
    feats, targets, offs = [], [], [0]
    for A in sets:
        for n in range(len(dims)):
            X, t = cprand_mlp_features(dims, n, R, A)
            feats.append(X)
            targets.append(t)
            for m in range(len(dims)):
                if m != n:
                    offs.append(offs[-1] + dims[m])
    dev = feats[0].device
    return torch.cat(feats), torch.cat(targets), torch.tensor(offs, dtype=torch.int64, device=dev)
