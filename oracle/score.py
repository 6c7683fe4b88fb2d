"""Factor-match score (eq. score, Section 4.2).

Test infrastructure (see oracle/__init__.py).

For one true and one computed component the score is the product over modes
of the cosines between matching factor vectors (lambda ignored).  The score
of a decomposition is the mean over the true components, maximised over the
assignment of computed components to true ones.
"""
import itertools

import numpy as np
from scipy.optimize import linear_sum_assignment


def component_scores(A_true, A_est):
    """(R_true, R_est) matrix of per-pair scores."""
    R1 = A_true[0].shape[1]
    R2 = A_est[0].shape[1]
    S = np.ones((R1, R2))
    for At, Ae in zip(A_true, A_est):
        nt = np.linalg.norm(At, axis=0)
        ne = np.linalg.norm(Ae, axis=0)
        C = (At.T @ Ae) / np.outer(np.where(nt > 0, nt, 1), np.where(ne > 0, ne, 1))
        S = S * C
    return S


def score(A_true, A_est):
    """Mean matched score; exhaustive over assignments for small ranks, the
    Hungarian method otherwise (the optimum is the same)."""
    S = component_scores(A_true, A_est)
    R1, R2 = S.shape
    if R1 <= 7 and R2 <= 7:
        best = -np.inf
        for perm in itertools.permutations(range(R2), R1):
            best = max(best, float(np.mean(S[np.arange(R1), list(perm)])))
        return best
    rows, cols = linear_sum_assignment(-S)
    return float(np.mean(S[rows, cols]))
