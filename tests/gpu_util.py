"""Helpers for the GPU parity tests: move oracle inputs to the device in the
library's layouts and bring results back."""
import numpy as np
import torch

from oracle.tensor import to_colmajor


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def view_of(X, dtype=torch.float32):
    """Column-major device view of a numpy tensor."""
    import paper_1701_06600_amd as P
    flat = dev(to_colmajor(X), dtype)
    return P.View(flat, X.shape)


def factors_dev(A, dtype=torch.float32):
    return [dev(M, dtype) for M in A]


def cplx_factors_dev(Ah, dtype=torch.complex64):
    return [None if M is None else dev(M, dtype) for M in Ah]


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
