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


def close(got, ref, tol, what=""):
    """Element-wise parity: every entry within tol times the largest |ref|
    of its column (the last axis of a matrix; the whole array for vectors
    and flat tensors), and the Frobenius relative error within tol too.
    Returns (worst scaled entry error, Frobenius relative error)."""
    g = np.asarray(got, dtype=np.complex128)
    r = np.asarray(ref, dtype=np.complex128)
    assert g.shape == r.shape, (what, g.shape, r.shape)
    if r.ndim == 2:
        scale = np.max(np.abs(r), axis=0, keepdims=True)
    else:
        scale = np.max(np.abs(r)) if r.size else 1.0
    scale = np.maximum(scale, 1e-300)
    ent = float(np.max(np.abs(g - r) / scale)) if r.size else 0.0
    fro = rel(g, r)
    assert ent <= tol and fro <= tol, "%s: worst entry %.3g (column-scaled), Frobenius %.3g, tol %.3g" % (
        what, ent, fro, tol)
    return ent, fro
