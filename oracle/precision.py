"""The BF16 precision form of the sampled least-squares step (a project
addition to Alg. 3): BF16 tensor entries and BF16 sampled Khatri-Rao rows
in the product, FP64 Gram and solve, and one step of iterative refinement
against the FP32 normal equations.

Test infrastructure (see oracle/__init__.py).

Rounding decisions are taken in the precision the GPU takes them in: a
sampled Khatri-Rao row is the FP32 product of the factor rows in increasing
mode order, and FP32 values go to BF16 by round-to-nearest-even.  Everything
after the rounding is summed in FP64 here.
"""
import numpy as np

from .cprand import sample_fibers


def bf16_round(x):
    """Round FP32 values to the nearest BF16 value (ties to even), returned
    as FP32: keep the top 16 bits of the IEEE single after adding half an
    ulp of the kept part plus the tie-breaking bit.  NaN is not handled
    (the method never produces one)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return r.astype(np.uint32).view(np.float32)


def skr_f32(idx, A, n):
    """Sampled Khatri-Rao rows formed in FP32, multiplying the rows of the
    factors m != n in increasing m (Alg. 2 in the GPU's precision)."""
    S = idx.shape[0]
    R = A[(n + 1) % len(A)].shape[1]
    Z = np.ones((S, R), dtype=np.float32)
    for m in range(len(A)):
        if m == n:
            continue
        Z = (Z * np.asarray(A[m], dtype=np.float32)[idx[:, m], :]).astype(np.float32)
    return Z


def bf16_normal_blocks(X32, idx, A32, n, w=None):
    """W = bf16(X_S) bf16(w z) and V = bf16(w z)^T bf16(z) for the sampled
    rows z of Alg. 2 (weights w, 1 for uniform sampling), both summed in
    FP64: the normal-equation blocks of the sampled LS with the product's
    inputs in BF16."""
    Z = skr_f32(idx, A32, n)
    zb = bf16_round(Z).astype(np.float64)
    wv = np.ones(idx.shape[0]) if w is None else np.asarray(w, dtype=np.float64)
    zw = bf16_round((wv[:, None] * zb).astype(np.float32)).astype(np.float64)
    Xs = bf16_round(sample_fibers(np.asarray(X32, dtype=np.float32), idx, n)).astype(np.float64)
    return Xs @ zw, zw.T @ zb


def refine_step(A0, V_lo, W_hi, V_hi):
    """One step of iterative refinement of A V = W: the residual is formed
    with the higher-precision blocks (W_hi, V_hi) and corrected with the
    lower-precision operator, A1 = A0 + (W_hi - A0 V_hi) V_lo^{-1}."""
    return A0 + np.linalg.solve(V_lo.T, (W_hi - A0 @ V_hi).T).T
