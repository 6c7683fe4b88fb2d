"""Philox4x64-10 counter-based random numbers, written from its published
definition (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11), vectorised over numpy uint64 arrays.

Test infrastructure (see oracle/__init__.py): nothing in the GPU library uses
this file.

The method draws three kinds of random numbers, and each is a pure function of
(seed, stream tag, counter) so that any implementation that follows the same
definition reproduces them bit for bit:

* sample multi-indices of the sampled least-squares step (uniform sampling
  with replacement, Section 3.2; a fresh draw for every mode and outer
  iteration, Section 4.2);
* the random sign flips D_m of the mixing operator (Section 2.2, Alg. 4);
* the fixed set of P-hat tensor entries of the sampled fit estimate
  (Section 3.4; the same entries at every iteration, Section 4.2).

A random 64-bit word u is mapped to [0, I) as floor(u * I / 2^64) (the high
word of the 128-bit product); the paper leaves this mapping open.
"""
import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

# Stream tags (second key word).
TAG_FACTORS = 0
TAG_LAMBDA = 1
TAG_NOISE = 2
TAG_SIGNS = 3
TAG_INIT = 4
TAG_SAMPLES = 5
TAG_FIT = 6
TAG_SPIKE = 7
TAG_MLP_INIT = 8
TAG_TRAIN = 9


def mulhilo64(a, b):
    """(high, low) 64-bit words of the 128-bit product a*b, elementwise."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    with np.errstate(over="ignore"):
        a_lo, a_hi = a & _M32, a >> _S32
        b_lo, b_hi = b & _M32, b >> _S32
        ll = a_lo * b_lo
        hl = a_hi * b_lo
        lh = a_lo * b_hi
        hh = a_hi * b_hi
        t = hl + (ll >> _S32)          # < 2^64: (2^32-1)^2 + 2^32-1
        u = lh + (t & _M32)
        hi = hh + (t >> _S32) + (u >> _S32)
        lo = a * b
    return hi, lo


def philox4x64_10(ctr, key):
    """Ten Philox rounds.  ctr: four uint64 arrays (broadcastable), key: two.

    One round maps (x0, x1, x2, x3) under key (k0, k1) to
    (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1, lo(M0*x0));
    the key is bumped by the Weyl constants (W0, W1) between rounds.
    Returns a (..., 4) uint64 array.
    """
    x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) for c in ctr)
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    k0 = np.uint64(key[0])
    k1 = np.uint64(key[1])
    with np.errstate(over="ignore"):
        for r in range(10):
            if r > 0:
                k0 = np.uint64(k0 + W0)
                k1 = np.uint64(k1 + W1)
            hi0, lo0 = mulhilo64(M0, x0)
            hi1, lo1 = mulhilo64(M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return np.stack([x0, x1, x2, x3], axis=-1)


def bounded(u, n):
    """Map uniform 64-bit words u to integers in [0, n): high word of u*n."""
    hi, _ = mulhilo64(u, np.uint64(n))
    return hi.astype(np.int64)


def sample_indices(dims, n, S, seed, t):
    """S i.i.d. uniform multi-indices over the modes other than n.

    Returns an (S, N) int64 array; column n holds -1.  Sample s of outer
    iteration t for mode n uses counter (s, t, n, b) under key
    (seed, TAG_SAMPLES); the k-th mode other than n takes word k % 4 of
    block b = k // 4.
    """
    N = len(dims)
    others = [m for m in range(N) if m != n]
    idx = np.full((S, N), -1, dtype=np.int64)
    s = np.arange(S, dtype=np.uint64)
    nblocks = (len(others) + 3) // 4
    for b in range(nblocks):
        words = philox4x64_10((s, t, n, b), (seed, TAG_SAMPLES))
        for w in range(4):
            k = 4 * b + w
            if k < len(others):
                m = others[k]
                idx[:, m] = bounded(words[:, w], dims[m])
    return idx


def sample_words(N, n, S, seed, t):
    """The raw words behind sample_indices: (S, N) uint64, column n unused."""
    others = [m for m in range(N) if m != n]
    out = np.zeros((S, N), dtype=np.uint64)
    s = np.arange(S, dtype=np.uint64)
    for b in range((len(others) + 3) // 4):
        words = philox4x64_10((s, t, n, b), (seed, TAG_SAMPLES))
        for w in range(4):
            k = 4 * b + w
            if k < len(others):
                out[:, others[k]] = words[:, w]
    return out


def sign_vectors(dims, seed):
    """Random signs D_m (Section 2.2): entry i of mode m is -1 when bit 63 of
    word 0 of Philox((i, m, 0, 0), (seed, TAG_SIGNS)) is set, else +1."""
    out = []
    for m, I in enumerate(dims):
        words = philox4x64_10((np.arange(I, dtype=np.uint64), m, 0, 0),
                              (seed, TAG_SIGNS))
        bit = (words[:, 0] >> np.uint64(63)).astype(np.int64)
        out.append((1 - 2 * bit).astype(np.int8))
    return out


def fit_indices(dims, P_hat, seed):
    """The fixed set of P_hat multi-indices (i.i.d. uniform, with replacement)
    of the sampled fit estimate, Section 3.4.  Entry p uses counter
    (p, 0, 0, b) under key (seed, TAG_FIT); mode k takes word k % 4 of block
    k // 4.  Returns a (P_hat, N) int64 array."""
    N = len(dims)
    idx = np.zeros((P_hat, N), dtype=np.int64)
    p = np.arange(P_hat, dtype=np.uint64)
    for b in range((N + 3) // 4):
        words = philox4x64_10((p, 0, 0, b), (seed, TAG_FIT))
        for w in range(4):
            k = 4 * b + w
            if k < N:
                idx[:, k] = bounded(words[:, w], dims[k])
    return idx
