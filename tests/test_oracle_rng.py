"""Pins of the oracle's Philox4x64-10 and index draws against an independent
implementation (numpy's Philox bit generator), a published known-answer
vector, and plain integer arithmetic."""
import numpy as np
import pytest

from oracle import philox


def _numpy_block(ctr, key):
    # numpy's bit generator increments the 256-bit counter before each block.
    c = [int(x) for x in ctr]
    c[0] -= 1
    for i in range(3):
        if c[i] < 0:
            c[i] += 2 ** 64
            c[i + 1] -= 1
    bg = np.random.Philox(counter=np.array(c, dtype=np.uint64),
                          key=np.array(key, dtype=np.uint64))
    return bg.random_raw(4)


@pytest.mark.parametrize("ctr,key", [
    ((1, 0, 0, 0), (0, 0)),
    ((5, 7, 11, 13), (123456789, 5)),
    ((0, 4, 0, 9), (2 ** 63 + 17, 2 ** 64 - 1)),
    ((2 ** 40 + 3, 199, 2, 1), (1701066002, 6)),
])
def test_philox_matches_numpy(ctr, key):
    mine = philox.philox4x64_10(tuple(np.uint64(c) for c in ctr), key)
    assert np.array_equal(mine, _numpy_block(ctr, key))


def test_philox_known_answer_zero():
    # Random123 known-answer vector for philox4x64-10, counter 0 and key 0.
    out = philox.philox4x64_10((0, 0, 0, 0), (0, 0))
    assert [int(x) for x in out] == [0x16554d9eca36314c, 0xdb20fe9d672d0fdc,
                                     0xd7e772cee186176b, 0x7e68b68aec7ba23b]


def test_philox_vectorised_equals_scalar():
    s = np.arange(37, dtype=np.uint64)
    vec = philox.philox4x64_10((s, 3, 1, 0), (99, philox.TAG_SAMPLES))
    for i in (0, 5, 36):
        one = philox.philox4x64_10((np.uint64(i), 3, 1, 0), (99, philox.TAG_SAMPLES))
        assert np.array_equal(vec[i], one)


def test_mulhilo_against_python_ints():
    rng = np.random.default_rng(0)
    a = rng.integers(0, 2 ** 63, size=500, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    b = rng.integers(0, 2 ** 63, size=500, dtype=np.uint64) * np.uint64(2)
    hi, lo = philox.mulhilo64(a, b)
    for x, y, h, l in zip(a, b, hi, lo):
        p = int(x) * int(y)
        assert int(h) == p >> 64 and int(l) == p & (2 ** 64 - 1)


def test_bounded_edges():
    u = np.array([0, 1, 2 ** 63, 2 ** 64 - 1], dtype=np.uint64)
    for n in (1, 2, 3, 2 ** 31 - 1):
        got = philox.bounded(u, n)
        want = [(int(x) * n) >> 64 for x in u]
        assert list(got) == want
        assert got.max() < n


def test_sample_indices_ranges_and_uniformity():
    dims = (7, 5, 11, 3, 2, 13)          # N = 6 -> two Philox blocks per sample
    n = 2
    idx = philox.sample_indices(dims, n, 20000, 1234, 7)
    assert (idx[:, n] == -1).all()
    for m, I in enumerate(dims):
        if m == n:
            continue
        col = idx[:, m]
        assert col.min() >= 0 and col.max() < I
        counts = np.bincount(col, minlength=I)
        expected = len(col) / I
        chi2 = float(np.sum((counts - expected) ** 2 / expected))
        # chi-square with I-1 dof: mean I-1, sd sqrt(2(I-1)); allow 6 sd
        assert chi2 < (I - 1) + 6 * np.sqrt(2 * (I - 1))


def test_sample_indices_depend_on_t_and_n():
    dims = (10, 10, 10)
    a = philox.sample_indices(dims, 0, 50, 5, 0)
    b = philox.sample_indices(dims, 0, 50, 5, 1)
    c = philox.sample_indices(dims, 1, 50, 5, 0)
    assert not np.array_equal(a, b)
    assert not np.array_equal(a[:, 1], c[:, 2])


def test_signs_balanced_and_fit_indices():
    signs = philox.sign_vectors((400, 1000), 77)
    for d in signs:
        assert set(np.unique(d)) <= {-1, 1}
        assert abs(float(d.mean())) < 0.15
    f = philox.fit_indices((4, 5, 6, 7, 8), 4096, 3)
    assert f.shape == (4096, 5)
    for k, I in enumerate((4, 5, 6, 7, 8)):
        assert f[:, k].min() >= 0 and f[:, k].max() < I
        assert len(np.unique(f[:, k])) == I
