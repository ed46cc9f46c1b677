"""Pins for oracle/philox.py: numpy's Philox4x64-10 (a library implementation of the
same published generator), a pure-integer scalar version, and the law of the maps."""
import numpy as np
import pytest
from scipy import stats

from oracle import philox


def numpy_block(counter, key):
    """numpy's Philox pre-increments its counter before producing a block."""
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64))
    st = bg.state
    c = [int(v) for v in counter]
    # counter - 1 with borrow across the four 64-bit words (wraps at zero)
    i = 0
    while i < 4 and c[i] == 0:
        c[i] = (1 << 64) - 1
        i += 1
    if i < 4:
        c[i] -= 1
    st["state"]["counter"] = np.array(c, dtype=np.uint64)
    st["buffer_pos"] = 4
    bg.state = st
    return [int(v) for v in bg.random_raw(4)]


CASES = [
    ((1, 0, 0, 0), (1, 2)),
    ((0, 0, 0, 0), (0, 0)),
    ((5, 3, 17, 511), (4, 0)),
    ((2 ** 64 - 1, 2 ** 63, 12345, 7), (2 ** 64 - 1, 99)),
    ((123, 1, 999, 4095), (0xDEADBEEF, 0xCAFEBABE)),
]


@pytest.mark.parametrize("counter,key", CASES)
def test_scalar_matches_numpy(counter, key):
    assert philox.philox4x64_scalar(counter, key) == numpy_block(counter, key)


@pytest.mark.parametrize("counter,key", CASES)
def test_vector_matches_scalar(counter, key):
    out = philox.philox4x64(*[np.array([v], dtype=np.uint64) for v in counter], key[0], key[1])
    assert [int(o[0]) for o in out] == philox.philox4x64_scalar(counter, key)


def test_vector_many_counters_match_numpy():
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2 ** 63, size=(20, 4), dtype=np.uint64)
    out = philox.philox4x64(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3], 77, 88)
    for j in range(20):
        ref = numpy_block(tuple(int(v) for v in ctr[j]), (77, 88))
        assert [int(o[j]) for o in out] == ref


def test_uniform_open_interval():
    w = np.array([0, 2 ** 64 - 1, 2 ** 12 - 1, 2 ** 63], dtype=np.uint64)
    u = philox.to_uniform(w)
    assert np.all(u > 0.0) and np.all(u < 1.0)
    assert u[0] == 2.0 ** -53 and u[2] == 2.0 ** -53
    assert u[1] == 1.0 - 2.0 ** -53
    assert u[3] == 0.5 + 2.0 ** -53
    # every 52-bit value maps exactly: (k + 1/2) 2^-52
    k = np.array([1, 12345, 2 ** 52 - 2], dtype=np.uint64)
    np.testing.assert_array_equal(philox.to_uniform(k << np.uint64(12)),
                                  (k.astype(np.float64) + 0.5) * 2.0 ** -52)


def test_normals_law():
    z = philox.normals(3, 1, philox.STREAM_XI, np.arange(200)[:, None], np.arange(50)[None, :], 9)
    x = z.ravel()
    assert abs(x.mean()) < 4.0 / np.sqrt(x.size)
    assert abs(x.var() - 1.0) < 5.0 * np.sqrt(2.0 / x.size)
    assert stats.kstest(x, "norm").pvalue > 1e-3
    # slot structure: normal i comes from block i // 4
    a = philox.normals(3, 1, 0, 7, 2, 9)
    b = philox.normals(3, 1, 0, 7, 2, 4)
    assert np.array_equal(a[:4], b)


def test_box_muller_slots_from_words():
    o = philox.philox4x64_scalar((0, philox.STREAM_XI, 5, 3), (9, 2))
    u = philox.to_uniform(np.array(o, dtype=np.uint64))
    R0 = np.sqrt(-2 * np.log(u[0]))
    R2 = np.sqrt(-2 * np.log(u[2]))
    ref = [R0 * np.cos(2 * np.pi * u[1]), R0 * np.sin(2 * np.pi * u[1]),
           R2 * np.cos(2 * np.pi * u[3]), R2 * np.sin(2 * np.pi * u[3])]
    got = philox.normals(9, 2, philox.STREAM_XI, 5, 3, 4)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-15)


def test_streams_independent():
    a = philox.normals(1, 0, philox.STREAM_XI, 0, 0, 8)
    b = philox.normals(1, 0, philox.STREAM_COMPLEMENT, 0, 0, 8)
    c = philox.normals(1, 1, philox.STREAM_XI, 0, 0, 8)
    assert not np.allclose(a, b) and not np.allclose(a, c)
