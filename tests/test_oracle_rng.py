"""Pins of the oracle's random-number layer (CPU only).

Philox4x64-10 is pinned bit-exactly to numpy's ``np.random.Philox`` (library
code implementing the same published generator).  numpy advances its counter
before generating, so its first block for counter c is Philox(c + 1).
"""
import numpy as np
import pytest
from scipy import stats

from oracle import philox as R


def _numpy_block(counter, key):
    # explicit uint64 arrays: a list of Python ints above 2^63 goes through float64
    bg = np.random.Philox(counter=np.array(counter, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_philox_matches_numpy(seed):
    rng = np.random.default_rng(seed)
    for _ in range(50):
        c = [int(x) for x in rng.integers(0, 2 ** 63, size=4, dtype=np.int64)]
        k = [int(x) for x in rng.integers(0, 2 ** 63, size=2, dtype=np.int64)]
        c[1] |= 1 << 63                       # exercise the top bit too
        want = _numpy_block(c, k)
        got = R.philox4x64(c[0] + 1, c[1], c[2], c[3], np.uint64(k[0]), np.uint64(k[1]))
        assert [int(g[0]) for g in got] == want


def test_philox_counter_carry_matches_numpy():
    # numpy's increment carries from word 0 into word 1
    c = [2 ** 64 - 1, 5, 7, 9]
    want = _numpy_block(c, [11, 13])
    got = R.philox4x64(0, 6, 7, 9, np.uint64(11), np.uint64(13))
    assert [int(g[0]) for g in got] == want


def test_philox_vectorised_equals_scalar():
    ids = np.arange(100, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    vec = R.philox4x64(ids, 17, 258, 0, np.uint64(5), np.uint64(6))
    for i in (0, 1, 50, 99):
        one = R.philox4x64(ids[i], 17, 258, 0, np.uint64(5), np.uint64(6))
        assert all(int(v[i]) == int(o[0]) for v, o in zip(vec, one))


def test_mulhilo_matches_python_bigint():
    rng = np.random.default_rng(7)
    a = rng.integers(0, 2 ** 63, size=1000, dtype=np.int64).astype(np.uint64) * np.uint64(2) + np.uint64(1)
    b = rng.integers(0, 2 ** 63, size=1000, dtype=np.int64).astype(np.uint64) * np.uint64(3)
    hi, lo = R.mulhilo64(a, b)
    for i in range(0, 1000, 37):
        p = int(a[i]) * int(b[i])
        assert int(hi[i]) == p >> 64 and int(lo[i]) == p & (2 ** 64 - 1)


def test_uniform_map_bits_and_fp32_exactness():
    w = [np.array([0xFFFFFFFFFFFFFFFF, 0, (5 << 41) | (3 << 9)], dtype=np.uint64)] * 4
    U = R.uniforms(w)
    assert U[0, 0] == (2 ** 23 - 0.5) * 2.0 ** -23 and U[0, 1] == (2 ** 23 - 0.5) * 2.0 ** -23
    assert U[1, 0] == 0.5 * 2.0 ** -23 and U[1, 1] == 0.5 * 2.0 ** -23
    assert U[2, 0] == 5.5 * 2.0 ** -23 and U[2, 1] == 3.5 * 2.0 ** -23
    ids = np.arange(200000, dtype=np.uint64)
    U = R.draw(ids, 3, 259, 1, 2)
    assert np.all((U > 0) & (U < 1))
    assert np.array_equal(U.astype(np.float32).astype(np.float64), U)


def test_uniform_chi2_and_independence():
    ids = np.arange(400000, dtype=np.uint64)
    U = R.draw(ids, 12, R.tag(0, R.COLL), 1607, 2)
    for k in range(8):
        counts = np.bincount((U[:, k] * 64).astype(int), minlength=64)
        assert stats.chisquare(counts).pvalue > 1e-4
    c = np.corrcoef(U.T)
    assert np.max(np.abs(c - np.eye(8))) < 0.01


def test_box_muller_normal_ks():
    ids = np.arange(300000, dtype=np.uint64)
    U = R.draw(ids, 0, R.tag(1, R.PARTNER), 9, 9)
    n0, n1 = R.box_muller(U[:, 0], U[:, 1])
    for n in (n0, n1):
        assert stats.kstest(n, "norm").pvalue > 1e-4
    assert abs(np.corrcoef(n0, n1)[0, 1]) < 0.01


def test_maxwell_velocity_moments():
    ids = np.arange(400000, dtype=np.uint64)
    U = R.draw(ids, 0, R.tag(0, R.INIT), 3, 4)
    v = R.maxwell_velocity(U[:, 1:5], 2.0)
    var = np.var(v, axis=0)
    assert np.allclose(var, 4.0, rtol=0.01)
    assert np.allclose(np.mean(v, axis=0), 0.0, atol=0.01)
