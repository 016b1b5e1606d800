"""Pins of the oracle's Philox4x64-10 and Wigner draw (library routine, statistics)."""
import numpy as np
import pytest

from oracle.philox import gaussian_pair, philox4x64_10, uniform_open


def numpy_block(ctr, key):
    """Philox block for counter ``ctr`` from numpy (which increments before use)."""
    c = list(ctr)
    # numpy adds one to the counter before generating: hand it ctr - 1
    borrow = 1
    prev = []
    for w in c:
        v = (w - borrow) % (1 << 64)
        borrow = 1 if (w < borrow) else 0
        prev.append(v)
    bg = np.random.Philox(counter=np.array(prev, dtype=np.uint64),
                          key=np.array(key, dtype=np.uint64))
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (5, 0)),
    ((123456789, 2, 63, 3), (1001, 0)),
    ((2**64 - 1, 2**63, 7, 2**40 + 3), (2**64 - 5, 2**33)),
    ((0, 1, 0, 0), (42, 0)),
])
def test_philox_matches_numpy(ctr, key):
    got = philox4x64_10([np.uint64(c) for c in ctr], [np.uint64(k) for k in key])
    assert [int(g) for g in got] == numpy_block(ctr, key)


def test_philox_vectorised_matches_scalar():
    rng = np.random.default_rng(0)
    c0 = rng.integers(0, 2**63, size=20, dtype=np.uint64)
    got = philox4x64_10([c0, np.uint64(1), np.uint64(2), np.uint64(3)], [np.uint64(9), np.uint64(0)])
    for i in range(20):
        ref = numpy_block((int(c0[i]), 1, 2, 3), (9, 0))
        assert [int(g[i]) for g in got] == ref


def test_uniform_open_open_interval():
    u = uniform_open(np.array([0, 2**64 - 1, 2**63], dtype=np.uint64))
    assert u[0] == 2.0 ** -53
    assert u[1] == 1.0 - 2.0 ** -53 and u[1] < 1.0
    assert u[2] == 0.5 + 2.0 ** -53


def test_gaussian_moments():
    n = 200000
    ctr = (np.arange(n, dtype=np.uint64), np.uint64(0), np.uint64(0), np.uint64(0))
    g_re, g_im = gaussian_pair(ctr, (np.uint64(77), np.uint64(0)))
    for g in (g_re, g_im):
        assert abs(g.mean()) < 5 / np.sqrt(n)
        assert abs(g.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(np.mean(g_re * g_im)) < 5 / np.sqrt(n)
    # fourth moment of a standard normal is 3
    assert abs(np.mean(g_re ** 4) - 3.0) < 5 * np.sqrt(96.0 / n)
