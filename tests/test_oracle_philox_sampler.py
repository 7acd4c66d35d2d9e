"""Pins of the oracle's noise and sampler (CPU only).

Philox4x64-10 is pinned bit-exactly to numpy's independent implementation
(numpy.random.Philox emits the block of counter + 1 after a state set to
counter).  The sampler is pinned by the second moments the squeezed-state
integral fixes (main text, squeezed input as a real coherent integral):
Var(alpha) = Var(beta) = sinh r cosh r, Cov(alpha, beta) = sinh^2 r.
"""
import numpy as np
import pytest

from oracle import philox, sampler


def _numpy_block(ctr, key):
    bg = np.random.Philox(counter=np.array(ctr, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("seed", [0, 1, 12345, 2**63 + 17])
def test_philox_matches_numpy(seed):
    rng = np.random.default_rng(seed % 1000)
    for _ in range(20):
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4, dtype=np.uint64)]
        key = [seed & (2**64 - 1), int(rng.integers(0, 2**63, dtype=np.uint64))]
        want = _numpy_block(ctr, key)
        c = [ctr[0] + 1] + ctr[1:]
        got = philox.philox4x64_10(*[np.uint64(x) for x in c], np.uint64(key[0]), np.uint64(key[1]))
        assert [int(g) for g in got] == want


def test_philox_vectorised_equals_scalar():
    g = np.arange(5, dtype=np.uint64)[:, None]
    p = np.arange(3, dtype=np.uint64)[None, :]
    out = philox.philox4x64_10(g, p, np.uint64(2), np.uint64(0), np.uint64(9), np.uint64(0))
    for i in range(5):
        for j in range(3):
            one = philox.philox4x64_10(np.uint64(i), np.uint64(j), np.uint64(2), np.uint64(0),
                                       np.uint64(9), np.uint64(0))
            assert [int(o[i, j]) for o in out] == [int(x) for x in one]


def test_mulhilo_against_python_ints():
    rng = np.random.default_rng(3)
    a = rng.integers(0, 2**64 - 1, size=1000, dtype=np.uint64)
    b = rng.integers(0, 2**64 - 1, size=1000, dtype=np.uint64)
    hi, lo = philox.mulhilo64(a, b)
    for x, y, h, l in zip(a[:200], b[:200], hi[:200], lo[:200]):
        prod = int(x) * int(y)
        assert int(h) == prod >> 64 and int(l) == prod & (2**64 - 1)


def test_box_muller_ranges_and_extremes():
    top = np.array([2**64 - 1], dtype=np.uint64)
    zero = np.array([0], dtype=np.uint64)
    w1, w2 = sampler.box_muller(top, zero)     # u = 1 exactly -> radius 0
    assert w1[0] == 0.0 and w2[0] == 0.0
    w1, w2 = sampler.box_muller(zero, zero)    # u = 2^-53, v = 0
    assert np.isfinite(w1[0]) and abs(w1[0] - np.sqrt(2 * 53 * np.log(2))) < 1e-12 and w2[0] == 0.0


def test_noise_independent_of_chunking():
    r = np.linspace(0.2, 1.3, 7)
    a1, b1, n1 = sampler.sample(r, 0, 30, seed=77)
    a2, b2, n2 = sampler.sample(r, 10, 20, seed=77)
    np.testing.assert_array_equal(a1[10:], a2)
    np.testing.assert_array_equal(b1[10:], b2)
    a3, _, _ = sampler.sample(r, 0, 30, seed=77, net=1)
    assert not np.allclose(a1, a3)


def test_sampler_second_moments():
    r = np.array([0.3, 1.0, 1.5, 0.7])
    E = 200_000
    a, b, n = sampler.sample(r, 0, E, seed=5)
    A, N = sampler.input_moments(r)
    for got, want, var in (((a * a).mean(0), A, 2 * A * A),
                           ((b * b).mean(0), A, 2 * A * A),
                           ((a * b).mean(0), N, A * A + N * N)):
        se = np.sqrt(var / E)
        assert np.all(np.abs(got - want) < 5 * se)
    np.testing.assert_allclose(n, (a * b).sum(1), rtol=1e-14)
    assert abs(np.corrcoef(a[:, 0], a[:, 1])[0, 1]) < 5 / np.sqrt(E)


def test_vacuum_modes_are_zero():
    a, b, n = sampler.sample(np.array([0.0, 0.8, 0.0]), 0, 100, seed=1)
    assert np.all(a[:, [0, 2]] == 0) and np.all(b[:, [0, 2]] == 0)
