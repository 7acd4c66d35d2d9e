"""Pins of the oracle's exact references against brute force, closed forms
and the numbers the paper prints (CPU only)."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import exact, fock

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _subunitary(M, seed, scale=1.1):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    return X / (np.linalg.norm(X, 2) * scale)


def test_lossless_law_vs_fock_bruteforce():
    """eq. Exact_multi_mode_squeezed_state against a Fock-space expansion,
    M = 4, Haar network."""
    U = synth.haar_unitary(4, 11)
    P, tail = fock.binned_probabilities(U, np.full(4, 0.5), np.zeros(4, int), 1, 30)
    assert tail < 1e-9
    ref = exact.lossless_uniform_total(4, 0.5, np.arange(29))
    np.testing.assert_allclose(P[:29], ref, atol=1e-14)
    assert np.all(ref[1::2] == 0)


@pytest.mark.parametrize("kind", ["haar", "random"])
def test_gaussian_pgf_joint_vs_fock(kind):
    """Determinant generating function (two single-mode bins, lossy,
    non-uniform squeezing) against brute force at M = 2."""
    r = np.array([0.4, 0.6])
    T = 0.8 * synth.haar_unitary(2, 7) if kind == "haar" else _subunitary(2, 3)
    Pf, tail = fock.binned_probabilities(T, r, np.array([0, 1]), 2, 30)
    Pe = exact.gaussian_joint2(T, r, np.array([0, 1]), 64, 64)
    assert np.abs(Pf[:20, :20] - Pe[:20, :20]).max() < 1e-9 + tail
    Pt = exact.gaussian_total(T, r, np.ones(2), 128)
    Pft = np.array([sum(Pf[a, m - a] for a in range(m + 1)) for m in range(25)])
    assert np.abs(Pt[:25] - Pft).max() < 1e-9 + tail
    # a single counted mode: the marginal of bin 0
    P0 = exact.gaussian_total(T, r, np.array([1.0, 0.0]), 128)
    assert np.abs(P0[:25] - Pf[:25].sum(axis=1)).max() < 1e-9 + tail


def test_transposed_network_is_detected():
    """A transposed T changes the binned law for an asymmetric network."""
    r = np.array([0.4, 0.6])
    T = _subunitary(2, 3)
    Pf, _ = fock.binned_probabilities(T, r, np.array([0, 1]), 2, 24)
    Pe_wrong = exact.gaussian_joint2(T.T, r, np.array([0, 1]), 64, 64)
    assert np.abs(Pf[:12, :12] - Pe_wrong[:12, :12]).max() > 1e-3


def test_uniform_loss_law_equals_determinant_and_lossless_limit():
    r = synth.squeezing_random_uniform(12, 0.3, 1.0, 5)
    T = 0.7 * synth.haar_unitary(12, 5)
    np.testing.assert_allclose(exact.uniform_loss_total(r, 0.7, 256),
                               exact.gaussian_total(T, r, np.ones(12), 256), atol=1e-14)
    np.testing.assert_allclose(exact.uniform_loss_total(np.full(10, 0.7), 1.0, 256),
                               exact.lossless_uniform_total(10, 0.7, np.arange(256)), atol=1e-14)


def test_closed_form_moments_vs_determinant():
    r = synth.squeezing_random_uniform(10, 0.4, 1.2, 8)
    T = _subunitary(10, 4, 1.05)
    for counted in (np.ones(10), (np.arange(10) < 4).astype(float)):
        P = exact.gaussian_total(T, r, counted, 512)
        m = np.arange(512)
        mean, var = exact.count_moments(T, r, counted)
        assert abs((m * P).sum() - mean) < 1e-10
        assert abs((m * m * P).sum() - (m * P).sum() ** 2 - var) < 1e-9
    # uniform-loss closed form: mean = t^2 sum N, var = sum t^2 N + t^4 N (2N+1)
    T = 0.9 * synth.haar_unitary(10, 2)
    N = np.sinh(r) ** 2
    mean, var = exact.count_moments(T, r, np.ones(10))
    assert abs(mean - 0.81 * N.sum()) < 1e-12
    assert abs(var - (0.81 * N + 0.81 ** 2 * N * (2 * N + 1)).sum()) < 1e-10


def test_probabilities_normalised_and_nonnegative():
    T = 0.5 * synth.haar_unitary(16, synth.SEED_BASE)
    P = exact.gaussian_total(T, np.ones(16), np.ones(16), 128)
    assert abs(P.sum() - 1) < 1e-12 and P.min() > -1e-15


def test_appendix_b_cutoffs():
    g = json.load(open(os.path.join(GOLDEN, "appB_cutoffs.json")))
    tol = g["tolerance_counts"]
    for M, mmax in zip(g["timing_M"], g["timing_m_max"]):
        assert abs(exact.cutoffs(M, g["r"], g["level"])[1] - mmax) <= tol
    for M, mmin in zip(g["timing_m_min_M"], g["timing_m_min"]):
        assert abs(exact.cutoffs(M, g["r"], g["level"])[0] - mmin) <= tol
    for M, mmax in zip(g["error_M"], g["error_m_max"]):
        assert abs(exact.cutoffs(M, g["r"], g["level"])[1] - mmax) <= tol


def test_pair_moments_vs_fock_and_single_mode():
    """<:n_1 n_2:> and <:n_i^2:> against brute-force Fock probabilities at
    M = 2 (lossy, asymmetric network); the squeezed-vacuum value
    <a^+2 a^2> = 3 sinh^4 r + sinh^2 r for one lossless mode; a transposed
    network changes them."""
    r = np.array([0.4, 0.6])
    T = _subunitary(2, 3)
    Pf, tail = fock.binned_probabilities(T, r, np.array([0, 1]), 2, 30)
    m = np.arange(Pf.shape[0], dtype=float)
    G = exact.pair_moments(T, r)
    tol = 1e-9 + 3600 * tail
    assert abs((m[:, None] * m[None, :] * Pf).sum() - G[0, 1]) < tol
    assert abs((m * (m - 1) * Pf.sum(axis=1)).sum() - G[0, 0]) < tol
    assert abs((m * (m - 1) * Pf.sum(axis=0)).sum() - G[1, 1]) < tol
    np.testing.assert_allclose(G, G.T, rtol=0, atol=1e-15)
    assert np.abs(exact.pair_moments(T.T, r) - G).max() > 1e-3
    for rr in (0.3, 1.1):
        s = np.sinh(rr) ** 2
        np.testing.assert_allclose(exact.pair_moments(np.eye(1), np.array([rr]))[0, 0],
                                   3 * s * s + s, rtol=1e-14)


def test_pair_moments_sum_to_count_factorial_moment():
    """sum over counted i, j of <:n_i n_j:> = <N (N - 1)> = var + mean^2 - mean
    of the bin count (closed-form mean and variance)."""
    r = synth.squeezing_random_uniform(9, 0.4, 1.2, 3)
    T = _subunitary(9, 6, 1.05)
    G = exact.pair_moments(T, r)
    for counted in (np.ones(9), (np.arange(9) % 3 == 0).astype(float)):
        mean, var = exact.count_moments(T, r, counted)
        sel = counted > 0
        np.testing.assert_allclose(G[np.ix_(sel, sel)].sum(), var + mean * mean - mean, rtol=1e-12)
