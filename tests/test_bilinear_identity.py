"""The identity the bilinear path rests on, checked with the oracle's own
sampling and propagation (CPU): for real alpha, beta and any mode set S,
sum_{j in S} alpha'_j beta'_j with alpha' = T alpha, beta' = T* beta equals
alpha^T W beta with W = T^T P_S T*; W is Hermitian with the real diagonal
sum_{j in S} |T_ja|^2, and only that diagonal enters the mean of n_S (the
amplitudes of different modes are uncorrelated)."""
import numpy as np

import synth
from oracle import estimator as oest
from oracle import sampler as osamp


def _network(M, seed):
    return synth.haar_unitary(M, seed) * np.linspace(0.6, 1.0, M)[:, None]


def test_bin_occupation_is_the_bilinear_form():
    M, E = 37, 400
    T = _network(M, 4)
    r = np.linspace(0.2, 1.1, M)
    a, b, _ = osamp.sample(r, 0, E, 11)
    ap, bp = oest.propagate(T, a, b)
    rng = np.random.default_rng(2)
    for S in (np.arange(M), np.flatnonzero(rng.random(M) < 0.4), np.array([5])):
        P = np.zeros(M)
        P[S] = 1.0
        W = T.T @ (P[:, None] * T.conj())
        direct = (ap[:, S] * bp[:, S]).sum(axis=1)
        bilinear = np.einsum("ka,ab,kb->k", a, W, b)
        np.testing.assert_allclose(bilinear, direct, rtol=0, atol=1e-12 * np.abs(direct).max())
        assert np.allclose(W, W.conj().T, atol=1e-15)
        np.testing.assert_allclose(W.diagonal().imag, 0.0, atol=1e-16)
        np.testing.assert_allclose(W.diagonal().real, (np.abs(T[S]) ** 2).sum(axis=0), rtol=1e-13)


def test_mean_of_n_S_needs_only_the_diagonal():
    """E[alpha_a beta_b] = delta_ab sinh^2 r_a, so E[n_S] = sum_a W_aa sinh^2 r_a:
    the sample mean of alpha^T W_off beta (W without its diagonal) vanishes
    within its standard error while the diagonal part carries the mean."""
    M, E = 24, 20000
    T = _network(M, 8)
    r = np.linspace(0.3, 1.0, M)
    a, b, _ = osamp.sample(r, 0, E, 19)
    W = T.T @ T.conj()
    D = np.diag(W.diagonal())
    off = np.einsum("ka,ab,kb->k", a, W - D, b)
    diag = np.einsum("ka,ab,kb->k", a, D, b)
    assert abs(off.mean().real) < 5 * off.real.std() / np.sqrt(E)
    assert abs(off.mean().imag) < 5 * off.imag.std() / np.sqrt(E)
    expect = (W.diagonal().real * np.sinh(r) ** 2).sum()
    assert abs(diag.mean().real - expect) < 5 * diag.real.std() / np.sqrt(E)
