"""Exact photon-count laws the matrix-P estimator converges to (FP64).

E1  lossless network, uniform squeezing: the total count is 0 for odd m and
    negative-binomial in m/2 for even m (eq. Exact_multi_mode_squeezed_state,
    p_S = 1 / (1 + sinh^2 r)).
E2  uniform loss T = t U (any unitary U), any squeezing profile: the paper
    states that an exact law exists (text after eq.
    Exact_multi_mode_squeezed_state).  Its generating function follows from the
    sampled Gaussian (oracle.sampler) because the +P expectation of
    exp(sum_b (z_b - 1) n_b) is the count generating function; for T = t U the
    bilinear form is t^2 alpha . beta and each mode gives
        E[exp(c alpha_j beta_j)] = (1 - 2 c N_j - c^2 N_j)^(-1/2),  c = t^2 (z-1).
E3  any T, any bins: the same expectation is a Gaussian integral,
        G(z_1..z_d) = det(I_2M - Sigma B(z))^(-1/2),
    Sigma = [[diag A, diag N], [diag N, diag A]],  B = [[0, W], [W^T, 0]],
    W = T^T diag(z_b(i) - 1 over counted outputs i) T*,
    evaluated on the unit circle through eigenvalue factorisations whose
    principal square roots are analytic in the closed unit disk.
E4  closed-form mean and variance of a bin count, and the normally ordered
    pair moments of single modes (Isserlis' theorem on the same Gaussian).
Cutoffs m_min / m_max of Appendix B (first and last count at which the
lossless law reaches a given level).

Probabilities are recovered from generating functions by numpy's FFT on a
grid of K points (aliasing mod K; K is chosen far beyond the support).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np
from scipy.special import gammaln

from .sampler import input_moments


# ---------------------------------------------------------------- E1
def lossless_uniform_total(M: int, r: float, m: np.ndarray) -> np.ndarray:
    """eq. Exact_multi_mode_squeezed_state, in log space."""
    m = np.asarray(m)
    nbar = np.sinh(r) ** 2
    p = 1.0 / (1.0 + nbar)
    k = m / 2.0
    half = M / 2.0
    with np.errstate(divide="ignore"):
        lp = (gammaln(half + k) - gammaln(k + 1.0) - gammaln(half)
              + half * np.log(p) + k * np.log1p(-p))
    out = np.exp(lp)
    return np.where((m % 2 == 0) & (m >= 0), out, 0.0)


def cutoffs(M: int, r: float, level: float = 1e-7):
    """(m_min, m_max): the first and last even count whose lossless
    probability is at least `level` (Appendix B uses 1e-7)."""
    nbar = np.sinh(r) ** 2
    mean = M * nbar
    sd = np.sqrt(M * nbar * (2 * nbar + 1) * 2)
    hi = int(mean + 20 * sd + 50)
    m = np.arange(0, hi + 1, 2)
    P = lossless_uniform_total(M, r, m)
    ok = m[P >= level]
    return int(ok.min()), int(ok.max())


# ---------------------------------------------------------------- E2
def uniform_loss_pgf(r: np.ndarray, t: float, z: np.ndarray) -> np.ndarray:
    """Total-count generating function for T = t U at points z (|z| <= 1).

    Each mode factor f_j(z) = 1 - 2 c N_j - c^2 N_j, c = t^2 (z - 1), is a
    quadratic in z with both roots outside the closed unit disk (they are
    1 - (1 +- coth r_j) / t^2); writing f_j(z) = f_j(0) (1 - z/z1)(1 - z/z2)
    makes every principal square root analytic on the disk."""
    r = np.asarray(r, dtype=np.float64)
    _, N = input_moments(r)
    z = np.asarray(z, dtype=np.complex128)
    u = t * t
    G = np.ones_like(z)
    for Nj, rj in zip(N, r):
        if Nj == 0.0:
            continue
        cth = 1.0 / np.tanh(rj)
        z1 = 1.0 - (1.0 + cth) / u
        z2 = 1.0 - (1.0 - cth) / u
        f0 = 1.0 + 2.0 * u * Nj - u * u * Nj
        G = G * (f0 ** -0.5) * (1.0 - z / z1) ** -0.5 * (1.0 - z / z2) ** -0.5
    return G


def probabilities_from_pgf(Gk: np.ndarray) -> np.ndarray:
    """P(m mod K) from samples of the generating function at z_k = e^{2 pi i k/K}
    (one axis per bin)."""
    return np.fft.fftn(Gk) / Gk.size


def unit_circle(K: int) -> np.ndarray:
    return np.exp(2j * np.pi * np.arange(K) / K)


def uniform_loss_total(r: np.ndarray, t: float, K: int) -> np.ndarray:
    """P(m), m = 0..K-1 (aliased mod K), for T = t U."""
    return probabilities_from_pgf(uniform_loss_pgf(r, t, unit_circle(K))).real


# ---------------------------------------------------------------- E3
def _sigma(r):
    A, N = input_moments(np.asarray(r, dtype=np.float64))
    return np.block([[np.diag(A), np.diag(N)], [np.diag(N), np.diag(A)]])


def _bilinear(T: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """B = [[0, W], [W^T, 0]] with W = T^T diag(weights) T*."""
    T = np.asarray(T, dtype=np.complex128)
    W = T.T @ (weights[:, None] * T.conj())
    M = T.shape[1]
    Z = np.zeros((M, M), dtype=np.complex128)
    return np.block([[Z, W], [W.T, Z]])


def _det_inv_sqrt_positive(Q: np.ndarray) -> float:
    """det(Q)^(-1/2) for a matrix whose determinant is real and positive
    (it equals the inverse square of a probability)."""
    sign, logdet = np.linalg.slogdet(Q)
    return float(np.exp(-0.5 * logdet))


def gaussian_pgf_total(T: np.ndarray, r: np.ndarray, counted: np.ndarray, z: np.ndarray):
    """G(z) of the count summed over the counted outputs (boolean mask).

    det(I - (z-1) Sigma B1) = det(Q - z Sigma B1), Q = I + Sigma B1, and
    det(Q)^(-1/2) = P(0) > 0; the remaining factors (1 - z nu_i)^(-1/2),
    nu = eig(Q^-1 Sigma B1), have |nu_i| < 1."""
    S = _sigma(r)
    SB = S @ _bilinear(T, np.asarray(counted, dtype=np.float64))
    Q = np.eye(SB.shape[0]) + SB
    p0 = _det_inv_sqrt_positive(Q)
    nu = np.linalg.eigvals(np.linalg.solve(Q, SB))
    z = np.asarray(z, dtype=np.complex128)
    G = np.full(z.shape, p0, dtype=np.complex128)
    for v in nu:
        G = G * (1.0 - z * v) ** -0.5
    return G


def gaussian_total(T, r, counted, K: int) -> np.ndarray:
    return probabilities_from_pgf(gaussian_pgf_total(T, r, counted, unit_circle(K))).real


def gaussian_pgf_joint2(T, r, bin_of_mode, K1: int, K2: int) -> np.ndarray:
    """G(z1, z2) of two bins on a K1 x K2 grid of the unit torus.

    With Q = I + Sigma B1 + Sigma B2 and R(z1) = Q - z1 Sigma B1:
        G(z1, 0)  = det(Q)^(-1/2) prod (1 - z1 nu_i)^(-1/2),
        G(z1, z2) = G(z1, 0) prod (1 - z2 mu_i(z1))^(-1/2),
    nu = eig(Q^-1 Sigma B1), mu(z1) = eig(R(z1)^-1 Sigma B2), all |.| < 1."""
    b = np.asarray(bin_of_mode)
    S = _sigma(r)
    SB1 = S @ _bilinear(T, (b == 0).astype(np.float64))
    SB2 = S @ _bilinear(T, (b == 1).astype(np.float64))
    Q = np.eye(SB1.shape[0]) + SB1 + SB2
    p0 = _det_inv_sqrt_positive(Q)
    nu = np.linalg.eigvals(np.linalg.solve(Q, SB1))
    z1s, z2s = unit_circle(K1), unit_circle(K2)
    G = np.empty((K1, K2), dtype=np.complex128)
    for a, z1 in enumerate(z1s):
        g1 = p0 * np.prod((1.0 - z1 * nu) ** -0.5)
        R = Q - z1 * SB1
        mu = np.linalg.eigvals(np.linalg.solve(R, SB2))
        row = np.full(K2, g1, dtype=np.complex128)
        for v in mu:
            row = row * (1.0 - z2s * v) ** -0.5
        G[a] = row
    return G


def gaussian_joint2(T, r, bin_of_mode, K1: int, K2: int) -> np.ndarray:
    return probabilities_from_pgf(gaussian_pgf_joint2(T, r, bin_of_mode, K1, K2)).real


# ---------------------------------------------------------------- E4
def count_moments(T: np.ndarray, r: np.ndarray, counted: np.ndarray):
    """Mean and variance of the count summed over the counted outputs:
        mean = sum_j W_jj N_j,
        var  = mean + sum_jk [N_j N_k |W_jk|^2 + A_j A_k Re(W_jk^2)],
    W = T^T P_S T* (Hermitian)."""
    T = np.asarray(T, dtype=np.complex128)
    A, N = input_moments(np.asarray(r, dtype=np.float64))
    w = np.asarray(counted, dtype=np.float64)
    W = T.T @ (w[:, None] * T.conj())
    mean = float(np.real(np.diag(W)) @ N)
    var = mean + float(N @ (np.abs(W) ** 2) @ N) + float(A @ np.real(W * W) @ A)
    return mean, var


def pair_moments(T: np.ndarray, r: np.ndarray) -> np.ndarray:
    """<:n_i n_j:> = <a_i^+ a_j^+ a_i a_j> of the lossy output of squeezed
    vacua (Isserlis' theorem on the Gaussian state):
        N_ii N_jj + |N_ij|^2 + |S_ij|^2,
    N = T diag(sinh^2 r) T^+  (the <a^+ a> correlations, up to conjugation),
    S = T diag(sinh r cosh r) T^T  (the <a a> correlations).
    Shape (M, M), real."""
    T = np.asarray(T, dtype=np.complex128)
    A, N = input_moments(np.asarray(r, dtype=np.float64))
    Nm = T @ (N[:, None] * T.conj().T)
    Sm = T @ (A[:, None] * T.T)
    d = np.real(np.diag(Nm))
    return d[:, None] * d[None, :] + np.abs(Nm) ** 2 + np.abs(Sm) ** 2
