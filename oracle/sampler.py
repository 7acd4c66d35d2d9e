"""Phase-space samples of multimode squeezed vacuum, in FP64 (test oracle).

Paper, main text "Applications to GBS": a squeezed input is an integral over
real coherent amplitudes with the even weight xi(alpha) = prod_j C_j
exp(-alpha_j^2 coth(r_j)/2), C_j = (2 pi sinh r_j)^(-1/2).  With the
unnormalised +P kernel ||alpha><beta*|| exp(-alpha.beta) the density matrix
is reproduced by the real-valued distribution

    P(alpha, beta)  proportional to  xi(alpha) xi(beta) exp(alpha . beta),

and the parity-projected matrix-P distribution (Omega_00 = 1, even in n) is
sampled the same way ("the +P sampling procedure ... can still be used").
Per mode this is a zero-mean real Gaussian pair with
    Var(alpha_j) = Var(beta_j) = A_j = sinh r_j cosh r_j,
    Cov(alpha_j, beta_j)      = N_j = sinh^2 r_j,
the inverse of the quadratic form [[coth r, -1], [-1, coth r]].  One exact
way to draw it from two independent normals w1, w2:
    alpha_j = sqrt(sinh(r_j)/2) (e^{r_j/2} w1 + e^{-r_j/2} w2)
    beta_j  = sqrt(sinh(r_j)/2) (e^{r_j/2} w1 - e^{-r_j/2} w2)
(r_j = 0 gives alpha = beta = 0, the vacuum).  The global photon number of the
sample is n = sum_j alpha_j beta_j (defined before eq. canonical-expansion).

Noise: for global sample index g, mode pair p = j // 2, network id `net` and
seed `seed`, one Philox4x64-10 call with counter (g, p, net, 0) and key
(seed, 0) gives four 64-bit words x0..x3.  Words (x0, x1) feed mode 2p and
(x2, x3) mode 2p + 1 through Box-Muller:
    u = ((x_even >> 11) + 1) * 2^-53   in (0, 1]
    v = (x_odd >> 11) * 2^-53          in [0, 1)
    w1 = sqrt(-2 ln u) cos(2 pi v),  w2 = sqrt(-2 ln u) sin(2 pi v).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import math

import numpy as np

from .philox import philox4x64_10

TWO_M53 = 2.0 ** -53


def box_muller(x_even: np.ndarray, x_odd: np.ndarray):
    u = ((x_even >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * TWO_M53
    v = (x_odd >> np.uint64(11)).astype(np.float64) * TWO_M53
    rho = np.sqrt(-2.0 * np.log(u))
    ang = 2.0 * math.pi * v
    return rho * np.cos(ang), rho * np.sin(ang)


def normals(M: int, g0: int, E: int, seed: int, net: int = 0):
    """w1, w2 of shape (E, M) for global samples g0 .. g0+E-1."""
    P = (M + 1) // 2
    g = np.arange(g0, g0 + E, dtype=np.uint64)[:, None]
    p = np.arange(P, dtype=np.uint64)[None, :]
    x0, x1, x2, x3 = philox4x64_10(g, p, np.uint64(net), np.uint64(0),
                                   np.uint64(seed), np.uint64(0))
    wa1, wa2 = box_muller(x0, x1)      # mode 2p
    wb1, wb2 = box_muller(x2, x3)      # mode 2p + 1
    w1 = np.empty((E, 2 * P))
    w2 = np.empty((E, 2 * P))
    w1[:, 0::2], w1[:, 1::2] = wa1, wb1
    w2[:, 0::2], w2[:, 1::2] = wa2, wb2
    return w1[:, :M], w2[:, :M]


def amplitudes(r: np.ndarray, w1: np.ndarray, w2: np.ndarray):
    """alpha, beta (E, M) from the normals; see the module docstring."""
    r = np.asarray(r, dtype=np.float64)
    s = np.sqrt(np.sinh(r) / 2.0)
    cp = s * np.exp(r / 2.0)
    cm = s * np.exp(-r / 2.0)
    alpha = cp * w1 + cm * w2
    beta = cp * w1 - cm * w2
    return alpha, beta


def sample(r: np.ndarray, g0: int, E: int, seed: int, net: int = 0):
    """alpha, beta (E, M) and the global photon number n (E,) of samples
    g0 .. g0+E-1."""
    r = np.asarray(r, dtype=np.float64)
    w1, w2 = normals(r.size, g0, E, seed, net)
    alpha, beta = amplitudes(r, w1, w2)
    n = np.sum(alpha * beta, axis=1)
    return alpha, beta, n


def input_moments(r: np.ndarray):
    """A_j = sinh r cosh r and N_j = sinh^2 r of the sampled Gaussian."""
    r = np.asarray(r, dtype=np.float64)
    return np.sinh(r) * np.cosh(r), np.sinh(r) ** 2
