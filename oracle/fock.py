"""Brute-force Fock-space count probabilities for M <= 4 modes (FP64).

The squeezed input of the paper (real coherent-state integral with weight
xi(alpha)) is, per mode, (cosh r)^(-1/2) exp(tanh(r) a^dag^2 / 2)|0>, obtained
by doing the Gaussian integral over alpha.  A linear network with unitary V
maps a^dag_j to sum_i V_ij a^dag_i, so the output state is

    (prod_j cosh r_j)^(-1/2) exp(x^T B x / 2)|0>,   B = V D V^T,  x = a^dag,

with D = diag(tanh r).  Loss is modelled as uncounted reservoir channels
(main text, "Computational results and losses"): a sub-unitary T is dilated to
the unitary [[T, (I - T T^dag)^(1/2)], [(I - T^dag T)^(1/2), -T^dag]], of which
only the columns fed by the squeezed inputs enter B.  The exponential is
expanded as a polynomial in the creation operators, truncated at total degree
n_max (exact for every Fock state with at most n_max photons); the amplitude of
|c> is coefficient * sqrt(prod c_i!).  Reservoir counts are summed out.

The missing probability is the chance that the input holds more than n_max
photons (the network conserves the total), returned alongside.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import math

import numpy as np


def _sqrtm_psd(H: np.ndarray) -> np.ndarray:
    w, U = np.linalg.eigh(H)
    return (U * np.sqrt(np.clip(w, 0.0, None))) @ U.conj().T


def input_photon_tail(r: np.ndarray, n_max: int) -> float:
    """P(total input photons > n_max) for product squeezed vacua."""
    dist = np.zeros(n_max + 1)
    dist[0] = 1.0
    for rj in np.asarray(r, dtype=np.float64):
        th = math.tanh(rj)
        single = np.zeros(n_max + 1)
        for k in range(n_max // 2 + 1):
            # |<2k|r>|^2 = tanh^2k (2k)! / (2^k k!)^2 / cosh r
            single[2 * k] = math.exp(2 * k * math.log(th) if th > 0 else (0.0 if k == 0 else -np.inf)) \
                * math.exp(math.lgamma(2 * k + 1) - 2 * (k * math.log(2) + math.lgamma(k + 1))) / math.cosh(rj)
        dist = np.convolve(dist, single)[: n_max + 1]
    return float(max(0.0, 1.0 - dist.sum()))


def output_pattern_probabilities(T: np.ndarray, r: np.ndarray, n_max: int):
    """Probabilities of the system output patterns c (array of shape
    (n_max + 1,) * M, reservoirs summed out) and the truncation bound."""
    T = np.asarray(T, dtype=np.complex128)
    r = np.asarray(r, dtype=np.float64)
    M = T.shape[0]
    lossless = np.allclose(T.conj().T @ T, np.eye(M), atol=1e-13)
    if lossless:
        V1 = T
    else:
        V1 = np.vstack([T, _sqrtm_psd(np.eye(M) - T.conj().T @ T)])
    nv = V1.shape[0]
    B = V1 @ np.diag(np.tanh(r)) @ V1.T
    D = n_max - (n_max % 2)
    shape = (D + 1,) * nv
    total = np.zeros(shape, dtype=np.complex128)
    term = np.zeros(shape, dtype=np.complex128)
    term[(0,) * nv] = 1.0
    total += term
    full = slice(None)
    for n in range(1, D // 2 + 1):
        new = np.zeros(shape, dtype=np.complex128)
        for i in range(nv):
            for j in range(i, nv):
                if i == j:
                    coef = 0.5 * B[i, i]
                    dst = [full] * nv
                    src = [full] * nv
                    dst[i] = slice(2, None)
                    src[i] = slice(0, -2)
                else:
                    coef = B[i, j]
                    dst = [full] * nv
                    src = [full] * nv
                    dst[i] = dst[j] = slice(1, None)
                    src[i] = src[j] = slice(0, -1)
                new[tuple(dst)] += coef * term[tuple(src)]
        term = new / n
        total += term
    fact = np.array([math.lgamma(c + 1) for c in range(D + 1)])
    logf = 0.0
    for ax in range(nv):
        sh = [1] * nv
        sh[ax] = D + 1
        logf = logf + fact.reshape(sh)
    norm = float(np.prod(1.0 / np.sqrt(np.cosh(r))))
    amp = total * np.exp(0.5 * logf) * norm
    prob = np.abs(amp) ** 2
    if nv > M:
        prob = prob.sum(axis=tuple(range(M, nv)))
    return prob, input_photon_tail(r, D)


def binned_probabilities(T, r, bin_of_mode, d: int, n_max: int):
    """Joint distribution of the d bin counts, shape (n_max + 1,) * d, plus
    the truncation bound.  Modes with bin -1 are summed out."""
    prob, tail = output_pattern_probabilities(T, r, n_max)
    M = prob.ndim
    D = prob.shape[0] - 1
    idx = np.indices(prob.shape)
    out = np.zeros((D + 1,) * d)
    sums = []
    for b in range(d):
        sel = [i for i in range(M) if bin_of_mode[i] == b]
        sums.append(sum(idx[i] for i in sel) if sel else np.zeros(prob.shape, dtype=int))
    keep = np.ones(prob.shape, dtype=bool)
    for s in sums:
        keep &= s <= D
    flat_idx = tuple(s[keep] for s in sums)
    np.add.at(out, flat_idx, prob[keep])
    return out, tail
