"""Plain FP64 matrix-P estimator of grouped photon-count probabilities.

Steps, in the paper's order (main text, "Applications to GBS" and
"Photon-counting observables"):

 1. samples (alpha, beta), n = alpha . beta          -> oracle.sampler
 2. alpha' = t alpha, beta' = t* beta                 (linear network; loss as
    uncounted reservoir channels makes t sub-unitary)
 3. n'_i = alpha'_i beta'_i, and for each bin S_b of counted modes
    n_b = sum_{i in S_b} n'_i; n_S = sum_b n_b
 4. per sample, eq. c-number-variable with
        g0(n_S, m) = (1 + pi_m exp(2 (n_S - n))) / (1 + exp(-2 n)),
        pi_m = (-1)^(total count),
    summed over all patterns c with the given bin counts m_b (multinomial
    theorem: sum_{sum c_i = m_b} prod n_i^c_i / c_i! = n_b^m_b / m_b!):
        G(m_1..m_d) = g0 * prod_b n_b^m_b exp(-n_b) / m_b!
    The n used in g0 is the global photon number of the inputs (it equals the
    sum over all outputs including the reservoirs); see the readings recorded
    with the tests.
 5. average G over each sub-ensemble of N_S samples; the estimate is the mean
    of the N_R sub-ensemble means and sigma_T = sd(sub-ensemble means) /
    sqrt(N_R) (Appendix A, eq. gen_probability_density and text after it).

G is evaluated directly for each count vector m in log space (no Fourier
transform), with the two terms of g0 arranged so that no exponential of a
large |n| overflows.  The +P estimator of Appendix A (g0 = 1) is provided for
comparison.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np
from scipy.special import gammaln

from . import sampler


def propagate(T: np.ndarray, alpha: np.ndarray, beta: np.ndarray):
    """alpha'_k = T alpha_k and beta'_k = T* beta_k for every sample row k."""
    T = np.asarray(T, dtype=np.complex128)
    return alpha @ T.T, beta @ T.conj().T


def bin_occupations(ap: np.ndarray, bp: np.ndarray, bin_of_mode: np.ndarray, d: int):
    """n_b = sum_{i in S_b} alpha'_i beta'_i, shape (E, d); modes with bin -1
    are not counted."""
    occ = ap * bp
    nb = np.zeros((occ.shape[0], d), dtype=np.complex128)
    for b in range(d):
        sel = np.asarray(bin_of_mode) == b
        nb[:, b] = occ[:, sel].sum(axis=1)
    return nb


def _log_poisson_numerator(nb: np.ndarray, m: np.ndarray):
    """m log(n_b) - log(m!) per sample and count, with 0^0 = 1; shape (E, K)."""
    m = np.asarray(m, dtype=np.float64)[None, :]
    nb = nb[:, None]
    zero = nb == 0
    with np.errstate(divide="ignore", invalid="ignore"):
        lg = np.where(zero, 0.0 + 0j, np.log(np.where(zero, 1.0, nb)))
        out = m * lg - gammaln(m + 1.0)
    out = np.where(zero & (m > 0), -np.inf + 0j, out)
    return out


def _parity_exponents(n: np.ndarray, nS: np.ndarray):
    """(a1, a2) with g0 * exp(-n_S) = exp(a1) + pi_m exp(a2), both finite for
    any sign and size of the real global number n."""
    c = np.log1p(np.exp(-2.0 * np.abs(n)))
    pos = n >= 0
    a1 = np.where(pos, -nS - c, 2.0 * n - nS - c)
    a2 = np.where(pos, nS - 2.0 * n - c, nS - c)
    return a1, a2


def pattern_probability(n: np.ndarray, nb: np.ndarray, counts: list, plus_p: bool = False):
    """Per-sample G for the joint counts of d bins.

    n: (E,) real global number; nb: (E, d) bin occupations; counts: list of d
    integer arrays (the count values of each bin).  Returns complex array of
    shape (E, len(counts[0]), ..., len(counts[d-1])).  plus_p=True gives the
    +P observable (g0 = 1)."""
    E, d = nb.shape
    assert len(counts) == d
    logs = 0.0
    for b in range(d):
        Lb = _log_poisson_numerator(nb[:, b], counts[b])
        shape = [E] + [1] * d
        shape[1 + b] = len(counts[b])
        logs = logs + Lb.reshape(shape)
    nS = nb.sum(axis=1)
    ex = (Ellipsis,) + (None,) * d
    if plus_p:
        return np.exp(logs - nS[ex])
    a1, a2 = _parity_exponents(np.asarray(n, dtype=np.float64), nS)
    tot = 0
    for b in range(d):
        shape = [1] * d
        shape[b] = len(counts[b])
        tot = tot + np.asarray(counts[b]).reshape(shape)
    parity = np.where(tot % 2 == 0, 1.0, -1.0)[None]
    return np.exp(logs + a1[ex]) + parity * np.exp(logs + a2[ex])


def subensemble_stats(sums: np.ndarray, counts: np.ndarray):
    """From per-sub-ensemble sums of G (N_R, ...) and sample counts (N_R,):
    sub-ensemble means, their mean P and sigma_T = sd / sqrt(N_R)."""
    Ps = sums / counts.reshape((-1,) + (1,) * (sums.ndim - 1))
    P = Ps.mean(axis=0)
    nr = Ps.shape[0]
    if nr > 1:
        sig = Ps.real.std(axis=0, ddof=1) / np.sqrt(nr)
    else:
        sig = np.full(P.shape, np.nan)
    return Ps, P, sig


def _distributions(windows, mode, d):
    """Count arrays of each distribution and the shape of the per-sample G."""
    counts = [np.arange(lo, lo + K) for lo, K in windows]
    if mode == "joint":
        return counts, tuple(len(c) for c in counts), 1
    nterm = d + 1 if mode == "marginals_and_total" else d
    assert len(counts) == nterm
    return counts, (nterm, max(len(c) for c in counts)), nterm


def accumulate(sums, T, r, seed, ns, bin_of_mode, d, windows, g_begin, g_end, mode="joint",
               g0=0, net=0, chunk=2000, plus_p=False):
    """Adds G of samples g0 + g_begin .. g0 + g_end - 1 into the per-sub-ensemble
    sums (sample g0 + i belongs to sub-ensemble i // ns), in chunks of `chunk`
    counted from g_begin.  A run can stop after any chunk and continue from
    the saved sums and the next sample index."""
    r = np.asarray(r, dtype=np.float64)
    counts, shape, nterm = _distributions(windows, mode, d)
    assert sums.shape[1:] == shape
    done = g_begin
    while done < g_end:
        c = min(chunk, g_end - done)
        alpha, beta, n = sampler.sample(r, g0 + done, c, seed, net)
        ap, bp = propagate(T, alpha, beta)
        nb = bin_occupations(ap, bp, bin_of_mode, d)
        sub = (np.arange(done, done + c)) // ns
        if mode == "joint":
            G = pattern_probability(n, nb, counts, plus_p)
        else:
            if nterm > d:  # the total of the counted modes, S = S_1 + .. + S_d
                nb = np.concatenate([nb, nb.sum(axis=1, keepdims=True)], axis=1)
            G = np.zeros((c,) + shape, dtype=np.complex128)
            for b in range(nterm):
                Gb = pattern_probability(n, nb[:, b:b + 1], [counts[b]], plus_p)
                G[:, b, :len(counts[b])] = Gb
        np.add.at(sums, sub, G)
        done += c
    return sums


def estimate(T, r, seed, E, n_sub, bin_of_mode, d, windows, mode="joint",
             g0=0, net=0, chunk=2000, plus_p=False):
    """Full oracle pipeline over samples g0 .. g0+E-1 split into n_sub equal
    sub-ensembles (E must be a multiple of n_sub).

    mode "joint": the d-dimensional joint distribution on the windows
    [(m_lo, K)] * d (d = 1 gives the total counts of the counted modes).
    mode "marginals": d separate one-bin distributions (S = S_b alone), each
    on its own window.
    mode "marginals_and_total": those d distributions plus the total count of
    all d bins (S = the union of the bins), d + 1 windows, the total last.
    Returns dict(P=real estimate, sigma=sigma_T, P_complex, Ps=sub-ensemble
    means, counts=list of count arrays)."""
    assert E % n_sub == 0
    ns = E // n_sub
    counts, shape, _ = _distributions(windows, mode, d)
    sums = np.zeros((n_sub,) + shape, dtype=np.complex128)
    accumulate(sums, T, r, seed, ns, bin_of_mode, d, windows, 0, E, mode=mode, g0=g0, net=net,
               chunk=chunk, plus_p=plus_p)
    Ps, P, sig = subensemble_stats(sums, np.full(n_sub, ns, dtype=np.float64))
    return dict(P=P.real, P_complex=P, sigma=sig, Ps=Ps, counts=counts)


def factorial_moment_samples(n: np.ndarray, nS: np.ndarray, kmax: int):
    """Per-sample normally ordered moments of the counted photon number,
    n_S^k tr[T^{p_k} Omega] with T_0 = tanh n for odd k and 1 for even k
    (eq. moment with the M = 2 weights given after eq. Lambda-identities).
    Shape (E, kmax)."""
    out = np.empty((nS.shape[0], kmax), dtype=np.complex128)
    th = np.tanh(n)
    for k in range(1, kmax + 1):
        out[:, k - 1] = nS ** k * (th if k % 2 else 1.0)
    return out


def pair_correlations(T, r, seed, E, n_sub, g0=0, net=0, chunk=2000):
    """Normally ordered pair moments <:n_i n_j:> of single output modes from
    the same ensemble (main text, eq. moment, with every output mode taken as
    its own group): the mixed second derivative of the per-sample generating
    function at z = 1 is n'_i n'_j, with the even-order weight 1 for both the
    parity-projected and the +P estimator.  Each sub-ensemble sums
    n'_i n'_j over its samples (a plain product of the occupation matrix with
    itself); then the sub-ensemble statistics of Appendix A.

    Samples g0 .. g0+E-1, n_sub equal sub-ensembles.  Returns dict(G2 = mean
    (M, M) complex, sigma = sigma_T of the real part, Ps = sub-ensemble means,
    abs_sums = per sub-ensemble sums of |n'_i||n'_j| (the scale of the
    rounding error of any evaluation of the sums))."""
    assert E % n_sub == 0
    ns = E // n_sub
    r = np.asarray(r, dtype=np.float64)
    M = np.asarray(T).shape[0]
    sums = np.zeros((n_sub, M, M), dtype=np.complex128)
    abs_sums = np.zeros((n_sub, M, M))
    done = 0
    while done < E:
        c = min(chunk, E - done)
        alpha, beta, _ = sampler.sample(r, g0 + done, c, seed, net)
        ap, bp = propagate(T, alpha, beta)
        occ = ap * bp
        sub = (np.arange(done, done + c)) // ns
        for s in np.unique(sub):
            x = occ[sub == s]
            sums[s] += x.T @ x
            a = np.abs(x)
            abs_sums[s] += a.T @ a
        done += c
    Ps, P, sig = subensemble_stats(sums, np.full(n_sub, ns, dtype=np.float64))
    return dict(G2=P, sigma=sig, Ps=Ps, abs_sums=abs_sums)
