"""Seeded synthetic inputs for the matrix-P Gaussian-boson-sampling workloads.

This module is shared by the tests, the benchmark and the oracle, and holds
none of the phase-space method's arithmetic.  It draws the things the paper's
experiments take as given: Haar-random linear networks scaled by a uniform
amplitude transmission (main text, "Applications to GBS"; loss as uncounted
reservoir channels, "Computational results and losses"), squeezing profiles
(uniform, uniform-random, or 0.89 + 0.1 w_i as in Appendix B), contiguous bin
partitions (eq. General_GCP), and count windows sized from the first two
moments of the total photon number.

The amplitude noise the method itself draws is NOT generated here: each side
(oracle and HIP library) implements the counter-based Philox4x64-10 generator
from its published definition.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 250312749

# Independent sub-streams of the input generator (the second Philox key word).
STREAM_T = 0x54          # Haar network
STREAM_R = 0x52          # squeezing profiles
STREAM_NET = 0x4E        # per-network parameters of the batched workload


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[int(seed) & (2**64 - 1), int(stream)]))


def haar_unitary(M: int, seed: int) -> np.ndarray:
    """Haar-random M x M unitary: QR of a complex Gaussian matrix with
    N(0, 1/2) real and imaginary parts, phase-fixed as Q * diag(R_ii/|R_ii|)."""
    rng = _rng(seed, STREAM_T)
    Z = (rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))) * math.sqrt(0.5)
    Q, R = np.linalg.qr(Z)
    d = np.diag(R)
    return Q * (d / np.abs(d))[None, :]


def transmission(M: int, t: float, seed: int) -> np.ndarray:
    """Lossy transmission matrix T = t * U_H (complex128, C order, T[i, j] maps
    input mode j to output mode i)."""
    return t * haar_unitary(M, seed)


def squeezing_uniform(M: int, r: float) -> np.ndarray:
    return np.full(M, float(r))


def squeezing_random_uniform(M: int, lo: float, hi: float, seed: int) -> np.ndarray:
    return _rng(seed, STREAM_R).uniform(lo, hi, size=M)


def squeezing_gaussian(M: int, mean: float, sd: float, seed: int) -> np.ndarray:
    """r_i = mean + sd * w_i with w_i ~ N(0, 1), clipped at 0 (Appendix B uses
    mean 0.89, sd 0.1)."""
    return np.clip(mean + sd * _rng(seed, STREAM_R).standard_normal(M), 0.0, None)


def contiguous_bins(M: int, d: int) -> np.ndarray:
    """bin_of_mode for d equal contiguous mode blocks (the last absorbs the
    remainder)."""
    size = M // d
    b = np.minimum(np.arange(M) // max(size, 1), d - 1)
    return b.astype(np.int32)


def all_modes_bin(M: int) -> np.ndarray:
    return np.zeros(M, dtype=np.int32)


def count_window(mean: float, sd: float, nsig: float = 9.0, align: int = 64) -> tuple[int, int]:
    """Window [m_lo, m_lo + K) covering mean +- nsig * sd (clipped at 0), with K
    rounded up to a multiple of `align`.  Sizing only: the moments passed in are
    rough (see uniform_loss_moments)."""
    half = nsig * sd + 4.0
    lo = max(0, int(math.floor(mean - half)))
    hi = int(math.ceil(mean + half)) + 1
    K = -(-(hi - lo) // align) * align
    return lo, K


def uniform_loss_moments(r: np.ndarray, t: float, frac: float = 1.0) -> tuple[float, float]:
    """Rough mean and standard deviation of the photon count in a bin holding a
    fraction `frac` of the outputs of T = t*U, used only to size windows.
    Exact for frac = 1; for a sub-block of a Haar network it ignores the
    off-diagonal network terms, which window margins absorb."""
    N = np.sinh(r) ** 2
    mean = frac * t * t * N.sum()
    var = mean + (frac * t * t) ** 2 * (N * (2 * N + 1)).sum()
    return float(mean), float(math.sqrt(var))


@dataclasses.dataclass
class Workload:
    """One synthetic configuration of the hot path."""
    name: str
    M: int
    t: float
    r: np.ndarray
    T: np.ndarray | None
    E: int                 # total samples
    n_sub: int             # sub-ensembles N_R
    seed: int              # amplitude-noise seed (Philox key word 0)
    bins: np.ndarray       # bin_of_mode, -1 = uncounted
    d: int
    windows: list          # [(m_lo, K)] per bin (or one for the total)
    chunk: int             # samples per chunk

    @property
    def samples_per_sub(self) -> int:
        return self.E // self.n_sub


def workload_small(seed_offset: int = 0, E: int = 10_000, n_sub: int = 10,
                   with_T: bool = True) -> Workload:
    """M = 16 modes, Haar x t = 0.5, r = 1, total counts m = 0..64 (K = 128)."""
    M, t = 16, 0.5
    seed = SEED_BASE + 0 + seed_offset
    T = transmission(M, t, seed) if with_T else None
    return Workload("M16_t0.5_r1", M, t, squeezing_uniform(M, 1.0), T, E, n_sub,
                    seed, all_modes_bin(M), 1, [(0, 128)], E)


def workload_m1000(E: int = 1_200_000, with_T: bool = True) -> Workload:
    """M = 1000, Haar x t = 0.9, r = 1, total counts, E = 1.2e6 in 1e5 chunks,
    N_S = 1e4 per sub-ensemble."""
    M, t = 1000, 0.9
    seed = SEED_BASE + 1
    r = squeezing_uniform(M, 1.0)
    mean, sd = uniform_loss_moments(r, t)
    T = transmission(M, t, seed) if with_T else None
    return Workload("M1000_t0.9_r1", M, t, r, T, E, max(1, E // 10_000), seed,
                    all_modes_bin(M), 1, [count_window(mean, sd)], 100_000)


def workload_m8000(E: int = 589_824, chunk: int = 65_536, with_T: bool = True) -> Workload:
    """M = 8000, Haar x t = 0.95, r = 1, total counts (window K = 4096)."""
    M, t = 8000, 0.95
    seed = SEED_BASE + 5
    r = squeezing_uniform(M, 1.0)
    mean, sd = uniform_loss_moments(r, t)
    T = transmission(M, t, seed) if with_T else None
    n_sub = max(1, E // 8192)
    return Workload("M8000_t0.95_r1", M, t, r, T, E, n_sub, seed, all_modes_bin(M), 1,
                    [count_window(mean, sd)], chunk)


def workload_m4000(E: int = 983_040, chunk: int = 65_536, ns: int = 8192,
                   with_T: bool = True) -> Workload:
    """M = 4000, Haar x t = 0.95, r_j ~ U[0.5, 1.5], four equal mode blocks:
    their four marginal distributions and the total (windows in that order;
    the block windows take 1.3x the independent-mode sd as margin for the
    network correlations inside a block)."""
    M, t = 4000, 0.95
    seed = SEED_BASE + 2
    r = squeezing_random_uniform(M, 0.5, 1.5, seed)
    T = transmission(M, t, seed) if with_T else None
    bins = contiguous_bins(M, 4)
    N = np.sinh(r) ** 2
    wins = []
    for b in range(4):
        Nb = N[bins == b]
        mb = t * t * Nb.sum()
        sb = math.sqrt(mb + (t * t) ** 2 * (Nb * (2 * Nb + 1)).sum())
        wins.append(count_window(mb, sb * 1.3))
    wins.append(count_window(*uniform_loss_moments(r, t)))
    return Workload("M4000_t0.95_rU[0.5,1.5]", M, t, r, T, E, E // ns, seed, bins, 4, wins, chunk)


BATCHED_SIZES = [500] * 4 + [1000] * 4 + [2000] * 4 + [4000] * 4


def batched_networks(E: int = 200_000, n_sub: int = 20, indices=None) -> list[dict]:
    """The sixteen networks of the batched workload (4 each of M = 500, 1000,
    2000, 4000; t ~ U[0.85, 0.99]; r = 1; total counts), as dicts with keys
    T, r, seed, net, E, n_sub, window, t.  `indices` selects networks (their
    parameters do not depend on the selection)."""
    rng = np.random.default_rng(SEED_BASE + 7)
    ts = [float(rng.uniform(0.85, 0.99)) for _ in BATCHED_SIZES]
    out = []
    for i, M in enumerate(BATCHED_SIZES):
        if indices is not None and i not in indices:
            continue
        t = ts[i]
        r = np.ones(M)
        out.append(dict(T=transmission(M, t, SEED_BASE + 100 + i), r=r, seed=SEED_BASE + 7, net=i,
                        E=E, n_sub=n_sub, window=count_window(*uniform_loss_moments(r, t)), t=t))
    return out
