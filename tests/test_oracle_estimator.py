"""Pins of the oracle's matrix-P estimator (CPU only): per-sample identities,
printed values of the paper, and statistical agreement with the exact laws."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import estimator, exact, sampler

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_g0_m4_worked_value():
    """Appendix A: for lossless total counts the matrix-P projector G_0(4)
    lies in (0, 0.4) with its largest values near 0.39."""
    g = json.load(open(os.path.join(GOLDEN, "g0_m4_density.json")))
    n = np.linspace(-25, 25, 200_001)
    n = n[n != 0]
    G = estimator.pattern_probability(n, n[:, None].astype(complex), [np.array([g["m"]])])[:, 0]
    assert np.all(np.abs(G.imag) <= 1e-14 * np.abs(G))
    lo, hi = g["range"]
    assert G.real.min() > lo and G.real.max() < hi
    assert abs(G.real.max() - g["peak_value_approx"]) < g["peak_tolerance"]
    # closed form given with the projector: g0(2m) = n^2m / ((2m)! cosh n)
    np.testing.assert_allclose(G.real, n ** 4 / (24 * np.cosh(n)), rtol=1e-12)


def test_lossless_odd_counts_vanish_per_sample():
    """g0(2m+1) = 0 when every channel is counted (n_S = n)."""
    rng = np.random.default_rng(0)
    n = rng.normal(3, 4, size=500)
    G = estimator.pattern_probability(n, n[:, None].astype(complex), [np.arange(40)])
    assert np.abs(G[:, 1::2]).max() < 1e-300 or np.abs(G[:, 1::2]).max() == 0.0
    assert np.abs(G[:, 0::2]).max() > 0


def test_generating_function_identity_per_sample():
    """sum_m G(m) z^m = cosh(n + n_S (z - 1)) / cosh(n) for each sample (the
    per-sample characteristic function of eq. c-number-variable)."""
    rng = np.random.default_rng(1)
    E = 64
    n = rng.normal(4, 3, size=E)
    nS = (0.6 * n + rng.normal(0, 0.7, E)) + 1j * rng.normal(0, 0.7, E)
    m = np.arange(160)
    G = estimator.pattern_probability(n, nS[:, None], [m])
    for z in (1.0, -1.0, np.exp(0.7j), 0.3 - 0.2j):
        lhs = (G * z ** m[None, :]).sum(1)
        rhs = np.cosh(n + nS * (z - 1)) / np.cosh(n)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-11, atol=1e-13)


def test_plus_p_generating_function():
    rng = np.random.default_rng(2)
    n = rng.normal(4, 1, 8)
    nS = n * 0.7 + 0.2j
    m = np.arange(120)
    G = estimator.pattern_probability(n, nS[:, None], [m], plus_p=True)
    z = np.exp(0.4j)
    np.testing.assert_allclose((G * z ** m).sum(1), np.exp(nS * (z - 1)), rtol=1e-12)


def test_joint_sums_to_marginal_and_total():
    rng = np.random.default_rng(3)
    E = 40
    n = rng.normal(5, 2, E)
    nb = np.stack([0.3 * n + 0.1j * rng.normal(size=E), 0.4 * n - 0.2j * rng.normal(size=E)], 1)
    m = np.arange(60)
    J = estimator.pattern_probability(n, nb, [m, m])
    M1 = estimator.pattern_probability(n, nb[:, :1], [m])
    np.testing.assert_allclose(J.sum(2), M1, rtol=1e-11, atol=1e-15)
    tot = estimator.pattern_probability(n, nb.sum(1, keepdims=True), [m])
    diag = np.stack([sum(J[:, a, k - a] for a in range(k + 1)) for k in range(60)], 1)
    np.testing.assert_allclose(diag, tot, rtol=1e-11, atol=1e-15)


def test_uniform_loss_invariant():
    """For T = t U every sample has n_S = t^2 n (unitary invariance of
    alpha . beta)."""
    r = np.linspace(0.3, 1.2, 12)
    T = 0.8 * synth.haar_unitary(12, 4)
    a, b, n = sampler.sample(r, 0, 200, seed=6)
    ap, bp = estimator.propagate(T, a, b)
    nS = estimator.bin_occupations(ap, bp, np.zeros(12, int), 1)[:, 0]
    np.testing.assert_allclose(nS, 0.64 * n, rtol=1e-12, atol=1e-12)


def _z(res, ref, rel_floor=1e-3):
    P, s = res["P"], res["sigma"]
    bulk = ref > rel_floor * ref.max()
    return np.abs((P - ref)[bulk] / s[bulk])


def test_small_workload_vs_determinant_law():
    """M = 16, Haar x 0.5, r = 1, E = 1e4: bulk bins within 5 sigma_T."""
    w = synth.workload_small()
    res = estimator.estimate(w.T, w.r, w.seed, w.E, w.n_sub, w.bins, 1, w.windows)
    ref = exact.gaussian_total(w.T, w.r, np.ones(16), 128)
    assert _z(res, ref).max() < 5
    assert abs(res["P"].sum() - 1) < 1e-12


def test_lossless_vs_negative_binomial():
    U = synth.haar_unitary(8, 3)
    res = estimator.estimate(U, np.full(8, 0.5), 99, 40_000, 20, np.zeros(8, int), 1, [(0, 64)])
    ref = exact.lossless_uniform_total(8, 0.5, np.arange(64))
    assert _z(res, ref).max() < 5
    assert np.abs(res["P_complex"][1::2]).max() < 1e-14


def _lossy_two_mode():
    r = np.array([0.4, 0.6])
    T = 0.8 * synth.haar_unitary(2, 7)
    return T, r


def test_global_n_reading_against_exact():
    """Lossy two-mode network, many samples: the global-n estimator agrees
    with the exact joint law; replacing the global n by the counted output
    photon number (a planted mistake) is rejected."""
    T, r = _lossy_two_mode()
    E, nsub = 200_000, 40
    res = estimator.estimate(T, r, 31, E, nsub, np.array([0, 1]), 2, [(0, 16), (0, 16)],
                             chunk=20_000)
    ref = exact.gaussian_joint2(T, r, np.array([0, 1]), 64, 64)[:16, :16]
    assert _z(res, ref).max() < 5
    # planted mistake: n := Re(n_S), the counted output number
    a, b, n = sampler.sample(r, 0, E, 31)
    ap, bp = estimator.propagate(T, a, b)
    nb = estimator.bin_occupations(ap, bp, np.array([0, 1]), 2)
    wrong = estimator.pattern_probability(nb.sum(1).real, nb, [np.arange(16)] * 2).real
    Ps = wrong.reshape(nsub, E // nsub, 16, 16).mean(1)
    z = np.abs(Ps.mean(0) - ref) / (Ps.std(0, ddof=1) / np.sqrt(nsub) + 1e-30)
    assert z.max() > 20


def test_two_bin_joint_vs_determinant_law():
    r = np.array([0.5, 0.8, 0.6, 0.7])
    T = 0.9 * synth.haar_unitary(4, 21)
    bins = np.array([0, 0, 1, 1])
    res = estimator.estimate(T, r, 5, 100_000, 25, bins, 2, [(0, 16), (0, 16)], chunk=20_000)
    ref = exact.gaussian_joint2(T, r, bins, 64, 64)[:16, :16]
    assert _z(res, ref).max() < 5


def test_marginal_mode_matches_single_bin_runs():
    r = np.array([0.5, 0.8, 0.6, 0.7, 1.0, 0.9])
    T = 0.9 * synth.haar_unitary(6, 2)
    bins = np.array([0, 0, 1, 1, 2, 2])
    res = estimator.estimate(T, r, 5, 2000, 4, bins, 3, [(0, 24)] * 3, mode="marginals")
    for b in range(3):
        only = np.where(bins == b, 0, -1)
        one = estimator.estimate(T, r, 5, 2000, 4, only, 1, [(0, 24)])
        np.testing.assert_allclose(res["P_complex"][b], one["P_complex"], rtol=1e-12, atol=1e-15)


def test_marginals_and_total_mode():
    """The d marginals plus the total: the first d distributions equal the
    marginal mode's, the last equals a one-bin run over the union of the bins
    (modes outside every bin stay uncounted), and that total agrees with the
    exact Gaussian law of the counted modes."""
    r = np.array([0.5, 0.8, 0.6, 0.7, 1.0, 0.9])
    T = 0.9 * synth.haar_unitary(6, 2)
    bins = np.array([0, 0, 1, 1, 2, -1])
    wins = [(0, 24)] * 3 + [(0, 40)]
    res = estimator.estimate(T, r, 5, 2000, 4, bins, 3, wins, mode="marginals_and_total")
    marg = estimator.estimate(T, r, 5, 2000, 4, bins, 3, wins[:3], mode="marginals")
    np.testing.assert_allclose(res["P_complex"][:3, :24], marg["P_complex"], rtol=1e-12, atol=1e-15)
    union = np.where(bins >= 0, 0, -1)
    tot = estimator.estimate(T, r, 5, 2000, 4, union, 1, [(0, 40)])
    np.testing.assert_allclose(res["P_complex"][3], tot["P_complex"], rtol=1e-12, atol=1e-15)
    big = estimator.estimate(T, r, 6, 200_000, 40, bins, 3, wins, mode="marginals_and_total",
                             chunk=20_000)
    ref = exact.gaussian_total(T, r, (bins >= 0).astype(int), 128)[:40]
    z = np.abs(big["P"][3] - ref) / np.maximum(big["sigma"][3], 1e-300)
    assert z[ref > 1e-4].max() < 5


def test_factorial_moments_vs_closed_form():
    """eq. moment with T_0 = tanh n: E[n_S] and E[n_S (n_S - 1)] ... reduce
    to the closed-form mean and variance."""
    r = np.linspace(0.4, 1.1, 6)
    T = 0.85 * synth.haar_unitary(6, 9)
    counted = np.array([1, 1, 1, 0, 0, 1])
    bins = np.where(counted == 1, 0, -1)
    a, b, n = sampler.sample(r, 0, 400_000, 13)
    ap, bp = estimator.propagate(T, a, b)
    nS = estimator.bin_occupations(ap, bp, bins, 1)[:, 0]
    f = estimator.factorial_moment_samples(n, nS, 2)
    mean, var = exact.count_moments(T, r, counted)
    f1, f2 = f[:, 0].real, f[:, 1].real
    assert abs(f1.mean() - mean) < 5 * f1.std() / np.sqrt(len(f1))
    assert abs((f2.mean() + mean - mean ** 2) - var) < 5 * f2.std() / np.sqrt(len(f2)) + 1e-9


@pytest.mark.parametrize("plus_p", [False, True])
def test_factorial_moments_orders_3_4_vs_exact_law(plus_p):
    """Normally ordered moments <:n^k:> are the factorial moments of the
    count, sum_m m!/(m-k)! P(m).  For T = t U the exact P(m) of the total
    count follows from the uniform-loss generating function; the oracle's
    per-sample moments (matrix-P weights tanh n on odd orders, or none for
    +P) must average to it for k = 1..4."""
    from scipy.special import gammaln
    rng = np.random.default_rng(21)
    M, t = 6, 0.9
    r = rng.uniform(0.3, 0.8, M)
    T = t * synth.haar_unitary(M, 31)
    a, b, n = sampler.sample(r, 0, 400_000, 17)
    ap, bp = estimator.propagate(T, a, b)
    nS = estimator.bin_occupations(ap, bp, np.zeros(M, int), 1)[:, 0]
    if plus_p:
        f = np.stack([nS ** k for k in range(1, 5)], axis=1)
    else:
        f = estimator.factorial_moment_samples(n, nS, 4)
    P = exact.uniform_loss_total(r, t, 256)
    m = np.arange(256)
    for k in range(1, 5):
        ff = np.exp(gammaln(m + 1) - gammaln(np.maximum(m - k + 1, 1)))
        ff[m < k] = 0.0
        want = float((ff * P).sum())
        x = f[:, k - 1].real
        se = x.std() / np.sqrt(len(x))
        assert abs(x.mean() - want) < 5 * se, (k, x.mean(), want, se)
        xi = f[:, k - 1].imag  # complex per sample under loss; the mean is real
        assert abs(xi.mean()) < 5 * xi.std() / np.sqrt(len(xi)) + 1e-12


@pytest.mark.parametrize("plus_p", [False, True])
def test_factorial_moments_are_derivatives_of_the_per_sample_law(plus_p):
    """Per sample, sum_m m!/(m-k)! G(m) over the count-space observable is the
    k-th derivative at z = 1 of its generating function, cosh(n + n_S (z-1)) /
    cosh n (matrix-P) or e^{n_S (z-1)} (+P): n_S^k tanh(n)^(k odd) or n_S^k.
    Two independent code paths (direct G(m) vs the moment formula) must agree
    exactly, which fixes where the tanh weight goes."""
    from scipy.special import gammaln
    rng = np.random.default_rng(5)
    E = 200
    n = rng.normal(1.0, 2.0, E)
    nS = (rng.normal(1.5, 1.5, E) + 1j * rng.normal(0, 0.5, E))
    m = np.arange(160)
    G = estimator.pattern_probability(n, nS[:, None], [m], plus_p=plus_p)
    if plus_p:
        f = np.stack([nS ** k for k in range(1, 6)], axis=1)
    else:
        f = estimator.factorial_moment_samples(n, nS, 5)
    for k in range(1, 6):
        ff = np.exp(gammaln(m + 1) - gammaln(np.maximum(m - k + 1, 1)))
        ff[m < k] = 0.0
        direct = (G * ff[None, :]).sum(axis=1)
        np.testing.assert_allclose(direct, f[:, k - 1], rtol=1e-9, atol=1e-12)


def _lossy_network(M, seed, t):
    """Haar unitary with mode-dependent input loss: sub-unitary, non-normal."""
    return synth.haar_unitary(M, seed) * np.asarray(t)[None, :]


def test_pair_correlations_are_count_space_mixed_moments():
    """Per sub-ensemble, the pair estimator equals the mixed moments of the
    count-space estimator with single-mode bins: sum m_1 m_2 G(m_1, m_2) for
    two modes and sum m (m - 1) G(m) for one (eq. moment via the per-sample
    law of eq. c-number-variable; the parity weights cancel exactly)."""
    M, E, n_sub, K = 5, 400, 4, 40
    r = np.array([0.3, 0.5, 0.45, 0.6, 0.35])
    T = _lossy_network(M, 21, [0.9, 0.7, 1.0, 0.8, 0.95])
    pc = estimator.pair_correlations(T, r, 5, E, n_sub, chunk=150)
    m = np.arange(K, dtype=float)
    for i in range(M):
        for j in range(i, M):
            bins = np.full(M, -1)
            if i == j:
                bins[i] = 0
                e = estimator.estimate(T, r, 5, E, n_sub, bins, 1, [(0, K)], chunk=150)
                ref = (e["Ps"] * (m * (m - 1))[None, :]).sum(axis=1)
            else:
                bins[i], bins[j] = 0, 1
                e = estimator.estimate(T, r, 5, E, n_sub, bins, 2, [(0, K), (0, K)], chunk=150)
                ref = (e["Ps"] * (m[:, None] * m[None, :])[None]).sum(axis=(1, 2))
            np.testing.assert_allclose(pc["Ps"][:, i, j], ref, rtol=1e-9, atol=1e-13)
            np.testing.assert_allclose(pc["Ps"][:, j, i], ref, rtol=1e-9, atol=1e-13)


def test_pair_correlations_vs_gaussian_closed_form():
    """Statistical agreement with Isserlis' closed form on a lossy,
    non-uniformly squeezed network; the closed form of the transposed network
    is rejected."""
    r = np.array([0.5, 0.8, 0.3, 0.6])
    T = _lossy_network(4, 31, [0.9, 0.6, 1.0, 0.75])
    pc = estimator.pair_correlations(T, r, 12, 200000, 40, chunk=20000)
    z = (pc["G2"].real - exact.pair_moments(T, r)) / pc["sigma"]
    assert np.abs(z).max() < 4.5, z
    z_wrong = (pc["G2"].real - exact.pair_moments(T.T, r)) / pc["sigma"]
    assert np.abs(z_wrong).max() > 10


def test_three_and_four_bin_joints_sum_to_lower_joints_per_sample():
    """Summing the joint law of d bins over the last bin's counts gives the
    joint law of the first d - 1 bins with the last bin's modes uncounted
    (eq. General_GCP; the parity weight of the dropped bin cancels), per
    sample, for d = 3 and d = 4."""
    rng = np.random.default_rng(5)
    E = 24
    n = rng.normal(5, 2, E)
    nb = np.stack([0.25 * n + 0.1j * rng.normal(size=E), 0.3 * n - 0.2j * rng.normal(size=E),
                   0.2 * n + 0.15j * rng.normal(size=E), 0.1 * n - 0.05j * rng.normal(size=E)], 1)
    m = np.arange(48)
    J2 = estimator.pattern_probability(n, nb[:, :2], [m, m])
    J3 = estimator.pattern_probability(n, nb[:, :3], [m, m, m])
    np.testing.assert_allclose(J3.sum(3), J2, rtol=1e-11, atol=1e-15)
    m4 = np.arange(24)
    J4 = estimator.pattern_probability(n * 0.5, nb * 0.5, [m4] * 4)
    J3h = estimator.pattern_probability(n * 0.5, nb[:, :3] * 0.5, [m4] * 3)
    np.testing.assert_allclose(J4.sum(4), J3h, rtol=1e-11, atol=1e-15)


def test_three_bin_joint_vs_fock():
    """Three single-mode bins of a lossy, non-normal 3-mode network: the
    estimator's joint law within 5 sigma_T of brute-force Fock probabilities
    in every bulk cell (P above 1e-3 of the peak: in the far tail the
    per-sample values are heavy-tailed and sigma_T from 30 sub-ensembles
    understates the spread), zero-mean normalised errors, and the total
    probability of the window."""
    from oracle import fock
    r = np.array([0.3, 0.45, 0.35])
    T = _lossy_network(3, 13, [0.9, 0.75, 0.85])
    bins = np.array([0, 1, 2])
    Pf, tail = fock.binned_probabilities(T, r, bins, 3, 14)
    K = 10
    est = estimator.estimate(T, r, 77, 60000, 30, bins, 3, [(0, K)] * 3, mode="joint",
                             chunk=3000)
    ref = Pf[:K, :K, :K]
    z = _z(est, ref)
    assert z.max() < 5, z.max()
    bulk = ref > 1e-3 * ref.max()
    assert abs(((est["P"] - ref)[bulk] / est["sigma"][bulk]).mean()) < 0.3
    assert abs(est["P"].sum() - ref.sum()) < 5 * np.sqrt((est["sigma"] ** 2).sum()) + tail


def _sigma_scale_replicas():
    """4000 independent runs of the oracle (N_R = 4 sub-ensembles of N_S = 50
    samples each, disjoint sample ranges) on a lossy four-mode network whose
    total-count law is known exactly (uniform loss).  Returns the runs' (P,
    sigma_T, sub-ensemble means) and the exact law."""
    M, t, r, K = 4, 0.8, 0.6, 16
    T = synth.transmission(M, t, 7)
    rr = np.full(M, r)
    n_sub, ns, runs = 4, 50, 4000
    out = []
    for rep in range(runs):
        o = estimator.estimate(T, rr, 99, n_sub * ns, n_sub, np.zeros(M, np.int32), 1, [(0, K)],
                               g0=rep * n_sub * ns, chunk=n_sub * ns)
        out.append((o["P"], o["sigma"], o["Ps"]))
    return out, exact.uniform_loss_total(rr, t, K)


def _pooled_ratio(runs, exact_P, stats=None):
    """Mean sigma_T^2 over mean (P - P_exact)^2, pooled over the bins above
    2 %; `stats` recomputes (P, sigma) from the sub-ensemble means (to plant
    mistakes)."""
    s2 = np.zeros_like(exact_P)
    mse = np.zeros_like(exact_P)
    for P, sig, Ps in runs:
        if stats is not None:
            P, sig = stats(Ps)
        s2 += sig ** 2
        mse += (P - exact_P) ** 2
    sel = exact_P > 0.02
    return s2[sel].sum() / mse[sel].sum()


def test_sigma_T_is_the_standard_error_of_P():
    """Appendix A: sigma_T, taken from the spread of the N_R sub-ensemble
    means, estimates the sampling error of P.  Since the estimator is unbiased
    for the exact law, E[sigma_T^2] must equal E[(P - P_exact)^2] over
    independent runs: a sigma_T without the 1/sqrt(N_R) (ratio 4 at N_R = 4)
    or with the biased sd (ddof 0: ratio 3/4) fails.  Over 4000 runs the
    pooled ratio scatters by about 0.04 between seeds."""
    runs, exact_P = _sigma_scale_replicas()
    ratio = _pooled_ratio(runs, exact_P)
    assert 0.88 < ratio < 1.14, ratio

    # planted mistakes in a copy of the statistics, on the same runs
    def ddof0(Ps):
        return Ps.mean(0).real, Ps.real.std(0, ddof=0) / np.sqrt(Ps.shape[0])

    def no_sqrt(Ps):
        return Ps.mean(0).real, Ps.real.std(0, ddof=1)

    for wrong in (ddof0, no_sqrt):
        rw = _pooled_ratio(runs, exact_P, wrong)
        assert not 0.88 < rw < 1.14, (wrong.__name__, rw)


def test_sigma_T_of_two_sub_ensembles():
    """With two sub-ensembles the estimate is the mean of the two halves' own
    estimates and sigma_T is half their difference (the standard error of a
    mean of two values).  The halves are run as separate one-sub-ensemble
    estimates of the same samples, so this also pins which samples form each
    sub-ensemble."""
    w = synth.workload_small(E=600, n_sub=2)
    whole = estimator.estimate(w.T, w.r, w.seed, 600, 2, w.bins, 1, w.windows, chunk=250)
    a = estimator.estimate(w.T, w.r, w.seed, 300, 1, w.bins, 1, w.windows, g0=0)
    b = estimator.estimate(w.T, w.r, w.seed, 300, 1, w.bins, 1, w.windows, g0=300)
    np.testing.assert_allclose(whole["P"], 0.5 * (a["P"] + b["P"]), rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(whole["sigma"], 0.5 * np.abs(a["P"] - b["P"]), rtol=1e-10,
                               atol=1e-16)
    assert np.all(np.isnan(a["sigma"]))


def test_resume_from_saved_sums_is_bit_identical(tmp_path):
    """Checkpoint and resume: run the oracle's accumulation to the end of
    chunk c, save the per-sub-ensemble sums and the next sample index, start
    a fresh accumulation from the file, and finish: the estimate is bit for
    bit the uninterrupted one (the noise is counter-based, so sample g is the
    same draw whenever it is made)."""
    w = synth.workload_small(E=3000, n_sub=6)
    ns, chunk = w.samples_per_sub, 400
    full = estimator.estimate(w.T, w.r, w.seed, w.E, w.n_sub, w.bins, 1, w.windows, chunk=chunk)
    sums = np.zeros((w.n_sub, w.windows[0][1]), dtype=np.complex128)
    stop = 3 * chunk  # after chunk c = 3, inside sub-ensemble 2
    estimator.accumulate(sums, w.T, w.r, w.seed, ns, w.bins, 1, w.windows, 0, stop, chunk=chunk)
    np.save(tmp_path / "sums.npy", sums)
    np.save(tmp_path / "next.npy", np.array([stop]))
    del sums
    sums2 = np.load(tmp_path / "sums.npy")
    nxt = int(np.load(tmp_path / "next.npy")[0])
    estimator.accumulate(sums2, w.T, w.r, w.seed, ns, w.bins, 1, w.windows, nxt, w.E, chunk=chunk)
    _, P, sig = estimator.subensemble_stats(sums2, np.full(w.n_sub, ns, dtype=np.float64))
    assert np.array_equal(P.real, full["P"]) and np.array_equal(sig, full["sigma"])
