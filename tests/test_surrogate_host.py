"""Host-side pieces of the surrogate, checked against closed forms: the
truncated cumulants of known distributions, the independent-mode baseline
against the exact count variance of a uniform-loss network (E4), and the
round trip between moments and targets."""
import math

import numpy as np
from scipy import stats

from oracle import exact
from paper_2503_12749_amd import surrogate as sg


def test_cumulants_of_poisson_and_negative_binomial():
    m = np.arange(0, 400)
    lam = 37.5
    P = stats.poisson.pmf(m, lam)
    np.testing.assert_allclose(sg.cumulants(m, P, trunc=1e9), [lam] * 4, rtol=1e-9)
    # the default 7-sigma window moves the fourth cumulant by ~5e-5 relative
    np.testing.assert_allclose(sg.cumulants(m, P), [lam] * 4, rtol=1e-4)
    # negative binomial (n, p): kappa_2 = n q / p^2, kappa_3 = n q (1 + q) / p^3,
    # kappa_4 = n q (1 + 4q + q^2) / p^4 with q = 1 - p
    n, p = 20.0, 0.4
    q = 1 - p
    want = [n * q / p, n * q / p ** 2, n * q * (1 + q) / p ** 3, n * q * (1 + 4 * q + q * q) / p ** 4]
    k = sg.cumulants(m, stats.nbinom.pmf(m, n, p), trunc=1e9)
    np.testing.assert_allclose(k, want, rtol=1e-8)


def test_truncation_drops_far_tail_only():
    m = np.arange(0, 300)
    P = stats.poisson.pmf(m, 50.0)
    P[290] += 1e-6  # a spurious far-tail value, as sampling noise leaves
    assert abs(sg.cumulants(m, P)[1] - 50.0) < 1e-4
    assert abs(sg.cumulants(m, P, trunc=1e9)[1] - 50.0) > 1e-3


def test_total_baseline_equals_exact_uniform_loss_variance():
    """For T = t U (U unitary) the total count's mean and variance are exact
    closed forms; the baseline reproduces them per mode."""
    rng = np.random.default_rng(1)
    M, t = 12, 0.9
    r = rng.uniform(0.5, 1.5, M)
    from synth import haar_unitary
    T = t * haar_unitary(M, 5)
    mean, var = exact.count_moments(T, r, np.ones(M, dtype=bool))
    b_mean, _, b_var = sg.independent_mode_baseline(t, r, 1)
    assert math.isclose(mean, M * b_mean, rel_tol=1e-12)
    assert math.isclose(var, M * b_var, rel_tol=1e-10)


def test_targets_round_trip():
    rng = np.random.default_rng(2)
    r = rng.uniform(0.5, 1.5, 64)
    kb = np.array([20.0, 30.0, 5.0, 2.0])
    kt = np.array([80.0, 150.0, 40.0, 9.0])
    y = sg.targets(64, 0.9, r, 4, kb, kt)
    kb2, kt2 = sg.moments_from_targets(64, 0.9, r, 4, y)
    np.testing.assert_allclose(kb2, kb, rtol=1e-12)
    np.testing.assert_allclose(kt2, kt, rtol=1e-12)
