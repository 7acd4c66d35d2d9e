"""Pair moments <:n_i n_j:> of single output modes (mp_mode_occupations +
mp_pair_correlations_accumulate through the C ABI) against the FP64 oracle
on identical noise.

Tolerances, per sub-ensemble sum and element (i, j):
  FP64: 1e-11 of sum_k |n'_ik| |n'_jk| (FP64 rounding of propagation and sums).
  FP32 / split: a propagated amplitude carries at most rel * ||alpha_k|| of
  error (rel: 2e-6 FP32, 2e-5 split BF16, 4e-6 split FP16 at M = 300, the
  bounds of the propagation parity test; doubled at M = 1000 for the sqrt(M)
  growth of the GEMM's rounding), so to first order
      |d(n'_ik n'_jk)| <= e_ik |n'_jk| + |n'_ik| e_jk,
      e_ik = rel (||alpha_k|| |beta'_ik| + ||beta_k|| |alpha'_ik|);
  the test allows twice the sum of that bound over the samples plus FP32
  rounding of the products and of the sums over a sub-ensemble's K samples:
  the kernel forms Im = P3 - P1 - P2 from three real products, whose sums
  round by up to (2 + 1 + 1) K u of sum_k |n'_ik| |n'_jk| (u = 2^-24; P3
  sums products of |Re| + |Im| <= sqrt(2) |n'|).
"""
import numpy as np
import pytest

import synth
from oracle import estimator as oest
from oracle import exact, sampler as osamp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
REL = {"fp32": 2e-6, "split_bf16": 2e-5, "split_fp16": 4e-6}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_12749_amd  # noqa: F401
    yield


def _network(M, seed, t_lo=0.7):
    """Haar unitary with mode-dependent input loss (non-normal)."""
    return synth.haar_unitary(M, seed) * np.linspace(t_lo, 1.0, M)[None, :]


def _tolerance(prec, a, b, ap, bp, rel_scale=1.0):
    """Per-element bound for the sum over one sub-ensemble's samples; a, b
    are the input amplitudes (E_s, M), ap, bp the oracle's propagated ones
    restricted to the compared modes (E_s, m)."""
    occ = np.abs(ap * bp)
    abs_sums = occ.T @ occ
    if prec == "fp64":
        return 1e-11 * abs_sums
    rel = REL[prec] * rel_scale
    na = np.linalg.norm(a, axis=1, keepdims=True)
    nb = np.linalg.norm(b, axis=1, keepdims=True)
    e = rel * (na * np.abs(bp) + nb * np.abs(ap))
    first = e.T @ occ + occ.T @ e
    K = ap.shape[0]
    return 2.0 * first + 4.0 * K * 2.0 ** -24 * abs_sums


@pytest.mark.parametrize("prec", ["fp64", "fp32", "split_bf16", "split_fp16"])
def test_pair_sums_match_oracle(prec):
    """M = 333 (three 128-mode tiles, the last ragged; five 64-mode tiles for
    FP64), 1000 samples in chunks of 384 over five sub-ensembles of 200, so
    sub-ensembles straddle chunks; every element of both triangles."""
    import paper_2503_12749_amd as mp
    M, E, n_sub, chunk, seed = 333, 1000, 5, 384, 41
    ns = E // n_sub
    T = _network(M, 3)
    r = np.linspace(0.4, 1.2, M)
    p = mp.PairPipeline(T, r, prec=prec, seed=seed, n_sub=n_sub, samples_per_sub=ns, chunk=chunk,
                        device=DEV)
    p.run()
    got = p.subensemble_sums()
    ref = oest.pair_correlations(T, r, seed, E, n_sub, chunk=chunk)
    a, b, _ = osamp.sample(r, 0, E, seed)
    ap, bp = oest.propagate(T, a, b)
    worst = 0.0
    for s in range(n_sub):
        sl = slice(s * ns, (s + 1) * ns)
        tol = _tolerance(prec, a[sl], b[sl], ap[sl], bp[sl])
        err = np.abs(got[s] - ref["Ps"][s] * ns)
        worst = max(worst, float((err / tol).max()))
        assert np.all(err <= tol), (s, (err / tol).max())
    print(f"{prec}: max err / tolerance = {worst:.3g}")


def test_pair_means_and_sigma_match_oracle():
    import paper_2503_12749_amd as mp
    M, E, n_sub, seed = 200, 1200, 6, 9
    T = _network(M, 5)
    r = np.full(M, 0.8)
    p = mp.PairPipeline(T, r, prec="fp64", seed=seed, n_sub=n_sub, samples_per_sub=E // n_sub,
                        chunk=500, device=DEV)
    p.run()
    G2, sig = p.result()
    ref = oest.pair_correlations(T, r, seed, E, n_sub, chunk=500)
    scale = ref["abs_sums"].sum(axis=0) / E
    assert np.all(np.abs(G2 - ref["G2"]) <= 1e-11 * scale)
    np.testing.assert_allclose(sig, ref["sigma"], rtol=1e-7, atol=1e-12 * scale.max())


def test_pair_full_size_m1000_sampled_modes():
    """The M = 1000 network (t = 0.9, r = 1) with 16384 samples in one chunk
    over 4 sub-ensembles, FP32: 40 sampled modes (first and last included)
    against the oracle's sums for those rows, and the symmetry of the whole
    matrix."""
    import paper_2503_12749_amd as mp
    M, E, n_sub, seed = 1000, 16384, 4, 250312751
    ns = E // n_sub
    T = 0.9 * synth.haar_unitary(M, seed)
    r = np.full(M, 1.0)
    p = mp.PairPipeline(T, r, prec="fp32", seed=seed, n_sub=n_sub, samples_per_sub=ns, chunk=E,
                        device=DEV)
    p.run()
    got = p.subensemble_sums()
    rng = np.random.default_rng(4)
    S = np.unique(np.concatenate([[0, M - 1], rng.choice(M, 38, replace=False)]))
    a, b, _ = osamp.sample(r, 0, E, seed)
    ap, bp = oest.propagate(T[S], a, b)
    ref = oest.pair_correlations(T[S], r, seed, E, n_sub, chunk=4096)
    for s in range(n_sub):
        sl = slice(s * ns, (s + 1) * ns)
        tol = _tolerance("fp32", a[sl], b[sl], ap[sl], bp[sl], rel_scale=2.0)
        err = np.abs(got[s][np.ix_(S, S)] - ref["Ps"][s] * ns)
        print(f"sub-ensemble {s}: max err / tolerance = {(err / tol).max():.3g}")
        assert np.all(err <= tol)
        sym = np.abs(got[s] - got[s].T)
        assert sym.max() <= 1e-4 * np.abs(got[s]).max()


def test_pair_moments_vs_closed_form_m64():
    """FP32 path, M = 64 lossy network, E = 2e5 in 50 sub-ensembles: every
    element within 5.5 sigma_T of Isserlis' closed form (sigma_T from 50
    sub-ensembles: Student t with 49 degrees of freedom), and the spread of
    the normalised errors close to 1."""
    import paper_2503_12749_amd as mp
    M, E, n_sub = 64, 200000, 50
    T = _network(M, 8)
    r = np.linspace(0.5, 1.0, M)
    p = mp.PairPipeline(T, r, prec="fp32", seed=17, n_sub=n_sub, samples_per_sub=E // n_sub,
                        chunk=65536, device=DEV)
    p.run()
    G2, sig = p.result()
    z = (G2.real - exact.pair_moments(T, r)) / sig
    print(f"max |z| = {np.abs(z).max():.2f}, rms z = {np.sqrt((z ** 2).mean()):.3f}")
    assert np.abs(z).max() < 5.5
    assert 0.8 < np.sqrt((z ** 2).mean()) < 1.2


def test_pair_unsplit_launch_m2000():
    """M = 2000 (136 tile pairs) with 16 sub-ensembles of 128 in one chunk:
    2176 items, so the FP32 launch sums each item in one workgroup (no sample
    pieces, no workspace); 40 sampled modes (first and last included) against
    the oracle."""
    import paper_2503_12749_amd as mp
    M, E, n_sub, seed = 2000, 2048, 16, 88
    ns = E // n_sub
    assert mp.mp_pair_correlations_workspace(M, E, "fp32", ns, 0) == 0
    T = _network(M, 12, t_lo=0.85)
    r = np.linspace(0.6, 1.1, M)
    p = mp.PairPipeline(T, r, prec="fp32", seed=seed, n_sub=n_sub, samples_per_sub=ns, chunk=E,
                        device=DEV)
    p.run()
    got = p.subensemble_sums()
    rng = np.random.default_rng(6)
    S = np.unique(np.concatenate([[0, M - 1], rng.choice(M, 38, replace=False)]))
    a, b, _ = osamp.sample(r, 0, E, seed)
    ap, bp = oest.propagate(T[S], a, b)
    ref = oest.pair_correlations(T[S], r, seed, E, n_sub, chunk=E)
    for s in range(n_sub):
        sl = slice(s * ns, (s + 1) * ns)
        tol = _tolerance("fp32", a[sl], b[sl], ap[sl], bp[sl], rel_scale=3.0)
        err = np.abs(got[s][np.ix_(S, S)] - ref["Ps"][s] * ns)
        assert np.all(err <= tol), (s, (err / tol).max())
