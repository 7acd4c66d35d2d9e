"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle on
identical seeded inputs and identical Philox noise.

Tolerances
  FP64 path: every binned probability within 1e-10 relative, with an
  absolute floor of 1e-14 * max P for tail bins (FP64 rounding of the sums);
  intermediate buffers within a few hundred ulps of their magnitude.
  FP32 / split-BF16 paths: operands are rounded to 24 / ~16 significant bits,
  so propagated amplitudes carry relative errors ~ sqrt(M) 2^-24 (FP32) and
  ~ sqrt(M) 2^-17 (split BF16) of the column norm; the probabilities must stay
  far inside the sampling error sigma_T.
"""
import os

import numpy as np
import pytest

import synth
from oracle import estimator as oest
from oracle import exact, sampler as osamp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_12749_amd as mp  # noqa: F401  (fails loudly if the library is missing)
    yield


def _pipe(T, r, **kw):
    import paper_2503_12749_amd as mp
    return mp.CountsPipeline(T, r, device=DEV, **kw)


def _p_close(P, ref, rel=1e-10, floor=1e-14, scale=None):
    scale = np.abs(ref).max() if scale is None else scale
    tol = rel * np.maximum(np.abs(ref), 1e-4 * scale) + floor * scale
    bad = np.abs(P - ref) > tol
    assert not bad.any(), (np.flatnonzero(bad)[:10], (P - ref)[bad][:5], ref[bad][:5])


def test_sampler_matches_oracle_fp64():
    r = np.concatenate([np.linspace(0.2, 1.5, 37), [0.0, 0.0]])
    M = r.size
    T = np.eye(M, dtype=np.complex128)
    p = _pipe(T, r, prec="fp64", seed=4242, windows=[(0, 64)], n_sub=1, samples_per_sub=1000,
              chunk=300)
    g0, E = 123, 257
    import paper_2503_12749_amd as mp
    mp.mp_sample(M, g0, E, p.r, p.seed, 3, "fp64", p.ab, p.n)
    a_gpu, b_gpu = p.alpha_beta(E)
    a, b, n = osamp.sample(r, g0, E, 4242, net=3)
    np.testing.assert_allclose(a_gpu, a, rtol=0, atol=1e-14 * np.abs(a).max())
    np.testing.assert_allclose(b_gpu, b, rtol=0, atol=1e-14 * np.abs(b).max())
    np.testing.assert_allclose(p.n[:E].cpu().numpy(), n, rtol=0, atol=1e-13 * np.abs(n).max())
    assert np.all(a_gpu[:, -2:] == 0) and np.all(b_gpu[:, -2:] == 0)
    # padding rows of the mode-major layout are zero
    ldm = mp.mp_ld_modes(M)
    raw = p.ab.view(torch.float64)[: ldm * 2 * E].reshape(2 * E, ldm)
    assert torch.all(raw[:, M:] == 0)


@pytest.mark.parametrize("M,E", [(16, 1000), (200, 333), (1, 7), (257, 130), (1000, 3000),
                                 (2049, 1100)])
def test_propagate_fp64_matches_oracle(M, E):
    """FP64 GEMM against the oracle element by element.  The FP64 tile is 128
    rows x 256 columns over 16-deep slabs: the cases span two to 34 row tiles
    (the last of the larger ones a partial group of eight in the tile order),
    8 to 136 slabs, and ragged last column tiles (2E = 14 ... 6000)."""
    T = 0.8 * synth.haar_unitary(M, 100 + M)
    r = synth.squeezing_random_uniform(M, 0.3, 1.2, M)
    p = _pipe(T, r, prec="fp64", seed=9, windows=[(0, 64)], n_sub=1, samples_per_sub=E, chunk=E)
    import paper_2503_12749_amd as mp
    mp.mp_sample(M, 0, E, p.r, p.seed, 0, "fp64", p.ab, p.n)
    mp.mp_propagate(M, E, p.T, "fp64", p.ab, p.C, p.ws_prop)
    ag, bg = p.propagated(E)
    a, b, n = osamp.sample(r, 0, E, 9)
    ao, bo = oest.propagate(T, a, b)
    scale = np.abs(ao).max()
    np.testing.assert_allclose(ag, ao, rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(bg, bo, rtol=0, atol=1e-13 * scale)
    # invariant of T = t U: sum_j alpha'_j beta'_j = t^2 n
    np.testing.assert_allclose((ag * bg).sum(1), 0.64 * n, rtol=0, atol=1e-12 * np.abs(n).max())


def _oracle(w_T, r, seed, E, n_sub, bins, d, windows, mode="joint", plus_p=False):
    return oest.estimate(w_T, r, seed, E, n_sub, bins, d, windows, mode=mode, plus_p=plus_p,
                         chunk=4000)


def test_small_workload_fp64_parity():
    """M = 16, Haar x 0.5, r = 1, E = 1e4 (10 x 1e3), total counts on m = 0..127."""
    w = synth.workload_small()
    p = _pipe(w.T, w.r, prec="fp64", seed=w.seed, windows=w.windows, n_sub=w.n_sub,
              samples_per_sub=w.samples_per_sub, chunk=w.chunk)
    p.run()
    P, Pi, s = p.result()
    ref = _oracle(w.T, w.r, w.seed, w.E, w.n_sub, w.bins, 1, w.windows)
    _p_close(P, ref["P"])
    _p_close(Pi, ref["P_complex"].imag, scale=ref["P"].max())
    np.testing.assert_allclose(s, ref["sigma"], rtol=1e-7, atol=1e-14 * ref["P"].max())
    assert abs(P.sum() - 1) < 1e-12


def test_chunking_and_subensemble_boundaries():
    """Chunks that straddle sub-ensembles (N_S = 100, chunks of 130, ragged M)
    give the oracle's result; a second run is bit-identical."""
    M = 200
    T = 0.9 * synth.haar_unitary(M, 77)
    r = synth.squeezing_random_uniform(M, 0.2, 0.6, 77)
    mean, sd = synth.uniform_loss_moments(r, 0.9)
    win = [synth.count_window(mean, sd, align=16)]
    p = _pipe(T, r, prec="fp64", seed=55, windows=win, n_sub=7, samples_per_sub=100, chunk=130)
    p.run()
    P1 = p.acc.clone()
    P, Pi, s = p.result()
    p.reset()
    p.run()
    assert torch.equal(P1, p.acc)
    ref = _oracle(T, r, 55, 700, 7, np.zeros(M, int), 1, win)
    _p_close(P, ref["P"])
    np.testing.assert_allclose(s, ref["sigma"], rtol=1e-7, atol=1e-14 * ref["P"].max())


def _fold(P_full, m_full, m_lo, K):
    """Oracle probabilities on counts m_full folded into the window's residues:
    entry l collects every m with m = m_lo + l (mod K)."""
    out = np.zeros(K)
    np.add.at(out, (m_full - m_lo) % K, P_full)
    return out


def test_marginals_total_uncounted_and_vacuum():
    """Three bins (one split into two runs), uncounted and vacuum modes,
    marginal distributions plus the total, with window offsets; counts outside
    a window alias into it mod K."""
    M = 40
    T = 0.85 * synth.haar_unitary(M, 5)
    r = synth.squeezing_random_uniform(M, 0.3, 1.0, 5)
    r[[3, 17]] = 0.0
    bins = np.array([0] * 10 + [1] * 10 + [-1] * 5 + [2] * 10 + [0] * 5, dtype=np.int32)
    wins = [(2, 64), (0, 48), (1, 40), (10, 96)]
    p = _pipe(T, r, prec="fp64", seed=8, bin_of_mode=bins, d=3, mode="marginals_and_total",
              windows=wins, n_sub=4, samples_per_sub=500, chunk=700)
    p.run()
    P, Pi, s = p.result()
    off = np.cumsum([0] + [k for _, k in wins])
    full = [(0, 160)] * 3
    ref = _oracle(T, r, 8, 2000, 4, bins, 3, full, mode="marginals")
    m = np.arange(160)
    for b in range(3):
        lo, K = wins[b]
        _p_close(P[off[b]:off[b + 1]], _fold(ref["P"][b], m, lo, K))
    tot = _oracle(T, r, 8, 2000, 4, np.where(bins >= 0, 0, -1), 1, [(0, 200)])
    _p_close(P[off[3]:], _fold(tot["P"], np.arange(200), *wins[3]))


def test_plus_p_estimator_parity():
    M = 12
    T = 0.7 * synth.haar_unitary(M, 3)
    r = np.full(M, 0.5)
    p = _pipe(T, r, prec="fp64", seed=2, windows=[(0, 64)], n_sub=5, samples_per_sub=400,
              chunk=2000, est="plus_p")
    p.run()
    P, _, s = p.result()
    ref = _oracle(T, r, 2, 2000, 5, np.zeros(M, int), 1, [(0, 64)], plus_p=True)
    _p_close(P, ref["P"])


def test_single_mode_negative_n_and_tiny_chunk():
    """M = 1 (n = alpha beta often negative), E below one tile."""
    T = np.array([[0.6 * np.exp(0.3j)]])
    r = np.array([0.5])
    p = _pipe(T, r, prec="fp64", seed=1, windows=[(0, 32)], n_sub=1, samples_per_sub=7, chunk=7)
    p.run()
    P, _, _ = p.result()
    ref = _oracle(T, r, 1, 7, 1, np.zeros(1, int), 1, [(0, 32)])
    _p_close(P, ref["P"])


def test_lossless_odd_counts_vanish():
    M = 24
    U = synth.haar_unitary(M, 31)
    p = _pipe(U, np.full(M, 0.5), prec="fp64", seed=3, windows=[(0, 64)], n_sub=4,
              samples_per_sub=500, chunk=2000)
    p.run()
    P, _, s = p.result()
    assert np.abs(P[1::2]).max() < 1e-13
    ref = exact.lossless_uniform_total(M, 0.5, np.arange(64))
    bulk = ref > 1e-3 * ref.max()
    assert np.all(np.abs(P - ref)[bulk] < 5 * s[bulk])


@pytest.mark.parametrize("M,E", [(300, 200), (2049, 1100)])
@pytest.mark.parametrize("prec,rel", [("fp32", 2e-6), ("split_bf16", 2e-5), ("split_fp16", 4e-6)])
def test_reduced_precision_propagation(prec, rel, M, E):
    """Every element against the oracle, relative to the largest per-sample
    norm of the propagated amplitudes.  M = 2049 (ldm 2176, with the split
    kernels' L2 prefetch) spans 17 row tiles of 256 and 68 slabs of 32."""
    T = 0.95 * synth.haar_unitary(M, 12)
    r = np.full(M, 1.0)
    p = _pipe(T, r, prec=prec, seed=5, windows=[(0, 64)], n_sub=1, samples_per_sub=E, chunk=E)
    import paper_2503_12749_amd as mp
    mp.mp_sample(M, 0, E, p.r, p.seed, 0, prec, p.ab, p.n)
    mp.mp_propagate(M, E, p.T, prec, p.ab, p.C, p.ws_prop)
    ag, bg = p.propagated(E)
    a, b, n = osamp.sample(r, 0, E, 5)
    ao, bo = oest.propagate(T, a, b)
    norm = np.linalg.norm(ao, axis=1, keepdims=True)
    assert np.abs(ag - ao).max() / norm.max() < rel
    assert np.abs(bg - bo).max() / norm.max() < rel
    nS = (ag * bg).sum(1)
    assert np.abs(nS - 0.9025 * n).max() < 50 * rel * np.abs(n).max()


def _fp16_network(T, M):
    """T with each real and imaginary part rounded to FP16 after the power-of-two
    prescale 2^floor(log2(M) / 2) (the packed operand of the one-sided split)."""
    e = 0
    while 4 ** (e + 1) <= M:
        e += 1
    sc = 2.0 ** e
    q = lambda x: np.float16(x * sc).astype(np.float64) / sc
    return q(T.real) + 1j * q(T.imag)


@pytest.mark.parametrize("M,E", [(300, 200), (2049, 1100)])
def test_split1_propagation(M, E):
    """The one-sided split (T as one FP16 value, samples hi/lo FP16, two
    products): every element against the oracle propagating with the
    FP16-rounded network, relative to the largest per-sample norm (4e-6, the
    split-FP16 bound: what remains is the samples' 2^-22 split and FP32
    accumulation); the distance to the unrounded network is the T rounding
    itself, below 2e-4 of the norm."""
    import paper_2503_12749_amd as mp
    prec = "split1_fp16"
    T = 0.95 * synth.haar_unitary(M, 12)
    r = np.full(M, 1.0)
    p = _pipe(T, r, prec=prec, seed=5, windows=[(0, 64)], n_sub=1, samples_per_sub=E, chunk=E)
    mp.mp_sample(M, 0, E, p.r, p.seed, 0, prec, p.ab, p.n)
    mp.mp_propagate(M, E, p.T, prec, p.ab, p.C, p.ws_prop)
    ag, bg = p.propagated(E)
    a, b, n = osamp.sample(r, 0, E, 5)
    ao, bo = oest.propagate(_fp16_network(T, M), a, b)
    norm = np.linalg.norm(ao, axis=1, keepdims=True).max()
    err = max(np.abs(ag - ao).max(), np.abs(bg - bo).max()) / norm
    at, bt = oest.propagate(T, a, b)
    dist = max(np.abs(ag - at).max(), np.abs(bg - bt).max()) / norm
    print(f"split1 M={M}: vs rounded network {err:.2e}, vs exact network {dist:.2e}")
    assert err < 4e-6
    assert dist < 2e-4
    nS = (ag * bg).sum(1)
    assert np.abs(nS - (ao * bo).sum(1)).max() < 200 * 4e-6 * np.abs(n).max()


@pytest.mark.parametrize("M,E", [(300, 201), (2049, 1100)])
def test_split1t_sampler_and_propagation(M, E):
    """The T-split one-sided form (T hi/lo FP16, samples as one FP16 value,
    two products).  Sampler: every stored amplitude is the oracle's rounded
    to FP16 (within half an FP16 ulp plus the FP32 evaluation's 5e-7 of the
    term scale), n is the sum over the stored values, and the padding columns
    of an odd E hold zeros.  GEMM: every element against the oracle
    propagating the stored (rounded) samples through the exact network, at
    the split's 2^-22 and FP32 accumulation (4e-6 of the largest per-sample
    norm); E = 201 leaves a ragged tile and a padded column pair."""
    import paper_2503_12749_amd as mp
    prec = "split1t_fp16"
    T = 0.95 * synth.haar_unitary(M, 12)
    r = np.linspace(0.5, 1.5, M)
    p = _pipe(T, r, prec=prec, seed=5, windows=[(0, 64)], n_sub=1, samples_per_sub=E, chunk=E)
    mp.mp_sample(M, 0, E, p.r, p.seed, 0, prec, p.ab, p.n)
    mp.mp_propagate(M, E, p.T, prec, p.ab, p.C, p.ws_prop)
    a_s, b_s = p.alpha_beta(E)
    a, b, n = osamp.sample(r, 0, E, 5)
    scale = np.abs(a).max()
    assert np.all(np.abs(a_s - a) <= 2.0 ** -11 * np.abs(a) + 5e-7 * scale + 1e-7)
    assert np.all(np.abs(b_s - b) <= 2.0 ** -11 * np.abs(b) + 5e-7 * scale + 1e-7)
    ng = p.n.cpu().numpy()
    assert np.abs(ng - (a_s * b_s).sum(1)).max() <= 1e-12 * np.abs(a_s * b_s).sum(1).max()
    if E % 2:
        h = p.ab.view(torch.float16).cpu().numpy()
        ldm = mp.mp_ld_modes(M)
        j = np.arange(ldm)
        for c in (E, E + 1 + E):  # the padding columns E and E2 + E
            assert not h[(c >> 1) * 2 * ldm + 64 * (j >> 5) + (j & 31) + 32].any()
    ag, bg = p.propagated(E)
    ao, bo = oest.propagate(T, a_s, b_s)
    norm = np.linalg.norm(ao, axis=1, keepdims=True).max()
    err = max(np.abs(ag - ao).max(), np.abs(bg - bo).max()) / norm
    at, bt = oest.propagate(T, a, b)
    dist = max(np.abs(ag - at).max(), np.abs(bg - bt).max()) / norm
    print(f"split1t M={M} E={E}: vs rounded samples {err:.2e}, vs unrounded samples {dist:.2e}")
    assert err < 4e-6
    assert dist < 1e-3


def _e4m3_table():
    """Values of the OCP e4m3 codes 0x00 .. 0x7E (4 exponent bits, bias 7,
    3 mantissa bits, subnormals below 2^-6), increasing with the code."""
    c = np.arange(127)
    e, m = c >> 3, c & 7
    return np.where(e > 0, np.ldexp(1.0 + m / 8.0, e - 7), np.ldexp(m / 8.0, -6))


def _e4m3_decode(codes):
    v = _e4m3_table()[np.asarray(codes) & 0x7F]
    return np.where(np.asarray(codes) & 0x80, -v, v)


def _e4m3_rne(x):
    """Codes of x rounded to the nearest e4m3 value, ties to the even code,
    saturating at 448: the rounding by the definition, over the code table."""
    tab = _e4m3_table()
    a = np.abs(np.asarray(x, dtype=np.float64))
    hi = np.clip(np.searchsorted(tab, a), 1, 126)
    lo = hi - 1
    dlo, dhi = a - tab[lo], tab[hi] - a
    code = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi, np.where(lo % 2 == 0, lo, hi)))
    code = np.where(a >= tab[126], 126, code)
    return (code | np.where(np.signbit(x), 0x80, 0)).astype(np.uint8)


def test_e4m3_reference_rounding():
    """The test-side e4m3 rounding against hand-checked values."""
    assert _e4m3_rne([1.0, 1.0625, 1.1875, 448.0, 1e6, -2.0 ** -9, 2.0 ** -10, 3 * 2.0 ** -10,
                      0.0]).tolist() == [0x38, 0x38, 0x3A, 0x7E, 0x7E, 0x81, 0x00, 0x02, 0x00]
    assert np.array_equal(_e4m3_decode(_e4m3_rne(_e4m3_table())), _e4m3_table())


@pytest.mark.parametrize("M,E", [(300, 201), (2049, 1100)])
def test_split1t_f8_sampler_packing_and_propagation(M, E):
    """The T-split form with an FP8 correction product.  Sampler: the FP16
    operand and n equal the T-split form's bit for bit, the e4m3 copy is the
    nearest-even e4m3 of every stored FP16 value, and the padding pairs of
    an odd E hold zeros.  Packing: T_hi is T 2^e within half an FP16 unit and
    the e4m3 remainder is the nearest-even e4m3 of (x - T_hi) 2^(18 - e).
    GEMM, every element against the oracle propagating the stored samples
    through the exact network: the network is kept to 2^-15 |x| per entry
    (remainder at most 2^-11 |x|, e4m3's relative rounding 2^-4) and the
    correction product's sample copy to 2^-15 of the product, so by
    Cauchy-Schwarz over a row of T (norm <= 1) |error| <= 2^-14 |beta| per
    element, plus FP32 accumulation; the bound is 2^-14 of the largest
    sample norm plus 4e-6 of the largest propagated norm."""
    import paper_2503_12749_amd as mp
    T = 0.95 * synth.haar_unitary(M, 12)
    r = np.linspace(0.5, 1.5, M)
    ldm = mp.mp_ld_modes(M)
    e2 = E + (E & 1)
    kw = dict(seed=5, windows=[(0, 64)], n_sub=1, samples_per_sub=E, chunk=E)
    q = _pipe(T, r, prec="split1t_fp16", **kw)
    mp.mp_sample(M, 0, E, q.r, q.seed, 0, "split1t_fp16", q.ab, q.n)
    p = _pipe(T, r, prec="split1t_f8", **kw)
    mp.mp_sample(M, 0, E, p.r, p.seed, 0, "split1t_f8", p.ab, p.n)
    assert mp.mp_ab_bytes(M, E, "split1t_f8") == 3 * ldm * 2 * e2
    raw = p.ab.view(torch.uint8).cpu().numpy()
    h16 = 4 * e2 * ldm  # bytes of the FP16 part
    assert np.array_equal(raw[:h16], q.ab.view(torch.uint8).cpu().numpy()[:h16])
    assert np.array_equal(p.n.cpu().numpy(), q.n.cpu().numpy())
    a_s, b_s = p.alpha_beta(E)
    j = np.arange(M)
    b8 = raw[h16:]

    def codes(c):
        c = np.asarray(c)[:, None]
        return b8[(c >> 1) * 2 * ldm + 128 * (j >> 6) + 64 * (c & 1) + (j & 63)]

    assert np.array_equal(codes(np.arange(E)), _e4m3_rne(a_s))
    assert np.array_equal(codes(e2 + np.arange(E)), _e4m3_rne(b_s))
    if E % 2:
        jj = np.arange(ldm)
        for c in (E, e2 + E):
            assert not b8[(c >> 1) * 2 * ldm + 128 * (jj >> 6) + 64 + (jj & 63)].any()
    # packing
    Td = torch.from_numpy(np.ascontiguousarray(T).view(np.float64).reshape(-1).copy()).to(DEV)
    packed = torch.empty(mp.mp_propagate_workspace(M, "split1t_f8"), dtype=torch.uint8, device=DEV)
    assert packed.numel() == 3 * 2 * ldm * ldm
    mp.mp_pack_transmission(M, Td, "split1t_f8", packed)
    praw = packed.cpu().numpy()
    hi = praw[: 4 * ldm * ldm].view(np.float16).astype(np.float64)
    lo8 = praw[4 * ldm * ldm:]
    e = int(np.floor(np.log2(M) / 2))
    rows = np.arange(2 * ldm)
    A = np.zeros((2 * ldm, ldm))
    A[:M, :M], A[ldm: ldm + M, :M] = T.real, T.imag
    x = np.ldexp(A, e)
    kk = np.arange(ldm)
    R, K = rows[:, None], kk[None, :]
    hi_rk = hi[(R >> 1) * 2 * ldm + 64 * (K >> 5) + (K & 31) + 32 * (R & 1)]
    lo_rk = lo8[(R >> 1) * 2 * ldm + 128 * (K >> 6) + 64 * (R & 1) + (K & 63)]
    assert np.all(np.abs(hi_rk - x) <= np.ldexp(np.abs(x), -11) + 2.0 ** -25)
    ref_lo = _e4m3_rne(np.ldexp(x - hi_rk, 18 - e).astype(np.float32))
    assert np.array_equal(lo_rk, ref_lo)
    # propagation
    mp.mp_propagate(M, E, p.T, "split1t_f8", p.ab, p.C, p.ws_prop)
    ag, bg = p.propagated(E)
    ao, bo = oest.propagate(T, a_s, b_s)
    norm = np.linalg.norm(ao, axis=1).max()
    snorm = max(np.linalg.norm(a_s, axis=1).max(), np.linalg.norm(b_s, axis=1).max())
    err = max(np.abs(ag - ao).max(), np.abs(bg - bo).max())
    print(f"split1t_f8 M={M} E={E}: max |error| {err:.2e} = {err / snorm:.2e} of the largest "
          f"sample norm (bound 2^-14 = {2.0 ** -14:.2e})")
    assert err <= 2.0 ** -14 * snorm + 4e-6 * norm


def test_split1t_f8_saturated_sample_copies():
    """Squeezing r = 7 on ten modes puts about 40 % of their amplitudes above
    448, e4m3's largest value (and far below FP16's 65504).  Their e4m3 copies
    saturate (the nearest-even rounding with saturation, as documented), the
    FP16 operand is unaffected, and the product stays finite: the correction
    term, at most 2^-11 of each entry's product, only loses the excess
    (|S| - 448)+, so by Cauchy-Schwarz over a row of T the error bound of the
    unsaturated case grows by at most 2^-11 of the norm of those excesses."""
    import paper_2503_12749_amd as mp
    M, E = 300, 201
    T = 0.95 * synth.haar_unitary(M, 13)
    r = np.full(M, 0.8)
    r[:10] = 7.0
    ldm = mp.mp_ld_modes(M)
    e2 = E + (E & 1)
    p = _pipe(T, r, prec="split1t_f8", seed=6, windows=[(0, 64)], n_sub=1, samples_per_sub=E,
              chunk=E)
    mp.mp_sample(M, 0, E, p.r, p.seed, 0, "split1t_f8", p.ab, p.n)
    a_s, b_s = p.alpha_beta(E)
    assert np.isfinite(a_s).all() and np.isfinite(b_s).all()
    over = (np.abs(a_s) > 448).sum() + (np.abs(b_s) > 448).sum()
    assert over > 200
    raw = p.ab.view(torch.uint8).cpu().numpy()
    b8 = raw[4 * e2 * ldm:]
    j = np.arange(M)

    def codes(c):
        c = np.asarray(c)[:, None]
        return b8[(c >> 1) * 2 * ldm + 128 * (j >> 6) + 64 * (c & 1) + (j & 63)]

    ca, cb = codes(np.arange(E)), codes(e2 + np.arange(E))
    assert np.array_equal(ca, _e4m3_rne(a_s)) and np.array_equal(cb, _e4m3_rne(b_s))
    assert set(np.unique(ca[np.abs(a_s) > 448] & 0x7F)) == {0x7E}
    mp.mp_propagate(M, E, p.T, "split1t_f8", p.ab, p.C, p.ws_prop)
    ag, bg = p.propagated(E)
    assert np.isfinite(ag).all() and np.isfinite(bg).all()
    ao, bo = oest.propagate(T, a_s, b_s)
    norm = np.linalg.norm(ao, axis=1).max()
    snorm = max(np.linalg.norm(a_s, axis=1).max(), np.linalg.norm(b_s, axis=1).max())
    excess = max(np.linalg.norm(np.maximum(np.abs(a_s) - 448, 0), axis=1).max(),
                 np.linalg.norm(np.maximum(np.abs(b_s) - 448, 0), axis=1).max())
    err = max(np.abs(ag - ao).max(), np.abs(bg - bo).max())
    bound = 2.0 ** -14 * snorm + 2.0 ** -11 * excess + 4e-6 * norm
    print(f"saturated e4m3 copies: max |error| {err:.3e}, bound {bound:.3e} "
          f"(excess norm {excess:.1f}, sample norm {snorm:.1f})")
    assert err <= bound


@pytest.mark.parametrize("prec", ["fp64", "fp32", "split_bf16", "split_fp16", "split1_fp16",
                                  "split1t_fp16", "split1t_f8"])
def test_pack_once_then_propagate_matches_propagate(prec):
    """mp_pack_transmission + mp_propagate_packed give the same bits as
    mp_propagate, over several tiles with ragged edges."""
    import paper_2503_12749_amd as mp
    M, E = 333, 301
    T = 0.9 * synth.haar_unitary(M, 19)
    r = np.linspace(0.5, 1.5, M)
    p = _pipe(T, r, prec=prec, seed=8, windows=[(0, 64)], n_sub=1, samples_per_sub=E, chunk=E)
    mp.mp_sample(M, 0, E, p.r, p.seed, 0, prec, p.ab, p.n)
    mp.mp_propagate(M, E, p.T, prec, p.ab, p.C, p.ws_prop)
    ref = p.C.clone()
    p.C.zero_()
    ws = torch.empty_like(p.ws_prop)
    mp.mp_pack_transmission(M, p.T, prec, ws)
    mp.mp_propagate_packed(M, E, prec, p.ab, p.C, ws)
    torch.cuda.synchronize()
    assert torch.equal(p.C, ref)


def test_sampler_fp32_matches_oracle():
    """The FP32 path draws the same noise and evaluates the Box-Muller radius
    and angle in FP32: each amplitude within 5e-7 of the scale of its terms
    (FP32 rounding of the coefficients and the products, a radius within a few
    FP32 ulps, an angle error of ~1e-7 rad times the radius), and n equal to
    the sum over the stored values.  E = 261 leaves a ragged group of
    samples."""
    import paper_2503_12749_amd as mp
    r = np.concatenate([np.linspace(0.2, 1.5, 139), [0.0]])
    M = r.size
    p = _pipe(np.eye(M, dtype=np.complex128), r, prec="fp32", seed=77, windows=[(0, 64)],
              n_sub=1, samples_per_sub=1000, chunk=300)
    g0, E = 5, 261
    mp.mp_sample(M, g0, E, p.r, p.seed, 2, "fp32", p.ab, p.n)
    a_gpu, b_gpu = p.alpha_beta(E)
    a, b, _ = osamp.sample(r, g0, E, 77, net=2)
    w1, w2 = osamp.normals(M, g0, E, 77, net=2)
    cp = np.sqrt(np.expm1(2 * r)) / 2
    cm = np.sqrt(-np.expm1(-2 * r)) / 2
    rho = np.hypot(w1, w2)
    tol = 5e-7 * (cp * np.abs(w1) + cm * np.abs(w2) + (cp + cm) * rho)
    assert np.all(np.abs(a_gpu - a) <= tol)
    assert np.all(np.abs(b_gpu - b) <= tol)
    n_gpu = p.n[:E].cpu().numpy()
    np.testing.assert_allclose(n_gpu, (a_gpu * b_gpu).sum(1), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_sampler_rounding_unbiased(prec):
    """The FP32 and split samplers round the FP64 Box-Muller values once, so
    on the same noise their mean of alpha^2, beta^2 and n = alpha beta over
    M = 4000 modes x 16384 samples equals the FP64 sampler's (itself equal to
    the oracle's to 1e-14) to 1e-8 relative.  Rounding errors average to
    ~1e-11 here; what remains is the FP32 rounding of the per-mode
    coefficients (~1e-9).  A biased FP32 logarithm in the radius moved these
    means by 3.7e-8."""
    import paper_2503_12749_amd as mp
    M, E, seed = 4000, 16384, 1234
    r = np.random.default_rng(5).uniform(0.5, 1.5, M)
    ldm = mp.mp_ld_modes(M)
    rd = torch.tensor(r, dtype=torch.float64, device="cuda:0")
    sums = {}
    for pr in ("fp64", prec):
        ab = torch.empty(mp.mp_ab_bytes(M, E, pr), dtype=torch.uint8, device="cuda:0")
        n = torch.empty(E, dtype=torch.float64, device="cuda:0")
        mp.mp_sample(M, 0, E, rd, seed, 0, pr, ab, n)
        if pr == "split_bf16":
            v = ab.view(torch.int16)[: 2 * ldm * 2 * E].reshape(2 * E, ldm // 32, 2, 32)
            hi = (v[:, :, 0, :].to(torch.int32) << 16).view(torch.float32).double()
            lo = (v[:, :, 1, :].to(torch.int32) << 16).view(torch.float32).double()
            v = (hi + lo).reshape(2 * E, ldm)[:, :M]
        else:
            dt = torch.float64 if pr == "fp64" else torch.float32
            v = ab.view(dt)[: ldm * 2 * E].reshape(2 * E, ldm)[:, :M].double()
        a, b = v[:E], v[E:]
        sums[pr] = ((a * a).sum().item(), (b * b).sum().item(), n.sum().item())
        del ab, n, v, a, b
    for got, ref in zip(sums[prec], sums["fp64"]):
        assert abs(got - ref) <= 1e-8 * abs(ref), (got, ref, (got - ref) / ref)


@pytest.mark.parametrize("prec,floor", [("fp32", 1e-7), ("split_bf16", 1e-6), ("split_fp16", 1e-6),
                                        ("split1_fp16", 1e-6), ("split1t_fp16", 1e-6),
                                        ("split1t_f8", 1e-6)])
def test_reduced_precision_counts_within_sigma(prec, floor):
    """M = 300, t = 0.9, r = 1: the reduced-precision estimate differs from the
    FP64 oracle on the same noise by far less than sigma_T.  Besides the
    operand rounding, the FP32 evaluation of chi (relative error ~1e-7 per
    term) leaves an absolute floor of order 1e-8 * max P on every bin, tails
    included."""
    M = 300
    T = 0.9 * synth.haar_unitary(M, 44)
    r = np.full(M, 1.0)
    mean, sd = synth.uniform_loss_moments(r, 0.9)
    win = [synth.count_window(mean, sd)]
    p = _pipe(T, r, prec=prec, seed=6, windows=win, n_sub=8, samples_per_sub=500, chunk=4000)
    p.run()
    P, _, s = p.result()
    ref = _oracle(T, r, 6, 4000, 8, np.zeros(M, int), 1, win)
    err = np.abs(P - ref["P"])
    print(f"{prec}: max |dP| = {err.max():.3e}, max |dP|/sigma over the bulk = "
          f"{(err / ref['sigma'])[ref['P'] > 1e-3 * ref['P'].max()].max():.3e}")
    assert np.all(err <= 0.05 * ref["sigma"] + floor * ref["P"].max())


def test_joint_two_bins_lossless_fp64():
    """Joint counts of two bins of a lossless network: both characteristic-
    function bands (around theta = 0 and theta = pi) contribute; odd totals
    vanish."""
    M = 8
    U = synth.haar_unitary(M, 13)
    r = np.full(M, 0.5)
    bins = np.array([0] * 4 + [1] * 4, dtype=np.int32)
    wins = [(0, 32), (0, 32)]
    p = _pipe(U, r, prec="fp64", seed=21, bin_of_mode=bins, d=2, mode="joint", windows=wins,
              n_sub=4, samples_per_sub=500, chunk=2000)
    p.run()
    P, _, s = p.result()
    P = P.reshape(32, 32)
    ref = _oracle(U, r, 21, 2000, 4, bins, 2, wins)
    _p_close(P, ref["P"])
    odd = (np.add.outer(np.arange(32), np.arange(32)) % 2) == 1
    assert np.abs(P[odd]).max() < 1e-13


def test_joint_two_bins_lossy_offsets_fp64():
    """Lossy network, window offsets and aliasing, chunks across sub-ensembles."""
    M = 40
    T = 0.85 * synth.haar_unitary(M, 17)
    r = synth.squeezing_random_uniform(M, 0.4, 0.9, 17)
    bins = np.array([0] * 20 + [1] * 20, dtype=np.int32)
    wins = [(3, 48), (1, 40)]
    p = _pipe(T, r, prec="fp64", seed=23, bin_of_mode=bins, d=2, mode="joint", windows=wins,
              n_sub=5, samples_per_sub=400, chunk=700)
    p.run()
    P, _, s = p.result()
    P = P.reshape(48, 40)
    full = _oracle(T, r, 23, 2000, 5, bins, 2, [(0, 96), (0, 96)])
    ref = np.zeros((48, 40))
    m = np.arange(96)
    np.add.at(ref, ((m[:, None] - 3) % 48, (m[None, :] - 1) % 40), full["P"])
    _p_close(P, ref)
    # sigma_T of the folded cells from the oracle's folded sub-ensemble estimates
    Ps = np.zeros((5, 48, 40))
    for k in range(5):
        np.add.at(Ps[k], ((m[:, None] - 3) % 48, (m[None, :] - 1) % 40), full["Ps"][k].real)
    sref = Ps.std(axis=0, ddof=1) / np.sqrt(5)
    np.testing.assert_allclose(s.reshape(48, 40), sref, rtol=1e-6, atol=1e-13 * ref.max())


def test_joint_m1000_fp32_subwindow():
    """Two halves of a 1000-mode network (Haar x 0.9, r = 1), FP32 path, the
    K = 768 windows of the two-bin workload; checked on a 40 x 40 block around
    the peak against the oracle on the same noise."""
    M = 1000
    T = 0.9 * synth.haar_unitary(M, synth.SEED_BASE + 1)
    r = np.full(M, 1.0)
    bins = synth.contiguous_bins(M, 2)
    mean, sd = synth.uniform_loss_moments(r, 0.9, frac=0.5)
    w = synth.count_window(mean, sd, nsig=9.0)
    wins = [w, w]
    E, nsub = 4096, 4
    p = _pipe(T, r, prec="fp32", seed=synth.SEED_BASE + 1, bin_of_mode=bins, d=2, mode="joint",
              windows=wins, n_sub=nsub, samples_per_sub=E // nsub, chunk=E)
    p.run()
    P, _, s = p.result()
    K = w[1]
    P = P.reshape(K, K)
    c = int(round(mean))
    blk = np.arange(c - 20, c + 20)
    ref = _oracle(T, r, synth.SEED_BASE + 1, E, nsub, bins, 2, [(c - 20, 40), (c - 20, 40)])
    got = P[np.ix_(blk - w[0], blk - w[0])]
    err = np.abs(got - ref["P"])
    print(f"joint m1000 fp32: max|dP| = {err.max():.3e}, max sigma = {ref['sigma'].max():.3e}")
    assert np.all(err <= 0.05 * ref["sigma"] + 1e-7 * ref["P"].max())
    assert abs(P.sum() - 1) < 1e-6
