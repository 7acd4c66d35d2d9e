"""The occupation-fused GEMM path (mp_propagate_counts) against the unfused
path (mp_propagate_packed + mp_binned_counts) on the same noise, and against
the FP64 oracle.  The fused path sums the occupations in FP32 within a
128-mode block and in FP64 across blocks instead of in FP64 per mode, so the
two agree to FP32 rounding: far inside sigma_T."""
import numpy as np
import pytest

import synth
from oracle import estimator as oest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_12749_amd  # noqa: F401
    yield


def _bins(M):
    """Three bins whose runs cross 128-mode blocks; bin 1 has two runs; a tail
    of uncounted modes."""
    b = np.full(M, -1, dtype=np.int32)
    b[0:100] = 0
    b[100:180] = 1
    b[260:300] = 1
    b[180:260] = 2
    return b


def _run(fused, prec, est, M=333, E=1000, n_sub=5, chunk=384, seed=71, t=0.9):
    import paper_2503_12749_amd as mp
    T = t * synth.haar_unitary(M, seed)
    r = np.linspace(0.4, 1.2, M)
    bins = _bins(M)
    N = np.sinh(r) ** 2
    wins = []
    for b in range(3):
        mb = t * t * N[bins == b].sum()
        sb = np.sqrt(mb + (t * t) ** 2 * (N[bins == b] * (2 * N[bins == b] + 1)).sum())
        wins.append(synth.count_window(mb, 1.5 * sb))
    mt, st = synth.uniform_loss_moments(r[bins >= 0], t)
    wins.append(synth.count_window(mt, 1.5 * st))
    p = mp.CountsPipeline(T, r, prec=prec, seed=seed, bin_of_mode=bins, d=3,
                          mode="marginals_and_total", windows=wins, n_sub=n_sub,
                          samples_per_sub=E // n_sub, chunk=chunk, est=est, device=DEV,
                          fused=fused)
    p.run()
    P, Pi, s = p.result()
    return P, s, T, r, bins, wins


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16", "split1_fp16", "split1t_fp16",
                                  "split1t_f8"])
@pytest.mark.parametrize("est", ["matrix_p", "plus_p"])
def test_fused_equals_unfused(prec, est):
    Pf, sf, *_ = _run(True, prec, est)
    Pu, su, *_ = _run(False, prec, est)
    scale = np.abs(Pu).max()
    assert np.all(np.abs(Pf - Pu) <= 1e-3 * su + 1e-6 * scale), np.abs(Pf - Pu).max()
    np.testing.assert_allclose(sf, su, rtol=1e-3, atol=1e-6 * scale)


def _run_joint(fused, prec, est, d, M=333, E=1000, n_sub=5, chunk=384, seed=73, t=0.9):
    """Joint distribution of the first d bins of _bins (d = 2: bin 2 uncounted)."""
    import paper_2503_12749_amd as mp
    T = t * synth.haar_unitary(M, seed)
    r = np.linspace(0.4, 1.2, M)
    bins = _bins(M)
    bins[bins >= d] = -1
    N = np.sinh(r) ** 2
    wins = []
    for b in range(d):
        mb = t * t * N[bins == b].sum()
        sb = np.sqrt(mb + (t * t) ** 2 * (N[bins == b] * (2 * N[bins == b] + 1)).sum())
        m_lo, K = synth.count_window(mb, 1.5 * sb)
        wins.append((m_lo, min(K, 256)))
    p = mp.CountsPipeline(T, r, prec=prec, seed=seed, bin_of_mode=bins, d=d, mode="joint",
                          windows=wins, n_sub=n_sub, samples_per_sub=E // n_sub, chunk=chunk,
                          est=est, device=DEV, fused=fused)
    p.run()
    P, Pi, s = p.result()
    return P, s


@pytest.mark.parametrize("prec,est,d", [("fp32", "matrix_p", 2), ("split_bf16", "matrix_p", 2),
                                        ("fp32", "plus_p", 2), ("fp32", "matrix_p", 3),
                                        ("split_bf16", "matrix_p", 3), ("split1t_f8", "matrix_p", 2),
                                        ("split1t_f8", "matrix_p", 3)])
def test_fused_joint_equals_unfused(prec, est, d):
    """Joint distributions of two and three bins through mp_propagate_counts:
    the bin sums come from the GEMM's partials instead of C, the rest of the
    joint path is shared, so the two agree to FP32 rounding (three chunks, one
    of them ragged)."""
    Pf, sf = _run_joint(True, prec, est, d)
    Pu, su = _run_joint(False, prec, est, d)
    scale = np.abs(Pu).max()
    assert abs(Pf.sum() - 1) < 1e-6
    assert np.all(np.abs(Pf - Pu) <= 1e-3 * su + 1e-6 * scale), np.abs(Pf - Pu).max()
    np.testing.assert_allclose(sf, su, rtol=1e-3, atol=1e-6 * scale)


def test_split1t_odd_chunks_fused_equals_unfused():
    """The T-split form in chunks of odd length (333, 333, 333 and 2 samples:
    padded column pairs in every chunk), marginals of three bins and the
    total: fused and unfused agree, and both stay far inside sigma_T of the
    FP64 oracle."""
    import paper_2503_12749_amd as mp
    M, E, n_sub = 300, 1001, 7
    T = 0.9 * synth.haar_unitary(M, 91)
    r = np.linspace(0.4, 1.2, M)
    bins = _bins(M)
    N = np.sinh(r) ** 2
    wins = []
    for b in range(3):
        mb = 0.81 * N[bins == b].sum()
        sb = np.sqrt(mb + 0.6561 * (N[bins == b] * (2 * N[bins == b] + 1)).sum())
        wins.append(synth.count_window(mb, 1.5 * sb))
    mt = 0.81 * N[bins >= 0].sum()
    st = np.sqrt(mt + 0.6561 * (N[bins >= 0] * (2 * N[bins >= 0] + 1)).sum())
    wins.append(synth.count_window(mt, 1.5 * st))
    out = []
    for fused in (True, False):
        p = mp.CountsPipeline(T, r, prec="split1t_fp16", seed=29, bin_of_mode=bins, d=3,
                              mode="marginals_and_total", windows=wins, n_sub=n_sub,
                              samples_per_sub=E // n_sub, chunk=333, device=DEV, fused=fused)
        p.run()
        out.append(p.result())
    (Pf, _, sf), (Pu, _, su) = out
    scale = np.abs(Pu).max()
    assert np.all(np.abs(Pf - Pu) <= 1e-3 * su + 1e-6 * scale), np.abs(Pf - Pu).max()
    mar = oest.estimate(T, r, 29, E, n_sub, bins, 3, wins[:3], mode="marginals", chunk=500)
    tot = oest.estimate(T, r, 29, E, n_sub, np.where(bins >= 0, 0, -1), 1, wins[3:], mode="joint",
                        chunk=500)
    off = 0
    for q in range(4):
        K = wins[q][1]
        Pr, sr = (mar["P"][q, :K], mar["sigma"][q, :K]) if q < 3 else (tot["P"], tot["sigma"])
        for P in (Pf, Pu):
            assert np.all(np.abs(P[off: off + K] - Pr) <= 0.05 * sr + 1e-6 * np.abs(Pr).max()), q
        off += K


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split1_fp16", "split1t_fp16", "split1t_f8"])
@pytest.mark.parametrize("M,E", [(1, 1), (1, 3), (5, 1), (5, 3)])
def test_tiny_chunks_fused_and_unfused(prec, M, E):
    """One mode or five, one sample or three (a single ragged tile, the
    T-split form's padded column pair, n often negative): fused and unfused
    agree to FP32 rounding, and both give the oracle's per-sample G(m) to the
    precision's rounding (the operands' 2^-11 to 2^-22 relative, times counts
    up to 31 in the exponent: within 2 % of max |P|)."""
    import paper_2503_12749_amd as mp
    rng = np.random.default_rng(M * 10 + E)
    T = 0.8 * synth.haar_unitary(M, 7) if M > 1 else np.array([[0.7 * np.exp(0.4j)]])
    r = rng.uniform(0.4, 1.2, M)
    out = []
    for fused in (True, False):
        p = mp.CountsPipeline(T, r, prec=prec, seed=13, windows=[(0, 32)], n_sub=1,
                              samples_per_sub=E, chunk=E, device=DEV, fused=fused)
        p.run()
        out.append(p.result()[0])
    ref = oest.estimate(T, r, 13, E, 1, np.zeros(M, int), 1, [(0, 32)], chunk=E)["P"]
    scale = np.abs(ref).max()
    assert np.all(np.abs(out[0] - out[1]) <= 1e-4 * scale), np.abs(out[0] - out[1]).max()
    for P in out:
        assert np.all(np.isfinite(P))
        assert np.abs(P - ref).max() <= 2e-2 * scale, np.abs(P - ref).max() / scale


def test_fused_matches_oracle():
    """Split-BF16 fused run against the FP64 oracle on the same noise, per
    distribution (three bin marginals and the total): far inside sigma_T."""
    P, s, T, r, bins, wins = _run(True, "split_bf16", "matrix_p")
    mar = oest.estimate(T, r, 71, 1000, 5, bins, 3, wins[:3], mode="marginals", chunk=500)
    tot = oest.estimate(T, r, 71, 1000, 5, np.where(bins >= 0, 0, -1), 1, wins[3:], mode="joint",
                        chunk=500)
    off = 0
    for q in range(4):
        K = wins[q][1]
        if q < 3:
            Pr, sr = mar["P"][q, :K], mar["sigma"][q, :K]
        else:
            Pr, sr = tot["P"], tot["sigma"]
        got = P[off: off + K]
        assert np.all(np.abs(got - Pr) <= 0.05 * sr + 1e-6 * np.abs(Pr).max()), q
        off += K


def test_full_size_m4000_fused_equals_unfused():
    """M = 4000 (32 blocks of 128 modes), one chunk of 65536 samples over 8
    sub-ensembles, total counts: fused and unfused split-BF16 agree."""
    import paper_2503_12749_amd as mp
    M, t, E, n_sub = 4000, 0.95, 65536, 8
    T = t * synth.haar_unitary(M, 5)
    r = np.full(M, 1.0)
    mean, sd = synth.uniform_loss_moments(r, t)
    win = synth.count_window(mean, sd)
    out = []
    for fused in (True, False):
        p = mp.CountsPipeline(T, r, prec="split_bf16", seed=9, windows=[win], n_sub=n_sub,
                              samples_per_sub=E // n_sub, chunk=E, device=DEV, fused=fused)
        p.run()
        out.append(p.result())
        del p
        torch.cuda.empty_cache()
    (Pf, _, sf), (Pu, _, su) = out
    assert np.all(np.abs(Pf - Pu) <= 1e-3 * su + 1e-7 * Pu.max()), np.abs(Pf - Pu).max()


def test_fused_rejects_unsupported_cases():
    import paper_2503_12749_amd as mp
    with pytest.raises(mp.MPError):
        mp.CountsPipeline(np.eye(8, dtype=complex), np.ones(8), prec="fp64", seed=1,
                          windows=[(0, 64)], n_sub=1, samples_per_sub=64, chunk=64, device=DEV,
                          fused=True).run()
    # joint distributions of more than four bins exist on no path
    bins = np.array([0, 0, 1, 1, 2, 2, 3, 4], dtype=np.int32)
    with pytest.raises(mp.MPError):
        mp.CountsPipeline(np.eye(8, dtype=complex), np.ones(8), prec="fp32", seed=1, bin_of_mode=bins,
                          d=5, mode="joint", windows=[(0, 8)] * 5, n_sub=1,
                          samples_per_sub=64, chunk=64, device=DEV, fused=True).run()
