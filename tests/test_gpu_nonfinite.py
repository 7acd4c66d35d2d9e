"""Non-finite values are reported, never absorbed.  mp_check_finite counts NaN
and infinite entries on the device.  Samples whose FP16 amplitudes overflow
(squeezing far beyond FP16's range: r = 12 gives amplitudes near 8e4 against
FP16's 65504) make the estimate NaN on every counting path: totals, marginals,
joint d = 2 and d = 3, both estimators, unfused and occupation-fused.  result()
therefore raises MP_ERR_NONFINITE instead of returning a finite but wrong P(m),
and so do a batched plan's result for that network (only) and the pair
moments.  Per-sample moments and histograms carry such samples as NaN, or in
the histogram's non-finite bin."""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NONFINITE = -6
M, E_TOTAL, CHUNK, N_SUB = 96, 512, 256, 4
FP16_FORMS = ["split_fp16", "split1_fp16", "split1t_fp16", "split1t_f8"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_12749_amd  # noqa: F401
    yield


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("n", [1, 255, 256, 257, 100_003, (1 << 20) + 5])
def test_check_finite_counts_nan_and_inf(n):
    import paper_2503_12749_amd as mp
    from paper_2503_12749_amd import _lib
    lib = _lib.load()
    rng = np.random.default_rng(1000 + n)
    x = rng.standard_normal(n)
    # finite extremes, which must not count
    for v in (np.finfo(np.float64).max, -np.finfo(np.float64).max, 5e-324, -0.0):
        x[rng.integers(0, n)] = v
    scratch = torch.empty(1, dtype=torch.int64, device=DEV)
    bad = ctypes.c_int64(-1)
    t = torch.from_numpy(x).to(DEV)
    assert lib.mp_check_finite(_vp(t), n, _vp(scratch), ctypes.byref(bad), None) == 0
    assert bad.value == 0
    idx = sorted(set(rng.choice(n, size=min(n, 9), replace=False).tolist()) | {0, n - 1})
    for i, j in enumerate(idx):
        x[j] = (np.nan, np.inf, -np.inf)[i % 3]
    t = torch.from_numpy(x).to(DEV)
    assert lib.mp_check_finite(_vp(t), n, _vp(scratch), ctypes.byref(bad), None) == NONFINITE
    assert bad.value == np.count_nonzero(~np.isfinite(x)) == len(idx)
    with pytest.raises(mp.MPError) as e:
        mp.mp_check_finite(t, scratch)
    assert e.value.status == NONFINITE


def _layout(name):
    """(d, mode, bin_of_mode, windows): a total, two marginals, joint d = 2, 3."""
    if name == "total":
        return 1, "joint", np.zeros(M, np.int32), [(0, 64)]
    d = 2 if name in ("marginals", "joint2") else 3
    bins = (np.arange(M) * d // M).astype(np.int32)
    mode = "marginals" if name == "marginals" else "joint"
    return d, mode, bins, [(0, 48 if d == 2 else 16)] * d


def _run(prec, layout, est, fused, r_big):
    import paper_2503_12749_amd as mp
    d, mode, bins, windows = _layout(layout)
    T = 0.9 * synth.haar_unitary(M, 7)
    r = np.ones(M)
    r[:4] = r_big  # the first bin's first modes
    p = mp.CountsPipeline(T, r, prec=prec, seed=4242, bin_of_mode=bins, d=d, mode=mode,
                          windows=windows, n_sub=N_SUB, samples_per_sub=E_TOTAL // N_SUB,
                          chunk=CHUNK, est=est, device=DEV, fused=fused)
    p.run()
    return mp, p


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("layout", ["total", "marginals", "joint2", "joint3"])
@pytest.mark.parametrize("prec", FP16_FORMS)
def test_fp16_overflow_is_reported(prec, layout, fused):
    mp, p = _run(prec, layout, "matrix_p", fused, 12.0)
    with pytest.raises(mp.MPError) as e:
        p.result()
    assert e.value.status == NONFINITE


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("layout", ["total", "marginals", "joint2", "joint3"])
def test_fp16_overflow_is_reported_plus_p(layout, fused):
    mp, p = _run("split1t_f8", layout, "plus_p", fused, 12.0)
    with pytest.raises(mp.MPError) as e:
        p.result()
    assert e.value.status == NONFINITE


@pytest.mark.parametrize("est", ["matrix_p", "plus_p"])
def test_fp16_overflow_is_reported_bilinear(est):
    """The bilinear form (one distribution): overflowing amplitudes reach its
    epilogue's sums as NaN, and result() raises."""
    import paper_2503_12749_amd as mp
    T = 0.9 * synth.haar_unitary(M, 7)
    r = np.ones(M)
    r[:4] = 12.0
    p = mp.CountsPipeline(T, r, prec="split1t_f8", seed=4242, windows=[(0, 64)], n_sub=N_SUB,
                          samples_per_sub=E_TOTAL // N_SUB, chunk=CHUNK, est=est, device=DEV,
                          bilinear=True)
    p.run()
    with pytest.raises(mp.MPError) as e:
        p.result()
    assert e.value.status == NONFINITE


@pytest.mark.parametrize("layout", ["total", "joint2", "joint3"])
def test_in_range_squeezing_stays_finite(layout):
    """Control: the same networks at r = 1 give a finite estimate."""
    _, p = _run("split1t_f8", layout, "matrix_p", True, 1.0)
    P, _, s = p.result()
    assert np.isfinite(P).all() and np.isfinite(s).all()


@pytest.mark.parametrize("est", ["matrix_p", "plus_p"])
def test_overflowing_samples_reach_moments_and_histogram(est):
    """Moments of the overflowing chunk are NaN; in the histogram of a count
    observable every sample whose n or occupation is not finite lands in the
    top (not finite) bin, and the rest are binned as usual."""
    import paper_2503_12749_amd as mp
    _, p = _run("split1t_fp16", "total", "matrix_p", False, 12.0)
    E = CHUNK
    p.run_chunk(0, E)  # C and n of samples [0, 256)
    nq = torch.empty(E * 2, dtype=torch.float64, device=DEV)
    allm = np.zeros(M, dtype=np.int32)
    mp.mp_occupations(M, E, p.C, p.prec, 1, allm, "marginals", nq)
    n = p.n[:E].cpu().numpy()
    z = nq.cpu().numpy().reshape(E, 2)
    bad = ~np.isfinite(z).all(axis=1)
    if est == "matrix_p":
        bad |= ~np.isfinite(n)
    assert 0 < bad.sum() < E
    kmax = 3
    acc = torch.zeros(kmax * 2, dtype=torch.float64, device=DEV)
    mp.mp_moments_accumulate(E, p.n, nq, 1, kmax, est, 1, E, 0, acc)
    assert not np.isfinite(acc.cpu().numpy()).any()
    n_bins = 10
    hist = torch.zeros(n_bins + 2, dtype=torch.float64, device=DEV)
    mp.mp_observable_histogram(E, p.n, nq, 1, 0, 2, est, -1.0, 0.2, n_bins, 1, E, 0, hist)
    h = hist.cpu().numpy()
    assert h.sum() == E
    assert h[-1] >= bad.sum()


def test_plan_reports_overflow_of_one_network_only():
    """A batched plan: the network whose FP16 amplitudes overflow raises
    MP_ERR_NONFINITE from result(); the other network's estimate is finite."""
    import paper_2503_12749_amd as mp
    nets = []
    for i, (Mi, r_big) in enumerate(((60, 1.0), (130, 12.0))):
        r = np.ones(Mi)
        r[:4] = r_big
        mean, sd = synth.uniform_loss_moments(np.ones(Mi), 0.9)
        nets.append(dict(T=synth.transmission(Mi, 0.9, 77 + i), r=r, seed=77, net=i, E=1024,
                         n_sub=4, window=synth.count_window(mean, sd)))
    plan = mp.Plan(nets, prec="split1t_f8")
    plan.launch()
    P, _, s = plan.result(0)
    assert np.isfinite(P).all() and np.isfinite(s).all() and abs(P.sum() - 1) < 1e-6
    with pytest.raises(mp.MPError) as e:
        plan.result(1)
    assert e.value.status == NONFINITE


@pytest.mark.parametrize("r_big,raises", [(12.0, True), (1.0, False)])
def test_pair_moments_report_overflow(r_big, raises):
    import paper_2503_12749_amd as mp
    Mi = 70
    r = np.full(Mi, 0.8)
    r[:3] = r_big
    p = mp.PairPipeline(0.9 * synth.haar_unitary(Mi, 5), r, prec="split_fp16", seed=9, n_sub=2,
                        samples_per_sub=256, chunk=512, device=DEV)
    p.run()
    if raises:
        with pytest.raises(mp.MPError) as e:
            p.result()
        assert e.value.status == NONFINITE
    else:
        G2, s = p.result()
        assert np.isfinite(G2).all() and np.isfinite(s).all()
