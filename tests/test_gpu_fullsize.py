"""Full-size checks at the workloads' real shapes and in the benchmark's launch
configuration (chunks of 65536 samples at M = 8000).  The oracle computes
sampled outputs one by one (single propagated samples), and whole-run
results are checked through properties that hold at any size: normalisation,
the closed-form mean and variance of the total count, the unitary invariant
n_S = t^2 n, and exact relations between the joint, marginal and total
distributions of the same noise.

Tolerances for sampled propagated columns are relative to the column norm:
2e-6 (FP32), 2e-5 (split BF16), 4e-6 (split FP16); see test_gpu_parity.
"""
import numpy as np
import pytest

import synth
from oracle import estimator as oest
from oracle import exact
from oracle import sampler as osamp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL = {"fp64": 1e-12, "fp32": 2e-6, "split_bf16": 2e-5, "split_fp16": 4e-6}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_12749_amd  # noqa: F401
    yield


@pytest.fixture(scope="module")
def m8000():
    return synth.workload_m8000(E=65536, chunk=65536)


def _release(*objs):
    for o in objs:
        del o
    torch.cuda.empty_cache()


def _sampled_columns(p, w, g0, E, cols):
    """GPU alpha', beta' of chunk-local samples `cols` vs the oracle's."""
    import paper_2503_12749_amd as mp
    ldm = mp.mp_ld_modes(w.M)
    dt = torch.float64 if p.prec == 0 else torch.float32
    Cv = p.C.view(dt)[: 2 * ldm * 2 * E].reshape(2 * E, 2 * ldm)
    worst = 0.0
    for k in cols:
        ca = Cv[k].double().cpu().numpy()
        cb = Cv[E + k].double().cpu().numpy()
        ag = ca[: w.M] + 1j * ca[ldm: ldm + w.M]
        bg = cb[: w.M] - 1j * cb[ldm: ldm + w.M]
        a, b, n = osamp.sample(w.r, g0 + k, 1, w.seed)
        ao, bo = oest.propagate(w.T, a, b)
        norm = np.linalg.norm(ao[0])
        worst = max(worst, np.abs(ag - ao[0]).max() / norm, np.abs(bg - bo[0]).max() / norm)
        # unitary invariant for T = t U
        nS = (ag * bg).sum()
        assert abs(nS - w.t ** 2 * n[0]) < 100 * REL[_name(p.prec)] * np.abs(ao[0] * bo[0]).sum()
    return worst


def _name(code):
    return {0: "fp64", 1: "fp32", 2: "split_bf16", 3: "split_fp16"}[code]


@pytest.mark.parametrize("prec", ["split_bf16", "fp32", "split_fp16"])
def test_m8000_bench_launch(m8000, prec):
    """M = 8000, t = 0.95, r = 1, one 65536-sample chunk through the unfused
    path (mp_propagate writing C, then the counting kernels reading C; the
    occupation-fused launch the benchmark times is compared with the oracle
    bin by bin in test_gpu_oracle_fullsize): sampled columns against the
    oracle, then the whole chunk's total-count distribution against the
    closed-form moments."""
    import paper_2503_12749_amd as mp
    w = m8000
    E = 65536
    p = mp.CountsPipeline(w.T, w.r, prec=prec, seed=w.seed, windows=w.windows, n_sub=8,
                          samples_per_sub=8192, chunk=E, device="cuda:0")
    mp.mp_sample(w.M, 0, E, p.r, w.seed, 0, prec, p.ab, p.n)
    mp.mp_propagate(w.M, E, p.T, prec, p.ab, p.C, p.ws_prop)
    rng = np.random.default_rng(1)
    cols = [0, 1, 4095, 32768, E - 1] + list(rng.integers(0, E, 5))
    worst = _sampled_columns(p, w, 0, E, cols)
    print(f"{prec}: worst sampled column error {worst:.2e}")
    assert worst < REL[prec]
    # n for the sampled samples
    ng = p.n.cpu().numpy()
    for k in cols[:5]:
        _, _, n = osamp.sample(w.r, k, 1, w.seed)
        assert abs(ng[k] - n[0]) < 1e3 * REL[prec] * abs(n[0]) + 1e-6
    p.counts_chunk(0, E)
    p.finalize()
    P, Pi, s = p.result()
    m = np.arange(w.windows[0][0], w.windows[0][0] + w.windows[0][1])
    N = np.sinh(w.r) ** 2
    mean_x = w.t ** 2 * N.sum()
    var_x = (w.t ** 2 * N + w.t ** 4 * N * (2 * N + 1)).sum()
    mean_g = (m * P).sum()
    var_g = ((m - mean_g) ** 2 * P).sum()
    tol_mean = 5 * (np.abs(m - mean_x) * s).sum()
    tol_var = 5 * ((m - mean_x) ** 2 * s).sum()
    print(f"{prec}: sum P - 1 = {P.sum() - 1:.2e}, mean {mean_g:.3f} vs {mean_x:.3f} (tol {tol_mean:.3f}),"
          f" var {var_g:.1f} vs {var_x:.1f} (tol {tol_var:.1f})")
    assert abs(P.sum() - 1) < 1e-8
    assert abs(mean_g - mean_x) < tol_mean
    assert abs(var_g - var_x) < tol_var
    assert np.abs(Pi).max() < 1e-6 * P.max()
    _release(p)


def test_m4000_precision_study_per_bin():
    """M = 4000, t = 0.95, r_j ~ U[0.5, 1.5], four equal mode blocks
    (marginals + total): the split-BF16 and split-FP16 estimates differ from
    the FP64 GPU path on the same noise by a small fraction of sigma_T in
    every bin, and the FP64 path's sampled columns match the oracle (the
    comparison with the oracle bin by bin is in test_gpu_oracle_fullsize)."""
    import paper_2503_12749_amd as mp
    M, t = 4000, 0.95
    seed = synth.SEED_BASE + 2
    r = synth.squeezing_random_uniform(M, 0.5, 1.5, seed)
    T = synth.transmission(M, t, seed)
    bins = synth.contiguous_bins(M, 4)
    N = np.sinh(r) ** 2
    wins = []
    for b in range(4):
        mb = t * t * N[bins == b].sum()
        sb = np.sqrt(mb + (t * t) ** 2 * (N[bins == b] * (2 * N[bins == b] + 1)).sum())
        wins.append(synth.count_window(mb, sb * 1.3))
    mt, st = synth.uniform_loss_moments(r, t)
    wins.append(synth.count_window(mt, st))
    E, nsub = 32768, 8
    res = {}
    w = synth.Workload("m4000", M, t, r, T, E, nsub, seed, bins, 4, wins, E)
    for prec in ("fp64", "split_bf16", "split_fp16"):
        p = mp.CountsPipeline(T, r, prec=prec, seed=seed, bin_of_mode=bins, d=4,
                              mode="marginals_and_total", windows=wins, n_sub=nsub,
                              samples_per_sub=E // nsub, chunk=E, device="cuda:0")
        mp.mp_sample(M, 0, E, p.r, seed, 0, prec, p.ab, p.n)
        mp.mp_propagate(M, E, p.T, prec, p.ab, p.C, p.ws_prop)
        if prec == "fp64":
            worst = _sampled_columns(p, w, 0, E, [0, 17, E - 1])
            assert worst < REL["fp64"]
        p.counts_chunk(0, E)
        p.finalize()
        res[prec] = p.result()
        _release(p)
    P64, _, s64 = res["fp64"]
    off = np.cumsum([0] + [k for _, k in wins])
    for prec in ("split_bf16", "split_fp16"):
        P, _, s = res[prec]
        for b in range(5):
            sl = slice(off[b], off[b + 1])
            err = np.abs(P[sl] - P64[sl])
            ratio = (err / np.maximum(s64[sl], 1e-300))[P64[sl] > 1e-3 * P64[sl].max()].max()
            print(f"{prec} bin {b}: max|P - P_fp64| = {err.max():.2e}, max ratio to sigma {ratio:.2e}")
            assert np.all(err <= 0.05 * s64[sl] + 1e-6 * P64[sl].max())
    # the marginal means add up to the total mean (exact per sample)
    mtot = 0.0
    for b in range(4):
        m = np.arange(wins[b][0], wins[b][0] + wins[b][1])
        mtot += (m * P64[off[b]:off[b + 1]]).sum()
    m = np.arange(wins[4][0], wins[4][0] + wins[4][1])
    assert abs(mtot - (m * P64[off[4]:]).sum()) < 1e-6 * mtot


def test_m1000_full_run_total_joint_consistency():
    """M = 1000, Haar x 0.9, r = 1, E = 1.2e6 in chunks of 1e5 (N_R = 120 x
    N_S = 1e4), FP32: the total-count run and the two-bin joint run on the
    same noise satisfy sum_{m1 + m2 = m} P_joint = P_total; the first
    sub-ensemble matches the oracle's."""
    import paper_2503_12749_amd as mp
    w = synth.workload_m1000()
    bins2 = synth.contiguous_bins(w.M, 2)
    mh, sh = synth.uniform_loss_moments(w.r, w.t, frac=0.5)
    wh = synth.count_window(mh, sh)
    p1 = mp.CountsPipeline(w.T, w.r, prec="fp32", seed=w.seed, windows=w.windows, n_sub=w.n_sub,
                           samples_per_sub=w.samples_per_sub, chunk=w.chunk, device="cuda:0")
    p1.run()
    Pt, _, st = p1.result()
    acc0 = p1.acc[: p1.entries * 2].cpu().numpy()
    _release(p1)
    p2 = mp.CountsPipeline(w.T, w.r, prec="fp32", seed=w.seed, bin_of_mode=bins2, d=2,
                           mode="joint", windows=[wh, wh], n_sub=w.n_sub,
                           samples_per_sub=w.samples_per_sub, chunk=w.chunk, device="cuda:0")
    p2.run()
    Pj, _, sj = p2.result()
    _release(p2)
    K = wh[1]
    Pj = Pj.reshape(K, K)
    m_tot = np.arange(w.windows[0][0], w.windows[0][0] + w.windows[0][1])
    diag = np.zeros_like(Pt)
    sums = np.add.outer(np.arange(K), np.arange(K)) + 2 * wh[0]
    ok = (sums >= m_tot[0]) & (sums <= m_tot[-1])
    np.add.at(diag, sums[ok] - m_tot[0], Pj[ok])
    err = np.abs(diag - Pt)
    print(f"m1000: max |sum_diag P_joint - P_total| = {err.max():.2e}, max sigma {st.max():.2e}")
    assert np.all(err <= 0.05 * st + 1e-7 * Pt.max())
    assert abs(Pt.sum() - 1) < 1e-8 and abs(Pj.sum() - 1) < 1e-6
    # first sub-ensemble: inverse DFT of its accumulator vs the oracle
    Kt = w.windows[0][1]
    chi = (acc0[0::2] + 1j * acc0[1::2]) / w.samples_per_sub
    P0 = np.fft.fft(chi).real / Kt
    ref = oest.estimate(w.T, w.r, w.seed, w.samples_per_sub, 1, w.bins, 1, w.windows, chunk=2500)
    s_ref = st * np.sqrt(w.n_sub)  # sd of one sub-ensemble estimate
    err0 = np.abs(P0 - ref["P"])
    print(f"m1000 sub-ensemble 0: max |dP| = {err0.max():.2e}, sd of one sub-ensemble {s_ref.max():.2e}")
    assert np.all(err0 <= 0.02 * s_ref + 1e-7 * ref["P"].max())


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_m8192_row_stride_without_prefetch(prec):
    """M = 8192: the operand rows lie a multiple of 32 KB apart, where the
    split kernels run their loop without the L2 prefetch.  T = t F D with F
    the unitary DFT matrix and D random phases (dense and unitary, cheap to
    build); one ragged chunk of E = 600 samples.  Sampled columns against the
    oracle, then the occupation-fused run against the unfused one on the same
    noise."""
    import types
    import paper_2503_12749_amd as mp
    M, t, E, n_sub = 8192, 0.9, 600, 2
    assert mp.mp_ld_modes(M) % 8192 == 0
    rng = np.random.default_rng(8192)
    j = np.arange(M)
    T = (t / np.sqrt(M)) * np.exp(-2j * np.pi * (np.outer(j, j) % M) / M)
    T *= np.exp(2j * np.pi * rng.random(M))[None, :]
    r = np.full(M, 0.5)
    mean, sd = synth.uniform_loss_moments(r, t)
    win = synth.count_window(mean, sd)
    w = types.SimpleNamespace(M=M, t=t, T=T, r=r, seed=31)
    p = mp.CountsPipeline(T, r, prec=prec, seed=w.seed, windows=[win], n_sub=n_sub,
                          samples_per_sub=E // n_sub, chunk=E, device="cuda:0")
    mp.mp_sample(M, 0, E, p.r, w.seed, 0, prec, p.ab, p.n)
    mp.mp_propagate(M, E, p.T, prec, p.ab, p.C, p.ws_prop)
    cols = [0, 1, 255, 256, 299, 300, 511, E - 1]
    worst = _sampled_columns(p, w, 0, E, cols)
    print(f"{prec} M=8192: worst sampled column error {worst:.2e}")
    assert worst < REL[prec]
    _release(p)
    out = []
    for fused in (True, False):
        q = mp.CountsPipeline(T, r, prec=prec, seed=w.seed, windows=[win], n_sub=n_sub,
                              samples_per_sub=E // n_sub, chunk=E, device="cuda:0", fused=fused)
        q.run()
        out.append(q.result())
        _release(q)
    (Pf, _, sf), (Pu, _, su) = out
    assert abs(Pf.sum() - 1) < 1e-8
    assert np.all(np.abs(Pf - Pu) <= 1e-3 * su + 1e-7 * Pu.max()), np.abs(Pf - Pu).max()


@pytest.mark.parametrize("prec", ["split1t_fp16", "split1t_f8"])
def test_m8192_pair_forms_without_prefetch(prec):
    """The two T-split forms at M = 8192, where they too run their loop
    without the L2 prefetch (same network and ragged chunk as above).
    Sampled columns of the C-writing GEMM against the oracle propagating the
    stored (FP16-rounded) samples through the exact network: the T-split FP16
    form within 4e-6 of the propagated norm (the split's 2^-22 and FP32
    accumulation), the FP8-correction form within 2^-14 of the largest sample
    norm plus that (the bound its parity test derives); then the
    occupation-fused run against the unfused one on the same noise."""
    import paper_2503_12749_amd as mp
    M, t, E, n_sub = 8192, 0.9, 600, 2
    assert mp.mp_ld_modes(M) % 8192 == 0
    rng = np.random.default_rng(8192)
    j = np.arange(M)
    T = (t / np.sqrt(M)) * np.exp(-2j * np.pi * (np.outer(j, j) % M) / M)
    T *= np.exp(2j * np.pi * rng.random(M))[None, :]
    r = np.full(M, 0.5)
    win = synth.count_window(*synth.uniform_loss_moments(r, t))
    p = mp.CountsPipeline(T, r, prec=prec, seed=31, windows=[win], n_sub=n_sub,
                          samples_per_sub=E // n_sub, chunk=E, device="cuda:0")
    mp.mp_sample(M, 0, E, p.r, 31, 0, prec, p.ab, p.n)
    mp.mp_propagate(M, E, p.T, prec, p.ab, p.C, p.ws_prop)
    a_s, b_s = p.alpha_beta(E)
    ag, bg = p.propagated(E)
    cols = [0, 1, 255, 256, 299, 300, 511, E - 1]
    ao, bo = oest.propagate(T, a_s[cols], b_s[cols])
    norm = np.linalg.norm(ao, axis=1).max()
    snorm = max(np.linalg.norm(a_s[cols], axis=1).max(), np.linalg.norm(b_s[cols], axis=1).max())
    err = max(np.abs(ag[cols] - ao).max(), np.abs(bg[cols] - bo).max())
    bound = 4e-6 * norm + (2.0 ** -14 * snorm if prec == "split1t_f8" else 0.0)
    print(f"{prec} M=8192: worst sampled column error {err:.2e} (bound {bound:.2e})")
    assert err <= bound
    _release(p)
    out = []
    for fused in (True, False):
        q = mp.CountsPipeline(T, r, prec=prec, seed=31, windows=[win], n_sub=n_sub,
                              samples_per_sub=E // n_sub, chunk=E, device="cuda:0", fused=fused)
        q.run()
        out.append(q.result())
        _release(q)
    (Pf, _, sf), (Pu, _, su) = out
    assert abs(Pf.sum() - 1) < 1e-8
    assert np.all(np.abs(Pf - Pu) <= 1e-3 * su + 1e-7 * Pu.max()), np.abs(Pf - Pu).max()


@pytest.mark.parametrize("prec", ["split1t_f8", "split_bf16", "fp32"])
def test_m8000_chunk_beyond_4gib(m8000, prec):
    """One chunk of 2^19 samples at M = 8000 through the occupation-fused path:
    the sample operand (25 GB for the default form, 34 GB for split-BF16 and
    FP32) puts byte offsets far past 2^32 in the sampler, the GEMM's operand
    loads and the epilogue's partials.  The accumulators equal those of the
    same samples in eight chunks of 2^16 bit for bit: each sample keeps its
    place within its 256-column tile, and every sub-ensemble lies inside one
    chunk either way."""
    import paper_2503_12749_amd as mp
    w = m8000
    big, small = 1 << 19, 1 << 16
    kw = dict(prec=prec, seed=w.seed, windows=w.windows, n_sub=big // 8192,
              samples_per_sub=8192, device="cuda:0", fused=True)
    p1 = mp.CountsPipeline(w.T, w.r, chunk=big, **kw)
    p1.run()
    acc1 = p1.acc.cpu().numpy()
    P1 = p1.result()[0]
    del p1
    torch.cuda.empty_cache()
    p2 = mp.CountsPipeline(w.T, w.r, chunk=small, **kw)
    p2.run()
    assert np.array_equal(p2.acc.cpu().numpy(), acc1)
    assert abs(P1.sum() - 1) < 1e-8
    del p2
    torch.cuda.empty_cache()
