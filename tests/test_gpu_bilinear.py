"""One count distribution through the bilinear form n_S = alpha^T W beta,
W = T^T P_S T* (the per-sample bin occupation of the main text's generating
function, rewritten for real alpha, beta): the packed W against W formed in
FP64 on the CPU, and binned P(m) against the FP64 oracle, which propagates
alpha' = T alpha and beta' = T* beta and sums alpha'_j beta'_j over S directly."""
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


def _network(M, seed):
    """Haar unitary with mode-dependent output loss, T = diag(l) U: W = U^T
    diag(l^2) P_S U* is dense even for S = all modes (with input loss, or
    uniform loss, W would be diagonal there and the GEMM's operand zero)."""
    return synth.haar_unitary(M, seed) * np.linspace(0.6, 1.0, M)[:, None]


def _e4m3_value(code):
    c = np.asarray(code, dtype=np.int64)
    sign = np.where(c & 0x80, -1.0, 1.0)
    ex, man = (c >> 3) & 15, c & 7
    mag = np.where(ex == 0, man * 2.0 ** -9, (1.0 + man / 8.0) * np.ldexp(1.0, ex - 7))
    return sign * mag


@pytest.mark.parametrize("subset", [False, True])
def test_packed_W_is_T_transpose_P_T_conj(subset):
    """Entries of the packed W (FP16 part plus the e4m3 remainder) against
    T^T P_S T* formed in FP64 by numpy: within 2^-15 of each entry (the
    packing's rounding, as for T) plus the e4m3 remainder's subnormal step."""
    import paper_2503_12749_amd as mp
    M = 300
    T = _network(M, 21)
    bins = np.zeros(M, np.int32)
    if subset:
        bins[np.random.default_rng(3).random(M) < 0.45] = -1
    ldm = mp.mp_ld_modes(M)
    Td = torch.from_numpy(np.ascontiguousarray(T).view(np.float64).reshape(-1).copy()).to(DEV)
    packed = torch.empty(mp.mp_bilinear_packed_bytes(M), dtype=torch.uint8, device=DEV)
    scratch = torch.empty(mp.mp_bilinear_workspace(M), dtype=torch.uint8, device=DEV)
    mp.mp_pack_bilinear(M, Td, bins, "split1t_f8", packed, scratch)
    praw = packed.cpu().numpy()
    hi = praw[: 4 * ldm * ldm].view(np.float16).astype(np.float64)
    lo8 = praw[4 * ldm * ldm: 6 * ldm * ldm]
    e = int(np.floor(np.log2(M) / 2))
    P = (bins >= 0).astype(np.float64)
    W = T.T @ (P[:, None] * T.conj())
    # the diagonal (real) in FP32 after the packed operand, the packed part without it
    D = praw[3 * 2 * ldm * ldm:].view(np.float32)[:ldm].astype(np.float64)
    np.testing.assert_allclose(D[:M], W.diagonal().real, rtol=2 ** -23, atol=0)
    assert not D[M:].any()
    W = W - np.diag(W.diagonal())
    A = np.zeros((2 * ldm, ldm))
    A[:M, :M], A[ldm: ldm + M, :M] = W.real, W.imag
    x = np.ldexp(A, e)
    R, K = np.arange(2 * ldm)[:, None], np.arange(ldm)[None, :]
    hi_rk = hi[(R >> 1) * 2 * ldm + 64 * (K >> 5) + (K & 31) + 32 * (R & 1)]
    lo_rk = _e4m3_value(lo8[(R >> 1) * 2 * ldm + 128 * (K >> 6) + 64 * (R & 1) + (K & 63)])
    got = hi_rk + np.ldexp(lo_rk, e - 18)
    err = np.abs(got - x)
    bound = 2.0 ** -15 * np.abs(x) + np.ldexp(2.0 ** -10, e - 18)
    print(f"packed W (subset={subset}): max |error| / bound = {(err / bound).max():.3f}")
    assert np.all(err <= bound)
    assert not got[M:ldm].any() and not got[ldm + M:].any() and not got[:, M:].any()


@pytest.mark.parametrize("est", ["matrix_p", "plus_p"])
@pytest.mark.parametrize("subset", [False, True])
def test_bilinear_counts_match_oracle(subset, est):
    """M = 300, E = 1104 in chunks of 511 (odd chunks: padded column pairs),
    three sub-ensembles of 368 straddling the chunks; S all modes or a
    scattered subset (about 75 runs of modes: beyond the 16 runs the
    occupation-fused epilogue takes, while S is inside W here).  P(m) within
    0.05 sigma_T + 1e-6 max P of the oracle; for S = all modes the T-form
    fused path on the same noise is printed beside it."""
    import paper_2503_12749_amd as mp
    M, E, n_sub, chunk, seed = 300, 1104, 3, 511, 17
    T = _network(M, 22)
    r = np.linspace(0.3, 0.9, M)
    bins = np.zeros(M, np.int32)
    if subset:
        bins[np.random.default_rng(5).random(M) < 0.5] = -1
    windows = [(0, 256)]
    kw = dict(prec="split1t_f8", seed=seed, bin_of_mode=bins, d=1, windows=windows, n_sub=n_sub,
              samples_per_sub=E // n_sub, chunk=chunk, est=est, device=DEV)
    pb = mp.CountsPipeline(T, r, bilinear=True, **kw)
    pb.run()
    Pb, Pib, sb = pb.result()
    ref = oest.estimate(T, r, seed, E, n_sub, bins, 1, windows, plus_p=(est == "plus_p"))
    bound = 0.05 * ref["sigma"] + 1e-6 * np.abs(ref["P"]).max()
    eb = np.abs(Pb - ref["P"])
    note = ""
    if not subset:
        pt = mp.CountsPipeline(T, r, fused=True, **kw)
        pt.run()
        Pt = pt.result()[0]
        note = f", T-form {(np.abs(Pt - ref['P']) / bound).max():.3f}"
    print(f"subset={subset} {est}: bilinear max |dP|/bound {(eb / bound).max():.3f}{note}")
    assert np.all(eb <= bound)
    assert abs(Pb.sum() - 1) < 1e-8
    assert np.isfinite(Pib).all()


def test_bilinear_rejects_what_it_does_not_cover():
    import paper_2503_12749_amd as mp
    M = 64
    T = _network(M, 2)
    r = np.full(M, 0.5)
    with pytest.raises(mp.MPError):
        mp.CountsPipeline(T, r, prec="split1t_fp16", seed=1, windows=[(0, 64)], n_sub=1,
                          samples_per_sub=128, chunk=128, bilinear=True)
    with pytest.raises(mp.MPError):
        mp.CountsPipeline(T, r, prec="split1t_f8", seed=1, bin_of_mode=np.arange(M) % 2, d=2,
                          mode="marginals", windows=[(0, 64)] * 2, n_sub=1, samples_per_sub=128,
                          chunk=128, bilinear=True)
