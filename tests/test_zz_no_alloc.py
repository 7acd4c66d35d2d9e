"""mp_propagate_counts_noalloc (the entry point that allocates nothing and
keeps its partials in the library's per-GPU scratch array) against
mp_propagate_counts with a caller workspace, through the C ABI, on identical
inputs: the accumulators must be identical bit for bit (same kernels, same
summation order; only the partials' storage differs).  Two calls in a row,
the second with a smaller input, so the second reads a scratch array that
still holds the first call's contents."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_12749_amd  # noqa: F401
    yield


def _dft_network(M, t, seed):
    """T = t F D: F the unitary DFT matrix, D random phases (dense, unitary
    up to t, cheap to build at large M)."""
    rng = np.random.default_rng(seed)
    j = np.arange(M)
    T = (t / np.sqrt(M)) * np.exp(-2j * np.pi * (np.outer(j, j) % M) / M)
    return T * np.exp(2j * np.pi * rng.random(M))[None, :]


def _both(M, T, r, prec, E, e0, bins, d, mode, windows, n_sub, ns, seed):
    """One chunk of E samples from global index e0: accumulators of the
    workspace entry point and of the no-allocation one."""
    import paper_2503_12749_amd as mp
    dev = torch.device("cuda:0")
    Td = torch.from_numpy(np.ascontiguousarray(T).view(np.float64).reshape(-1).copy()).to(dev)
    rd = torch.from_numpy(np.asarray(r, dtype=np.float64).copy()).to(dev)
    ab = torch.empty(mp.mp_ab_bytes(M, E, prec), dtype=torch.uint8, device=dev)
    n = torch.empty(E, dtype=torch.float64, device=dev)
    packed = torch.empty(mp.mp_propagate_workspace(M, prec), dtype=torch.uint8, device=dev)
    m_lo = [w[0] for w in windows]
    K = [w[1] for w in windows]
    ent = mp.mp_acc_entries(d, mode, K)
    mp.mp_pack_transmission(M, Td, prec, packed)
    mp.mp_sample(M, e0, E, rd, seed, 0, prec, ab, n)
    ws = torch.empty(mp.mp_propagate_counts_workspace(M, E, d, bins, mode, K, n_sub, ns, e0),
                     dtype=torch.uint8, device=dev)
    acc_ws = torch.zeros(n_sub * ent * 2, dtype=torch.float64, device=dev)
    acc_na = torch.zeros_like(acc_ws)
    mp.mp_propagate_counts(M, E, prec, "matrix_p", ab, n, packed, d, bins, mode, m_lo, K, n_sub,
                           ns, e0, acc_ws, ws)
    mp.mp_propagate_counts_noalloc(M, E, prec, "matrix_p", ab, n, packed, d, bins, mode, m_lo, K,
                                   n_sub, ns, e0, acc_na)
    torch.cuda.synchronize()
    return acc_ws.cpu().numpy(), acc_na.cpu().numpy(), ws.numel()


@pytest.mark.parametrize("prec", ["split_bf16", "fp32", "split1t_fp16", "split1t_f8"])
def test_noalloc_matches_workspace_entry_point(prec):
    import paper_2503_12749_amd as mp
    # call 1: M = 8000, total counts, 16384 samples (about half the scratch)
    M, t = 8000, 0.95
    T = _dft_network(M, t, 80)
    r = np.ones(M)
    win = synth.count_window(*synth.uniform_loss_moments(r, t))
    E1, ns1 = 16384, 4096
    a, b, need = _both(M, T, r, prec, E1, 0, synth.all_modes_bin(M), 1, "joint", [win],
                       E1 // ns1, ns1, 17)
    print(f"{prec} call 1: M={M} E={E1}, scratch need {need / 2**20:.1f} MiB", flush=True)
    assert need <= mp._lib.MP_NOALLOC_SCRATCH_BYTES
    assert np.any(a != 0)
    assert np.array_equal(a, b), np.abs(a - b).max()
    # call 2: smaller, M = 1000, two bins (marginals + total), a ragged chunk
    # starting inside a sub-ensemble
    w = synth.workload_m1000(E=12_000, with_T=True)
    bins = synth.contiguous_bins(w.M, 2)
    half = synth.count_window(*synth.uniform_loss_moments(w.r, w.t, frac=0.5))
    E2, ns2, e0 = 2999, 1000, 1500
    a2, b2, need2 = _both(w.M, w.T, w.r, prec, E2, e0, bins, 2, "marginals_and_total",
                          [half, half, w.windows[0]], 5, ns2, w.seed)
    print(f"{prec} call 2: M={w.M} E={E2} e0={e0}, scratch need {need2 / 2**20:.2f} MiB",
          flush=True)
    assert np.any(a2 != 0)
    assert np.array_equal(a2, b2), np.abs(a2 - b2).max()
