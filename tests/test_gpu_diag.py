"""The matrix-core rate probe (mp_mfma_sustained): it runs for every kind,
reports the launch's flop count (4 waves per compute unit, 16 MFMA chains
per wave for FP16, FP32 and the FP16 + FP8 mix, 32 for FP64, iters rounds), leaves finite values
in its sink, and rejects invalid arguments."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_12749_amd  # noqa: F401
    yield


@pytest.mark.parametrize("kind,flops_per_round", [(0, 16 * 2 * 32 * 32 * 16),
                                                   (1, 16 * 2 * 32 * 32 * 2),
                                                   (2, 32 * 2 * 16 * 16 * 4),
                                                   (3, 16 * (4 * 2 * 32 * 32 * 16 + 2 * 32 * 32 * 64))])
def test_probe_runs_and_counts_flops(kind, flops_per_round):
    import paper_2503_12749_amd as mp
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    sink = torch.full((cus * 256,), float("nan"), dtype=torch.float64, device="cuda:0")
    flops = mp.mp_mfma_sustained(kind, 7, sink)
    torch.cuda.synchronize()
    assert flops == cus * 4 * 7 * flops_per_round  # 4 waves per CU, 7 rounds
    v = sink.cpu().numpy()
    assert np.all(np.isfinite(v)) and np.all(v > 0)


def test_probe_rejects_bad_arguments():
    import paper_2503_12749_amd as mp
    sink = torch.empty(16, dtype=torch.float64, device="cuda:0")
    with pytest.raises(mp.MPError):
        mp.mp_mfma_sustained(0, 10, sink)  # sink smaller than 256 values per CU
    big = torch.empty(512 * 256, dtype=torch.float64, device="cuda:0")
    with pytest.raises(mp.MPError):
        mp.mp_mfma_sustained(4, 10, big)
