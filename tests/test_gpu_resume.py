"""Checkpoint and resume of a chunked run: stop after chunk c, save the
per-sub-ensemble accumulators and the next sample index to disk, continue in
a fresh pipeline from the file; the result equals the uninterrupted run bit
for bit (counter-based noise, same chunk boundaries, deterministic sums)."""
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


@pytest.mark.parametrize("prec,fused", [("fp64", False), ("split1_fp16", True), ("split1t_fp16", True),
                                        ("split1t_f8", True), ("split_bf16", True),
                                        ("split1t_f8", "bilinear")])
def test_resume_from_checkpoint_file(prec, fused, tmp_path):
    import paper_2503_12749_amd as mp
    w = synth.workload_m1000(E=60_000)
    chunk, ns = 7_000, 6_000  # chunks straddle sub-ensemble boundaries
    kw = dict(prec=prec, seed=w.seed, windows=w.windows, n_sub=w.E // ns, samples_per_sub=ns,
              chunk=chunk, device="cuda:0", fused=fused is True, bilinear=fused == "bilinear")
    full = mp.CountsPipeline(w.T, w.r, **kw)
    full.run(w.E)
    P0, _, s0 = full.result()
    del full
    a = mp.CountsPipeline(w.T, w.r, **kw)
    stop = 4 * chunk
    g = 0
    while g < stop:
        a.run_chunk(g, chunk)
        g += chunk
    st = a.checkpoint(g)
    np.savez(tmp_path / "ckpt.npz", acc=st["acc"], next_g=st["next_g"])
    del a
    torch.cuda.empty_cache()
    f = np.load(tmp_path / "ckpt.npz")
    b = mp.CountsPipeline(w.T, w.r, **kw)
    nxt = b.restore({"acc": f["acc"], "next_g": int(f["next_g"])})
    b.run(w.E - nxt, g_start=nxt)
    P1, _, s1 = b.result()
    assert np.array_equal(P0, P1) and np.array_equal(s0, s1)
    assert abs(P1.sum() - 1) < 1e-8
