"""Batched plans: one captured hipGraph, one persistent grouped GEMM launch
with the occupation-fused epilogue over networks of uneven M.  A plan's
result for each network must equal the single-network fused pipeline on the
same noise bit for bit (the grouped launch runs the same tile code), replays
must be identical, and the autotuner's choice must be cached and reused."""
import json

import numpy as np
import pytest

import synth
from oracle import estimator as oest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_12749_amd  # noqa: F401
    yield


def _nets(Ms, E, n_sub, seed0=900):
    rng = np.random.default_rng(seed0)
    nets = []
    for i, M in enumerate(Ms):
        t = float(rng.uniform(0.85, 0.99))
        r = np.ones(M)
        mean, sd = synth.uniform_loss_moments(r, t)
        nets.append(dict(T=synth.transmission(M, t, seed0 + i), r=r, seed=seed0, net=i, E=E,
                         n_sub=n_sub, window=synth.count_window(mean, sd), t=t))
    return nets


def _single(n, prec):
    """The single-network pipeline a plan reproduces: the occupation-fused
    path for FP32 and the split precisions."""
    import paper_2503_12749_amd as mp
    p = mp.CountsPipeline(n["T"], n["r"], prec=prec, seed=n["seed"], net=n["net"],
                          windows=[n["window"]], n_sub=n["n_sub"],
                          samples_per_sub=n["E"] // n["n_sub"], chunk=n["E"],
                          fused=prec != "fp64")
    p.run()
    return p.result()


@pytest.mark.parametrize("prec", ["split_fp16", "split_bf16", "split1_fp16", "split1t_fp16",
                                  "split1t_f8"])
def test_plan_equals_single_network_runs(prec, tmp_path):
    import paper_2503_12749_amd as mp
    nets = _nets([60, 130, 300, 520], E=4096, n_sub=4)
    cache = tmp_path / "tune.json"
    plan = mp.Plan(nets, prec=prec, tune_cache=cache)
    info = plan.info()
    assert 0 <= info["order"] < 3 and info["prefetch"] in (0, 1) and info["tuned_ms"] > 0
    assert len(info["tiles"]) == len(nets)
    if prec.startswith("split1"):  # one tile width
        assert info["tiles"] == [(128, 128)] * len(nets)
    first = []
    for rep in range(3):
        plan.launch()
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda:0")
        torch.cuda.synchronize()
        assert torch.isfinite(x.sum())
        res = [plan.result(i) for i in range(len(nets))]
        if rep == 0:
            first = res
        for a, b in zip(res, first):
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])
    for i, n in enumerate(nets):
        P, Pi, s = _single(n, prec)
        assert np.array_equal(first[i][0], P), i
        assert np.array_equal(first[i][2], s), i
        assert abs(P.sum() - 1) < 1e-8
    # the cache holds the choice and a second plan reuses it
    data = json.loads(cache.read_text())
    assert len(data) == 1
    plan2 = mp.Plan(nets, prec=prec, tune_cache=cache)
    assert plan2.info()["order"] == info["order"]
    assert plan2.info()["prefetch"] == info["prefetch"]
    assert plan2.info()["tuned_ms"] == pytest.approx(info["tuned_ms"], rel=1e-3)
    assert plan2.info()["tiles"] == info["tiles"]
    plan.close()
    plan2.close()


@pytest.mark.parametrize("prec", ["split_fp16", "split_bf16"])
def test_plan_tile_widths_from_cache(prec, tmp_path):
    """Tile widths per network (128 modes by 128 or 64 samples) read from the
    tuning cache: a plan forced to mixed widths, with ragged sample tails in
    both, gives the same bits as the tuned plan and the single-network runs;
    an entry with a malformed width list is ignored (the plan retunes)."""
    import paper_2503_12749_amd as mp
    nets = _nets([70, 200, 330, 600], E=4000, n_sub=4, seed0=123)
    cache = tmp_path / "tune.json"
    plan = mp.Plan(nets, prec=prec, tune_cache=cache)
    info = plan.info()
    assert all(t[0] == 128 and t[1] in (64, 128) for t in info["tiles"])
    plan.launch()
    ref = [plan.result(i) for i in range(len(nets))]
    plan.close()
    data = json.loads(cache.read_text())
    (key, entry), = data.items()
    for widths in ("2,4,2,4", "2,2,2,2", "4,4,4,4"):
        entry["nj"] = widths
        cache.write_text(json.dumps({key: entry}))
        p2 = mp.Plan(nets, prec=prec, tune_cache=cache)
        assert [t[1] for t in p2.info()["tiles"]] == [32 * int(w) for w in widths.split(",")]
        assert p2.info()["order"] == entry["order"]
        p2.launch()
        for i in range(len(nets)):
            P, Pi, s = p2.result(i)
            assert np.array_equal(P, ref[i][0]) and np.array_equal(s, ref[i][2]), (widths, i)
        p2.close()
    for i, n in enumerate(nets):
        P, _, s = _single(n, prec)
        assert np.array_equal(ref[i][0], P) and np.array_equal(ref[i][2], s), i
    entry["nj"] = "2,3,2,4"
    cache.write_text(json.dumps({key: entry}))
    p3 = mp.Plan(nets, prec=prec, tune_cache=cache)
    assert len(json.loads(cache.read_text())) == 1  # retuned and stored under the same key
    assert "3" not in json.loads(cache.read_text())[key]["nj"]
    p3.close()


def test_plan_chunked_passes_and_fp64_oracle():
    """FP64 plan (one GEMM per network inside the graph) over two passes per
    network against the oracle."""
    import paper_2503_12749_amd as mp
    nets = _nets([16, 40, 70], E=2000, n_sub=4, seed0=77)
    plan = mp.Plan(nets, prec="fp64", chunk=1000)
    plan.launch()
    for i, n in enumerate(nets):
        P, _, s = plan.result(i)
        ref = oest.estimate(n["T"], n["r"], n["seed"], n["E"], n["n_sub"], np.zeros(len(n["r"]), int),
                            1, [n["window"]], net=n["net"], chunk=1000)
        tol = 1e-10 * np.maximum(np.abs(ref["P"]), 1e-4 * ref["P"].max()) + 1e-14 * ref["P"].max()
        assert np.all(np.abs(P - ref["P"]) <= tol), i
    plan.close()


@pytest.mark.parametrize("prec", ["fp32", "split1_fp16"])
def test_plan_fused_per_network_two_passes(prec):
    """FP32 plans (the occupation-fused GEMM and its counts per network inside
    the graph) and one-sided split plans (one grouped launch per pass) over
    two passes per network: bit-identical to the fused single-network
    pipeline run in the same chunks."""
    import paper_2503_12749_amd as mp
    nets = _nets([50, 140, 260], E=2048, n_sub=4, seed0=311)
    plan = mp.Plan(nets, prec=prec, chunk=1024)
    grouped = prec != "fp32"
    assert plan.info()["tiles"] == [(128, 128) if grouped else (0, 0)] * len(nets)
    for rep in range(2):
        plan.launch()
        for i, n in enumerate(nets):
            P, _, s = plan.result(i)
            p = mp.CountsPipeline(n["T"], n["r"], prec=prec, seed=n["seed"], net=n["net"],
                                  windows=[n["window"]], n_sub=n["n_sub"],
                                  samples_per_sub=n["E"] // n["n_sub"], chunk=1024, fused=True)
            p.run()
            Pr, _, sr = p.result()
            assert np.array_equal(P, Pr) and np.array_equal(s, sr), (rep, i)
            assert abs(P.sum() - 1) < 1e-8
    plan.close()


@pytest.mark.parametrize("prec", ["split_bf16", "split1_fp16", "split1t_fp16", "split1t_f8"])
def test_plan_split_uneven_passes(prec):
    """Split plans over chunks of 2048 with networks of one and two passes:
    in the second pass the finished networks have no work items and no
    partials; every network equals the fused single-network pipeline run in
    the same chunks, bit for bit."""
    import paper_2503_12749_amd as mp
    nets = _nets([90, 200, 330], E=4096, n_sub=4, seed0=515)
    nets[1]["E"] = 2048
    nets[1]["n_sub"] = 2
    plan = mp.Plan(nets, prec=prec, chunk=2048)
    plan.launch()
    for i, n in enumerate(nets):
        P, _, s = plan.result(i)
        p = mp.CountsPipeline(n["T"], n["r"], prec=prec, seed=n["seed"], net=n["net"],
                              windows=[n["window"]], n_sub=n["n_sub"],
                              samples_per_sub=n["E"] // n["n_sub"], chunk=2048, fused=True)
        p.run()
        Pr, _, sr = p.result()
        assert np.array_equal(P, Pr) and np.array_equal(s, sr), i
        assert abs(P.sum() - 1) < 1e-8
    plan.close()


@pytest.mark.parametrize("prec", ["split1t_fp16", "split_fp16", "split1t_f8"])
def test_plan_odd_ensembles(prec):
    """Odd sample counts per pass (999 and 333: the T-split form's padded
    column pairs inside a grouped launch, ragged 64- and 128-sample tiles):
    every network equals the fused single-network pipeline, bit for bit."""
    import paper_2503_12749_amd as mp
    nets = _nets([77, 150, 260], E=999, n_sub=3, seed0=808)
    nets[1]["E"] = 333
    nets[1]["n_sub"] = 1
    plan = mp.Plan(nets, prec=prec, chunk=999)
    plan.launch()
    for i, n in enumerate(nets):
        P, _, s = plan.result(i)
        p = mp.CountsPipeline(n["T"], n["r"], prec=prec, seed=n["seed"], net=n["net"],
                              windows=[n["window"]], n_sub=n["n_sub"],
                              samples_per_sub=n["E"] // n["n_sub"], chunk=999, fused=True)
        p.run()
        Pr, _, sr = p.result()
        assert np.array_equal(P, Pr), i
        assert np.array_equal(s, sr) or (n["n_sub"] == 1 and np.isnan(s).all() and np.isnan(sr).all()), i
        assert abs(P.sum() - 1) < 1e-8
    plan.close()


def _binned_nets(Ms, E, n_sub, seed0, mode, d):
    """Networks whose outputs are split into d bins (the first d - 1 equal
    blocks, the rest the last bin, one mode uncounted), with windows from the
    per-bin uniform-loss moments."""
    nets = _nets(Ms, E, n_sub, seed0)
    for n in nets:
        M = len(n["r"])
        bins = np.minimum(np.arange(M) * d // M, d - 1).astype(np.int32)
        bins[M // 3] = -1
        wins = []
        for b in range(d):
            frac = (bins == b).sum() / M
            mean, sd = synth.uniform_loss_moments(n["r"], n["t"], frac=frac)
            wins.append(synth.count_window(mean, sd))
        if mode == "marginals_and_total":
            mean, sd = synth.uniform_loss_moments(n["r"], n["t"], frac=(bins >= 0).sum() / M)
            wins.append(synth.count_window(mean, sd))
        if mode == "joint":
            cap = 192 if d == 2 else 32
            wins = [(lo, min(K, cap)) for lo, K in wins]
        n.update(bin_of_mode=bins, d=d, mode=mode, windows=wins)
        del n["window"]
    return nets


@pytest.mark.parametrize("prec,mode,d", [("split1t_fp16", "marginals_and_total", 3),
                                         ("split_fp16", "marginals_and_total", 2),
                                         ("split_bf16", "joint", 2),
                                         ("split_fp16", "joint", 3),
                                         ("split1t_f8", "marginals", 2),
                                         ("fp32", "marginals", 3),
                                         ("fp64", "joint", 2)])
def test_plan_binned_equals_single_network_runs(prec, mode, d):
    """Plans over binned distributions (marginals of d bins with or without
    the total, joint grids of two and three bins; an uncounted mode; two
    passes for the larger networks): every network's accumulators finalise to
    the same bits
    as the single-network pipeline in the same chunks (the occupation-fused
    path; FP64 through C)."""
    import paper_2503_12749_amd as mp
    nets = _binned_nets([90, 200, 330], E=2048, n_sub=4, seed0=717, mode=mode, d=d)
    nets[0]["E"] = 1024
    nets[0]["n_sub"] = 2
    plan = mp.Plan(nets, prec=prec, chunk=1024)
    plan.launch()
    for i, n in enumerate(nets):
        P, _, s = plan.result(i)
        p = mp.CountsPipeline(n["T"], n["r"], prec=prec, seed=n["seed"], net=n["net"],
                              bin_of_mode=n["bin_of_mode"], d=d, mode=mode, windows=n["windows"],
                              n_sub=n["n_sub"], samples_per_sub=n["E"] // n["n_sub"], chunk=1024,
                              fused=prec != "fp64")
        p.run()
        Pr, _, sr = p.result()
        assert P.shape == Pr.shape, (i, P.shape, Pr.shape)
        assert np.array_equal(P, Pr) and np.array_equal(s, sr), i
    plan.close()


def test_plan_rejects_bad_networks():
    import paper_2503_12749_amd as mp
    nets = _nets([32], E=1000, n_sub=3)
    with pytest.raises(mp.MPError):
        mp.Plan(nets, prec="split_fp16")
