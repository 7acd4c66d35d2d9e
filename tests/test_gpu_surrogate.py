"""The surrogate's HIP kernels against the FP64 MLP oracle (forward, loss,
gradients, Adam), reproducibility of training, and what the trained network
gains over running the method on every candidate of a sweep."""
import time

import numpy as np
import pytest

from oracle import mlp as omlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_12749_amd  # noqa: F401
    yield


def _net(width, seed=0, batch=64):
    from paper_2503_12749_amd.surrogate import Mlp
    return Mlp(width=width, batch_max=batch, seed=seed)


@pytest.mark.parametrize("width", [(5, 16, 12, 4), (5, 256, 256, 256, 8)])
def test_forward_loss_and_gradients_match_oracle(width):
    net = _net(width)
    rng = np.random.default_rng(3)
    X = rng.normal(size=(64, width[0]))
    Y = rng.normal(size=(64, width[-1]))
    p = net.params.cpu().numpy().astype(np.float64)
    loss, g = net.loss_grad_raw(X, Y)
    Xr = X.astype(np.float32).astype(np.float64)
    Yr = Y.astype(np.float32).astype(np.float64)
    ref_loss, ref_g = omlp.loss_grad(p, width, Xr, Yr)
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    # per layer, relative to the layer's gradient norm (FP32 activations and sums)
    off = 0
    for l in range(len(width) - 1):
        n = (width[l] + 1) * width[l + 1]
        a, b = g[off: off + n], ref_g[off: off + n]
        assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b), l
        off += n
    pred = net.predict_raw(X)
    ref_pred, _ = omlp.forward(p, width, Xr)
    np.testing.assert_allclose(pred, ref_pred, rtol=0, atol=1e-5 * np.abs(ref_pred).max())


def test_adam_step_matches_formula():
    width = (5, 16, 12, 4)
    net = _net(width)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(32, 5)).astype(np.float32)
    Y = rng.normal(size=(32, 4)).astype(np.float32)
    for wd in (0.0, 0.5):
        p0 = net.params.cpu().numpy().astype(np.float64)
        m0 = net.m.cpu().numpy().astype(np.float64)
        v0 = net.v.cpu().numpy().astype(np.float64)
        Xd, Yd = net._dev(X), net._dev(Y)
        net.step_raw(Xd, Yd, 32, 1e-2, weight_decay=wd)
        k = net.step_count
        g = net.grads.cpu().numpy().astype(np.float64)
        m = 0.9 * m0 + 0.1 * g
        v = 0.999 * v0 + 0.001 * g * g
        mh, vh = m / (1 - 0.9 ** k), v / (1 - 0.999 ** k)
        want = p0 - 1e-2 * (mh / (np.sqrt(vh) + 1e-8) + wd * p0)
        np.testing.assert_allclose(net.params.cpu().numpy(), want, rtol=1e-5, atol=1e-7)
        w16 = net.w16.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
        np.testing.assert_array_equal(w16.view(np.float32).astype(np.float64),
                                      omlp.bf16_round(net.params.cpu().numpy()))


def test_training_is_reproducible_and_learns():
    width = (5, 64, 64, 64, 8)
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, size=(400, 5))
    Y = np.stack([np.sin(X @ rng.normal(size=5)) for _ in range(8)], 1)
    runs = []
    for _ in range(2):
        net = _net(width, seed=11, batch=128)
        hist = net.fit(X, Y, steps=400, batch=128, lr=3e-3, seed=1, log_every=50)
        runs.append((net.params.cpu().numpy(), hist))
    assert np.array_equal(runs[0][0], runs[1][0])
    hist = runs[0][1]
    assert hist[-1][1] < 0.1 * hist[0][1]


def test_surrogate_screens_faster_than_the_method():
    """Trained on method runs at M in [100, 400] (E = 1024 per sweep), the
    network predicts the mean and variance per mode of bin 0 for held-out
    sweeps at M = 800 (twice the largest training size): the mean to within
    a percent, and the bin variance much closer than the independent-mode
    baseline it corrects.  It answers a 256-candidate sweep orders of
    magnitude faster than the method would."""
    from paper_2503_12749_amd import surrogate as sg
    rng = np.random.default_rng(7)
    runner = sg.MethodRunner()
    sweeps = sg.sample_sweeps(400, rng, M_range=(100, 400), n_grid=6)
    t0 = time.perf_counter()
    X, Y = sg.generate(runner, sweeps, E=1024)
    t_method_each = (time.perf_counter() - t0) / len(sweeps)
    net = sg.Mlp(batch_max=256, seed=3)
    net.fit(X, Y, steps=300, batch=256, lr=2e-3, weight_decay=1.0, seed=2)
    held = sg.sample_sweeps(8, np.random.default_rng(8), M_range=(800, 800), n_grid=1)
    Xh = np.stack([sg.features(*s) for s in held])
    Yh = np.stack([runner.run(*s, E=4096, net=50000 + i)[0] for i, s in enumerate(held)])
    pred = net.predict(Xh)
    err = np.abs(pred - Yh) / np.abs(Yh)
    base = np.abs(1.0 - Yh) / np.abs(Yh)
    print("held-out M=800 bin-0 mean err", np.round(err[:, 0], 4), "var err", np.round(err[:, 1], 4),
          "baseline-only var err", np.round(base[:, 1], 4))
    assert err[:, 0].mean() < 0.01 and err[:, 0].max() < 0.03
    assert err[:, 4].mean() < 0.01
    assert err[:, 1].mean() < 0.5 * base[:, 1].mean()
    cands = np.stack([sg.features(800, 0.95, a, b, 1) for a in np.linspace(0.6, 1.4, 16)
                      for b in np.linspace(0.0, 0.3, 16)])
    t0 = time.perf_counter()
    net.predict(cands)
    t_pred = time.perf_counter() - t0
    gain = 256 * t_method_each / t_pred
    print(f"256 candidates: surrogate {t_pred * 1e3:.2f} ms vs method ~{256 * t_method_each:.2f} s"
          f" at E=1024 (gain {gain:.0f}x)")
    assert gain > 100
