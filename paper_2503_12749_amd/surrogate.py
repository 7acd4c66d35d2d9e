"""Learned surrogate for parameter sweeps of the matrix-P method.

A 4-layer MLP (5 -> 256 -> 256 -> 256 -> 8, SiLU, BF16 weight copies, FP32
accumulation) maps sweep parameters (modes M, transmission t, mean and spread
of the squeezing profile, number of bins d) to the first eight cumulants of
the photon count of the first of d equal mode bins, per mode of that bin.
Training data come from the method itself (CountsPipeline runs); training,
inference and the Adam updates run in the library's HIP kernels
(mp_mlp_*).  Screening: the network ranks candidate squeezing profiles at a
size outside its training range, and the method, run on the selected
candidates, judges the predictions and replaces any that miss.

Cumulants per mode of a bin are size-independent to leading order (the count
of a large bin is a sum of many weakly dependent contributions), which is what
lets a network trained at M <= 2000 screen at M = 8000.

Run as a module to generate data, train and screen:
    python -m paper_2503_12749_amd.surrogate --sweeps 20000 --E 10000
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import time

import numpy as np

from . import CountsPipeline, _lib, _ptr, _stream
from ._lib import MlpShape

WIDTH = (5, 256, 256, 256, 8)
N_CUM = 8


# ---------------------------------------------------------------- features / targets

def features(M, t, rbar, sr, d):
    """Network inputs, each of order one."""
    return np.array([math.log(M) / math.log(2000.0), (t - 0.9) * 10.0, rbar - 1.0, sr * 3.0,
                     1.0 / d], dtype=np.float64)


def cumulants_from_distribution(m, P, kmax=N_CUM):
    """Cumulants kappa_1..kappa_kmax of a count distribution given on counts m
    (central moments, then the moment-cumulant recursion)."""
    P = np.asarray(P, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    P = P / P.sum()
    mu = float((m * P).sum())
    c = [1.0, 0.0] + [float(((m - mu) ** k * P).sum()) for k in range(2, kmax + 1)]
    kap = [0.0, mu]
    for n in range(2, kmax + 1):
        v = c[n]
        for k in range(2, n - 1):
            v -= math.comb(n - 1, k - 1) * kap[k] * c[n - k]
        kap.append(v)
    return np.array(kap[1:])


def squeezing_profile(M, rbar, sr, seed):
    rng = np.random.Generator(np.random.Philox(key=[int(seed) & (2**64 - 1), 0x53]))
    return np.clip(rbar + sr * rng.standard_normal(M), 0.5, 1.5)


# ---------------------------------------------------------------- method runs

class MethodRunner:
    """Runs the method for sweep points; keeps one Haar network per M (an
    input, drawn from the seeded generator) and scales it by t."""

    def __init__(self, prec="split_fp16", device="cuda:0", seed=2503):
        import synth
        self.synth = synth
        self.prec, self.device, self.seed = prec, device, seed
        self._haar = {}

    def haar(self, M):
        if M not in self._haar:
            self._haar[M] = self.synth.haar_unitary(M, self.seed + M)
        return self._haar[M]

    def run(self, M, t, rbar, sr, d, E, net, n_sub=10, chunk=None):
        """Cumulants per mode of bin 0 (the first M // d modes) and the run's
        distribution (m, P, sigma)."""
        r = squeezing_profile(M, rbar, sr, self.seed * 7919 + net)
        Mb = M // d
        bins = np.full(M, -1, dtype=np.int32)
        bins[:Mb] = 0
        # rough moments of bin 0 (network correlations ignored, hence the margin)
        mean, sd = self.synth.uniform_loss_moments(r, t, frac=Mb / M)
        win = self.synth.count_window(mean, sd * 1.6 + 2.0, nsig=10.0)
        ns = E // n_sub
        E = ns * n_sub  # whole sub-ensembles only
        chunk = min(chunk or E, E)
        p = CountsPipeline(t * self.haar(M), r, prec=self.prec, seed=self.seed, net=net,
                           bin_of_mode=bins, d=1, windows=[win], n_sub=n_sub,
                           samples_per_sub=ns, chunk=chunk, device=self.device)
        p.run(E)
        P, _, s = p.result()
        m = np.arange(win[0], win[0] + win[1])
        return cumulants_from_distribution(m, P) / Mb, (m, P, s)


def sample_sweeps(n, rng, M_range=(100, 2000), t_range=(0.8, 0.99), bins=(1, 2, 4),
                  n_grid=24):
    """Sweep points drawn uniformly from the training box; M is log-uniform on
    a grid of n_grid multiples of 4 (so that every bin count divides it and a
    few Haar networks serve all sweeps)."""
    grid = np.unique(np.round(np.exp(np.linspace(math.log(M_range[0]), math.log(M_range[1]),
                                                 n_grid)) / 4).astype(int) * 4)
    out = []
    for _ in range(n):
        M = int(rng.choice(grid))
        d = int(rng.choice(bins))
        out.append((M, float(rng.uniform(*t_range)), float(rng.uniform(0.5, 1.5)),
                    float(rng.uniform(0.0, 0.3)), d))
    return out


def generate(runner, sweeps, E, log_every=0):
    X = np.stack([features(*s) for s in sweeps])
    Y = np.empty((len(sweeps), N_CUM))
    t0 = time.perf_counter()
    for i, s in enumerate(sweeps):
        Y[i], _ = runner.run(*s, E=E, net=i)
        if log_every and (i + 1) % log_every == 0:
            print(f"[surrogate] {i + 1}/{len(sweeps)} sweeps, {time.perf_counter() - t0:.1f} s",
                  flush=True)
    return X, Y


# ---------------------------------------------------------------- network

class Mlp:
    """Device-resident MLP: FP32 master parameters, BF16 copy, Adam moments."""

    def __init__(self, width=WIDTH, batch_max=512, seed=0, device="cuda:0"):
        import torch
        self.torch = torch
        self.width = tuple(width)
        self.shape = MlpShape(len(width) - 1, (ctypes.c_int32 * 9)(*(list(width) + [0] * (9 - len(width)))))
        lib = _lib.load()
        self.n = int(lib.mp_mlp_param_count(ctypes.byref(self.shape)))
        rng = np.random.default_rng(seed)
        init = []
        for l in range(len(width) - 1):
            I, O = width[l], width[l + 1]
            init.append(rng.normal(0.0, math.sqrt(2.0 / I), I * O))
            init.append(np.zeros(O))
        dev = torch.device(device)
        self.params = torch.from_numpy(np.concatenate(init).astype(np.float32)).to(dev)
        self.w16 = torch.empty(self.n, dtype=torch.int16, device=dev)
        self.grads = torch.zeros(self.n, dtype=torch.float32, device=dev)
        self.m = torch.zeros(self.n, dtype=torch.float32, device=dev)
        self.v = torch.zeros(self.n, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.batch_max = batch_max
        self.ws = torch.empty(int(lib.mp_mlp_workspace(ctypes.byref(self.shape), batch_max)),
                              dtype=torch.uint8, device=dev)
        self.device = dev
        self.step_count = 0
        self.x_mean = np.zeros(width[0])
        self.x_std = np.ones(width[0])
        self.y_mean = np.zeros(width[-1])
        self.y_std = np.ones(width[-1])
        _lib.check(lib.mp_mlp_round(ctypes.byref(self.shape), _ptr(self.params), _ptr(self.w16),
                                    _stream(None)))

    # raw (already normalised) device calls
    def _dev(self, a):
        return self.torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(self.device)

    def loss_grad_raw(self, X, Y):
        lib = _lib.load()
        Xd, Yd = self._dev(X), self._dev(Y)
        _lib.check(lib.mp_mlp_loss_grad(ctypes.byref(self.shape), _ptr(self.w16), _ptr(self.params),
                                        _ptr(Xd), _ptr(Yd), len(X), _ptr(self.grads), _ptr(self.loss),
                                        _ptr(self.ws), self.ws.numel(), _stream(None)))
        return float(self.loss.item()), self.grads.cpu().numpy().astype(np.float64)

    def step_raw(self, Xd, Yd, batch, lr):
        lib = _lib.load()
        _lib.check(lib.mp_mlp_loss_grad(ctypes.byref(self.shape), _ptr(self.w16), _ptr(self.params),
                                        _ptr(Xd), _ptr(Yd), batch, _ptr(self.grads), _ptr(self.loss),
                                        _ptr(self.ws), self.ws.numel(), _stream(None)))
        self.step_count += 1
        _lib.check(lib.mp_mlp_adam(ctypes.byref(self.shape), _ptr(self.params), _ptr(self.grads),
                                   _ptr(self.m), _ptr(self.v), _ptr(self.w16), lr, 0.9, 0.999, 1e-8,
                                   self.step_count, _stream(None)))

    def predict_raw(self, X):
        lib = _lib.load()
        out = np.empty((len(X), self.width[-1]))
        for i in range(0, len(X), self.batch_max):
            Xd = self._dev(X[i: i + self.batch_max])
            Yd = self.torch.empty((len(Xd), self.width[-1]), dtype=self.torch.float32, device=self.device)
            _lib.check(lib.mp_mlp_forward(ctypes.byref(self.shape), _ptr(self.w16), _ptr(self.params),
                                          _ptr(Xd), len(Xd), _ptr(Yd), _ptr(self.ws), self.ws.numel(),
                                          _stream(None)))
            out[i: i + len(Xd)] = Yd.cpu().numpy()
        return out

    # normalised interface
    def fit(self, X, Y, steps=3000, batch=256, lr=2e-3, seed=0, log_every=0):
        self.x_mean, self.x_std = X.mean(0), X.std(0) + 1e-8
        self.y_mean, self.y_std = Y.mean(0), Y.std(0) + 1e-12
        Xn = (X - self.x_mean) / self.x_std
        Yn = (Y - self.y_mean) / self.y_std
        Xd, Yd = self._dev(Xn), self._dev(Yn)
        rng = np.random.default_rng(seed)
        hist = []
        batch = min(batch, self.batch_max, len(X))
        for s in range(steps):
            idx = self.torch.from_numpy(rng.choice(len(X), batch, replace=False)).to(self.device)
            lr_s = lr * 0.5 * (1 + math.cos(math.pi * s / steps))
            self.step_raw(Xd[idx].contiguous(), Yd[idx].contiguous(), batch, lr_s)
            if log_every and (s % log_every == 0 or s == steps - 1):
                hist.append((s, float(self.loss.item())))
        return hist

    def predict(self, X):
        Xn = (np.atleast_2d(X) - self.x_mean) / self.x_std
        return self.predict_raw(Xn) * self.y_std + self.y_mean


# ---------------------------------------------------------------- screening

def screen(mlp, runner, M, t, d, candidates, E_judge, top, tol_sigma=4.0):
    """Ranks candidate (rbar, sr) profiles by predicted mean count per mode
    closest to the middle of the candidates' range, runs the method on the
    `top` best, and keeps the method's value wherever the prediction misses
    by more than tol_sigma of the method's error."""
    X = np.stack([features(M, t, rb, sr, d) for rb, sr in candidates])
    t0 = time.perf_counter()
    pred = mlp.predict(X)
    t_pred = time.perf_counter() - t0
    target = 0.5 * (pred[:, 0].min() + pred[:, 0].max())
    order = np.argsort(np.abs(pred[:, 0] - target))[:top]
    judged = []
    t0 = time.perf_counter()
    for q in order:
        rb, sr = candidates[q]
        y, (m, P, s) = runner.run(M, t, rb, sr, d, E=E_judge, net=100000 + int(q),
                                  chunk=min(E_judge, 65536), n_sub=max(2, E_judge // 8192))
        Mb = M // d
        sig_mean = float(np.sqrt(((m - y[0] * Mb) ** 2 * s ** 2).sum())) / Mb
        miss = abs(pred[q, 0] - y[0]) > tol_sigma * max(sig_mean, 1e-12)
        judged.append(dict(candidate=[rb, sr], predicted=pred[q].tolist(), method=y.tolist(),
                           sigma_mean_per_mode=sig_mean, fallback=bool(miss)))
    t_method = time.perf_counter() - t0
    return dict(t_predict_s=t_pred, t_method_s=t_method, n_candidates=len(candidates),
                judged=judged)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sweeps", type=int, default=20000)
    ap.add_argument("--E", type=int, default=10000)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--screen-M", type=int, default=8000)
    ap.add_argument("--screen-E", type=int, default=1_000_000)
    ap.add_argument("--candidates", type=int, default=256)
    ap.add_argument("--top", type=int, default=8)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    rng = np.random.default_rng(2503)
    runner = MethodRunner()
    sweeps = sample_sweeps(args.sweeps, rng)
    t0 = time.perf_counter()
    X, Y = generate(runner, sweeps, args.E, log_every=max(1, args.sweeps // 20))
    t_gen = time.perf_counter() - t0
    mlp = Mlp()
    t0 = time.perf_counter()
    hist = mlp.fit(X, Y, steps=args.steps, log_every=max(1, args.steps // 20))
    t_train = time.perf_counter() - t0
    cands = [(float(a), float(b)) for a in np.linspace(0.6, 1.4, 16) for b in np.linspace(0.0, 0.3, 16)]
    cands = cands[: args.candidates]
    res = screen(mlp, runner, args.screen_M, 0.95, 1, cands, args.screen_E, args.top)
    res.update(t_generate_s=t_gen, t_train_s=t_train, loss_history=hist, sweeps=args.sweeps,
               E=args.E)
    text = json.dumps(res, indent=1)
    if args.out:
        open(args.out, "w").write(text)
    print(text)


if __name__ == "__main__":
    main()
