"""Learned surrogate for parameter sweeps of the matrix-P method.

A 4-layer MLP (5 -> 256 -> 256 -> 256 -> 8, SiLU, BF16 weight copies, FP32
accumulation) maps sweep parameters (modes M, transmission t, mean and spread
of the squeezing profile, number of equal bins d) to the first four cumulants
per mode of two counts: that of the first bin (M / d modes) and the total.
Each target is a ratio to the value it would have for independent modes (the
single-mode photon-number law of a squeezed vacuum after uniform loss t^2,
averaged over the run's squeezing profile), so the network learns the
correction that the network's mode correlations make, a number of order one
whose dependence on M is weak.  Training data come from the method itself
(CountsPipeline runs); training, inference and the Adam updates run in the
library's HIP kernels (mp_mlp_*).  Screening: the network ranks candidate
squeezing profiles at a size outside its training range, and the method, run
on the selected candidates, checks the predictions and replaces any that
miss.

Run as a module to generate data, train and screen:
    python -m paper_2503_12749_amd.surrogate --sweeps 4000 --E 10000
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import sys
import time

import numpy as np

from . import CountsPipeline, _lib, _ptr, _stream
from ._lib import MlpShape

WIDTH = (5, 256, 256, 256, 8)
N_CUM = 4           # cumulants per count
TRUNC_SIGMA = 7.0   # cumulants are taken over mean +- 7 sd of the distribution


# ---------------------------------------------------------------- features / targets

def features(M, t, rbar, sr, d):
    """Network inputs, each of order one; 1/sqrt(M) is the scale of the
    finite-size corrections."""
    return np.array([10.0 / math.sqrt(M), (t - 0.9) * 10.0, rbar - 1.0, sr * 3.0, 1.0 / d],
                    dtype=np.float64)


def independent_mode_baseline(t, r, d):
    """Per-mode mean and variances of the counts for independent modes.

    A squeezed vacuum of squeezing r has mean N = sinh^2 r and photon-number
    variance 2N(N+1); after uniform loss t^2 a mode's count has mean t^2 N and
    variance t^2 N + t^4 N (2N + 1).  For the bin of M/d modes the excess
    term is diluted by the fraction of each input's light that stays in the
    bin (1/d for a uniform spread).  Returns (mean, var_bin, var_total) per
    mode, averaged over the profile r."""
    N = np.sinh(np.asarray(r, dtype=np.float64)) ** 2
    EN, EN2 = float(N.mean()), float((N * (2.0 * N + 1.0)).mean())
    t2 = t * t
    return t2 * EN, t2 * EN + t2 * t2 * EN2 / d, t2 * EN + t2 * t2 * EN2


def cumulants(m, P, kmax=N_CUM, trunc=TRUNC_SIGMA):
    """kappa_1..kappa_kmax (kmax <= 4) of a count distribution P on counts m,
    over the counts within trunc standard deviations of the mean (outside that
    range the estimate holds only sampling noise)."""
    m = np.asarray(m, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    P = P / P.sum()
    mu = float((m * P).sum())
    sd = math.sqrt(max(float(((m - mu) ** 2 * P).sum()), 0.0))
    keep = np.abs(m - mu) <= trunc * sd
    m, P = m[keep], P[keep] / P[keep].sum()
    mu = float((m * P).sum())
    c = [float(((m - mu) ** k * P).sum()) for k in range(5)]
    kap = [mu, c[2], c[3], c[4] - 3.0 * c[2] ** 2]
    return np.array(kap[:kmax])


def targets(M, t, r, d, kap_bin, kap_tot):
    """Cumulants per mode over the independent-mode baseline."""
    mean, vb, vt = independent_mode_baseline(t, r, d)
    kb = np.asarray(kap_bin) / (M // d)
    kt = np.asarray(kap_tot) / M
    return np.array([kb[0] / mean, kb[1] / vb, kb[2] / vb, kb[3] / vb,
                     kt[0] / mean, kt[1] / vt, kt[2] / vt, kt[3] / vt])


def moments_from_targets(M, t, r, d, y):
    """Inverse of targets(): (bin cumulants, total cumulants) of the counts."""
    mean, vb, vt = independent_mode_baseline(t, r, d)
    y = np.asarray(y, dtype=np.float64)
    kb = np.array([y[0] * mean, y[1] * vb, y[2] * vb, y[3] * vb]) * (M // d)
    kt = np.array([y[4] * mean, y[5] * vt, y[6] * vt, y[7] * vt]) * M
    return kb, kt


def squeezing_profile(M, rbar, sr, seed):
    """r_j = clip(rbar + sr w_j, 0.5, 1.5), w_j standard normal (seeded)."""
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

    def profile(self, M, rbar, sr, net):
        return squeezing_profile(M, rbar, sr, self.seed * 7919 + net)

    def run(self, M, t, rbar, sr, d, E, net, n_sub=8, chunk=None):
        """One method run: the marginal of bin 0 (the first M // d modes) and
        the total count from the same samples.  Returns the 8 targets and the
        two distributions as (m, P, sigma) triples."""
        r = self.profile(M, rbar, sr, net)
        Mb = M // d
        d_run = 1 if d == 1 else 2
        bins = np.zeros(M, dtype=np.int32)
        bins[Mb:] = 1
        # windows from the independent-mode moments, widened for the
        # correlations that the network adds
        spans = [(Mb / M, 1.6)] + ([((M - Mb) / M, 1.6)] if d > 1 else []) + [(1.0, 1.2)]
        wins = []
        for frac, widen in spans:
            mean, sd = self.synth.uniform_loss_moments(r, t, frac=frac)
            wins.append(self.synth.count_window(mean, sd * widen + 2.0, nsig=10.0))
        ns = E // n_sub
        E = ns * n_sub  # whole sub-ensembles only
        chunk = min(chunk or E, E)
        p = CountsPipeline(t * self.haar(M), r, prec=self.prec, seed=self.seed, net=net,
                           bin_of_mode=bins, d=d_run, mode="marginals_and_total", windows=wins,
                           n_sub=n_sub, samples_per_sub=ns, chunk=chunk, device=self.device)
        p.run(E)
        P, _, s = p.result()
        out, off = [], 0
        for lo, K in wins:
            out.append((np.arange(lo, lo + K), P[off: off + K], s[off: off + K]))
            off += K
        kb = cumulants(out[0][0], out[0][1])
        kt = cumulants(out[-1][0], out[-1][1])
        return targets(M, t, r, d, kb, kt), (out[0], out[-1])


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


def generate(runner, sweeps, E, net0=0, log_every=0):
    X = np.stack([features(*s) for s in sweeps])
    Y = np.empty((len(sweeps), 2 * N_CUM))
    t0 = time.perf_counter()
    for i, s in enumerate(sweeps):
        Y[i], _ = runner.run(*s, E=E, net=net0 + i)
        if log_every and (i + 1) % log_every == 0:
            # progress goes to stderr: stdout carries the caller's result line
            print(f"[surrogate] {i + 1}/{len(sweeps)} sweeps, {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
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

    def step_raw(self, Xd, Yd, batch, lr, weight_decay=0.0):
        lib = _lib.load()
        _lib.check(lib.mp_mlp_loss_grad(ctypes.byref(self.shape), _ptr(self.w16), _ptr(self.params),
                                        _ptr(Xd), _ptr(Yd), batch, _ptr(self.grads), _ptr(self.loss),
                                        _ptr(self.ws), self.ws.numel(), _stream(None)))
        self.step_count += 1
        _lib.check(lib.mp_mlp_adam(ctypes.byref(self.shape), _ptr(self.params), _ptr(self.grads),
                                   _ptr(self.m), _ptr(self.v), _ptr(self.w16), lr, 0.9, 0.999, 1e-8,
                                   weight_decay, self.step_count, _stream(None)))

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
    def fit(self, X, Y, steps=300, batch=256, lr=2e-3, weight_decay=1.0, seed=0, log_every=0):
        """Mini-batch Adam with decoupled weight decay and a cosine learning
        rate.  The sweeps are noisy method estimates and the targets vary
        slowly, so training is short and strongly regularised: longer runs fit
        the noise and extrapolate worse in M."""
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
            self.step_raw(Xd[idx].contiguous(), Yd[idx].contiguous(), batch, lr_s, weight_decay)
            if log_every and (s % log_every == 0 or s == steps - 1):
                hist.append((s, float(self.loss.item())))
        return hist

    def predict(self, X):
        Xn = (np.atleast_2d(X) - self.x_mean) / self.x_std
        return self.predict_raw(Xn) * self.y_std + self.y_mean


# ---------------------------------------------------------------- screening

def screen(mlp, runner, M, t, d, candidates, E_check, top, tol_mean=0.01, tol_var=0.05,
           net0=100000):
    """Predicts the bin-0 cumulants of every candidate (rbar, sr) profile,
    selects the `top` candidates whose Fano factor (variance / mean) is
    closest to the middle of the predicted range, and runs the method on
    them.  The method's values replace a prediction (fallback) when the
    predicted mean or variance misses the method's by more than tol_mean or
    tol_var relative.  Each checked entry also carries the error of the
    independent-mode baseline alone, the part the network corrects."""
    profs = [runner.profile(M, rb, sr, net0 + q) for q, (rb, sr) in enumerate(candidates)]
    t0 = time.perf_counter()
    X = np.stack([features(M, t, rb, sr, d) for rb, sr in candidates])
    y = mlp.predict(X)
    mom = [moments_from_targets(M, t, r, d, yq) for r, yq in zip(profs, y)]
    t_pred = time.perf_counter() - t0
    fano = np.array([kb[1] / kb[0] for kb, _ in mom])
    target = 0.5 * (fano.min() + fano.max())
    order = np.argsort(np.abs(fano - target))[:top]
    checked = []
    t0 = time.perf_counter()
    for q in order:
        rb, sr = candidates[q]
        yq, ((m, P, s), _) = runner.run(M, t, rb, sr, d, E=E_check, net=net0 + int(q),
                                        chunk=min(E_check, 65536), n_sub=max(2, E_check // 8192))
        kb, _ = moments_from_targets(M, t, profs[q], d, yq)
        pb, _ = mom[q]
        base, _ = moments_from_targets(M, t, profs[q], d, np.ones(2 * N_CUM))
        sig_mean = float(np.sqrt(((m - kb[0]) ** 2 * s ** 2).sum()))
        e_mean = abs(pb[0] - kb[0]) / kb[0]
        e_var = abs(pb[1] - kb[1]) / kb[1]
        checked.append(dict(candidate=[rb, sr], predicted_mean=float(pb[0]),
                           predicted_var=float(pb[1]), method_mean=float(kb[0]),
                           method_var=float(kb[1]), sigma_mean=sig_mean,
                           mean_rel_err=float(e_mean), var_rel_err=float(e_var),
                           baseline_mean_rel_err=float(abs(base[0] - kb[0]) / kb[0]),
                           baseline_var_rel_err=float(abs(base[1] - kb[1]) / kb[1]),
                           fallback=bool(e_mean > tol_mean or e_var > tol_var)))
    t_method = time.perf_counter() - t0
    return dict(t_predict_s=t_pred, t_method_s=t_method, n_candidates=len(candidates),
                checked=checked)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sweeps", type=int, default=4000)
    ap.add_argument("--E", type=int, default=10000)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--screen-M", type=int, default=8000)
    ap.add_argument("--screen-E", type=int, default=1_048_576)
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
    res = screen(mlp, runner, args.screen_M, 0.95, 4, cands, args.screen_E, args.top)
    res.update(t_generate_s=t_gen, t_train_s=t_train, loss_history=hist, sweeps=args.sweeps,
               E=args.E)
    text = json.dumps(res, indent=1)
    if args.out:
        open(args.out, "w").write(text)
    print(text)


if __name__ == "__main__":
    main()
