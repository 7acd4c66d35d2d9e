"""Benchmark of the matrix-P hot path on one MI355X.

Workload: M = 8000 modes, Haar network x t = 0.95, r = 1 on every mode,
total-count distribution on the window [8083, 8083 + 3840) (mean 9972,
sd 209), sub-ensembles of 8192 samples.  One step = one chunk of 65536
samples through the whole path: mp_sample -> mp_propagate_counts (the mixed
MFMA GEMM whose epilogue forms the per-sample occupations, then the counting
kernels; --unfused writes C and counts from it).  The default mixed path is
the one-sided split (T as one FP16 value, samples hi/lo FP16, two products);
the three-product split-BF16 path and the FP32 path are timed on the same
workload.  All consume the same noise, so the ensemble size the criterion
needs is the same for all; the criterion job (pack T, the chunks that size
needs, inverse DFT) is timed end to end for each.

Prints one JSON line (last line of stdout).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "samples·M²/s and seconds to binned P(m) at 1σ≤1e-3, M=8000, mixed vs FP32"
# The split forms are priced against the dense FP16 (BF16) peak: the product
# they deliver is an FP16-operand contraction (the T-split form's FP8 MFMA only
# computes its correction term).
PEAKS_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "split_bf16": 2500.0, "split_fp16": 2500.0,
                "split1_fp16": 2500.0, "split1t_fp16": 2500.0, "split1t_f8": 2500.0}
# MFMA products per real multiply-add of the split forms, in FP16-product
# equivalents (hi*hi + hi*lo + lo*hi; one-sided: A*hi + A*lo or hi*B + lo*B;
# the FP8 correction form: one FP16 product and one FP8 product, which issues
# at twice the FP16 rate)
PRODUCTS = {"split_bf16": 3, "split_fp16": 3, "split1_fp16": 2, "split1t_fp16": 2,
            "split1t_f8": 1.5}
DTYPES = {"split_bf16": "split-bf16 (fp32 acc)", "split_fp16": "split-fp16 (fp32 acc)",
          "split1_fp16": "fp16 x split-fp16 (fp32 acc)",
          "split1t_fp16": "split-fp16 x fp16 (fp32 acc)",
          "split1t_f8": "fp16 x fp16 + e4m3 x e4m3 correction (fp32 acc)", "fp32": "fp32",
          "fp64": "f64"}
HBM_PEAK_GBS = 8000.0
# the GEMM kernel each precision runs: occupation-fused, C-writing
GEMM_KERNELS = {"split1t_f8": ("gemm_split1t8_occ", "gemm_split1t8_pp"),
                "split1t_fp16": ("gemm_split1t_occ", "gemm_split1t_pp"),
                "split1_fp16": ("gemm_split1_occ", "gemm_split1_pp"),
                "split_bf16": ("gemm_split_occ<bf16>", "gemm_split_256_pp<bf16>"),
                "split_fp16": ("gemm_split_occ<f16>", "gemm_split_256_pp<f16>"),
                "fp32": ("gemm_f32_pp<true>", "gemm_f32_pp<false>"),
                "fp64": ("gemm_f64_pp", "gemm_f64_pp")}

# FETCH_SIZE / WRITE_SIZE of the GEMM kernel at this workload (rocprofv3 --pmc,
# one counter per run, per dispatch), scaled by the factors a 1 GiB copy gives
# (fetch x2, write x1); valid only for the GEMM source they were taken from.
# Commands and per-kernel figures: profiles/m8000_gemm_traffic.md.
TRAFFIC = {
    ("split1t_f8", True): {"source_sha256_16": "7df0e3e2fad6d5c8",
                           "fetch_bytes": 3.696e7 * 1024 * 2, "write_bytes": 9.677e4 * 1024},
    ("split_bf16", True): {"source_sha256_16": "7df0e3e2fad6d5c8",
                           "fetch_bytes": 4.916e7 * 1024 * 2, "write_bytes": 9.677e4 * 1024},
    ("fp32", True): {"source_sha256_16": "7df0e3e2fad6d5c8",
                     "fetch_bytes": 4.903e7 * 1024 * 2, "write_bytes": 9.677e4 * 1024},
    # gemm_split1t8_bilin on the dense-W network of the bilinear_m8000 workload
    ("bilinear", True): {"source_sha256_16": "7df0e3e2fad6d5c8",
                         "fetch_bytes": 1.955e7 * 1024 * 2, "write_bytes": 3.231e5 * 1024},
}


def gemm_traffic_gb(prec, fused):
    """Counter-derived bytes per GEMM launch in GB, or None when the GEMM
    source has changed since the counters were taken."""
    import hashlib
    rec = TRAFFIC.get((prec, fused))
    if rec is None:
        return None
    src = os.path.join(ROOT, "paper_2503_12749_amd", "csrc", "propagate.hip")
    with open(src, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()[:16]
    if digest != rec["source_sha256_16"]:
        return None
    return round((rec["fetch_bytes"] + rec["write_bytes"]) / 1e9, 2)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed_run(mp, torch, pipe, steps, warmup, g_start=0):
    """Packs T, runs warmup + steps chunks; returns (seconds, per-launch GEMM
    ms, last g, pack ms)."""
    stream = torch.cuda.current_stream()
    E = pipe.chunk
    g = g_start
    pk = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    pk[0].record(stream)
    mp.mp_pack_transmission(pipe.M, pipe.T, pipe.prec, pipe.ws_prop)
    pk[1].record(stream)
    pipe.packed = True
    for _ in range(warmup):
        pipe.run_chunk(g, E)
        g += E
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        mp.mp_sample(pipe.M, g, E, pipe.r, pipe.seed, pipe.net, pipe.prec, pipe.ab, pipe.n)
        ev[i][0].record(stream)
        if pipe.fused:
            # GEMM with the occupation epilogue, then the counting kernels
            mp.mp_propagate_counts(pipe.M, E, pipe.prec, pipe.est, pipe.ab, pipe.n, pipe.ws_prop,
                                   pipe.d, pipe.bins, pipe.mode, pipe.m_lo, pipe.K, pipe.n_sub,
                                   pipe.ns, g, pipe.acc, pipe.ws_counts)
            ev[i][1].record(stream)
        else:
            mp.mp_propagate_packed(pipe.M, E, pipe.prec, pipe.ab, pipe.C, pipe.ws_prop)
            ev[i][1].record(stream)
            pipe.counts_chunk(g, E)
        g += E
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    gemm_ms = [a.elapsed_time(b) for a, b in ev]
    return secs, gemm_ms, g, pk[0].elapsed_time(pk[1])


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info()
                    if d.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def cpu_baseline(w, budget_s, synth):
    """The FP64 oracle on the host cores (never tuned): the M = 8000 workload
    on a bounded sample (whole pipeline: sampling, complex128 propagation,
    count-space G(m)), its propagation alone, both again on one core, and the
    M = 16 and M = 1000 configurations end to end."""
    from threadpoolctl import threadpool_limits
    from oracle import estimator, sampler

    def whole(wl, E, chunk):
        t = time.perf_counter()
        estimator.estimate(wl.T, wl.r, wl.seed, E, 1, wl.bins, 1, wl.windows, chunk=chunk)
        dt = time.perf_counter() - t
        return E * wl.M ** 2 / dt, dt

    def propagation(wl, E):
        a, b, _ = sampler.sample(wl.r, 0, E, wl.seed)
        t = time.perf_counter()
        estimator.propagate(wl.T, a, b)
        dt = time.perf_counter() - t
        return E * wl.M ** 2 / dt, dt

    threads = _blas_threads()
    E0 = 32
    _, dt = whole(w, E0, E0)
    E = int(max(E0, min(16384, E0 * budget_s / max(dt, 1e-3))))
    E = max(E0, (E // E0) * E0)
    rate, dt = whole(w, E, min(E, 512))
    prop_rate, prop_dt = propagation(w, 1024)
    with threadpool_limits(1):
        rate1, dt1 = whole(w, 64, 64)
        prop1, pdt1 = propagation(w, 128)
    c1 = synth.workload_small()
    c1_rate, c1_dt = whole(c1, c1.E, 2000)
    m1 = synth.workload_m1000(E=2000)
    m1_rate, m1_dt = whole(m1, 2000, 500)
    m1_prop, _ = propagation(m1, 2000)
    return {"value": rate, "unit": "samples·M²/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{E} samples of the M=8000 workload through the FP64 oracle "
                      f"(sampling, complex128 propagation, direct count-space G(m) on the "
                      f"{w.windows[0][1]}-count window), {dt:.1f} s",
            "os_cpu_count": os.cpu_count(), "blas_threads": int(threads),
            "legs": {
                "m8000_whole_pipeline": {"samples_M2_per_s": rate, "samples": E, "s": dt,
                                         "threads": int(threads)},
                "m8000_propagation_only": {"samples_M2_per_s": prop_rate, "samples": 1024,
                                           "s": prop_dt, "threads": int(threads)},
                "m8000_whole_pipeline_1_core": {"samples_M2_per_s": rate1, "samples": 64,
                                                "s": dt1, "threads": 1},
                "m8000_propagation_only_1_core": {"samples_M2_per_s": prop1, "samples": 128,
                                                  "s": pdt1, "threads": 1},
                "m16_whole_pipeline": {"samples_M2_per_s": c1_rate, "samples": c1.E,
                                       "s": c1_dt, "threads": int(threads),
                                       "workload": "M=16, Haar x t=0.5, r=1, E=1e4, K=128"},
                "m1000_whole_pipeline": {"samples_M2_per_s": m1_rate, "samples": 2000,
                                         "s": m1_dt, "threads": int(threads),
                                         "workload": "M=1000, Haar x t=0.9, r=1, window "
                                                     f"{m1.windows[0]}"},
                "m1000_propagation_only": {"samples_M2_per_s": m1_prop, "samples": 2000,
                                           "threads": int(threads)},
            }}


def criterion_job(mp, torch, w, prec, E_need, chunk, ns, fused):
    """The seconds-to-criterion job, timed end to end: pack T, run
    ceil(E_need / chunk) chunks (sample + fused GEMM + counts), finalize the
    inverse DFT; returns (seconds, samples, achieved max sigma_T / max P)."""
    n_chunks = max(1, math.ceil(E_need / chunk))
    E = n_chunks * chunk
    pipe = mp.CountsPipeline(w.T, w.r, prec=prec, seed=w.seed, windows=w.windows,
                             n_sub=E // ns, samples_per_sub=ns, chunk=chunk, fused=fused)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pipe.run(E)  # packs T on the first chunk, finalizes after the last
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    P, _, sig = pipe.result()
    del pipe
    torch.cuda.empty_cache()
    return secs, E, float(sig.max() / P.max())


def sustained_fp16_tflops(mp, torch, kind=0):
    """Executed TFLOP/s of the library's matrix-core probe with no memory
    traffic over about 50 ms: kind 0 back-to-back v_mfma_f32_32x32x16_f16,
    kind 3 the FP8-correction GEMM's mix (four of those and one FP8 MFMA per
    chain and round)."""
    iters = 200000 if kind == 0 else 80000
    sink = torch.empty(512 * 256, dtype=torch.float64, device="cuda:0")
    mp.mp_mfma_sustained(kind, 1000, sink)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    flops = mp.mp_mfma_sustained(kind, iters, sink)
    b.record()
    torch.cuda.synchronize()
    return flops / (a.elapsed_time(b) * 1e-3) / 1e12


def run_m8000(args, mp, torch, synth):
    """The headline workload (see the module docstring)."""
    t = time.perf_counter()
    E_total = args.chunk * (args.warmup + args.steps)
    w = synth.workload_m8000(E=E_total, chunk=args.chunk) if args.M == 8000 else None
    if w is None:
        M = args.M
        r = synth.squeezing_uniform(M, 1.0)
        mean, sd = synth.uniform_loss_moments(r, 0.95)
        w = synth.Workload(f"M{M}_t0.95_r1", M, 0.95, r, synth.transmission(M, 0.95, synth.SEED_BASE + 5),
                           E_total, E_total // 8192, synth.SEED_BASE + 5, synth.all_modes_bin(M), 1,
                           [synth.count_window(mean, sd)], args.chunk)
    log(f"[bench] workload {w.name}: Haar network ready in {time.perf_counter() - t:.1f} s")
    ns = 8192
    n_sub = E_total // ns

    results = {}
    legs = [(args.prec, args.steps), (args.compare, args.compare_steps)]
    if args.also and args.also != args.prec:
        legs.append((args.also, args.compare_steps))
    for prec, steps in legs:
        if not prec:
            continue
        fused = not args.unfused and prec != "fp64"
        pipe = mp.CountsPipeline(w.T, w.r, prec=prec, seed=w.seed, windows=w.windows,
                                 n_sub=n_sub, samples_per_sub=ns, chunk=args.chunk,
                                 fused=fused)
        secs, gemm_ms, g, pack_ms = timed_run(mp, torch, pipe, steps,
                                              args.warmup if prec == args.prec else 1)
        t0 = time.perf_counter()
        # statistics over the sub-ensembles completed so far
        done_sub = g // ns
        mp.mp_counts_finalize(1, "joint", pipe.K, done_sub, ns, pipe.acc, pipe.P_re, pipe.P_im,
                              pipe.sigma, None)
        torch.cuda.synchronize()
        fin_s = time.perf_counter() - t0
        P, _, sig = pipe.result()
        E_run = done_sub * ns
        crit = 1e-3 * P.max()
        if prec == args.prec:
            E_need = E_run * (sig.max() / crit) ** 2
        else:  # same noise, same accuracy: the main precision's estimate of E
            E_need = results[args.prec]["E_needed"]
        per_sample = secs / (steps * args.chunk)
        # secondary reading of the criterion: absolute sigma_T <= 1e-3, reached after a
        # handful of samples; sigma_T needs two sub-ensembles, so the run is at least 2 N_S
        E_abs = E_run * (sig.max() / 1e-3) ** 2
        secs_abs = max(E_abs, 2 * ns) * per_sample + fin_s + 1e-3 * pack_ms
        del pipe
        torch.cuda.empty_cache()
        job_s, job_E, job_ratio = criterion_job(mp, torch, w, prec, E_need, args.chunk, ns, fused)
        results[prec] = dict(
            secs=secs, steps=steps, ms_per_step=1e3 * secs / steps,
            value=steps * args.chunk * w.M ** 2 / secs,
            gemm_ms=float(np.mean(gemm_ms)), gemm_ms_all=[round(x, 3) for x in gemm_ms],
            sigma_max=float(sig.max()), P_max=float(P.max()), sumP=float(P.sum()),
            E_run=E_run, E_needed=float(E_need),
            seconds_to_criterion=job_s,
            criterion_job={"samples": job_E, "seconds": job_s,
                           "achieved_sigma_max_over_P_max": job_ratio,
                           "what": "pack T, ceil(E_needed / chunk) chunks of sample + GEMM + "
                                   "counts, inverse DFT; timed end to end"},
            seconds_to_criterion_extrapolated=float(E_need * per_sample + fin_s + 1e-3 * pack_ms),
            E_needed_absolute=float(E_abs), seconds_to_criterion_absolute=float(secs_abs),
            finalize_s=fin_s, pack_ms=pack_ms,
            mean=float((np.arange(w.windows[0][0], w.windows[0][0] + w.windows[0][1]) * P).sum()))
        log(f"[bench] {prec}: {results[prec]['ms_per_step']:.1f} ms/step, GEMM {results[prec]['gemm_ms']:.1f} ms, "
            f"{results[prec]['value']:.3e} samples*M^2/s, sigma_max {sig.max():.2e} (P_max {P.max():.2e}), "
            f"E needed {E_need:.3g}; criterion job {job_E} samples in {job_s:.3f} s, "
            f"sigma/P_max {job_ratio:.3e}")

    main_r = results[args.prec]
    flops = 8.0 * w.M ** 2 * args.chunk
    achieved = flops / (main_r["gemm_ms"] * 1e-3) / 1e12
    peak = PEAKS_TFLOPS[args.prec]
    roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": (gemm_traffic_gb(args.prec, not args.unfused)
                        if w.M == 8000 and args.chunk == 65536 else None),
            "traffic_unit": "GB per launch (FETCH_SIZE x2 + WRITE_SIZE x1, calibrated on a 1 GiB copy)",
            "kernel": (f"{GEMM_KERNELS[args.prec][0]} (mp_propagate_counts: the GEMM with the "
                       f"occupation epilogue; the timed call includes the counting kernels)"
                       if not args.unfused
                       else f"{GEMM_KERNELS[args.prec][1]} (mp_propagate_packed)"),
            "algorithmic_flops_per_launch": flops}
    if args.prec in PRODUCTS:
        roof["executed_mfma_frac"] = round(PRODUCTS[args.prec] * achieved / peak, 4)
        roof["mfma_products"] = PRODUCTS[args.prec]
        if args.prec != "split_bf16":
            # the FP16 matrix cores' sustained rate on this machine with no memory
            # traffic (about one GEMM's duration), as context for the fraction
            sust = sustained_fp16_tflops(mp, torch)
            roof["sustained_fp16_mfma_tflops_measured"] = round(sust, 1)
            roof["executed_frac_of_sustained"] = round(PRODUCTS[args.prec] * achieved / sust, 4)
        if args.prec == "split1t_f8":
            # the same probe running this kernel's own instruction mix: its
            # product of depth 64 is half of the mix's executed flops
            mix = sustained_fp16_tflops(mp, torch, kind=3)
            roof["sustained_f16_f8_mix_tflops_measured"] = round(mix, 1)
            roof["frac_of_sustained_mix"] = round(achieved / (0.5 * mix), 4)
    out = {
        "metric": METRIC,
        "value": main_r["value"],
        "unit": "samples·M²/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES.get(args.prec, args.prec),
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: M={w.M}, Haar x t={w.t}, r=1, total counts on window "
                        f"[{w.windows[0][0]}, {w.windows[0][0] + w.windows[0][1]}), "
                        f"{args.chunk} samples per step, sub-ensembles of {ns}",
            "precision": args.prec,
            "seconds_to_criterion": main_r["seconds_to_criterion"],
            "criterion_job": main_r["criterion_job"],
            "seconds_to_criterion_extrapolated": main_r["seconds_to_criterion_extrapolated"],
            "criterion_absolute": {"criterion": "max_m sigma_T(m) <= 1e-3 (absolute)",
                                   "E_needed": main_r["E_needed_absolute"],
                                   "seconds": main_r["seconds_to_criterion_absolute"]},
            "criterion": "max_m sigma_T(m) <= 1e-3 * max_m P(m)",
            "E_needed": main_r["E_needed"],
            "sigma_max": main_r["sigma_max"], "P_max": main_r["P_max"], "sum_P": main_r["sumP"],
            "gemm_ms": main_r["gemm_ms"], "pack_ms": main_r["pack_ms"],
        },
        "roofline": roof,
    }
    for key, prec in (("compare", args.compare), ("also", args.also)):
        if prec and prec in results and prec != args.prec:
            c = results[prec]
            out["config"][key] = {
                "precision": prec, "value": c["value"], "steps": c["steps"],
                "ms_per_step": c["ms_per_step"], "gemm_ms": c["gemm_ms"],
                "gemm_ms_all": c["gemm_ms_all"],
                "seconds_to_criterion": c["seconds_to_criterion"],
                "criterion_job": c["criterion_job"],
                "speedup_mixed_vs_this": main_r["value"] / c["value"],
                "criterion_speedup_mixed_vs_this": c["seconds_to_criterion"] / main_r["seconds_to_criterion"],
                "gemm_tflops": 8.0 * w.M ** 2 * args.chunk / (c["gemm_ms"] * 1e-3) / 1e12,
            }
    if args.compare in results:
        out["config"]["compare"]["speedup_mixed_vs_compare"] = \
            main_r["value"] / results[args.compare]["value"]
    if args.bilinear and args.M == 8000 and args.prec == "split1t_f8":
        # the same distribution through the bilinear form, on a network whose W is
        # dense (the headline network's W is a multiple of the identity)
        out["config"]["one_distribution_bilinear_form"] = dict(
            network="diag(l) x the same Haar unitary, l ~ U[0.9, 1] (W dense)",
            **_bilinear_pair(mp, torch, w, _dense_w_network(w, synth), "dense_W", args.chunk,
                             8192, 3))
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 CPU oracle on bounded samples ...")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget, synth)
    return out



def _timed(torch, fn):
    """Wall time of fn() between two device synchronisations, in seconds."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def _envelope(metric, value, unit, ms, workload, dtype, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": dtype, "data": "synthetic", "config": {"workload": workload}}
    out["config"].update(extra)
    return out


def run_joint_m1000(args, mp, torch, synth):
    """M = 1000, Haar x 0.9, r = 1, E = 1.2e6 in chunks of 1e5 (120 sub-ensembles
    of 1e4), FP32: the total-count run and the two-bin joint run (halves of
    500 modes) on the same noise, each timed as a whole job (pack, all chunks,
    finalize) after one untimed run."""
    w = synth.workload_m1000()
    bins2 = synth.contiguous_bins(w.M, 2)
    mh, sh = synth.uniform_loss_moments(w.r, w.t, frac=0.5)
    wh = synth.count_window(mh, sh)
    res = {}
    for name, kw in (("total", dict(windows=w.windows)),
                     ("joint2", dict(bin_of_mode=bins2, d=2, mode="joint", windows=[wh, wh]))):
        p = mp.CountsPipeline(w.T, w.r, prec="fp32", seed=w.seed, n_sub=w.n_sub,
                              samples_per_sub=w.samples_per_sub, chunk=w.chunk, **kw)
        p.run()

        def job():
            p.reset()
            p.packed = False
            p.run()
        secs = _timed(torch, job)
        P, _, sig = p.result()
        res[name] = dict(s=secs, P=P, sigma=sig)
        log(f"[bench] joint_m1000 {name}: {secs:.3f} s for E={w.E}")
        del p
        torch.cuda.empty_cache()
    K = wh[1]
    Pj = res["joint2"]["P"].reshape(K, K)
    Pt, st = res["total"]["P"], res["total"]["sigma"]
    m_tot = np.arange(w.windows[0][0], w.windows[0][0] + w.windows[0][1])
    diag = np.zeros_like(Pt)
    sums = np.add.outer(np.arange(K), np.arange(K)) + 2 * wh[0]
    ok = (sums >= m_tot[0]) & (sums <= m_tot[-1])
    np.add.at(diag, sums[ok] - m_tot[0], Pj[ok])
    sj = res["joint2"]["s"]
    return _envelope(
        "samples·M²/s of the two-bin joint run, M=1000, FP32", w.E * w.M ** 2 / sj, "samples·M²/s",
        1e3 * sj / (w.E / w.chunk),
        f"M1000_t0.9_r1: E={w.E} in chunks of {w.chunk}, {w.n_sub} sub-ensembles, total window "
        f"{tuple(w.windows[0])}, joint windows {tuple(wh)} x {tuple(wh)}", "fp32",
        total_run_s=res["total"]["s"], joint_run_s=sj,
        total_samples_M2_per_s=w.E * w.M ** 2 / res["total"]["s"],
        joint_vs_total_max_abs=float(np.abs(diag - Pt).max()), total_sigma_max=float(st.max()),
        joint_sum_P=float(Pj.sum()), joint_P_max=float(Pj.max()))


def run_precision_m4000(args, mp, torch, synth):
    """M = 4000, Haar x 0.95, r_j ~ U[0.5, 1.5], four equal mode blocks (their
    marginals and the total), E = 983040 in chunks of 65536 (120 sub-ensembles
    of 8192): every precision on the same noise, each result compared with
    the FP64 GPU path (itself pinned to the oracle) bin by bin, in units of
    the FP64 run's sigma_T."""
    chunk, ns = 65536, 8192
    w = synth.workload_m4000(E=15 * chunk, chunk=chunk, ns=ns)
    M, T, r, seed, bins, wins = w.M, w.T, w.r, w.seed, w.bins, w.windows
    E = w.E
    res = {}
    for prec in ("fp64", "fp32", "split_bf16", "split_fp16", "split1_fp16", "split1t_fp16",
                 "split1t_f8"):
        p = mp.CountsPipeline(T, r, prec=prec, seed=seed, bin_of_mode=bins, d=4,
                              mode="marginals_and_total", windows=wins, n_sub=E // ns,
                              samples_per_sub=ns, chunk=chunk)
        p.run_chunk(0, chunk)  # untimed: first launches
        p.reset()

        def job():
            p.packed = False
            p.run()
        secs = _timed(torch, job)
        res[prec] = (secs,) + p.result()
        log(f"[bench] precision_m4000 {prec}: {secs:.3f} s")
        del p
        torch.cuda.empty_cache()
    off = np.cumsum([0] + [k for _, k in wins])
    s64, P64, sig64 = res["fp64"][0], res["fp64"][1], res["fp64"][3]
    per = {}
    for prec in ("fp32", "split_bf16", "split_fp16", "split1_fp16", "split1t_fp16", "split1t_f8"):
        secs, P = res[prec][0], res[prec][1]
        rows = []
        for b in range(5):
            sl = slice(off[b], off[b + 1])
            err = np.abs(P[sl] - P64[sl])
            bulk = P64[sl] > 1e-3 * P64[sl].max()
            rows.append({"dist": f"bin {b}" if b < 4 else "total", "max_abs_err": float(err.max()),
                         "max_err_over_sigma": float((err / sig64[sl])[bulk].max()),
                         "sigma_max": float(sig64[sl].max())})
        per[prec] = {"run_s": secs, "samples_M2_per_s": E * M ** 2 / secs,
                     "speedup_vs_fp64": s64 / secs, "per_distribution": rows}
    sb = res["split_bf16"][0]
    return _envelope(
        "samples·M²/s, M=4000 four-bin run, split-BF16 (error vs FP64 per bin in config)",
        E * M ** 2 / sb, "samples·M²/s", 1e3 * sb / (E / chunk),
        f"M4000_t0.95_rU[0.5,1.5]: 4 equal bins + total, E={E} in chunks of {chunk}, "
        f"{E // ns} sub-ensembles", "split-bf16 (fp32 acc)",
        fp64_run_s=s64, fp64_samples_M2_per_s=E * M ** 2 / s64, precisions=per)


def run_precision_m8000(args, mp, torch, synth):
    """The headline workload at the criterion's sample count: M = 8000, Haar x
    0.95, r = 1, total counts, E = 11 chunks of 65536 (88 sub-ensembles of
    8192, max sigma_T / max P about 1e-3), every precision through the
    benchmark's launch (the occupation-fused GEMM; FP64 through C) on the same
    noise, each compared with the FP64 GPU path bin by bin in units of its
    sigma_T."""
    chunk, ns = 65536, 8192
    E = 11 * chunk
    w = synth.workload_m8000(E=E, chunk=chunk)
    res = {}
    for prec in ("fp64", "split1t_f8", "split1t_f8_bilinear", "split1t_fp16", "split1_fp16",
                 "split_bf16", "fp32"):
        bil = prec.endswith("_bilinear")
        p = mp.CountsPipeline(w.T, w.r, prec=prec.replace("_bilinear", ""), seed=w.seed,
                              windows=w.windows, n_sub=E // ns, samples_per_sub=ns, chunk=chunk,
                              fused=prec != "fp64" and not bil, bilinear=bil)
        secs = _timed(torch, p.run)
        res[prec] = (secs,) + p.result()
        log(f"[bench] precision_m8000 {prec}: {secs:.3f} s")
        del p
        torch.cuda.empty_cache()
    s64, P64, sig64 = res["fp64"][0], res["fp64"][1], res["fp64"][3]
    bulk = P64 > 1e-3 * P64.max()
    per = {}
    for prec in ("split1t_f8", "split1t_f8_bilinear", "split1t_fp16", "split1_fp16", "split_bf16",
                 "fp32"):
        secs, P = res[prec][0], res[prec][1]
        err = np.abs(P - P64)
        per[prec] = {"run_s": secs, "max_abs_err": float(err.max()),
                     "max_err_over_sigma": float((err / sig64)[bulk].max()),
                     "mean_err_over_sigma": float((err / sig64)[bulk].mean())}
        log(f"[bench] precision_m8000 {prec}: max |P - P64| / sigma_T = "
            f"{per[prec]['max_err_over_sigma']:.3e}")
    main = res["split1t_f8"][0]
    return _envelope(
        "samples·M²/s, M=8000 run to max sigma_T <= 1e-3 max P, T-split with the FP8 "
        "correction (error vs FP64 per bin in config)",
        E * w.M ** 2 / main, "samples·M²/s", 1e3 * main / (E / chunk),
        f"M8000_t0.95_r1: total counts, E={E} in chunks of {chunk}, {E // ns} sub-ensembles",
        DTYPES["split1t_f8"], fp64_run_s=s64,
        sigma_max_over_P_max=float(sig64.max() / P64.max()), precisions=per)


def _bilinear_pair(mp, torch, w, T, name, chunk, ns, steps):
    """The T form and the bilinear form of one network (FP8-correction
    precision, one total-count distribution): ms per step, the GEMM call (HIP
    events), the first chunk with packing T or forming W, the criterion job
    (10 chunks) end to end, and the largest difference of the two forms' P(m)
    on the same noise in units of sigma_T."""
    E_job = 10 * chunk
    res = {}
    for form, kw in (("T_form", dict(fused=True)), ("bilinear", dict(bilinear=True))):
        n_sub = (steps + 2) * chunk // ns
        p = mp.CountsPipeline(T, w.r, prec="split1t_f8", seed=w.seed, windows=w.windows,
                              n_sub=n_sub, samples_per_sub=ns, chunk=chunk, **kw)
        first = _timed(torch, lambda: p.run_chunk(0, chunk))
        p.run_chunk(chunk, chunk)
        stream = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            g = (2 + i) * chunk
            mp.mp_sample(p.M, g, chunk, p.r, p.seed, p.net, p.prec, p.ab, p.n)
            ev[i][0].record(stream)
            if form == "bilinear":
                mp.mp_propagate_counts_bilinear(p.M, chunk, p.prec, p.est, p.ab, p.n, p.ws_prop,
                                                p.m_lo[0], p.K[0], p.n_sub, p.ns, g, p.acc,
                                                p.ws_counts)
            else:
                mp.mp_propagate_counts(p.M, chunk, p.prec, p.est, p.ab, p.n, p.ws_prop, p.d, p.bins,
                                       p.mode, p.m_lo, p.K, p.n_sub, p.ns, g, p.acc, p.ws_counts)
            ev[i][1].record(stream)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        gemm = float(np.median([a.elapsed_time(b) for a, b in ev]))
        del p
        torch.cuda.empty_cache()
        job = mp.CountsPipeline(T, w.r, prec="split1t_f8", seed=w.seed, windows=w.windows,
                                n_sub=E_job // ns, samples_per_sub=ns, chunk=chunk, **kw)
        job_s = _timed(torch, lambda: job.run(E_job))
        P, _, sig = job.result()
        del job
        torch.cuda.empty_cache()
        flops = (4 if form == "bilinear" else 8) * w.M ** 2 * chunk
        res[form] = {"ms_per_step": ms, "gemm_call_ms": gemm,
                     "first_chunk_ms_with_pack": 1e3 * first, "job_s": job_s, "job_samples": E_job,
                     "sigma_max_over_P_max": float(sig.max() / P.max()),
                     "gemm_algorithmic_tflops": flops / gemm / 1e9, "_P": P, "_sig": sig}
        log(f"[bench] bilinear {name} {form}: {ms:.2f} ms/step, GEMM call {gemm:.2f} ms, "
            f"first chunk {1e3 * first:.1f} ms, job {job_s:.3f} s")
    a, b = res["T_form"], res["bilinear"]
    bulk = a["_P"] > 1e-3 * a["_P"].max()
    res["max_diff_over_sigma"] = float((np.abs(a["_P"] - b["_P"]) / a["_sig"])[bulk].max())
    res["step_speedup"] = a["ms_per_step"] / b["ms_per_step"]
    res["job_speedup"] = a["job_s"] / b["job_s"]
    for f in ("T_form", "bilinear"):
        del res[f]["_P"], res[f]["_sig"]
    log(f"[bench] bilinear {name}: step {res['step_speedup']:.2f}x, job {res['job_speedup']:.2f}x, "
        f"max |P_T - P_bilinear| / sigma_T {res['max_diff_over_sigma']:.2e}")
    return res


def _dense_w_network(w, synth):
    """The headline network's Haar unitary with mode-dependent output loss
    l_j ~ U[0.9, 1]: T = diag(l) U, so W = T^T T* is dense (for the headline
    network itself W = 0.9025 I and the bilinear GEMM's operand is zero)."""
    l = np.random.default_rng(synth.SEED_BASE + 77).uniform(0.9, 1.0, w.M)
    return l[:, None] * (w.T / w.t)


def run_bilinear_m8000(args, mp, torch, synth):
    """One count distribution through the bilinear form n_S = alpha^T W beta
    (W = T^T P_S T*, formed once; the GEMM applies W's off-diagonal part to
    beta alone: 4 M^2 flops per sample instead of 8 M^2) against the T form,
    both in the FP8-correction precision, at M = 8000 on two networks: the
    headline one (Haar x 0.95, total counts: W = 0.9025 I, so the GEMM's
    operand is zero and draws less power than a general one) and the same Haar
    unitary with output loss l_j ~ U[0.9, 1] (W dense), the representative
    case, which gives the line's value."""
    chunk, ns = args.chunk, 8192
    steps = max(args.steps, 3)
    w = synth.workload_m8000(E=chunk, chunk=chunk)
    nets = {"haar_x0.95": w.T, "output_loss_0.9_1": _dense_w_network(w, synth)}
    res = {name: _bilinear_pair(mp, torch, w, T, name, chunk, ns, steps)
           for name, T in nets.items()}
    rep_ = res["output_loss_0.9_1"]["bilinear"]
    out = _envelope(
        "samples·M²/s, one count distribution at M=8000 through the bilinear form (general network)",
        chunk * w.M ** 2 / (rep_["ms_per_step"] / 1e3), "samples·M²/s", rep_["ms_per_step"],
        "M8000_r1: total counts on [8083, 11923), 65536 samples per step; networks Haar x 0.95 "
        "(W = 0.9025 I) and diag(l) Haar with l ~ U[0.9, 1] (W dense)",
        DTYPES["split1t_f8"], networks=res)
    achieved = rep_["gemm_algorithmic_tflops"]
    out["roofline"] = {
        "bound": "mfma", "achieved": round(achieved, 2), "peak": PEAKS_TFLOPS["split1t_f8"],
        "unit": "TFLOP/s", "frac": round(achieved / PEAKS_TFLOPS["split1t_f8"], 4),
        "traffic": gemm_traffic_gb("bilinear", True),
        "traffic_unit": "GB per launch (FETCH_SIZE x2 + WRITE_SIZE x1, calibrated on a 1 GiB copy)",
        "kernel": "gemm_split1t8_bilin (mp_propagate_counts_bilinear, dense-W network: the GEMM "
                  "with the bilinear epilogue; the timed call includes the counting kernels)",
        "algorithmic_flops_per_launch": 4.0 * w.M ** 2 * chunk}
    return out


def _batched_leg(mp, torch, nets, chunk, label, prec="split_fp16"):
    """One plan over `nets` (tuned, tuning cache in a temporary file), the same
    plan with every network forced to the 128-sample tile (three-product
    splits, which have two tile widths), and the networks run one after
    another through the fused CountsPipeline; seconds per job (best of three)
    and whether they agree bit for bit."""
    tmp = tempfile.TemporaryDirectory(prefix="mpgbs_tune_")
    cache = os.path.join(tmp.name, "tune.json")
    t0 = time.perf_counter()
    plan = mp.Plan(nets, prec=prec, chunk=chunk, tune_cache=cache)
    create_s = time.perf_counter() - t0
    plan.launch()
    plan_s = min(_timed(torch, plan.launch) for _ in range(3))
    info = plan.info()
    res = [plan.result(i)[0] for i in range(len(nets))]
    plan.close()
    log(f"[bench] {label}: tuned plan {plan_s:.4f} s, {info}")
    wide_s, same = None, True
    if not prec.startswith("split1"):  # the one-sided forms have one tile width
        # the same order and prefetch with every network on the 128-sample tile
        with open(cache) as f:
            (key, entry), = json.load(f).items()
        entry["nj"] = ",".join(["4"] * len(nets))
        with open(cache, "w") as f:
            json.dump({key: entry}, f)
        wide = mp.Plan(nets, prec=prec, chunk=chunk, tune_cache=cache)
        wide.launch()
        wide_s = min(_timed(torch, wide.launch) for _ in range(3))
        same = all(np.array_equal(wide.result(i)[0], res[i]) for i in range(len(nets)))
        wide.close()
    tmp.cleanup()
    seq_s = 0.0
    for i, n in enumerate(nets):
        p = mp.CountsPipeline(n["T"], n["r"], prec=prec, seed=n["seed"], net=n["net"],
                              windows=[n["window"]], n_sub=n["n_sub"],
                              samples_per_sub=n["E"] // n["n_sub"], chunk=chunk, fused=True)
        p.run()

        def job():  # T stays packed, as in the plan
            p.reset()
            p.run()
        seq_s += min(_timed(torch, job) for _ in range(3))
        same = same and np.array_equal(p.result()[0], res[i])
        del p
        torch.cuda.empty_cache()
    log(f"[bench] {label}: all 128-sample tiles {wide_s} s, sequential {seq_s:.4f} s, "
        f"same bits {same}")
    return dict(precision=prec, plan_s=plan_s, plan_all_128_sample_tiles_s=wide_s,
                sequential_s=seq_s, speedup_vs_sequential=seq_s / plan_s,
                tile_choice_speedup=None if wide_s is None else wide_s / plan_s,
                plan_create_s=create_s, plan_info=info, same_bits_plan_wide_sequential=same)


def run_batched(args, mp, torch, synth):
    """16 networks (4 each of M = 500, 1000, 2000, 4000), t ~ U[0.85, 0.99],
    r = 1, E = 2e5 each (20 sub-ensembles of 1e4): one plan (a captured
    hipGraph with one persistent grouped GEMM launch with the
    occupation-fused epilogue per pass over chunks of 1e5) against the same
    networks run one after another through the fused CountsPipeline.  The
    line of record runs the default mixed precision (the T-split form with
    its correction product in FP8); further legs run the T-split FP16 form
    (two FP16 products), the three-product split FP16, whose plans also
    choose a tile width per size class, and the latter at E = 4096 (4
    sub-ensembles of 1024), where a single network offers the 256 compute
    units few GEMM tiles."""
    E, n_sub, chunk = 200_000, 20, 100_000
    Ms = synth.BATCHED_SIZES
    work = sum(E * M ** 2 for M in Ms)
    log("[bench] batched: creating the plans (autotuned order, prefetch, tiles)")
    main = _batched_leg(mp, torch, synth.batched_networks(E=E, n_sub=n_sub), chunk,
                        "batched T-split FP8 correction", prec="split1t_f8")
    tsplit = _batched_leg(mp, torch, synth.batched_networks(E=E, n_sub=n_sub), chunk,
                          "batched T-split", prec="split1t_fp16")
    tsplit["samples_M2_per_s"] = work / tsplit["plan_s"]
    three = _batched_leg(mp, torch, synth.batched_networks(E=E, n_sub=n_sub), chunk,
                         "batched three-product split")
    three["samples_M2_per_s"] = work / three["plan_s"]
    small = _batched_leg(mp, torch, synth.batched_networks(E=4096, n_sub=4), 4096,
                         "batched three-product E=4096")
    small["samples_M2_per_s"] = sum(4096 * M ** 2 for M in Ms) / small["plan_s"]
    plan_s = main["plan_s"]
    return _envelope(
        "samples·M²/s over 16 uneven networks in one plan, split-FP16", work / plan_s,
        "samples·M²/s", 1e3 * plan_s,
        "16 networks: 4 x M in {500, 1000, 2000, 4000}, t ~ U[0.85, 0.99], r = 1, E = 2e5 "
        "each in chunks of 1e5, total counts", DTYPES["split1t_f8"],
        **main, algorithmic_tflops_whole_job=8.0 * work / plan_s / 1e12,
        t_split_fp16=tsplit, three_product_split_fp16=three,
        three_product_split_fp16_e4096=small)


def run_surrogate(args, mp, torch, synth):
    """The learned surrogate end to end: method-generated training sweeps
    (M in [100, 2000], t in [0.8, 0.99], rbar in [0.5, 1.5], s_r in [0, 0.3],
    d in {1, 2, 4}; E = 1e4 each), GPU training, then screening of 256
    candidate profiles at M = 8000, t = 0.95, d = 4 with the method
    (E = 2^20 per checked candidate) as the check."""
    from paper_2503_12749_amd import surrogate as sg
    rng = np.random.default_rng(2503)
    runner = sg.MethodRunner()
    sweeps = sg.sample_sweeps(args.sweeps, rng)
    t0 = time.perf_counter()
    X, Y = sg.generate(runner, sweeps, E=args.sweep_E, log_every=max(1, args.sweeps // 10))
    gen_s = time.perf_counter() - t0
    net = sg.Mlp(seed=3)
    t0 = time.perf_counter()
    hist = net.fit(X, Y, steps=300, batch=256, lr=2e-3, weight_decay=1.0, seed=2, log_every=50)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    cands = [(float(a), float(b)) for a in np.linspace(0.6, 1.4, 16) for b in np.linspace(0.0, 0.3, 16)]
    log("[bench] surrogate: screening at M=8000")
    res = sg.screen(net, runner, 8000, 0.95, 4, cands, 1 << 20, 8)
    errs = [{k: j[k] for k in ("mean_rel_err", "var_rel_err", "baseline_mean_rel_err",
                               "baseline_var_rel_err", "fallback")} for j in res["checked"]]
    per_method = res["t_method_s"] / len(res["checked"])
    return _envelope(
        "candidates screened per second by the surrogate, M=8000 (method time per candidate in config)",
        len(cands) / res["t_predict_s"], "candidates/s", 1e3 * res["t_predict_s"],
        f"surrogate: {args.sweeps} training sweeps at E={args.sweep_E}, screening 256 profiles at M=8000, "
        f"t=0.95, d=4, check E=2^20", "bf16 weights, fp32 accumulate",
        generate_s=gen_s, train_s=train_s, loss_first_last=[hist[0][1], hist[-1][1]],
        predict_s_256=res["t_predict_s"], method_s_per_candidate=per_method,
        speedup_vs_method=per_method * len(cands) / res["t_predict_s"],
        fallback_rule="method replaces a prediction off by > 1 % (mean) or > 5 % (variance)",
        checked=errs)


def _golden(name):
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        return json.load(f)


def run_plusp_m20(args, mp, torch, synth):
    """Appendix A comparison: a lossless 20-mode Haar network with r = 0.5 on
    every mode, E = 2.4e8 samples (120 sub-ensembles of 2e6) through the FP64
    path.  From the same samples: the total-count distribution with the
    matrix-P and the +P estimators (errors against the exact law at
    E = 2.4e5 and 2.4e8), and densities of the per-sample observables
    G_+(3), G_+(4) (bins of 0.05) and G_0(4) (bins of 0.001)."""
    M, r0 = 20, 0.5
    seed = synth.SEED_BASE + 11
    T = synth.haar_unitary(M, seed)
    r = np.full(M, r0)
    n_sub, ns, chunk = 120, 2_000_000, 1_000_000
    E = n_sub * ns
    small = 240_000  # the smaller ensemble of the comparison: 120 x 2000
    win = (0, 64)
    ref = np.asarray(_golden("lossless_m20_r0.5.json")["P"])
    hists = {"G+(3)": ("plus_p", 3, -20.0 + 1e-9, 0.05, 800),
             "G+(4)": ("plus_p", 4, -20.0 + 1e-9, 0.05, 800),
             "G0(4)": ("matrix_p", 4, -0.05 + 1e-9, 0.001, 500)}
    pipes = {est: mp.CountsPipeline(T, r, prec="fp64", seed=seed, windows=[win], n_sub=n_sub,
                                    samples_per_sub=ns, chunk=chunk, est=est)
             for est in ("matrix_p", "plus_p")}
    p = pipes["matrix_p"]
    nq = torch.empty(chunk * 2, dtype=torch.float64, device="cuda:0")
    hbuf = {k: torch.zeros(n_sub * (v[4] + 2), dtype=torch.float64, device="cuda:0")
            for k, v in hists.items()}
    allm = np.zeros(M, dtype=np.int32)
    # the small ensemble: its own sub-ensembles (120 x 2000) over the first samples
    small_p = {est: mp.CountsPipeline(T, r, prec="fp64", seed=seed, windows=[win], n_sub=120,
                                      samples_per_sub=small // 120, chunk=small, est=est)
               for est in ("matrix_p", "plus_p")}
    for est, sp in small_p.items():
        sp.run()
    t0 = time.perf_counter()
    mp.mp_pack_transmission(M, p.T, "fp64", p.ws_prop)
    for g in range(0, E, chunk):
        mp.mp_sample(M, g, chunk, p.r, seed, 0, "fp64", p.ab, p.n)
        mp.mp_propagate_packed(M, chunk, "fp64", p.ab, p.C, p.ws_prop)
        for est, q in pipes.items():
            mp.mp_binned_counts(M, chunk, p.C, p.n, "fp64", est, 1, allm, "joint", [win[0]],
                                [win[1]], n_sub, ns, g, q.acc, q.ws_counts)
        mp.mp_occupations(M, chunk, p.C, "fp64", 1, allm, "marginals", nq)
        for k, (est, m, lo, w, nb) in hists.items():
            mp.mp_observable_histogram(chunk, p.n, nq, 1, 0, m, est, lo, w, nb, n_sub, ns, g,
                                       hbuf[k])
        if (g // chunk) % 40 == 0:
            log(f"[bench] plusp_m20: {g + chunk} / {E} samples")
    for q in pipes.values():
        q.finalize()
    torch.cuda.synchronize()
    run_s = time.perf_counter() - t0
    res = {}
    for label, group in (("E=2.4e5", small_p), ("E=2.4e8", pipes)):
        for est, q in group.items():
            P, _, sig = q.result()
            err = np.abs(P - ref)
            bulk = ref > 1e-6 * ref.max()
            res[f"{est} {label}"] = {"max_abs_err_vs_exact": float(err.max()),
                                     "sigma_T_max": float(np.nanmax(sig)),
                                     "max_err_over_sigma_bulk": float((err / sig)[bulk].max()),
                                     "max_abs_P_odd_m": float(np.abs(P[1::2]).max()),
                                     "sum_P": float(P.sum())}
    dens = {}
    for k, (est, m, lo, w, nb) in hists.items():
        d = torch.empty(nb + 2, dtype=torch.float64, device="cuda:0")
        s = torch.empty(nb + 2, dtype=torch.float64, device="cuda:0")
        mp.mp_subensemble_stats(n_sub, ns, nb + 2, 1, 1.0 / w, hbuf[k], d, s)
        counts = hbuf[k].cpu().numpy().reshape(n_sub, nb + 2).sum(0)
        dd = d.cpu().numpy()
        centers = lo + w * (np.arange(nb) + 0.5)
        occupied = np.flatnonzero(counts[1:-1])
        inner = (centers > -0.5) & (centers < 0.5)
        entry = {"below_range": int(counts[0]), "above_range": int(counts[-1]),
                 "lowest_occupied_bin_center": float(centers[occupied[0]]) if occupied.size else None,
                 "highest_occupied_bin_center": float(centers[occupied[-1]]) if occupied.size else None,
                 "fraction_outside_[-0.5,0.5]": float(1.0 - counts[1:-1][inner].sum() / E)}
        if k == "G0(4)":
            lo_peak = (centers < 0.1)
            hi_peak = (centers > 0.3)
            entry["peak_near_0"] = float(centers[lo_peak][np.argmax(dd[1:-1][lo_peak])])
            entry["peak_high"] = float(centers[hi_peak][np.argmax(dd[1:-1][hi_peak])])
        dens[k] = entry
    mpe = res["matrix_p E=2.4e8"]["max_abs_err_vs_exact"]
    ppe = res["plus_p E=2.4e8"]["max_abs_err_vs_exact"]
    return _envelope(
        "max |P - P_exact|, +P over matrix-P, lossless M=20, r=0.5, E=2.4e8", ppe / mpe,
        "ratio", 1e3 * run_s,
        "M20_r0.5 lossless Haar, FP64, E=2.4e8 in 120 sub-ensembles of 2e6 (comparison at 2.4e5: "
        "120 x 2000), total counts m = 0..63", "f64",
        run_s=run_s, estimators=res, densities=dens,
        density_bins={k: {"estimator": v[0], "m": v[1], "o_min": v[2], "width": v[3],
                          "n_bins": v[4]} for k, v in hists.items()})


def run_moments_m1000(args, mp, torch, synth):
    """Many tests from one ensemble (main text): the M = 1000, t = 0.9, r = 1
    FP32 workload (E = 1.2e6, chunks of 1e5) yields the two half-bin
    marginals and the total count distribution and, from the same samples,
    the normally ordered moments k = 1..4 of the halves and the total.  The
    first two are compared with the closed forms; timing with and without the
    moments."""
    w = synth.workload_m1000()
    bins = synth.contiguous_bins(w.M, 2)
    mh, sh = synth.uniform_loss_moments(w.r, w.t, frac=0.5)
    wh = synth.count_window(mh, sh)
    wins = [wh, wh, tuple(w.windows[0])]
    kmax, nd = 4, 3
    p = mp.CountsPipeline(w.T, w.r, prec="fp32", seed=w.seed, bin_of_mode=bins, d=2,
                          mode="marginals_and_total", windows=wins, n_sub=w.n_sub,
                          samples_per_sub=w.samples_per_sub, chunk=w.chunk)
    nq = torch.empty(w.chunk * nd * 2, dtype=torch.float64, device="cuda:0")
    acc = torch.zeros(w.n_sub * nd * kmax * 2, dtype=torch.float64, device="cuda:0")

    def job(with_moments):
        p.reset()
        acc.zero_()
        p.packed = False
        for g in range(0, w.E, w.chunk):
            p.run_chunk(g, w.chunk)
            if with_moments:
                mp.mp_occupations(w.M, w.chunk, p.C, "fp32", 2, bins, "marginals_and_total", nq)
                mp.mp_moments_accumulate(w.chunk, p.n, nq, nd, kmax, "matrix_p", w.n_sub,
                                         w.samples_per_sub, g, acc)
        p.finalize()
    job(True)
    base_s = _timed(torch, lambda: job(False))
    full_s = _timed(torch, lambda: job(True))
    mean = torch.empty(nd * kmax * 2, dtype=torch.float64, device="cuda:0")
    sig = torch.empty(nd * kmax, dtype=torch.float64, device="cuda:0")
    mp.mp_subensemble_stats(w.n_sub, w.samples_per_sub, nd * kmax, 2, 1.0, acc, mean, sig)
    mom = mean.cpu().numpy().reshape(nd, kmax, 2)[..., 0]
    smom = sig.cpu().numpy().reshape(nd, kmax)
    gold = _golden("m1000_count_moments.json")["dists"]
    rows = []
    for q in range(nd):
        mu, var = gold[q]["mean"], gold[q]["var"]
        f2_exact = var - mu + mu * mu  # <:n^2:> = Var - mean + mean^2
        rows.append({"dist": gold[q]["name"], "moments": mom[q].tolist(), "sigma_T": smom[q].tolist(),
                     "k1_minus_exact_over_sigma": float((mom[q][0] - mu) / smom[q][0]),
                     "k2_minus_exact_over_sigma": float((mom[q][1] - f2_exact) / smom[q][1])})
    return _envelope(
        "extra time of moments k=1..4 for 2 bins + total from the counts ensemble, M=1000, FP32",
        (full_s - base_s) / base_s, "fraction of the counts run", 1e3 * full_s,
        f"M1000_t0.9_r1: E={w.E} in chunks of {w.chunk}, {w.n_sub} sub-ensembles, halves "
        f"window {tuple(wh)}, total window {tuple(w.windows[0])}", "fp32 (fp64 moments)",
        counts_run_s=base_s, counts_and_moments_run_s=full_s, moments=rows)


def run_pairs_m1000(args, mp, torch, synth):
    """Normally ordered pair moments <:n_i n_j:> of all 1000 output modes from
    the M = 1000, t = 0.9, r = 1 FP32 ensemble (E = 1.2e6 in chunks of 1e5, 120
    sub-ensembles of 1e4).  Each chunk: sample, propagate, mode occupations,
    pair sums; the two pair kernels are timed with HIP events on the launch
    stream; the whole job is timed after one untimed run.  The estimates are
    compared with Isserlis' closed form at the stored entries (every diagonal
    element and 2048 off-diagonal pairs)."""
    w = synth.workload_m1000()
    p = mp.PairPipeline(w.T, w.r, prec="fp32", seed=w.seed, n_sub=w.n_sub,
                        samples_per_sub=w.samples_per_sub, chunk=w.chunk)
    stream = torch.cuda.current_stream()
    n_chunks = -(-w.E // w.chunk)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(n_chunks)]

    def job():
        p.acc.zero_()
        p.packed = False
        for c, g in enumerate(range(0, w.E, w.chunk)):
            E = min(w.chunk, w.E - g)
            if not p.packed:
                mp.mp_pack_transmission(p.M, p.T, p.prec, p.ws_prop)
                p.packed = True
            mp.mp_sample(p.M, g, E, p.r, p.seed, p.net, p.prec, p.ab, p.n)
            mp.mp_propagate_packed(p.M, E, p.prec, p.ab, p.C, p.ws_prop)
            ev[c][0].record(stream)
            mp.mp_mode_occupations(p.M, E, p.C, p.prec, p.X)
            ev[c][1].record(stream)
            mp.mp_pair_correlations_accumulate(p.M, E, p.X, p.prec, p.n_sub, p.ns, g, p.acc,
                                               p.workspace(g, E))
            ev[c][2].record(stream)
        p.finalize()
    job()
    secs = _timed(torch, job)
    occ_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    pair_ms = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    G2, sig = p.result()
    gold = _golden("m1000_pair_moments.json")
    i, j = np.array(gold["i"]), np.array(gold["j"])
    z = (G2.real[i, j] - np.array(gold["value"])) / sig[i, j]
    diag = i == j
    M, E_c = w.M, w.chunk
    flops = 4.0 * M * (M + 1) * E_c  # 8 flops per complex product-sum, i <= j
    nb = -(-M // 128)
    # three real MFMA products (6 flops) per tile element and sample, full tiles
    executed = 6.0 * nb * (nb + 1) / 2 * 128 * 128 * E_c
    achieved = flops / (pair_ms * 1e-3) / 1e12
    occ_bytes = M * E_c * (16 + 8)  # C read (4 FP32 per mode), X written (2 FP32)
    log(f"[bench] pairs m1000: job {secs:.3f} s, mode occupations {occ_ms:.3f} ms, pair sums "
        f"{pair_ms:.3f} ms per chunk ({achieved:.1f} TFLOP/s), max |z| {np.abs(z).max():.2f}")
    return _envelope(
        "pair moments <:n_i n_j:> of all modes, M=1000, FP32: ensemble samples per second",
        w.E / secs, "samples/s", 1e3 * secs,
        f"M1000_t0.9_r1: E={w.E} in chunks of {w.chunk}, {w.n_sub} sub-ensembles, all "
        f"{M * (M + 1) // 2} pairs i <= j", "fp32 (fp64 sums across chunks)",
        job_s=secs, mode_occupations_ms_per_chunk=occ_ms, pair_sums_ms_per_chunk=pair_ms,
        roofline={"bound": "mfma", "kernel": "pair_corr_f32", "achieved": round(achieved, 2),
                  "peak": PEAKS_TFLOPS["fp32"], "unit": "TFLOP/s",
                  "frac": round(achieved / PEAKS_TFLOPS["fp32"], 4),
                  "algorithmic_flops_per_launch": flops, "executed_flops_per_launch": executed,
                  "traffic": None},
        mode_occupations_GBps=occ_bytes / (occ_ms * 1e-3) / 1e9,
        closed_form_check={"entries": int(len(z)), "max_abs_z": float(np.abs(z).max()),
                           "rms_z": float(np.sqrt((z ** 2).mean())),
                           "rms_z_diagonal": float(np.sqrt((z[diag] ** 2).mean())),
                           "frac_within_3_sigma": float((np.abs(z) < 3).mean())})


def run_joint3_m300(args, mp, torch, synth):
    """Joint distribution of three bins (main text, higher-dimensional
    binning): lossless Haar network, M = 300, r = 0.5 on every mode, bins of
    100 contiguous modes, window [0, 128) per bin (2.1e6 cells), E = 1.2e6 in
    chunks of 1e5 (120 sub-ensembles of 1e4), FP32.  Each chunk: sample,
    propagate, then mp_binned_counts (occupations, factor tables, the two
    box contractions), timed with HIP events; the finalize (inverse DFT of
    120 sub-ensemble grids) timed apart; the whole job timed after one
    untimed run.  Checks: P vanishes for odd m_1 + m_2 + m_3 (lossless), and
    the distribution of the total m_1 + m_2 + m_3 < 128 against the exact
    lossless law (sd bound: the sum of the cells' sigma_T)."""
    M, K = 300, 128
    seed = synth.SEED_BASE + 40
    T = synth.haar_unitary(M, seed)
    r = np.full(M, 0.5)
    bins = synth.contiguous_bins(M, 3)
    E, ns, chunk = 1_200_000, 10_000, 100_000
    p = mp.CountsPipeline(T, r, prec="fp32", seed=seed, bin_of_mode=bins, d=3, mode="joint",
                          windows=[(0, K)] * 3, n_sub=E // ns, samples_per_sub=ns, chunk=chunk)
    stream = torch.cuda.current_stream()
    n_chunks = E // chunk
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(n_chunks)]
    fin = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def job():
        p.reset()
        p.packed = False
        for c in range(n_chunks):
            g = c * chunk
            if not p.packed:
                mp.mp_pack_transmission(p.M, p.T, p.prec, p.ws_prop)
                p.packed = True
            mp.mp_sample(p.M, g, chunk, p.r, p.seed, p.net, p.prec, p.ab, p.n)
            mp.mp_propagate_packed(p.M, chunk, p.prec, p.ab, p.C, p.ws_prop)
            ev[c][0].record(stream)
            p.counts_chunk(g, chunk)
            ev[c][1].record(stream)
        fin[0].record(stream)
        p.finalize()
        fin[1].record(stream)
    job()
    secs = _timed(torch, job)
    counts_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    fin_ms = fin[0].elapsed_time(fin[1])
    P = p.result()[0].reshape(K, K, K)
    sig = p.result()[2].reshape(K, K, K)
    # box half-widths of the last chunk: the first 8 ints of the counting
    # workspace (term 0 around theta = 0, term 1 around theta = pi)
    band = p.ws_counts[:32].view(torch.int32).cpu().numpy()
    widths = [[int(min(2 * h + 1, K)) if h >= 0 else 0 for h in band[4 * t: 4 * t + 3]]
              for t in range(2)]
    box_cells = sum(int(np.prod(w)) for w in widths)
    flops = 8.0 * box_cells * chunk
    achieved = flops / (counts_ms * 1e-3) / 1e12
    m = np.arange(K)
    tot_idx = m[:, None, None] + m[None, :, None] + m[None, None, :]
    odd = tot_idx % 2 == 1
    Ptot = np.bincount(tot_idx.ravel(), weights=P.ravel(), minlength=3 * K)[:K]
    Stot = np.bincount(tot_idx.ravel(), weights=sig.ravel(), minlength=3 * K)[:K]
    gold = np.array(_golden("lossless_m300_r0.5.json")["P"])
    bulk = gold > 1e-4 * gold.max()
    zt = np.abs(Ptot - gold)[bulk] / Stot[bulk]
    log(f"[bench] joint3 m300: job {secs:.3f} s, counts {counts_ms:.2f} ms per chunk "
        f"({achieved:.1f} TFLOP/s over the boxes {widths}), finalize {fin_ms:.1f} ms, "
        f"max odd |P| / max P {np.abs(P[odd]).max() / P.max():.2e}, total-law max z {zt.max():.2f}")
    return _envelope(
        "joint distribution of three bins, M=300 lossless, r=0.5: ensemble samples per second",
        E / secs, "samples/s", 1e3 * secs,
        f"M300_lossless_r0.5: 3 bins of 100 modes, windows [0,{K}) each ({K ** 3} cells), "
        f"E={E} in chunks of {chunk}, {E // ns} sub-ensembles", "fp32 (fp64 sums across chunks)",
        job_s=secs, counts_ms_per_chunk=counts_ms, finalize_ms=fin_ms, box_widths=widths,
        roofline={"bound": "mfma", "kernel": "jointd_sum_f32 (both terms; the timed call also "
                  "holds the occupation and factor-table kernels)", "achieved": round(achieved, 2),
                  "peak": PEAKS_TFLOPS["fp32"], "unit": "TFLOP/s",
                  "frac": round(achieved / PEAKS_TFLOPS["fp32"], 4),
                  "algorithmic_flops_per_launch": flops, "traffic": None},
        checks={"max_abs_P_odd_over_max_P": float(np.abs(P[odd]).max() / P.max()),
                "total_law_max_abs_err_over_sigma_bound": float(zt.max()),
                "total_law_max_abs_err": float(np.abs(Ptot - gold)[bulk].max()),
                "sum_P_window": float(P.sum())})


def run_scaling_appb(args, mp, torch, synth):
    """Appendix B scaling workloads.  Run time: lossless Haar networks,
    r = 0.89, M = 128 .. 8192, E = 1.2e6 (120 sub-ensembles of 1e4, chunks of
    1.2e5), total counts on the printed windows [m_min, m_max], each job
    timed whole (packing, all chunks, finalize) after one untimed chunk, for
    the default mixed precision (the FP8-correction T-split form), split-BF16
    and FP32.  Errors: max sigma_T for M = 16 .. 1024
    with r_i = 0.89 + 0.1 w_i and t in {1, 0.995, 1 - 1/m_max} (printed
    m_max), FP64, windows of +-9 sd around the closed-form mean."""
    g = _golden("appB_cutoffs.json")
    E, ns, chunk = 1_200_000, 10_000, 120_000
    n_sub = E // ns
    timing = []
    for M, mmin, mmax in zip(g["timing_M"], g["timing_m_min"], g["timing_m_max"]):
        seed = synth.SEED_BASE + 20
        T = synth.haar_unitary(M, seed + M)
        r = np.full(M, 0.89)
        K = -(-(mmax - mmin + 1) // 64) * 64
        row = {"M": M, "window": [mmin, K]}
        for prec in ("split1t_f8", "split_bf16", "fp32"):
            p = mp.CountsPipeline(T, r, prec=prec, seed=seed, windows=[(mmin, K)], n_sub=n_sub,
                                  samples_per_sub=ns, chunk=chunk)
            p.run_chunk(0, chunk)

            def job():
                p.reset()
                p.packed = False
                p.run()
            secs = _timed(torch, job)
            P, _, sig = p.result()
            row[prec] = {"run_s": secs, "max_sigma_T": float(sig.max()), "sum_P": float(P.sum())}
            del p
            torch.cuda.empty_cache()
        log(f"[bench] scaling M={M}: FP8-correction {row['split1t_f8']['run_s']:.3f} s, "
            f"split-BF16 {row['split_bf16']['run_s']:.3f} s, fp32 {row['fp32']['run_s']:.3f} s")
        timing.append(row)
    for a, b in zip(timing, timing[1:]):
        b["exponent_vs_previous_M"] = float(np.log(b["split1t_f8"]["run_s"] / a["split1t_f8"]["run_s"])
                                            / np.log(b["M"] / a["M"]))
    errors = []
    for M, mmax in zip(g["error_M"], g["error_m_max"]):
        seed = synth.SEED_BASE + 30
        r = synth.squeezing_gaussian(M, 0.89, 0.1, seed + M)
        U = synth.haar_unitary(M, seed + 1000 + M)
        row = {"M": M}
        for name, t in (("t=1", 1.0), ("t=0.995", 0.995), ("t=1-1/m_max", 1.0 - 1.0 / mmax)):
            mean, sd = synth.uniform_loss_moments(r, t)
            win = synth.count_window(mean, sd)
            p = mp.CountsPipeline(t * U, r, prec="fp64", seed=seed, windows=[win], n_sub=n_sub,
                                  samples_per_sub=ns, chunk=chunk)
            p.run()
            P, _, sig = p.result()
            row[name] = {"max_sigma_T": float(sig.max()), "window": list(win),
                         "sum_P": float(P.sum())}
            del p
        log(f"[bench] scaling errors M={M}: " + ", ".join(f"{k} {v['max_sigma_T']:.2e}"
                                                           for k, v in row.items() if k != "M"))
        errors.append(row)
        torch.cuda.empty_cache()
    top = timing[-1]["split1t_f8"]["run_s"]
    return {"metric": "seconds for the lossless M=8192 total-count job (E=1.2e6), default mixed "
                      "precision",
            "value": top, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1,
            "ms_per_step": 1e3 * top, "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": DTYPES["split1t_f8"], "data": "synthetic",
            "config": {"workload": "Appendix B: lossless Haar, r=0.89, M=128..8192, E=1.2e6; "
                                   "max sigma_T for M=16..1024, r_i=0.89+0.1 w_i, three losses",
                       "timing": timing, "errors": errors}}


def run_mfma_peak(args, mp, torch, synth):
    """The matrix cores' sustained rate with no memory traffic (the library's
    probe: one workgroup of four waves per CU, 256 accumulator registers of
    independent MFMA chains per wave on register-resident operands), per
    instruction the GEMMs use, timed
    with events; against the published dense peaks."""
    sink = torch.empty(512 * 256, dtype=torch.float64, device="cuda:0")
    out = {}
    # about 50 ms per launch, the length of one GEMM of the benchmark (the
    # clock settles under load within milliseconds)
    # kind 3: 4 FP16 MFMAs and one e4m3 32x32x64 MFMA per chain and round, the
    # FP8-correction GEMM's mix; its peak when each instruction ran at its
    # published rate: (4 x 32768 + 131072) flops in 4 x 32768 / 2500 +
    # 131072 / 5000 TFLOP/s-time units
    mix_peak = (4 * 32768 + 131072) / (4 * 32768 / 2500.0 + 131072 / 5000.0)
    for kind, name, peak, iters in ((0, "fp16 32x32x16", 2500.0, 200000),
                                    (1, "fp32 32x32x2", 157.3, 100000),
                                    (2, "fp64 16x16x4", 78.6, 50000),
                                    (3, "fp16 x4 + fp8 32x32x64", mix_peak, 80000)):
        mp.mp_mfma_sustained(kind, 100, sink)  # first launch
        best = None
        for _ in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            flops = mp.mp_mfma_sustained(kind, iters, sink)
            b.record()
            torch.cuda.synchronize()
            s = a.elapsed_time(b) * 1e-3
            best = s if best is None else min(best, s)
        tf = flops / best / 1e12
        out[name] = {"tflops": tf, "published_peak": peak, "fraction": tf / peak, "ms": 1e3 * best}
        log(f"[bench] mfma_peak {name}: {tf:.1f} TFLOP/s = {100 * tf / peak:.1f} % of {peak}")
    f16 = out["fp16 32x32x16"]
    return _envelope("TFLOP/s of back-to-back FP16 MFMA (no memory traffic)", f16["tflops"],
                     "TFLOP/s", f16["ms"], "matrix-core probe: 4 waves per CU, 256 accumulator registers per wave",
                     "f16 (fp32 acc)", kinds=out)


def run_copy(args, mp, torch, synth):
    """A plain 1 GiB device-to-device copy, three times: the reference for
    scaling the FETCH_SIZE and WRITE_SIZE counters to bytes."""
    n = 1 << 30
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    secs = [_timed(torch, lambda: dst.copy_(src)) for _ in range(3)]
    return _envelope("GB/s of a 1 GiB device copy (counter calibration)", 2 * n / min(secs) / 1e9,
                     "GB/s", 1e3 * min(secs), "1 GiB device-to-device copy", "u8",
                     bytes_read=n, bytes_written=n)

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="split1t_f8")
    ap.add_argument("--compare", default="fp32", help="second precision timed ('' to skip)")
    ap.add_argument("--compare-steps", type=int, default=5)
    ap.add_argument("--also", default="split_bf16",
                    help="m8000: a further mixed precision timed beside the main one ('' to skip)")
    ap.add_argument("--chunk", type=int, default=65536)
    ap.add_argument("--M", type=int, default=8000)
    ap.add_argument("--cpu-budget", type=float, default=45.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bilinear", dest="bilinear", action="store_false",
                    help="m8000: skip the one-distribution bilinear-form comparison leg")
    ap.add_argument("--unfused", action="store_true",
                    help="m8000: write C and count from it instead of the occupation-fused GEMM")
    ap.add_argument("--workload", default="m8000",
                    choices=["m8000", "joint_m1000", "precision_m4000", "precision_m8000", "batched",
                             "surrogate",
                             "plusp_m20", "moments_m1000", "pairs_m1000", "joint3_m300",
                             "scaling_appb", "copy", "mfma_peak", "bilinear_m8000"],
                    help="m8000 (default) is the headline metric; the others measure the other "
                         "configurations of the hot path and print their own JSON line")
    ap.add_argument("--sweeps", type=int, default=20000, help="surrogate: training sweeps")
    ap.add_argument("--sweep-E", type=int, default=10000, help="surrogate: samples per sweep")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library "
              f"computes on one device; sharding the samples over GPUs is not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2503_12749_amd as mp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    runners = {"m8000": run_m8000, "joint_m1000": run_joint_m1000,
               "precision_m4000": run_precision_m4000, "precision_m8000": run_precision_m8000,
               "batched": run_batched,
               "surrogate": run_surrogate, "plusp_m20": run_plusp_m20,
               "moments_m1000": run_moments_m1000, "pairs_m1000": run_pairs_m1000,
               "joint3_m300": run_joint3_m300,
               "scaling_appb": run_scaling_appb,
               "copy": run_copy, "mfma_peak": run_mfma_peak,
               "bilinear_m8000": run_bilinear_m8000}
    out = runners[args.workload](args, mp, torch, synth)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
