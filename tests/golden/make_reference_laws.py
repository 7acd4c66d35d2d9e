"""Writes exact reference values used by bench.py's comparison workloads.
Calls only oracle/ (and synth/ for the seeded networks):

  lossless_m20_r0.5.json   exact total-count law of a lossless 20-mode network
                           with r = 0.5 on every mode (eq.
                           Exact_multi_mode_squeezed_state), m = 0..63
  m1000_count_moments.json closed-form mean and variance (E4: W = T^T P_S T*)
                           of the two half-bins and the total of the M = 1000,
                           t = 0.9, r = 1 Haar workload
  lossless_m300_r0.5.json  exact total-count law of a lossless 300-mode network
                           with r = 0.5 on every mode, m = 0..127 (the total
                           of the three-bin joint workload)
  m1000_pair_moments.json  Isserlis closed form of <:n_i n_j:> for the same
                           workload at every diagonal element and 2048
                           seeded off-diagonal pairs (i < j)

Run from the repository root:  python tests/golden/make_reference_laws.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import exact  # noqa: E402


def main():
    m = np.arange(64)
    P = exact.lossless_uniform_total(20, 0.5, m)
    json.dump({"source": "eq. Exact_multi_mode_squeezed_state (lossless, identical r), M = 20, r = 0.5",
               "M": 20, "r": 0.5, "m": m.tolist(), "P": P.tolist()},
              open(os.path.join(HERE, "lossless_m20_r0.5.json"), "w"), indent=1)
    m = np.arange(128)
    P = exact.lossless_uniform_total(300, 0.5, m)
    json.dump({"source": "eq. Exact_multi_mode_squeezed_state (lossless, identical r), M = 300, r = 0.5",
               "M": 300, "r": 0.5, "m": m.tolist(), "P": P.tolist()},
              open(os.path.join(HERE, "lossless_m300_r0.5.json"), "w"), indent=1)
    w = synth.workload_m1000()
    bins = synth.contiguous_bins(w.M, 2)
    out = {"source": "closed-form count moments (mean sum_j W_jj N_j, variance with the N N |W|^2 "
                     "and A A Re W^2 terms), W = T^T P_S T*, for the M = 1000, t = 0.9, r = 1 "
                     "Haar workload (synth.workload_m1000)",
           "dists": []}
    for name, counted in (("bin 0", bins == 0), ("bin 1", bins == 1), ("total", bins >= 0)):
        mean, var = exact.count_moments(w.T, w.r, counted)
        out["dists"].append({"name": name, "mean": mean, "var": var})
    json.dump(out, open(os.path.join(HERE, "m1000_count_moments.json"), "w"), indent=1)
    G = exact.pair_moments(w.T, w.r)
    rng = np.random.default_rng(2503)
    i = rng.integers(0, w.M, 4 * 2048)
    j = rng.integers(0, w.M, 4 * 2048)
    keep = np.unique(np.stack([np.minimum(i, j), np.maximum(i, j)], 1)[i != j], axis=0)[:2048]
    pairs = np.concatenate([np.stack([np.arange(w.M)] * 2, 1), keep])
    json.dump({"source": "<:n_i n_j:> = N_ii N_jj + |N_ij|^2 + |S_ij|^2, N = T diag(sinh^2 r) T^+, "
                         "S = T diag(sinh r cosh r) T^T (Isserlis), M = 1000, t = 0.9, r = 1 Haar "
                         "workload (synth.workload_m1000)",
               "i": pairs[:, 0].tolist(), "j": pairs[:, 1].tolist(),
               "value": [float(G[a, b]) for a, b in pairs]},
              open(os.path.join(HERE, "m1000_pair_moments.json"), "w"))


if __name__ == "__main__":
    main()
