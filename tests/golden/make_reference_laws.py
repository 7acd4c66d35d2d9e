"""Writes exact reference values used by bench.py's comparison workloads.
Calls only oracle/ (and synth/ for the seeded networks):

  lossless_m20_r0.5.json   exact total-count law of a lossless 20-mode network
                           with r = 0.5 on every mode (eq.
                           Exact_multi_mode_squeezed_state), m = 0..63
  m1000_count_moments.json closed-form mean and variance (E4: W = T^T P_S T*)
                           of the two half-bins and the total of the M = 1000,
                           t = 0.9, r = 1 Haar workload

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


if __name__ == "__main__":
    main()
