"""Write the FP64 oracle's risk measures of the full paper-scale workload.

Run from the repository root:

    python tests/golden/make_paper_golden.py [--threads T] [--trials N]

It draws the 800,000-trial x 1,000-event YET and the 16-XELT layer from the
seeded input generator, runs the FP64 oracle (Algorithm 1, section 2.2, with
the secondary uncertainty of section 3) over every trial in plain-sampling
mode, and writes:

* ``paper_800k_oracle.json``: PML and TVaR (section 2.4) of the whole YLT at
  return periods 10, 50, 100 and 250 years, the same for the largest
  occurrence loss per trial (occurrence exceedance), the largest gross loss of
  any trial (the scale of the per-trial tolerance), and run facts;
* ``paper_800k_oracle_sample.npz``: the year loss and gross loss of every
  100th trial, for per-trial checks of the full-size launch.

Only ``oracle/`` computes; the input generator draws tables and holds none of
the method's arithmetic.  About 45 minutes on 8 host threads.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle                                     # noqa: E402
from paper_1310_2274_amd import synth             # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
RPS = [10.0, 50.0, 100.0, 250.0]
SAMPLE_STRIDE = 100


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0, help="OpenMP threads (0 = all)")
    ap.add_argument("--trials", type=int, default=800_000)
    ap.add_argument("--out", default=os.path.join(HERE, "paper_800k_oracle"))
    a = ap.parse_args()

    oracle.build(force=False)
    wl = synth.paper_scale(a.trials)
    layer = wl.layers[0]
    N, K, C = wl.n_trials, wl.events_per_trial, wl.catalog_size
    ylt = np.empty(N)
    gross = np.empty(N)
    omax = np.empty(N)
    t0 = time.time()
    block = synth.YET_BLOCK
    for lo in range(0, N, block):
        hi = min(N, lo + block)
        rows = synth.make_yet_rows(np.arange(lo, hi), N, K, C, wl.yet_seed)
        y, g, o = oracle.run_layer(layer, rows, np.arange(lo, hi), C, wl.seed,
                                   mode=oracle.MODE_PLAIN, threads=a.threads)
        ylt[lo:hi], gross[lo:hi], omax[lo:hi] = y, g, o
        print(f"[golden] trials {lo}..{hi - 1} done, {time.time() - t0:.0f} s", flush=True)
    secs = time.time() - t0

    pml, tvar = oracle.risk_measures(ylt, RPS)
    opml, otvar = oracle.risk_measures(omax, RPS)
    rec = {
        "source": ("FP64 oracle (oracle/ara_oracle.c, plain sampling) over every trial of the "
                   "paper-scale synthetic workload; PML = k-th largest year loss, TVaR = mean of "
                   "the k largest, k = floor(N/RP) (section 2.4)"),
        "command": "python tests/golden/make_paper_golden.py" + (
            f" --trials {a.trials}" if a.trials != 800_000 else ""),
        "workload": wl.name,
        "n_trials": N, "events_per_trial": K, "catalog_size": C,
        "n_elts": len(layer.elts), "seed": wl.seed,
        "return_periods": RPS,
        "pml": pml.tolist(), "tvar": tvar.tolist(),
        "oep_pml": opml.tolist(), "oep_tvar": otvar.tolist(),
        "max_gross": float(gross.max()),
        "mean_ylt": math.fsum(ylt.tolist()) / N,
        "zero_trials": int((ylt == 0.0).sum()),
        "capped_trials": int((ylt >= layer.agg_limit).sum()),
        "sample_stride": SAMPLE_STRIDE,
        "oracle_seconds": round(secs, 1),
        "oracle_threads": a.threads or oracle.max_threads(),
    }
    with open(a.out + ".json", "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    idx = np.arange(0, N, SAMPLE_STRIDE, dtype=np.int64)
    np.savez_compressed(a.out + "_sample.npz", trial=idx, ylt=ylt[idx], gross=gross[idx])
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
