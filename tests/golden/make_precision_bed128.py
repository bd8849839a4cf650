#!/usr/bin/env python3
"""Writes precision_bed128.json: the FP64 oracle's results on the 128^3 pool with
one bubble (R = 12) and 1,400 spheres (R = 4, density ratio 2.5), TRT tau = 0.55,
g = 2e-5, after 1,000 steps.  These are the reference values for the storage-form
accuracy report (total mass, bubble rise velocity, mean particle drag).

Definitions (the paper gives none):
  rise velocity  v = (z_c(T) - z_c(T-10)) / 10, z_c the gas-volume centroid of
                 the bubble (id 1, not the atmosphere);
  mean drag      the mean over particles of F_z, averaged over steps T-9..T.

Calls only the oracle.  Run from the repository root:
    python tests/golden/make_precision_bed128.py [--threads 8]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_1712_07028_amd import workloads as W  # noqa: E402

STEPS = 1000


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--steps", type=int, default=STEPS)
    args = ap.parse_args()
    O.build(force=False)
    w = W.bubble_bed_128()
    n = w.particles.n
    t0 = time.perf_counter()
    o = O.Oracle(w, n_threads=args.threads)
    M0, R0 = o.mass()
    o.step(args.steps - 10)
    b0 = o.bubbles()
    drag = []
    for _ in range(10):
        o.step(1)
        drag.append(float(o.particles_get(n)["F"][:, 2].mean()))
    b1 = o.bubbles()
    M1, R1 = o.mass()
    out = {
        "workload": w.name, "steps": args.steps,
        "mass0": M0, "mass": M1, "ledger": R1,
        "rise_velocity": (b1[1]["centroid"][2] - b0[1]["centroid"][2]) / 10.0,
        "bubble_V": b1[1]["V"], "bubble_centroid_z": b1[1]["centroid"][2],
        "mean_drag_z": float(np.mean(drag)),
        "source": "oracle/fsl_oracle.c via tests/golden/make_precision_bed128.py",
    }
    o.close()
    with open(os.path.join(HERE, "precision_bed128.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out), f"({time.perf_counter() - t0:.0f} s)")


if __name__ == "__main__":
    main()
