"""Writes pair_counts.json: the number of unique particle pairs closer than
the cutoff a (minimum image on periodic axes) in the seeded workload inputs,
rounded to FP32 as the GPU runs see them.  The benchmark divides the
short-range pair sum's algorithmic flops (28 + 4p per unique pair within a)
by its measured time; each count is keyed by the first 16 hex digits of the
SHA-256 of the FP32 positions so that a changed input recipe is detected.

Counts come from scipy's k-d tree (exact pair counting; free axes get a
period far larger than the box, so they never wrap).
Usage: python tests/golden/make_pair_counts.py
"""
import hashlib
import json
import os
import sys

import numpy as np
from scipy.spatial import cKDTree

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from paper_2510_05961_amd import workloads as WL  # noqa: E402


def count(cfg):
    c = WL.WORKLOADS[cfg]
    pos, _, box = WL.make_config(cfg, 1.0)
    p32 = np.ascontiguousarray(pos.astype(np.float32))
    key = hashlib.sha256(p32.tobytes()).hexdigest()[:16]
    p = p32.astype(np.float64)
    period = []
    for k in range(3):
        if (c["periodic"] >> k) & 1:
            p[:, k] = np.mod(p[:, k], box[k])
            period.append(box[k])
        else:
            period.append(1e6)
    t = cKDTree(p, boxsize=period)
    n = (t.count_neighbors(t, c["a"]) - len(p)) // 2
    return {"pairs": int(n), "n": len(p), "cutoff": c["a"], "positions_sha256_16": key}


if __name__ == "__main__":
    out = {str(cfg): count(cfg) for cfg in (2, 3, 4)}
    with open(os.path.join(HERE, "pair_counts.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(out)
