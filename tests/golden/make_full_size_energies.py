"""Writes full_size_energies.json: the FP64 oracle's energy of the full-size
workloads (the water box, the slab and the Gaussian-charge box), evaluated on
the FP32-rounded seeded inputs that the FP32 runs use.

Calls only the oracle and the seeded input generators.  Run from the repo
root:  python tests/golden/make_full_size_energies.py [cfg ...]
The JSON also records a SHA-256 prefix of the FP32 input bytes, so a reader
can tell that its inputs are the ones these energies belong to.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2510_05961_amd import workloads as WL  # noqa: E402

OUT = os.path.join(HERE, "full_size_energies.json")


def input_digest(pos32, q32):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(pos32, dtype=np.float32).tobytes())
    h.update(np.ascontiguousarray(q32, dtype=np.float32).tobytes())
    return h.hexdigest()[:16]


def main(cfgs):
    O.build(force=False)
    try:
        rec = json.load(open(OUT))
    except (OSError, ValueError):
        rec = {}
    for cfg in cfgs:
        c = WL.WORKLOADS[cfg]
        pos, q, box = WL.make_config(cfg, 1.0)
        pos32, q32 = pos.astype(np.float32), q.astype(np.float32)
        per = [bool((c["periodic"] >> k) & 1) for k in range(3)]
        o = O.OracleMSM(box, per, c["p"], c["h"], c["a"], c["L"])
        t0 = time.time()
        r = o.compute(pos32.astype(np.float64), q32.astype(np.float64))
        dt = time.time() - t0
        rec[str(cfg)] = {"workload": c["name"], "n": int(len(q)), "E": r["E"],
                         "sum_abs_q_phi_half": 0.5 * float(np.sum(np.abs(q32 * r["phi"]))),
                         "input_sha256_16": input_digest(pos32, q32),
                         "oracle_seconds": round(dt, 1), "threads": O.num_threads()}
        print(cfg, rec[str(cfg)], flush=True)
        with open(OUT, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [2, 4, 3])
