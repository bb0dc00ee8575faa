"""Writes edp_batch64.json: the C oracle's plain EDP (j = 1) of every instance of the 64-instance
uneven batch (synth.batch_problems(64): stereo 160x120..640x480 with 16-64 disparities, int16;
motion 9x9..21x21 labels at 160x120..320x240, int32) -- per instance its energy and the SHA-256 of
its int32 labels.  Calls only oracle/ and synth/; the instances are solved in parallel processes
(about a minute on 8 cores).

    python tests/golden/make_batch64.py
"""
import hashlib
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import cref  # noqa: E402

N = 64


def solve_one(i):
    p = synth.batch_problems(1, first_seed=i)[0]
    r = cref.edp(p.cost, p.qx, p.qy, p.lam, p.trunc, p.mode, 1, "lrms")
    labels = np.ascontiguousarray(r["labels"], dtype=np.int32)
    H, W, Q = p.cost.shape
    return {"index": i, "name": p.name, "width": W, "height": H, "qx": p.qx, "qy": p.qy, "lam": p.lam,
            "trunc": p.trunc, "mode": p.mode, "dtype": str(p.cost.dtype), "cost_sha256": p.sha256(),
            "energy": r["energy"], "labels_sha256": hashlib.sha256(labels.tobytes()).hexdigest()}


def main():
    cref.build()
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        rows = pool.map(solve_one, range(N), chunksize=1)
    out = {"workload": "batch_problems(64)", "iterations": 1,
           "source": "C oracle, plain EDP (Algorithm 1, one iteration), linear RMS minimum search",
           "instances": rows}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "edp_batch64.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}: {len(rows)} instances")


if __name__ == "__main__":
    main()
