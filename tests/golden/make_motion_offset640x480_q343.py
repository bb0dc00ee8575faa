"""Writes edp_motion_offset640x480_q343.json: the C oracle's plain EDP (j = 1) on the workload of
three label dimensions, motion with a brightness offset 640x480 with 7 x 7 x 7 labels
(synth.workload("motion_offset640x480"), seed 0) -- its energy and the SHA-256 of its int32
labels.  Calls only oracle/ and synth/; about a minute on one core.

    python tests/golden/make_motion_offset640x480_q343.py
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import cref  # noqa: E402


def main():
    p = synth.workload("motion_offset640x480")
    r = cref.edp(p.cost, p.qx, p.qy, p.lam, p.trunc, p.mode, 1, "grms", qz=p.qz)
    labels = np.ascontiguousarray(r["labels"], dtype=np.int32)
    out = {"workload": p.name, "cost_sha256": p.sha256(), "qx": p.qx, "qy": p.qy, "qz": p.qz, "lam": p.lam,
           "trunc": p.trunc, "mode": p.mode, "iterations": 1, "energy": r["energy"],
           "labels_sha256": hashlib.sha256(labels.tobytes()).hexdigest(),
           "source": "C oracle, plain EDP (Algorithm 1, one iteration), general RMS minimum search over "
                     "three label dimensions"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "edp_motion_offset640x480_q343.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
