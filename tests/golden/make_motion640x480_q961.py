"""Writes edp_motion640x480_q961.json: the C oracle's plain EDP (j = 1) on the 961-label motion
workload 640x480 (synth.workload("motion640x480"), seed 0) -- its energy and the SHA-256 of its
int32 labels.  Calls only oracle/ and synth/; about two minutes on one core.

    python tests/golden/make_motion640x480_q961.py
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
    p = synth.workload("motion640x480")
    r = cref.edp(p.cost, p.qx, p.qy, p.lam, p.trunc, p.mode, 1, "grms")
    labels = np.ascontiguousarray(r["labels"], dtype=np.int32)
    out = {"workload": p.name, "cost_sha256": p.sha256(), "qx": p.qx, "qy": p.qy, "lam": p.lam,
           "trunc": p.trunc, "mode": p.mode, "iterations": 1, "energy": r["energy"],
           "labels_sha256": hashlib.sha256(labels.tobytes()).hexdigest(),
           "source": "C oracle, plain EDP (Algorithm 1, one iteration), general RMS minimum search"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "edp_motion640x480_q961.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
