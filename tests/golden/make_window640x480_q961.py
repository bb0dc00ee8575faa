"""Writes edp_window640x480_q961.json: the oracle's label-window EDP (j = 1, 7 x 7 windows) on the
961-label motion workload 640x480 (synth.workload("motion640x480"), seed 0).

Round 0: window centres from the oracle's network forward pass (oracle/cnn_ref: pooled input,
the four dilated convolutions in float64 on bf16-rounded operands, window decoding) with the
committed weights paper_1410_7922_amd/weights/window_net_31x31.npz (read as data), then the C
oracle's windowed EDP.  Round 1: centres re-centred on the round-0 labels (cnn_ref.recenter), then
the windowed EDP again.  Stored: SHA-256 of every centre array and label array, and the energies.
Calls only oracle/ and synth/ for arithmetic; a few minutes on one core.

    python tests/golden/make_window640x480_q961.py
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import cnn_ref, cref  # noqa: E402

WEIGHTS = os.path.join(ROOT, "paper_1410_7922_amd", "weights", "window_net_31x31.npz")
WIN, SCALE = 7, 250


def sha(a, dtype=np.int32):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def oracle_centres(cost, qx, qy):
    """Window centres of the network for an int32 cost volume, computed by the oracle."""
    with np.load(WEIGHTS, allow_pickle=False) as f:
        params = cnn_ref.params_from_flat(f["params"])
        mode = int(f["pool_mode"])
    return cnn_ref.network_centres(cost, qx, qy, params, SCALE, WIN, mode)


def main():
    p = synth.workload("motion640x480")
    cen0 = oracle_centres(p.cost, p.qx, p.qy)
    r0 = cref.edp_window(p.cost, cen0, WIN, p.qx, p.qy, p.lam, p.trunc, p.mode, 1)
    cen1 = cnn_ref.recenter(r0["labels"], p.qx, p.qy, WIN)
    r1 = cref.edp_window(p.cost, cen1, WIN, p.qx, p.qy, p.lam, p.trunc, p.mode, 1)
    out = {"workload": p.name, "cost_sha256": p.sha256(), "qx": p.qx, "qy": p.qy, "lam": p.lam,
           "trunc": p.trunc, "mode": p.mode, "iterations": 1, "win": WIN, "scale": SCALE,
           "rounds": [{"centres_sha256": sha(cen0), "energy": r0["energy"], "labels_sha256": sha(r0["labels"])},
                      {"centres_sha256": sha(cen1), "energy": r1["energy"], "labels_sha256": sha(r1["labels"])}],
           "source": "oracle network forward (cnn_ref) on the committed weights, C oracle windowed EDP; "
                     "round 1 re-centred on the round-0 labels"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "edp_window640x480_q961.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
