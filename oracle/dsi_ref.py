"""Data cost (DSI) oracle -- TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 2 eq. Cost_value: C(x, v) = min(|I1(x + v) - I0(x)|^l2, C_max), l2 = 1 or 2
(Sec. 5.1 uses both).  Sec. 5.1 eq. Cost_cmp, the composite three-view cost:
C(x, v) = min(C_{0->1}(x, v), C_{0->2}(x, -v)).

Readings: a displaced position outside the image costs C_max for that view
(the paper does not say; this is the usual choice and what the synthetic
workloads use).  Label q = iy * qx + ix has the displacement
v = (ox + sx * ix, oy + sy * iy) with sx, sy = +1 or -1, so rectified stereo
with I1 the right image is qy = 1, ox = 0, sx = -1 (label d compares
I0(x, y) with I1(x - d, y)) and motion within [-r, r]^2 is ox = oy = -r,
sx = sy = +1.  All arithmetic is on int64.
"""
from __future__ import annotations

import numpy as np


def view_cost(i0: np.ndarray, i1: np.ndarray, dx: int, dy: int, l2: int, cmax: int) -> np.ndarray:
    """min(|I1(x + dx, y + dy) - I0(x, y)|^l2, cmax) for every pixel, cmax where x + v leaves the image."""
    H, W = i0.shape
    yy, xx = np.mgrid[0:H, 0:W]
    X, Y = xx + dx, yy + dy
    inside = (X >= 0) & (X < W) & (Y >= 0) & (Y < H)
    moved = i1[np.clip(Y, 0, H - 1), np.clip(X, 0, W - 1)].astype(np.int64)
    d = np.abs(moved - i0.astype(np.int64)) ** l2
    return np.where(inside, np.minimum(d, cmax), cmax)


def dsi(i0, i1, qx: int, qy: int, ox: int, oy: int, sx: int, sy: int, l2: int, cmax: int, i2=None) -> np.ndarray:
    """The cost volume [H][W][qx * qy] int64; with i2, the composite cost of eq. Cost_cmp."""
    i0, i1 = np.asarray(i0), np.asarray(i1)
    H, W = i0.shape
    out = np.empty((H, W, qx * qy), np.int64)
    for iy in range(qy):
        for ix in range(qx):
            dx, dy = ox + sx * ix, oy + sy * iy
            c = view_cost(i0, i1, dx, dy, l2, cmax)
            if i2 is not None:
                c = np.minimum(c, view_cost(i0, np.asarray(i2), -dx, -dy, l2, cmax))
            out[:, :, iy * qx + ix] = c
    return out
