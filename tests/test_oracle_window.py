"""Pins of the windowed-EDP oracle (the plain EDP on a cost volume masked outside each vertex's
label box) against facts that do not depend on it: a box covering the label space is the plain
EDP; a one-label box forces its label; with lambda = 0 each vertex takes its in-box cost minimum;
costs outside the boxes do not matter; the result never beats the exhaustive box-restricted
minimum on tiny grids."""
import itertools

import numpy as np
import pytest

import synth
from oracle import cref
from oracle import edp_ref as R


def _centers(rng, H, W, qx, qy, win):
    r = win // 2
    cx = rng.integers(r, qx - r, size=(H, W))
    cy = rng.integers(r, qy - r, size=(H, W))
    return np.stack([cx, cy], -1).astype(np.int32)


@pytest.mark.parametrize("mode", [0, 1])
def test_full_box_is_plain_edp(mode):
    p = synth.random_problem(3, 9, 7, 5, 4, 6, 2, mode, 0, 60)
    cen = np.zeros((7, 9, 2), np.int32)
    cen[..., 0], cen[..., 1] = 2, 2
    for j in (1, 2):
        w = cref.edp_window(p.cost, cen, 9, 5, 4, 6, 2, mode, j)
        ref = cref.edp(p.cost, 5, 4, 6, 2, mode, j)
        assert np.array_equal(w["labels"], ref["labels"]) and w["energy"] == ref["energy"]


def test_one_label_box_forces_the_centre():
    rng = np.random.default_rng(1)
    p = synth.random_problem(4, 8, 6, 7, 7, 5, 3, 0, 0, 99)
    cen = _centers(rng, 6, 8, 7, 7, 1)
    w = cref.edp_window(p.cost, cen, 1, 7, 7, 5, 3, 0)
    lab = cen[..., 1] * 7 + cen[..., 0]
    assert np.array_equal(w["labels"], lab)
    assert w["energy"] == R.energy(p.cost, lab, 7, 7, 5, 3, 0, True)


def test_zero_lambda_takes_the_in_box_minimum():
    rng = np.random.default_rng(2)
    p = synth.random_problem(5, 10, 6, 9, 9, 0, 3, 0, 0, 40)      # small range: many ties
    cen = _centers(rng, 6, 10, 9, 9, 3)
    w = cref.edp_window(p.cost, cen, 3, 9, 9, 0, 3, 0)
    c = p.cost.reshape(6, 10, 9, 9)
    for y in range(6):
        for x in range(10):
            cx, cy = cen[y, x]
            box = c[y, x, cy - 1:cy + 2, cx - 1:cx + 2]
            iy, ix = np.unravel_index(np.argmin(box), box.shape)   # row-major first minimum
            assert w["labels"][y, x] == (cy - 1 + iy) * 9 + (cx - 1 + ix)


def test_costs_outside_the_boxes_do_not_matter():
    rng = np.random.default_rng(3)
    p = synth.random_problem(6, 7, 9, 11, 11, 4, 2, 0, 0, 80)
    cen = _centers(rng, 9, 7, 11, 11, 5)
    w = cref.edp_window(p.cost, cen, 5, 11, 11, 4, 2, 0)
    c2 = p.cost.reshape(9, 7, 11, 11).copy()
    vy, vx = np.mgrid[0:11, 0:11]
    for y in range(9):
        for x in range(7):
            cx, cy = cen[y, x]
            out = (np.abs(vx - cx) > 2) | (np.abs(vy - cy) > 2)
            c2[y, x][out] = rng.integers(-1000, 1000, size=int(out.sum()))
    w2 = cref.edp_window(c2.reshape(9, 7, 121), cen, 5, 11, 11, 4, 2, 0)
    assert np.array_equal(w["labels"], w2["labels"])


def test_never_below_the_exhaustive_box_minimum():
    rng = np.random.default_rng(4)
    for trial in range(3):
        p = synth.random_problem(7 + trial, 2, 2, 5, 1, 4, 2, 0, 0, 30)
        cen = np.stack([rng.integers(1, 4, size=(2, 2)), np.zeros((2, 2), np.int64)], -1).astype(np.int32)
        w = cref.edp_window(p.cost, cen, 3, 5, 1, 4, 2, 0)
        boxes = [range(cen[y, x, 0] - 1, cen[y, x, 0] + 2) for y in range(2) for x in range(2)]
        best = min(R.energy(p.cost, np.array(l).reshape(2, 2), 5, 1, 4, 2, 0, True)
                   for l in itertools.product(*boxes))
        assert w["energy"] >= best
        for y in range(2):
            for x in range(2):
                assert abs(int(w["labels"][y, x]) - int(cen[y, x, 0])) <= 1
