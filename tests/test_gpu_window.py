"""GPU parity of the label-window EDP (edp_solve_windowed) with the oracle's windowed EDP (the
plain EDP on a cost volume masked outside each vertex's box): bit-exact labels and energies on
random and motion problems, boxes of several sizes, both truncation modes, several iterations
and launch shapes, and the case of a box that covers the whole label space."""
import numpy as np
import pytest
import torch

import paper_1410_7922_amd as edp
import synth
from oracle import cref

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def centers_for(rng, H, W, qx, qy, win, smooth=False):
    r = win // 2
    if smooth:                                   # piecewise-constant blocks, like decoded windows
        cx = np.repeat(np.repeat(rng.integers(r, qx - r, size=((H + 1) // 2, (W + 1) // 2)), 2, 0), 2, 1)[:H, :W]
        cy = np.repeat(np.repeat(rng.integers(r, qy - r, size=((H + 1) // 2, (W + 1) // 2)), 2, 0), 2, 1)[:H, :W]
    else:
        cx = rng.integers(r, qx - r, size=(H, W))
        cy = rng.integers(r, qy - r, size=(H, W))
    return np.ascontiguousarray(np.stack([cx, cy], -1).astype(np.int32))


def gpu_win(p, cen, win, iterations=1, cost_bound=0, waves=0, chunk=0, fuse=0):
    lab, e = edp.solve_windowed(torch.from_numpy(np.ascontiguousarray(p.cost, np.int32)).to(DEV),
                                torch.from_numpy(cen).to(DEV), win, p.qx, p.qy, p.lam, p.trunc, p.mode, iterations,
                                cost_bound=cost_bound or int(np.abs(p.cost).max()) + 1, waves=waves, chunk=chunk,
                                fuse=fuse)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), int(e.item())


CASES = [
    # W, H, q, win, lam, T, mode, iterations, smooth centres
    (13, 9, 9, 3, 5, 2, 0, 1, False),
    (17, 11, 15, 5, 9, 3, 0, 1, False),
    (21, 14, 31, 7, 15, 3, 0, 1, True),
    (21, 14, 31, 7, 15, 3, 0, 2, False),
    (12, 19, 11, 7, 6, 2, 1, 1, False),
    (1, 9, 9, 5, 4, 2, 0, 1, False),
    (9, 1, 9, 5, 4, 2, 0, 2, False),
    (40, 37, 31, 7, 15, 3, 0, 1, True),
    # T <= 3 runs the general RMS window between frames, larger T the linear RMS transform
    (15, 10, 13, 5, 7, 1, 0, 1, False),
    (17, 11, 15, 5, 9, 4, 0, 1, False),
    (14, 12, 21, 7, 6, 6, 1, 2, True),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}q{c[2]}w{c[3]}m{c[6]}j{c[7]}")
def test_windowed_matches_oracle(case):
    W, H, q, win, lam, T, mode, j, smooth = case
    rng = np.random.default_rng(W * 7 + H + q)
    p = synth.random_problem(W + H, W, H, q, q, lam, T, mode, 0, 900)
    cen = centers_for(rng, H, W, q, q, win, smooth)
    ref = cref.edp_window(p.cost, cen, win, q, q, lam, T, mode, j)
    for waves, chunk, fuse in ((0, 0, 0), (1, 1, 1), (3, 8, 2)):
        note(f"window {p.name} win {win} j{j} waves {waves} chunk {chunk} fuse {fuse}")
        lab, e = gpu_win(p, cen, win, j, waves=waves, chunk=chunk, fuse=fuse)
        assert np.array_equal(lab, ref["labels"]), (waves, chunk, fuse)
        assert e == ref["energy"], (waves, chunk, fuse)


def test_full_box_equals_plain_edp():
    p = synth.random_problem(77, 23, 17, 7, 7, 5, 2, 0, 0, 300)
    cen = np.full((17, 23, 2), 3, np.int32)
    note("window covering the label space")
    lab, e = gpu_win(p, cen, 7)
    ref = cref.edp(p.cost, 7, 7, 5, 2, 0, 1)
    assert np.array_equal(lab, ref["labels"]) and e == ref["energy"]


def test_motion_31x31_mid_size_matches_oracle():
    p = synth.motion_problem(seed=5, W=96, H=72, r=15)
    rng = np.random.default_rng(8)
    gt = p.meta["gt"]
    # windows around the planted flow, perturbed by up to two labels and clamped
    cx = np.clip(gt % 31 + rng.integers(-2, 3, gt.shape), 3, 27)
    cy = np.clip(gt // 31 + rng.integers(-2, 3, gt.shape), 3, 27)
    cen = np.ascontiguousarray(np.stack([cx, cy], -1).astype(np.int32))
    note("window motion 96x72 31x31")
    lab, e = gpu_win(p, cen, 7, cost_bound=2500)
    ref = cref.edp_window(p.cost, cen, 7, 31, 31, p.lam, p.trunc, p.mode, 1)
    assert np.array_equal(lab, ref["labels"]) and e == ref["energy"]


def test_wide_label_axis_at_the_shift_limit():
    # centres along x anywhere in [3, 130]: neighbouring frames differ by up to 127 labels, the
    # largest shift the frames' 8-bit shift codes hold (qx - win = 127)
    p = synth.random_problem(91, 12, 10, 134, 9, 5, 3, 0, 0, 400)
    rng = np.random.default_rng(91)
    cen = centers_for(rng, 10, 12, 134, 9, 7)
    cen[0, 0, 0], cen[0, 1, 0] = 3, 130
    note("window 12x10 with 134x9 labels, shifts up to 127")
    lab, e = gpu_win(p, cen, 7)
    ref = cref.edp_window(p.cost, cen, 7, 134, 9, 5, 3, 0, 1)
    assert np.array_equal(lab, ref["labels"]) and e == ref["energy"]
