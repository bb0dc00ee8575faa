"""GPU parity of the EDP solve over three label dimensions (the tiles of edp_tiles_3d: every lane
holds its labels at each label of the third dimension, whose operator runs inside the lane; the
wide tile of edp_wide_tiles_3d: the third dimension spread over the wavefronts of a vertex, its
operator exchanging them through LDS) against the C oracle, bit-exact: labels and energy.

Cases cover every 3D tile, the four minimum searches the scans compile (general RMS windows of
one and two steps, the linear RMS, the walked window of the squared prior), both truncation
modes, int16 and int32 costs, one and two iterations, padded label spaces (every dimension short
of the tile), a label space along z only, single vertices, rows and columns, ragged grids that
span several workgroup bands, both lane splits, the batch path with 2D and 3D instances mixed,
the energy kernel on random labellings, and the 640 x 480 workload with 343 labels checked
through properties that hold at any size.
"""
import numpy as np
import pytest
import torch

import paper_1410_7922_amd as edp
import synth
from oracle import cref
from oracle import edp_ref as R

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def gpu_edp(p, qz, iterations, tile=-1, prior=0, split=0, waves=0, fuse=0):
    lab, e = edp.solve(torch.from_numpy(np.ascontiguousarray(p.cost)).to(DEV), p.qx, p.qy, p.lam, p.trunc, p.mode,
                       iterations=iterations, cost_bound=int(np.abs(p.cost).max()) + 1, tile=tile, prior=prior,
                       split=split, waves=waves, fuse=fuse, qz=qz)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), int(e.item())


def search_of(lam_T_prior):
    T, prior = lam_T_prior
    return "grms" if (prior == 1 or T <= 3) else "lrms"


CASES = [
    # W, H, qx, qy, qz, lam, T, mode, prior, lo, hi, dtype, iterations
    (13, 11, 7, 7, 7, 40, 3, 0, 0, 0, 2500, np.int32, 1),     # the workload's label space, window of 2
    (13, 11, 7, 7, 7, 40, 3, 1, 0, 0, 2500, np.int32, 2),     # joint truncation, two iterations
    (9, 10, 8, 8, 8, 9, 2, 0, 0, -40, 300, np.int32, 1),     # full tile, window of 1, negative costs
    (11, 9, 5, 6, 3, 6, 5, 0, 0, 0, 90, np.int16, 1),        # linear RMS (T = 5), padding everywhere
    (11, 9, 5, 6, 3, 6, 5, 1, 0, 0, 90, np.int32, 2),        # linear RMS, joint
    (10, 8, 6, 5, 7, 3, 4, 0, 1, 0, 400, np.int32, 1),       # squared prior, walked window (T = 4)
    (10, 8, 4, 4, 4, 5, 3, 1, 1, 0, 400, np.int16, 1),       # squared prior, window of 2, joint
    (9, 7, 1, 1, 8, 7, 3, 0, 0, 0, 200, np.int32, 1),        # a label space along z only
    (1, 1, 7, 7, 7, 40, 3, 0, 0, 0, 2500, np.int32, 1),      # single vertex
    (1, 37, 4, 3, 4, 7, 3, 0, 0, 0, 200, np.int16, 1),       # single column, many bands
    (33, 1, 4, 3, 4, 7, 3, 1, 0, 0, 200, np.int32, 1),       # single row
    (7, 45, 3, 2, 2, 4, 2, 0, 0, 0, 60, np.int32, 2),        # tall ragged grid, small space
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}q{c[2]}x{c[3]}x{c[4]}T{c[6]}m{c[7]}p{c[8]}j{c[12]}")
def test_three_dimensional_tiles_against_oracle(case):
    W, H, qx, qy, qz, lam, T, mode, prior, lo, hi, dt, j = case
    p = synth.random_problem(W * 17 + H * 5 + qx + qy + qz + j, W, H, qx, qy, lam, T, mode, lo, hi, dt, qz=qz)
    ref = cref.edp(p.cost, qx, qy, lam, T, mode, j, search_of((T, prior)), prior=prior, qz=qz)
    tiles = edp.tiles_3d(qx, qy, qz)
    wide = edp.wide_tiles_3d(qx, qy, qz)
    assert tiles and wide
    for tile in [-1] + tiles + (wide if T <= 3 else []):
        note(f"r3 {p.name} T{T} mode {mode} prior {prior} j{j} tile {tile}")
        lab, e = gpu_edp(p, qz, j, tile, prior)
        assert np.array_equal(lab, ref["labels"]), tile
        assert e == ref["energy"], tile
    if T > 3:
        # the wide tiles take the window search of at most two steps per side only
        with pytest.raises(edp.EdpError) as err:
            gpu_edp(p, qz, j, wide[0], prior)
        assert err.value.status == -5


@pytest.mark.parametrize("split,waves,fuse", [(2, 0, 0), (1, 1, 1), (2, 3, 2)])
def test_lane_splits_and_launch_shapes(split, waves, fuse):
    """The 16-lane 3D tiles with both searches of a step on one lane set or on two halves, and
    other workgroup shapes: the same labels."""
    p = synth.random_problem(77, 14, 19, 4, 4, 6, 3, 0, 0, 120, np.int32, qz=4)
    ref = cref.edp(p.cost, 4, 4, 6, 3, 0, 1, "grms", qz=4)
    for tile in (20, 21):
        note(f"r3 split {split} waves {waves} fuse {fuse} tile {tile}")
        lab, e = gpu_edp(p, 4, 1, tile, split=split, waves=waves, fuse=fuse)
        assert np.array_equal(lab, ref["labels"]) and e == ref["energy"], tile


@pytest.mark.parametrize("waves,fuse", [(1, 1), (2, 2), (1, 2)])
def test_wide_tile_launch_shapes(waves, fuse):
    """The wide 3D tile with one or two scanlines per workgroup and one or two scans per launch,
    on a grid of several workgroup bands with a ragged last band, j = 2: the same labels."""
    p = synth.random_problem(91, 23, 17, 7, 6, 9, 3, 0, 0, 400, np.int32, qz=5)
    ref = cref.edp(p.cost, 7, 6, 9, 3, 0, 2, "grms", qz=5)
    note(f"r3 wide tile rows {waves} fuse {fuse}")
    lab, e = gpu_edp(p, 5, 2, 25, waves=waves, fuse=fuse)
    assert np.array_equal(lab, ref["labels"]) and e == ref["energy"]


def test_lambda_zero_is_winner_take_all():
    p = synth.random_problem(5, 21, 17, 7, 7, 0, 3, 0, -50, 50, np.int32, qz=7)
    lab, _ = gpu_edp(p, 7, 2)
    assert np.array_equal(lab, R.wta(p.cost))


def test_offset_workload_crop_against_oracle():
    """A 64 x 48 crop of the motion-with-brightness-offset workload (7 x 7 x 7 labels)."""
    p = synth.motion_offset_problem(0, W=96, H=64)
    c = np.ascontiguousarray(p.cost[8:56, 16:80])
    crop = synth.Problem(c, 7, 7, p.lam, p.trunc, p.mode, qz=7)
    for j in (1, 2):
        ref = cref.edp(c, 7, 7, p.lam, p.trunc, p.mode, j, "grms", qz=7)
        note(f"r3 offset crop 64x48 j{j}")
        lab, e = gpu_edp(crop, 7, j)
        assert np.array_equal(lab, ref["labels"]) and e == ref["energy"], j


def test_energy_kernel_three_dimensions():
    """edp_energy of random labellings equals the oracle's energy (both priors and modes)."""
    rng = np.random.default_rng(3)
    p = synth.random_problem(8, 37, 29, 5, 3, 7, 3, 0, -100, 100, np.int32, qz=6)
    for mode, prior in ((0, 0), (1, 0), (0, 1), (1, 1)):
        lab = rng.integers(0, 5 * 3 * 6, size=(29, 37)).astype(np.int32)
        e, bad = edp.energy(torch.from_numpy(p.cost).to(DEV), torch.from_numpy(lab).to(DEV), 5, 3, 7, 3, mode,
                            cost_bound=101, prior=prior, qz=6)
        assert int(e.item()) == cref.energy(p.cost, lab, 5, 3, 7, 3, mode, True, prior=prior, qz=6)
        assert int(bad.item()) == 0


def test_batch_mixes_two_and_three_dimensional_instances():
    probs = [synth.random_problem(40 + i, 9 + i, 7 + 2 * i, 4, 3, 5, 3, i % 2, 0, 80, np.int32, qz=(3 if i % 2 else 1))
             for i in range(4)]
    costs = [torch.from_numpy(np.ascontiguousarray(q.cost)).to(DEV) for q in probs]
    params = [dict(qx=q.qx, qy=q.qy, qz=q.qz, lam=q.lam, trunc=q.trunc, mode=q.mode, iterations=1, cost_bound=81)
              for q in probs]
    plan = edp.BatchPlan(costs, params)
    note("r3 batch of 2D and 3D instances")
    labels, energies = plan.solve()
    plan.check()
    torch.cuda.synchronize()
    for i, q in enumerate(probs):
        ref = cref.edp(q.cost, q.qx, q.qy, q.lam, q.trunc, q.mode, 1, "grms", qz=q.qz)
        assert np.array_equal(labels[i].cpu().numpy(), ref["labels"]), i
        assert int(energies[i].item()) == ref["energy"], i


def test_full_size_offset_workload_against_golden():
    """The 640 x 480 workload with 343 labels at full size, on the built-in tile and on each tile of
    three label dimensions: labels and energy equal the C oracle's (its golden, written by
    tests/golden/make_motion_offset640x480_q343.py)."""
    import hashlib
    import json
    import os
    p = synth.workload("motion_offset640x480")
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "edp_motion_offset640x480_q343.json")) as f:
        g = json.load(f)
    assert g["cost_sha256"] == p.sha256()
    cost = torch.from_numpy(p.cost).to(DEV)
    for tile in [-1] + edp.tiles_3d(7, 7, 7) + edp.wide_tiles_3d(7, 7, 7):
        note(f"r3 640x480 q343 golden tile {tile}")
        lab, e = edp.solve(cost, 7, 7, p.lam, p.trunc, p.mode, iterations=1, cost_bound=2501, qz=7, tile=tile)
        torch.cuda.synchronize()
        sha = hashlib.sha256(np.ascontiguousarray(lab.cpu().numpy(), np.int32).tobytes()).hexdigest()
        assert sha == g["labels_sha256"] and int(e.item()) == g["energy"], tile


def test_full_size_offset_workload_properties():
    """The 640 x 480 workload with 343 labels, in the launch configuration the benchmark times: every
    label in range, the reported energy equal to the oracle's energy of the returned labels, below
    winner-take-all's by far; and with lambda = 0 the labels are winner-take-all's exactly."""
    p = synth.workload("motion_offset640x480")
    cost = torch.from_numpy(p.cost).to(DEV)
    note("r3 640x480 q343 solve")
    lab, e = edp.solve(cost, 7, 7, p.lam, p.trunc, p.mode, iterations=1, cost_bound=2501, qz=7)
    torch.cuda.synchronize()
    lab = lab.cpu().numpy()
    assert lab.min() >= 0 and lab.max() < 343
    e_ref = cref.energy(p.cost, lab, 7, 7, p.lam, p.trunc, p.mode, True, qz=7)
    assert int(e.item()) == e_ref
    assert e_ref < 0.5 * cref.energy(p.cost, R.wta(p.cost), 7, 7, p.lam, p.trunc, p.mode, True, qz=7)
    note("r3 640x480 q343 lambda 0")
    lab0, _ = edp.solve(cost, 7, 7, 0, p.trunc, p.mode, iterations=1, cost_bound=2501, qz=7)
    torch.cuda.synchronize()
    assert np.array_equal(lab0.cpu().numpy(), R.wta(p.cost))
