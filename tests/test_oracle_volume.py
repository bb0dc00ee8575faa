"""Pins of the oracle's EDP on a three-dimensional grid (D = 3; no GPU).

Sec. 4.2 states eq. DP_2D_1 and eq. DP_2D_base for any image dimension D: 2D directional sums,
each M applied to S_k / D.  With D = 3 the scanning procedure is read as the eight raster scans
of a volume (x innermost; the x order alternates fastest, then y, then z), each computing its
three directions' sums.  Expected values: a two-voxel example worked by hand
(tests/golden/edp_volume_1x1x2_q2.json), reductions to the already pinned image EDP (a volume
one voxel thick along z, or along x, is an image under the same recursion with D = 3), lambda = 0,
planted labels, exhaustive enumeration, and the Python and C oracles against each other.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import cref
from oracle import edp_ref as R

GOLD = os.path.join(os.path.dirname(__file__), "golden", "edp_volume_1x1x2_q2.json")


def test_two_voxel_example_worked_by_hand():
    g = json.load(open(GOLD))
    v = g["volume"]
    cost = np.array(g["cost_zq"], np.int32).reshape(2, 1, 1, 2)
    seen = {}
    r = R.edp_volume(cost, v["qx"], v["qy"], v["lambda"], v["trunc"], v["mode"], v["iterations"],
                     trace=lambda it, sc, s: seen.__setitem__(sc, {k: a[:, 0, 0].tolist() for k, a in s.items()}))
    for scan, key in ((3, "after_scan_4"), (7, "after_scan_8")):
        for k, want in g[key].items():
            assert seen[scan][k] == want, (scan, k)
    assert r["marginal"][:, 0, 0].tolist() == g["marginal_zq"]
    assert r["labels"].ravel().tolist() == g["labels_z"] and r["energy"] == g["energy"]
    assert R.volume_exhaustive(cost, 2, 1, 1, 1, 0) == g["exhaustive_min_energy"]
    for search in ("sfms", "lrms", "grms"):
        c = cref.edp_volume(cost, 2, 1, 1, 1, 0, 1, search, marginal=True)
        assert c["marginal"][:, 0, 0].tolist() == g["marginal_zq"]
        assert c["labels"].ravel().tolist() == g["labels_z"] and c["energy"] == g["energy"]


@pytest.mark.parametrize("qx,qy,mode,j", [(4, 1, 0, 1), (3, 3, 1, 1), (3, 2, 0, 2)])
def test_one_voxel_thick_along_z_is_the_image_edp_twice(qx, qy, mode, j):
    """Z = 1: every z term is 0 (off the grid), scans 5-8 repeat the x, y orders of scans 1-4,
    and the 6-connected energy is the 4-connected one, so j volume iterations are 2j image
    iterations with D = 3."""
    p = synth.random_problem(qx * 7 + qy + j, 6, 5, qx, qy, lam=7, trunc=2, mode=mode, lo=-30, hi=60)
    a = R.edp(p.cost, qx, qy, 7, 2, mode, 2 * j, divisor=3)
    b = R.edp_volume(p.cost[None], qx, qy, 7, 2, mode, j)
    assert np.array_equal(b["marginal"][0], a["marginal"]) and np.array_equal(b["labels"][0], a["labels"])
    assert b["energy"] == a["energy"]
    c = cref.edp_volume(p.cost[None], qx, qy, 7, 2, mode, j, "lrms", marginal=True)
    assert np.array_equal(c["marginal"][0], a["marginal"]) and c["energy"] == a["energy"]


@pytest.mark.parametrize("qx,qy,mode,j", [(4, 1, 0, 1), (2, 3, 1, 2)])
def test_one_voxel_thick_along_x_is_the_image_edp(qx, qy, mode, j):
    """W = 1: the x terms vanish, consecutive scans that differ only in the x order compute the
    same sums (a scan repeated at once is idempotent), and the remaining order is P1..P4 on the
    (y, z) image with y along the image's x: j volume iterations are j image iterations, D = 3."""
    p = synth.random_problem(qx * 5 + qy + 11 * j, 5, 6, qx, qy, lam=5, trunc=2, mode=mode, lo=-20, hi=50)
    a = R.edp(p.cost, qx, qy, 5, 2, mode, j, divisor=3)                  # image [Z = 6][H = 5]
    vol = np.ascontiguousarray(p.cost[:, :, None, :])                    # volume [Z][H][W = 1]
    b = R.edp_volume(vol, qx, qy, 5, 2, mode, j)
    assert np.array_equal(b["marginal"][:, :, 0], a["marginal"]) and np.array_equal(b["labels"][:, :, 0], a["labels"])
    assert b["energy"] == a["energy"]
    c = cref.edp_volume(vol, qx, qy, 5, 2, mode, j, "grms", marginal=True)
    assert np.array_equal(c["marginal"][:, :, 0], a["marginal"]) and c["energy"] == a["energy"]


def test_lambda_zero_is_winner_take_all():
    p = synth.random_volume(3, 5, 4, 3, 6, 1, lam=0, trunc=2, lo=-40, hi=40)
    r = R.edp_volume(p.cost, 6, 1, 0, 2, 0, 1)
    assert np.array_equal(r["labels"], np.argmin(p.cost, axis=-1))
    c = cref.edp_volume(p.cost, 6, 1, 0, 2, 0, 2, "lrms")
    assert np.array_equal(c["labels"], np.argmin(p.cost, axis=-1))


def test_planted_constant_label_and_single_voxel():
    cost = np.full((3, 4, 5, 9), 500, np.int32)
    cost[..., 4] = 0
    for mode in (0, 1):
        r = R.edp_volume(cost, 3, 3, 9, 2, mode, 1)
        assert (r["labels"] == 4).all() and r["energy"] == 0
        c = cref.edp_volume(cost, 3, 3, 9, 2, mode, 1, "grms")
        assert (c["labels"] == 4).all() and c["energy"] == 0
    one = np.array([[[[5, -3, 2, -3]]]], np.int32)
    r = R.edp_volume(one, 4, 1, 3, 1, 0, 3)
    assert r["labels"].ravel().tolist() == [1] and r["energy"] == -3


def test_energy_by_hand():
    """2 x 1 x 2 volume, 3 labels, labels (x, z): (0,0) -> 0, (1,0) -> 2, (0,1) -> 1, (1,1) -> 1;
    lambda 2, T 1: pairs along x: |0-2|, |1-1|; along z: |0-1|, |2-1| -> 2 (1 + 0 + 1 + 1) = 6."""
    cost = np.zeros((2, 1, 2, 3), np.int32)
    cost[0, 0, 0, 0], cost[0, 0, 1, 2], cost[1, 0, 0, 1], cost[1, 0, 1, 1] = 4, -1, 2, 3
    lab = np.array([[[0, 2]], [[1, 1]]])
    assert R.energy_volume(cost, lab, 3, 1, 2, 1, 0) == 8 + 6
    assert cref.energy_volume(cost, lab, 3, 1, 2, 1, 0) == 8 + 6
    # T 5: 2 (2 + 0 + 1 + 1) = 8
    assert cref.energy_volume(cost, lab, 3, 1, 2, 5, 0) == 8 + 8


@pytest.mark.parametrize("mode", [0, 1])
def test_energy_not_below_exhaustive_minimum(mode):
    """2 x 2 x 2 voxels with 2 labels (256 labellings) and a 2 x 1 x 2 volume with 2 x 2 labels."""
    for seed in range(3):
        p = synth.random_volume(seed, 2, 2, 2, 2, 1, lam=6, trunc=2, mode=mode, lo=0, hi=30)
        r = R.edp_volume(p.cost, 2, 1, 6, 2, mode, 2)
        assert r["energy"] >= R.volume_exhaustive(p.cost, 2, 1, 6, 2, mode)
        q = synth.random_volume(seed + 7, 2, 1, 2, 2, 2, lam=4, trunc=1, mode=mode, lo=0, hi=20)
        r = R.edp_volume(q.cost, 2, 2, 4, 1, mode, 1)
        assert r["energy"] >= R.volume_exhaustive(q.cost, 2, 2, 4, 1, mode)


@pytest.mark.parametrize("qx,qy,mode,prior,j", [(5, 1, 0, 0, 1), (3, 3, 1, 0, 2), (4, 2, 0, 1, 1), (6, 1, 1, 1, 1)])
def test_python_and_c_agree(qx, qy, mode, prior, j):
    p = synth.random_volume(qx + 3 * qy + 5 * j + prior, 5, 4, 3, qx, qy, lam=8, trunc=2, mode=mode, lo=-20, hi=60)
    r = R.edp_volume(p.cost, qx, qy, 8, 2, mode, j, "sfms", prior=prior)
    for search in (("sfms", "grms") if prior else ("sfms", "lrms", "grms")):
        c = cref.edp_volume(p.cost, qx, qy, 8, 2, mode, j, search, marginal=True, prior=prior)
        assert np.array_equal(c["marginal"], r["marginal"]), search
        assert np.array_equal(c["labels"], r["labels"]) and c["energy"] == r["energy"]


def test_volume_workload_crop():
    """The volume workload: the oracle's EDP on a crop recovers most planted levels and lowers
    the energy far below winner-take-all's (soft check, fixed seed)."""
    p = synth.volume_problem(0, W=32, H=24, Z=16)
    r = cref.edp_volume(p.cost, 32, 1, p.lam, p.trunc, p.mode, 1, "grms")
    w = np.argmin(p.cost, axis=-1)
    assert r["energy"] < 0.7 * cref.energy_volume(p.cost, w, 32, 1, p.lam, p.trunc, p.mode)
    assert (r["labels"] == p.meta["gt"]).mean() > 0.8


def test_sums_grow_geometrically_with_the_volume_extent():
    """The cardinality argument of eq. DP_2D_base_1 balances only at D = 2: with D = 3 the supports
    of the summed terms count (2 x H Z + W H Z) / 3 voxels instead of x H Z, and the sums grow
    geometrically with the extent of the volume.  Recorded on the volume workload after one
    iteration: doubling the side of a cube multiplies the largest sum by more than 30 (8 -> 16,
    12 -> 24), while on images of the same costs 2.25 times the side adds less than half."""
    peak = {}
    for n in (8, 12, 16, 24):
        p = synth.volume_problem(0, W=n, H=n, Z=n)
        peak[n] = cref.edp_volume(p.cost, 32, 1, p.lam, p.trunc, p.mode, 1, "grms")["max_abs_sum"]
    assert peak[16] > 30 * peak[8] and peak[24] > 30 * peak[12], peak
    flat = []
    for n in (16, 36):
        img = synth.volume_problem(0, W=n, H=n, Z=1).cost[0]
        flat.append(cref.edp(img, 32, 1, 60, 3, 0, 1, "grms")["max_abs_sum"])
    assert flat[1] < 1.5 * flat[0], flat
