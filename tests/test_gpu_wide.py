"""GPU parity of the wide-vertex EDP scans (a vertex's labels on several wavefronts that exchange
the label rows at their slab edges through LDS every step) against the C oracle, bit-exact.

Cases span one and several slabs, padded label spaces, both truncation modes and both priors,
int16 and int32 costs, one and two iterations, one to the largest number of scanlines per
workgroup, one and two scans per launch, single rows and columns, and grids whose scans cross
many workgroup bands (tagged hand-off rows used alternately by consecutive bands) with a
partial last band.
"""
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


def gpu_edp(p, iterations, tile, waves=0, fuse=0, prior=0):
    lab, e = edp.solve(torch.from_numpy(np.ascontiguousarray(p.cost)).to(DEV), p.qx, p.qy, p.lam, p.trunc, p.mode,
                       iterations=iterations, cost_bound=int(np.abs(p.cost).max()) + 1, tile=tile, waves=waves,
                       fuse=fuse, prior=prior)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), int(e.item())




CASES = [
    # W, H, qx, qy, lam, T, mode, prior, lo, hi, dtype, iterations
    (7, 9, 31, 31, 15, 3, 0, 0, 0, 2500, np.int32, 1),
    (7, 9, 31, 31, 15, 3, 1, 0, 0, 2500, np.int32, 2),
    (12, 14, 32, 32, 9, 2, 0, 0, -40, 300, np.int32, 1),   # one-step window, negative costs
    (10, 13, 20, 27, 6, 3, 1, 0, 0, 90, np.int16, 1),      # padded rows and columns, joint
    (9, 11, 17, 9, 5, 3, 0, 1, 0, 400, np.int32, 1),       # squared prior, few label rows
    (9, 11, 12, 30, 4, 3, 1, 1, 0, 400, np.int32, 2),      # squared prior, joint
    (1, 1, 31, 31, 15, 3, 0, 0, 0, 2500, np.int32, 1),     # single vertex
    (1, 23, 16, 16, 7, 3, 0, 0, 0, 200, np.int16, 1),      # single column, many bands
    (29, 1, 16, 16, 7, 3, 0, 0, 0, 200, np.int32, 1),      # single row
    (15, 16, 2, 2, 3, 2, 0, 0, 0, 20, np.int32, 1),        # tiny label space on a wide tile
    (6, 41, 31, 31, 15, 3, 0, 0, 0, 2500, np.int32, 1),    # tall: many workgroup bands, partial last
    (6, 7, 64, 64, 5, 2, 0, 0, 0, 300, np.int32, 1),       # 4096 labels, eight wavefronts per vertex
    (7, 9, 40, 40, 6, 3, 1, 0, 0, 200, np.int16, 1),       # 1600 labels padded to 64 x 64, joint
    (9, 5, 57, 23, 4, 3, 0, 1, 0, 300, np.int32, 2),       # 64 x 32 tile, squared prior, two iterations
    (5, 11, 20, 50, 6, 3, 0, 0, -50, 100, np.int32, 1),    # 32 x 64 tile, negative costs
]


def max_rows(tile):
    # at most 8 compute wavefronts per workgroup (py / 4 per scanline)
    return 8 // (edp.tile_info(tile)[2] // 4)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}q{c[2]}x{c[3]}m{c[6]}p{c[7]}j{c[11]}")
def test_wide_tiles_against_oracle(case):
    W, H, qx, qy, lam, T, mode, prior, lo, hi, dt, j = case
    p = synth.random_problem(W * 13 + H * 3 + qx + j, W, H, qx, qy, lam, T, mode, lo, hi, dt)
    ref = cref.edp(p.cost, qx, qy, lam, T, mode, j, "grms", prior=prior)
    tiles = edp.wide_tiles(qx, qy)
    assert tiles
    for tile in tiles:
        mr = max_rows(tile)
        for waves, fuse in sorted({(0, 0), (1, 2), (min(2, mr), 1), (mr, 2)}):
            note(f"wide {p.name} prior {prior} j{j} tile {tile} rows {waves} fuse {fuse}")
            lab, e = gpu_edp(p, j, tile, waves, fuse, prior)
            assert np.array_equal(lab, ref["labels"]), (tile, waves, fuse)
            assert e == ref["energy"], (tile, waves, fuse)


def test_wide_tile_is_the_built_in_choice_for_961_labels():
    """31x31 labels with T = 3 run on the wide tile of four wavefronts per vertex by default."""
    assert 16 in edp.wide_tiles(31, 31)
    assert edp.tile_info(16) == (16, 2, 16, 2)


def test_wide_tiles_reused_workspace():
    """Two different instances of one shape solved one after the other in one workspace (the tagged
    hand-off rows are cleared and their tags restart), then the first again."""
    ws = edp.Workspace(DEV)
    probs = [synth.random_problem(s, 5, 37, 31, 31, 15, 3, 0, 0, 2500, np.int32) for s in (1, 2)]
    refs = [cref.edp(p.cost, 31, 31, 15, 3, 0, 1, "grms") for p in probs]
    for k in (0, 1, 0):
        p = probs[k]
        note(f"wide reuse {p.name}")
        lab, e = edp.solve(torch.from_numpy(p.cost).to(DEV), 31, 31, 15, 3, 0, iterations=1, cost_bound=2501,
                           tile=16, waves=2, ws=ws)
        torch.cuda.synchronize()
        assert np.array_equal(lab.cpu().numpy(), refs[k]["labels"])
        assert int(e.item()) == refs[k]["energy"]
