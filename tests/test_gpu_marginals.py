"""GPU parity of the min-marginal scanline DP (Sec. 4.1, eqs. DP_1D_3 and DP_1D_5) against the
oracle's min-marginals, bit-exact: labels (smallest argmin of each column's marginal), the marginal
excess over each column's minimum, row optima; and, at full size, against the GPU's standard DP."""
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


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def oracle_marginals(p, prior):
    """Per row: S_Omega from the oracle (straightforward search), its smallest argmins and excess."""
    H, W, Q = p.cost.shape
    marg = np.stack([R.dp_min_marginals(p.cost[y], p.qx, p.qy, p.lam, p.trunc, p.mode, prior=prior)
                     for y in range(H)])
    return np.argmin(marg, axis=2).astype(np.int32), (marg - marg.min(axis=2, keepdims=True)).astype(np.int64)


CASES = [
    # W, H, qx, qy, lam, T, mode, prior, lo, hi, dtype
    (1, 3, 5, 1, 4, 2, 0, 0, -9, 9, np.int32),
    (2, 1, 3, 1, 3, 1, 0, 0, 0, 9, np.int32),
    (37, 13, 16, 1, 9, 3, 0, 0, -60, 255, np.int32),
    (50, 9, 32, 1, 11, 2, 0, 0, 0, 50, np.int16),
    (23, 70, 64, 1, 4, 6, 0, 0, 0, 120, np.int16),     # linear RMS (wide window)
    (19, 11, 5, 1, 0, 1, 0, 0, 0, 3, np.int32),         # lambda = 0, ties
    (21, 7, 4, 4, 6, 2, 0, 0, -20, 80, np.int32),
    (21, 7, 4, 4, 6, 3, 1, 0, -20, 80, np.int32),
    (17, 6, 15, 15, 15, 3, 0, 0, 0, 2500, np.int32),
    (9, 5, 31, 31, 15, 3, 0, 0, 0, 2500, np.int32),
    (30, 6, 24, 1, 2, 3, 0, 1, 0, 60, np.int16),        # squared prior, window
    (25, 5, 40, 1, 1, 6, 0, 1, 0, 60, np.int16),        # squared prior, walked window
    (14, 6, 7, 5, 2, 2, 1, 1, -10, 60, np.int32),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}q{c[2]}x{c[3]}T{c[5]}m{c[6]}p{c[7]}")
def test_marginals_all_tiles(case):
    W, H, qx, qy, lam, T, mode, prior, lo, hi, dt = case
    p = synth.random_problem(W * 23 + H + prior, W, H, qx, qy, lam, T, mode, lo, hi, dt)
    lab_ref, exc_ref = oracle_marginals(p, prior)
    _, row_ref, tot_ref = cref.dp_scanline(p.cost, qx, qy, lam, T, mode, "sfms", prior=prior)
    for tile in edp.tiles(qx, qy):
        note(f"dp marginals {p.name} T{T} prior {prior} tile {tile}")
        lab, exc, row, tot = edp.dp_marginals(to_dev(p.cost), qx, qy, lam, T, mode, cost_bound=max(abs(lo), hi) + 1,
                                              tile=tile, prior=prior, marginal=True)
        torch.cuda.synchronize()
        assert np.array_equal(lab.cpu().numpy(), lab_ref), tile
        assert np.array_equal(exc.cpu().numpy().astype(np.int64), exc_ref), tile
        assert np.array_equal(row.cpu().numpy(), row_ref), tile
        assert int(tot.item()) == tot_ref, tile


def test_marginals_stereo_workload_full_size():
    """Full stereo 384x288: sampled rows against the oracle; at every row and column, the marginal
    minimum is the row optimum of the GPU's standard DP, and where every column of a row has a
    unique minimiser the labels are the standard DP's (Sec. 4.1: exact for a unique optimum)."""
    p = synth.workload("stereo384x288")
    cost = to_dev(p.cost)
    note("dp marginals stereo384x288")
    lab, exc, row, tot = edp.dp_marginals(cost, p.qx, 1, p.lam, p.trunc, 0, cost_bound=50, marginal=True)
    dlab, drow, dtot = edp.dp_scanline(cost, p.qx, 1, p.lam, p.trunc, 0, cost_bound=50)
    torch.cuda.synchronize()
    lab, exc, row = lab.cpu().numpy(), exc.cpu().numpy(), row.cpu().numpy()
    dlab, drow = dlab.cpu().numpy(), drow.cpu().numpy()
    assert np.array_equal(row, drow) and int(tot.item()) == int(dtot.item())
    assert (exc.min(axis=2) == 0).all() and (exc >= 0).all()
    unique_rows = ((exc == 0).sum(axis=2) == 1).all(axis=1)
    assert unique_rows.sum() > 0
    assert np.array_equal(lab[unique_rows], dlab[unique_rows])
    for y in (0, 143, 287):
        marg = R.dp_min_marginals(p.cost[y], p.qx, 1, p.lam, p.trunc, 0)
        assert np.array_equal(lab[y], np.argmin(marg, axis=1))
        assert np.array_equal(exc[y], marg - marg.min(axis=1, keepdims=True))


def test_marginals_without_marginal_output_and_workspace_reuse():
    ws = edp.Workspace()
    for seed in (1, 2):
        p = synth.random_problem(seed, 40, 19, 12, 1, 5, 2, 0, 0, 40, np.int16)
        lab_ref, _ = oracle_marginals(p, 0)
        lab, exc, row, tot = edp.dp_marginals(to_dev(p.cost), 12, 1, 5, 2, 0, cost_bound=41, ws=ws)
        torch.cuda.synchronize()
        assert exc is None
        assert np.array_equal(lab.cpu().numpy(), lab_ref)


def test_data_cost_and_marginals_replay_from_a_graph():
    """edp_dsi and edp_dp_marginals enqueue kernels only: captured into a hipGraph they give the
    eager results on every replay, with eager work and synchronisations between the replays."""
    m = synth.workload("motion320x240")
    i0, i1 = (to_dev(f) for f in m.meta["frames"])
    ws = edp.Workspace()
    cost = torch.empty((240, 320, 225), dtype=torch.int32, device=DEV)
    edp.dsi(i0, i1, 15, 15, -7, -7, 1, 1, 2, 2500, out=cost)
    lab0, exc0, row0, tot0 = edp.dp_marginals(cost, 15, 15, 15, 3, 0, cost_bound=2500, ws=ws, marginal=True)
    torch.cuda.synchronize()
    ref = (lab0.clone(), exc0.clone(), row0.clone(), tot0.clone())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    note("graph capture of edp_dsi + edp_dp_marginals")
    with torch.cuda.graph(g, stream=side):
        edp.dsi(i0, i1, 15, 15, -7, -7, 1, 1, 2, 2500, out=cost)
        out = edp.dp_marginals(cost, 15, 15, 15, 3, 0, cost_bound=2500, ws=ws, marginal=True)
    for r in range(3):
        cost.zero_()
        for t in out:
            t.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(cost.cpu().numpy(), m.cost), r
        for got, want in zip(out, ref):
            assert torch.equal(got, want), r
