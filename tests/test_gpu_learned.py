"""GPU checks of the learned-window path: the proposal (pooled input, network, decoding) feeds the
windowed EDP, whose result equals the oracle's windowed EDP for those windows; the trained
network's windows beat windows proposed without it (an untrained network, the per-pixel cost
minimum) on held-out instances; the gap judge falls back to the plain EDP exactly when the gap
exceeds its bound."""
import numpy as np
import pytest
import torch

from paper_1410_7922_amd import binding as B
from paper_1410_7922_amd.learned import LearnedWindowEDP, window_hit_rate
from paper_1410_7922_amd.window import WindowNet
import synth
from oracle import cref

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def cost_of(seed, W, H):
    i0, i1, _, _ = synth.motion_frames(seed=seed, W=W, H=H, r=15)
    return B.dsi_motion(torch.from_numpy(i0).to(DEV), torch.from_numpy(i1).to(DEV), 15, 2500)


def test_learned_windows_feed_an_exact_windowed_solve():
    solver = LearnedWindowEDP.pretrained(DEV)
    cost = cost_of(20001, 64, 48)
    note("learned proposal + windowed solve vs oracle, 64x48")
    lab, e, cen = solver.solve_windowed(cost)
    torch.cuda.synchronize()
    ref = cref.edp_window(cost.cpu().numpy(), cen.cpu().numpy(), 7, 31, 31, 15, 3, 0, 1)
    assert np.array_equal(lab.cpu().numpy(), ref["labels"])
    assert int(e.item()) == ref["energy"]
    # refinement rounds keep every result exact for its windows
    lab2, e2, cen2 = solver.solve_refined(cost, 1)
    torch.cuda.synchronize()
    ref2 = cref.edp_window(cost.cpu().numpy(), cen2.cpu().numpy(), 7, 31, 31, 15, 3, 0, 1)
    assert np.array_equal(lab2.cpu().numpy(), ref2["labels"]) and int(e2.item()) == ref2["energy"]


def test_trained_network_gains_over_proposals_without_it():
    trained = LearnedWindowEDP.pretrained(DEV)
    untrained = LearnedWindowEDP(WindowNet(DEV, seed=7))
    gaps = {"trained": [], "untrained": [], "cost minimum": []}
    hits = {"trained": [], "untrained": []}
    for seed in (30001, 30002, 30003, 30004):
        cost = cost_of(seed, 160, 120)
        lab_p, e_p = trained.solve_plain(cost)
        ep = int(e_p.item())
        for name, solver in (("trained", trained), ("untrained", untrained)):
            lab, e, cen = solver.solve_windowed(cost)
            gaps[name].append(solver.judge(int(e.item()), ep))
            hits[name].append(window_hit_rate(cen, lab_p, 31, 7))
        wta = torch.argmin(cost, dim=2).to(torch.int32)
        cen = B.window_recenter(wta, 31, 31, 7, torch.empty((120, 160, 2), dtype=torch.int32, device=DEV))
        lab, e, _ = trained.solve_windowed(cost, cen)
        gaps["cost minimum"].append(trained.judge(int(e.item()), ep))
    mean = {k: float(np.mean(v)) for k, v in gaps.items()}
    note(f"mean energy gaps {mean}, window hit rates trained {np.mean(hits['trained']):.3f} "
         f"untrained {np.mean(hits['untrained']):.3f}")
    assert np.mean(hits["trained"]) > 0.7 > 0.2 > np.mean(hits["untrained"])
    assert mean["trained"] < 0.5 * mean["untrained"]
    assert mean["trained"] < 0.5 * mean["cost minimum"]


def test_gap_judge_and_fallback():
    cost = cost_of(40001, 96, 64)
    solver = LearnedWindowEDP.pretrained(DEV, max_gap=-1.0)      # every gap exceeds it
    note("gap judge: forced fallback")
    out = solver.solve(cost)
    lab_p, e_p = solver.solve_plain(cost)
    torch.cuda.synchronize()
    assert out["fallback"] and out["energy"] == int(e_p.item())
    assert torch.equal(out["labels"], lab_p)
    solver.max_gap = 1e9                                           # no gap exceeds it
    out = solver.solve(cost, e_plain=int(e_p.item()))
    lab_w, e_w, _ = solver.solve_windowed(cost)
    torch.cuda.synchronize()
    assert not out["fallback"] and out["energy"] == int(e_w.item())
    assert torch.equal(out["labels"], lab_w)
    assert out["gap"] == pytest.approx((int(e_w.item()) - int(e_p.item())) / int(e_p.item()))
