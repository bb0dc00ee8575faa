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


def test_windowed_solve_640x480_equals_oracle_golden():
    """The full-size windowed solve (640x480, 961 labels, 7x7 windows) with the network's centres
    as the oracle computes them (cnn_ref forward pass on the committed weights), and one round
    re-centred on its labels, against the oracle's energies and label hashes
    (tests/golden/edp_window640x480_q961.json, written by make_window640x480_q961.py)."""
    import hashlib
    import json
    import os
    from oracle import cnn_ref
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "golden", "edp_window640x480_q961.json")) as f:
        g = json.load(f)
    p = synth.workload("motion640x480")
    assert p.sha256() == g["cost_sha256"]
    weights = os.path.join(os.path.dirname(here), "paper_1410_7922_amd", "weights", "window_net_31x31.npz")
    with np.load(weights, allow_pickle=False) as f:
        params = cnn_ref.params_from_flat(f["params"])
        mode = int(f["pool_mode"])
    note("oracle network centres 640x480")
    cen = cnn_ref.network_centres(p.cost, 31, 31, params, g["scale"], g["win"], mode)
    sha = lambda a: hashlib.sha256(np.ascontiguousarray(a, np.int32).tobytes()).hexdigest()
    assert sha(cen) == g["rounds"][0]["centres_sha256"], "the oracle's centres differ from the golden's"
    cost = torch.from_numpy(p.cost).to(DEV)
    cen_t = torch.from_numpy(cen).to(DEV)
    for rnd in g["rounds"]:
        note(f"windowed solve 640x480 against the oracle golden, centres {rnd['centres_sha256'][:12]}")
        assert sha(cen_t.cpu().numpy()) == rnd["centres_sha256"]
        lab, e = B.solve_windowed(cost, cen_t, g["win"], 31, 31, g["lam"], g["trunc"], g["mode"], 1, cost_bound=2500)
        assert int(e.item()) == rnd["energy"]
        assert sha(lab.cpu().numpy()) == rnd["labels_sha256"]
        cen_t = B.window_recenter(lab, 31, 31, g["win"], torch.empty_like(cen_t))
