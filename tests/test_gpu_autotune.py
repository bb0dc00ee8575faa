"""GPU check of the launch-shape autotuner: it returns a valid shape for a label space, every
candidate it timed gave the built-in shape's result (the tuner raises otherwise), and batch
tuning shares one shape per tile."""
import numpy as np
import pytest
import torch

import paper_1410_7922_amd as edp
from paper_1410_7922_amd import autotune as AT
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def test_tune_and_batch_merge():
    print("[gpu] autotune", flush=True)
    probs = [synth.stereo_problem(seed=s, W=96, H=64, Q=q) for s, q in ((1, 24), (2, 20), (3, 40))]
    probs.append(synth.motion_problem(seed=4, W=64, H=48, r=4))
    costs = [torch.from_numpy(p.cost).to(DEV) for p in probs]
    params = [dict(qx=p.qx, qy=p.qy, lam=p.lam, trunc=p.trunc, mode=p.mode, iterations=1,
                   cost_bound=50 if p.cost.dtype == np.int16 else 2500) for p in probs]
    shape = AT.tune(costs[0], params[0], reps=1)
    assert shape["tile"] in edp.tiles(24) and shape["ms"] > 0
    tun = AT.tune_batch(costs, params, AT.TuneCache(None), reps=1)
    by_tile = {}
    for t in tun:
        by_tile.setdefault(t["tile"], set()).add(tuple(t.values()))
    assert all(len(v) == 1 for v in by_tile.values())
    plan = edp.BatchPlan(costs, params, tun)
    lab, en = plan.solve()
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        l1, e1 = edp.solve(costs[i], p.qx, p.qy, p.lam, p.trunc, p.mode, 1, cost_bound=params[i]["cost_bound"])
        torch.cuda.synchronize()
        assert torch.equal(l1, lab[i]) and int(e1.item()) == int(en[i].item())
    plan.close()


def test_tune_three_label_dimensions_and_squared_prior():
    """The tuner times the problem it is given: three label dimensions (its tiles, the wide one
    included) and the squared prior; the tuned batch returns the oracle's labels and energies."""
    from oracle import cref
    print("[gpu] autotune 3D and squared prior", flush=True)
    p3 = synth.random_problem(61, 20, 14, 7, 7, 40, 3, 0, 0, 2500, np.int32, qz=7)
    psq = synth.random_problem(62, 24, 16, 9, 1, 5, 3, 0, 0, 400, np.int32)
    probs = [(p3, dict(qx=7, qy=7, qz=7, lam=40, trunc=3, mode=0, iterations=1, cost_bound=2501)),
             (psq, dict(qx=9, qy=1, lam=5, trunc=3, mode=0, iterations=1, cost_bound=401, prior=edp.PRIOR_SQUARED))]
    costs = [torch.from_numpy(np.ascontiguousarray(p.cost)).to(DEV) for p, _ in probs]
    params = [q for _, q in probs]
    shape = AT.tune(costs[0], params[0], reps=1)
    assert shape["tile"] in edp.tiles_3d(7, 7, 7) + edp.wide_tiles_3d(7, 7, 7) and shape["ms"] > 0
    assert AT.key_of(7, 7, torch.int32, 0, 20, 14, 1, 7, 0).endswith(":z7")
    tun = AT.tune_batch(costs, params, AT.TuneCache(None), reps=1)
    assert tun[1]["tile"] in edp.tiles(9)
    plan = edp.BatchPlan(costs, params, tun)
    lab, en = plan.solve()
    plan.check()
    torch.cuda.synchronize()
    for i, (p, q) in enumerate(probs):
        ref = cref.edp(p.cost, q["qx"], q["qy"], q["lam"], q["trunc"], q["mode"], 1, "grms",
                       prior=q.get("prior", 0), qz=q.get("qz", 1))
        assert np.array_equal(lab[i].cpu().numpy(), ref["labels"]), i
        assert int(en[i].item()) == ref["energy"], i
    plan.close()
