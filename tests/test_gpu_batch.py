"""GPU parity of the batched persistent solve (edp_batch_plan_create / edp_batch_solve):
every instance bit-exact against the CPU oracle or against the single-instance solve, eagerly
and replayed from a captured hipGraph."""
import hashlib
import json
import os

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


def params_of(p, iterations=1, cost_bound=0):
    return dict(qx=p.qx, qy=p.qy, lam=p.lam, trunc=p.trunc, mode=p.mode, iterations=iterations,
                cost_bound=cost_bound or int(np.abs(p.cost).max()) + 1)


def small_mix():
    """Uneven instances over several launch classes: dtypes, label spaces, modes, iterations and
    explicit launch shapes, some sharing a class."""
    P = [
        (synth.stereo_problem(seed=1, W=64, H=40, Q=16), 1, None),
        (synth.stereo_problem(seed=2, W=96, H=72, Q=32), 1, None),
        (synth.stereo_problem(seed=3, W=40, H=100, Q=32), 1, None),
        (synth.random_problem(4, 33, 21, 9, 9, 7, 3, 0, 0, 900), 1, None),
        (synth.random_problem(5, 17, 29, 7, 5, 5, 2, 1, -20, 60), 2, None),
        (synth.random_problem(6, 50, 9, 32, 1, 11, 4, 0, 0, 50, np.int16), 1, dict(waves=2, fuse=1)),
        (synth.random_problem(7, 23, 45, 32, 1, 11, 4, 0, 0, 50, np.int16), 1, dict(waves=2, fuse=1)),
        (synth.random_problem(8, 1, 7, 5, 1, 3, 1, 0, 0, 9), 1, None),
        (synth.random_problem(9, 9, 1, 5, 1, 3, 1, 0, 0, 9), 1, None),
        (synth.random_problem(10, 31, 17, 20, 1, 9, 2, 0, 0, 70, np.int16), 3, dict(split=2, waves=3)),
    ]
    return P


def test_batch_small_mix_vs_oracle():
    mix = small_mix()
    costs = [torch.from_numpy(p.cost).to(DEV) for p, _, _ in mix]
    params = [params_of(p, j) for p, j, _ in mix]
    plan = edp.BatchPlan(costs, params, [t for _, _, t in mix])
    classes, launches = plan.info()
    note(f"batch small mix: {len(mix)} instances, {classes} classes, {launches} launches")
    assert classes >= 4
    labels, energies = plan.solve()
    torch.cuda.synchronize()
    for i, (p, j, _) in enumerate(mix):
        ref = cref.edp(p.cost, p.qx, p.qy, p.lam, p.trunc, p.mode, j, "lrms")
        assert np.array_equal(labels[i].cpu().numpy(), ref["labels"]), i
        assert int(energies[i].item()) == ref["energy"], i
    plan.close()


def test_batch_graph_replays_match_eager():
    mix = small_mix()
    costs = [torch.from_numpy(p.cost).to(DEV) for p, _, _ in mix]
    params = [params_of(p, j) for p, j, _ in mix]
    refs = [cref.edp(p.cost, p.qx, p.qy, p.lam, p.trunc, p.mode, j, "lrms") for p, j, _ in mix]
    plan = edp.BatchPlan(costs, params, [t for _, _, t in mix])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.solve()                       # warm up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.solve()
    x = torch.randn(512, 512, device=DEV)
    for r in range(3):
        note(f"batch graph replay {r}")
        for lab in plan.labels:
            lab.fill_(-1)
        plan.energies.fill_(0)
        x = torch.tanh(x @ x.T / 512.0)     # unrelated eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(mix)):
            assert np.array_equal(plan.labels[i].cpu().numpy(), refs[i]["labels"]), (r, i)
            assert int(plan.energies[i].item()) == refs[i]["energy"], (r, i)
    del g
    plan.close()


def test_batch_workload_64_instances():
    """Every instance of the 64-instance batch against the C oracle's energy and label hash
    (tests/golden/edp_batch64.json, written by tests/golden/make_batch64.py from oracle/ and synth/
    only), and against the single-instance solve."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "edp_batch64.json")) as f:
        golden = json.load(f)["instances"]
    probs = synth.batch_problems(64)
    assert len(golden) == len(probs)
    costs = [torch.from_numpy(p.cost).to(DEV) for p in probs]
    bounds = [50 if p.cost.dtype == np.int16 else 2500 for p in probs]
    params = [params_of(p, 1, b) for p, b in zip(probs, bounds)]
    plan = edp.BatchPlan(costs, params)
    classes, launches = plan.info()
    note(f"batch workload: 64 instances, {classes} classes, {launches} launches")
    labels, energies = plan.solve()
    torch.cuda.synchronize()
    plan.check()
    for i, p in enumerate(probs):
        g = golden[i]
        assert g["cost_sha256"] == p.sha256(), f"instance {i}: the generator's cost volume changed"
        lab = np.ascontiguousarray(labels[i].cpu().numpy(), np.int32)
        assert hashlib.sha256(lab.tobytes()).hexdigest() == g["labels_sha256"], f"instance {i} ({p.name}) labels"
        assert int(energies[i].item()) == g["energy"], f"instance {i} ({p.name}) energy"
    ws = edp.Workspace()
    for i, p in enumerate(probs):
        lab, e = edp.solve(costs[i], p.qx, p.qy, p.lam, p.trunc, p.mode, 1, cost_bound=bounds[i], ws=ws)
        assert torch.equal(lab, labels[i]), i
        assert int(e.item()) == int(energies[i].item()), i
    plan.close()


@pytest.mark.parametrize("fuse", [2, 1])
def test_wide_tiles_repeated_batch_solves(fuse):
    """The motion instances of up to 16 x 16 labels of the 64-instance workload on the two-wavefront
    wide tile with one scanline per workgroup (every scanline a workgroup band: workgroups move
    between instances and bands all the time), solved five times in one plan: every solve equals
    the C oracle's golden.  The first band of a scan takes zeros from its ring; the ring must not
    show the workgroup's previous band to either wavefront of the vertex."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "edp_batch64.json")) as f:
        golden = json.load(f)["instances"]
    probs = synth.batch_problems(64)
    idx = [i for i in range(64) if i % 2 == 1 and probs[i].qx <= 16]
    costs = [torch.from_numpy(probs[i].cost).to(DEV) for i in idx]
    params = [params_of(probs[i], 1, 2500) for i in idx]
    plan = edp.BatchPlan(costs, params, [dict(tile=18, waves=1, fuse=fuse)] * len(idx))
    note(f"wide tile 18, one scanline per workgroup, fuse {fuse}: {len(idx)} instances x 5 solves")
    for rep in range(5):
        labels, energies = plan.solve()
        torch.cuda.synchronize()
        plan.check()
        for j, i in enumerate(idx):
            lab = np.ascontiguousarray(labels[j].cpu().numpy(), np.int32)
            assert hashlib.sha256(lab.tobytes()).hexdigest() == golden[i]["labels_sha256"], (rep, i)
            assert int(energies[j].item()) == golden[i]["energy"], (rep, i)
    plan.close()
