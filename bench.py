#!/usr/bin/env python
"""Benchmark of the MI355X EDP / scanline-DP library; prints one JSON line.

Step = one plain EDP solve (Algorithm 1 with j = 1: the four scans, the
marginal and argmin, the 4-connected energy) of the motion workload 640 x 480
with 31 x 31 = 961 labels (int32 truncated squared-difference costs, lambda
15, T 3, per-dimension truncation), with the cost volume resident in HBM.
value = pixel-labels / s = W * H * Q / step.  The learned-window EDP on the
same kind of instances is reported beside it (extra.learned_window_640x480).

roofline: the dominant kernel (the EDP scan) timed live with HIP events
recorded by the library around every scan launch on the benchmark's stream;
algorithmic bytes per scan: the cost volume, the two sums of the other
directions it reads and the sums it writes that later scans read.
cpu_baseline: the C oracle (one thread) on a band of rows of the same volume.

Only one GPU is used: --gpus N with N > 1 exits with an error message.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class HipEvents:
    """hipEvent_t handles from the HIP runtime already loaded by torch."""

    def __init__(self, n):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.arr = (ctypes.c_void_p * n)()
        for i in range(n):
            h = ctypes.c_void_p()
            if self.hip.hipEventCreate(ctypes.byref(h)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.arr[i] = h
        self.n = n

    def ms(self, a, b):
        out = ctypes.c_float()
        if self.hip.hipEventElapsedTime(ctypes.byref(out), self.arr[a], self.arr[b]) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(out.value)

    def view(self, first, count):
        return (ctypes.c_void_p * count).from_buffer(self.arr, first * ctypes.sizeof(ctypes.c_void_p))

    def close(self):
        for i in range(self.n):
            self.hip.hipEventDestroy(self.arr[i])


def scan_bytes_per_pl(csize, iteration_first=False):
    """Algorithmic bytes per pixel-label of the four scans of one EDP iteration (T-form), per scan.

    Every scan reads C and the two sums of the other directions (in the first iteration three of
    those eight reads are of arrays that still hold zeros and are skipped: P1 both, P2 T-y).  Sums
    written that a later step reads: P1 T+x (its T+y is consumed inside the scan), P2 T-x and T+y,
    P3 T+x (its T-y likewise), P4 T-x and T-y.  The default counts all eight reads, 4 C + 56 B
    per pixel-label over the four scans (72 B with int32 costs); iteration_first gives the bytes
    the first iteration moves.
    """
    reads = [0, 1, 2, 2] if iteration_first else [2, 2, 2, 2]
    writes = [1, 2, 1, 2]
    return [csize + 4 * r + 4 * w for r, w in zip(reads, writes)]


def solve_bytes_per_pl(csize):
    """Algorithmic bytes per pixel-label of one solve with j = 1: the four scans (all eight
    old-sum reads counted) and the marginal (C and the four sums)."""
    return sum(scan_bytes_per_pl(csize)) + csize + 16


def kernel_source_hash(names):
    """Hash of the kernel sources' code: comments and whitespace do not count, so a comment
    edit keeps the recorded counters valid while any change to the code does not."""
    import re
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1410_7922_amd", "csrc", n)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel_key, src_hash):
    path = os.path.join(PROFILES, f"{kernel_key}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != src_hash:
        return None            # the kernel changed since the counters were taken
    return rec.get("bytes_per_launch")


def bench_edp(edp, torch, prob, steps, warmup, tile, chunk, iterations=1, fuse=0):
    dev = torch.device("cuda:0")
    cost = torch.from_numpy(prob.cost).to(dev)
    bound = int(abs(prob.cost).max()) + 1
    ws = edp.Workspace()
    H, W, Q = prob.cost.shape
    labels = torch.empty((H, W), dtype=torch.int32, device=dev)
    energy = torch.empty(1, dtype=torch.int64, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    nlaunch = (4 if fuse == 1 else 2) * iterations     # scan launches per solve
    ev = HipEvents(2 * nlaunch * steps)
    kw = dict(mode=prob.mode, iterations=iterations, cost_bound=bound, tile=tile, chunk=chunk, ws=ws,
              labels=labels, energy=energy, fuse=fuse, prior=prob.prior, status=status, check=False, qz=prob.qz)
    for _ in range(warmup):
        edp.solve(cost, prob.qx, prob.qy, prob.lam, prob.trunc, **kw)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for k in range(steps):
        edp.solve(cost, prob.qx, prob.qy, prob.lam, prob.trunc, events=ev.view(2 * nlaunch * k, 2 * nlaunch), **kw)
    stop.record()
    torch.cuda.synchronize()
    edp.check_status(status, "edp_solve")
    total_ms = start.elapsed_time(stop)
    launch_ms = [[ev.ms(2 * nlaunch * k + 2 * p, 2 * nlaunch * k + 2 * p + 1) for p in range(nlaunch)]
                 for k in range(steps)]
    ev.close()
    return {"ms_per_step": total_ms / steps, "launch_ms": launch_ms, "labels": labels.cpu().numpy(),
            "energy": int(energy.item()), "cost": cost}


# the sources each scan kernel is built from: its recorded counters stay valid while these are unchanged
SCAN_SOURCES = {"edp_pass_kernel": ["edp_pass_kernel.hpp", "edp_device.hpp"],
                "edp_pass_mv_kernel": ["edp_pass_kernel.hpp", "edp_device.hpp", "edp_pass_mv.hpp"]}


def scan_roofline(prob, r, traffic_key=None, kernel="edp_pass_kernel", note=""):
    """Roofline of the EDP scan kernel: algorithmic bytes of the scans of one solve (all eight old-sum
    reads counted) over the summed duration of the scan launches, timed by HIP events on the
    benchmark's stream; traffic: HBM bytes per launch from the recorded rocprofv3 counters, while
    the kernel's source is unchanged since they were taken.  With the wide tiles the last scan also
    forms the marginal and the labels; the marginal's bytes are not counted here."""
    import numpy as np
    H, W, Q = prob.cost.shape
    pl = H * W * Q
    csize = prob.cost.dtype.itemsize
    per_scan = scan_bytes_per_pl(csize)
    launch_ms = np.array(r["launch_ms"]).mean(axis=0)          # [scan launches]
    alg_bytes = float(sum(per_scan) * pl)
    achieved = alg_bytes / (launch_ms.sum() / 1e3) / 1e9
    src_hash = kernel_source_hash(SCAN_SOURCES[kernel])
    traffic = measured_traffic(traffic_key, src_hash) if traffic_key else None
    return {"bound": "hbm", "kernel": f"{kernel}{note} ({len(launch_ms)} scan launches per solve)",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic, "alg_bytes_per_pl_scans": sum(per_scan),
            "alg_bytes_per_launch": alg_bytes / len(launch_ms), "mean_launch_ms": launch_ms.tolist(),
            "source_hash": src_hash}


BATCH_TUNING = os.path.join(ROOT, "paper_1410_7922_amd", "tuned", "batch64_gfx950.json")


def bench_batch(edp, torch, steps, warmup):
    """The 64-instance uneven stereo / motion batch, one plan, solves replayed from a hipGraph, with
    the built-in launch shapes and with the autotuned ones (read from the committed tuning cache;
    keys missing from it are tuned here)."""
    import numpy as np
    import synth
    from paper_1410_7922_amd import autotune
    t0 = time.perf_counter()
    probs = synth.batch_problems(64)
    log(f"batch inputs generated in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    costs = [torch.from_numpy(p.cost).to(dev) for p in probs]
    params = [dict(qx=p.qx, qy=p.qy, lam=p.lam, trunc=p.trunc, mode=p.mode, iterations=1,
                   cost_bound=50 if p.cost.dtype == np.int16 else 2500) for p in probs]
    pl = sum(p.pixel_labels for p in probs)
    cache = autotune.TuneCache(BATCH_TUNING if os.path.exists(BATCH_TUNING) else None)
    t1 = time.perf_counter()
    tuned = autotune.tune_batch(costs, params, cache)
    tune_s = time.perf_counter() - t1

    def run(tunings):
        plan = edp.BatchPlan(costs, params, tunings)
        classes, launches = plan.info()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(max(1, warmup)):
                plan.solve()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(steps):
            plan.solve()
        stop.record()
        torch.cuda.synchronize()
        eager_ms = start.elapsed_time(stop) / steps
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            plan.solve()
        g.replay()
        torch.cuda.synchronize()
        start.record()
        for _ in range(steps):
            g.replay()
        stop.record()
        torch.cuda.synchronize()
        graph_ms = start.elapsed_time(stop) / steps
        energies = plan.energies.cpu().tolist()
        del g
        plan.close()
        return {"classes": classes, "launches_per_solve": launches, "graph_ms_per_solve": graph_ms,
                "eager_ms_per_solve": eager_ms, "pixel_labels_per_s": pl / (graph_ms / 1e3),
                "energy_sum": int(sum(energies))}

    def sequential():
        """The same 64 instances as 64 consecutive edp_solve calls on one stream (built-in shapes)."""
        ws = edp.Workspace()
        outs = [(torch.empty(c.shape[:2], dtype=torch.int32, device=dev), torch.empty(1, dtype=torch.int64, device=dev))
                for c in costs]
        status = torch.empty(1, dtype=torch.int32, device=dev)

        def once():
            for c, pr, (lab, en) in zip(costs, params, outs):
                edp.solve(c, pr["qx"], pr["qy"], pr["lam"], pr["trunc"], pr["mode"], 1, cost_bound=pr["cost_bound"],
                          ws=ws, labels=lab, energy=en, status=status, check=False)
        once()
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(steps):
            once()
        stop.record()
        torch.cuda.synchronize()
        edp.check_status(status, "edp_solve")
        ms = start.elapsed_time(stop) / steps
        return {"ms_per_solve_of_all": ms, "pixel_labels_per_s": pl / (ms / 1e3),
                "energy_sum": int(sum(int(en.item()) for _, en in outs))}

    seq = sequential()
    default = run(None)
    tuned_r = run(tuned)
    assert seq["energy_sum"] == default["energy_sum"]
    assert tuned_r["energy_sum"] == default["energy_sum"]        # launch shapes never change results
    best = tuned_r if tuned_r["graph_ms_per_solve"] < default["graph_ms_per_solve"] else default

    def best_ms(*rs):
        return min(x["graph_ms_per_solve"] for x in rs)
    return {"workload": "64 instances: stereo 160x120..640x480 Q 16-64 int16, motion 9x9..21x21 labels int32",
            "pixel_labels": pl, "sequential_solves": seq, "built_in_shapes": default, "autotuned_shapes": tuned_r,
            "speedup_over_sequential": seq["ms_per_solve_of_all"] / best_ms(default, tuned_r),
            "alg_bytes": sum(solve_bytes_per_pl(c.element_size()) * c.numel() for c in costs),
            "autotune_seconds": tune_s, "pixel_labels_per_s": best["pixel_labels_per_s"],
            "graph_ms_per_solve": best["graph_ms_per_solve"],
            "hbm_frac_alg": sum(solve_bytes_per_pl(c.element_size()) * c.numel() for c in costs)
            / (best["graph_ms_per_solve"] / 1e3) / 1e9 / HBM_PEAK_GBS}


def bench_dp_marginals(edp, torch, steps, warmup, rows=8192, cols=1024, q=64, seed=0):
    """The min-marginal scanline DP (labels only) on the DP sweep workload of bench_dp.  Algorithmic
    bytes per pixel-label: forward sweep 2 B cost read + 2 B forward term written, backward sweep
    the same two read; plus a 4 B label per pixel."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    cost = torch.randint(0, 51, (rows, cols, q), generator=g, device=dev, dtype=torch.int16)
    ws = edp.Workspace()
    ev = HipEvents(4 * steps)
    for _ in range(warmup):
        edp.dp_marginals(cost, q, 1, 20, 2, cost_bound=51, ws=ws)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for k in range(steps):
        edp.dp_marginals(cost, q, 1, 20, 2, cost_bound=51, ws=ws, events=ev.view(4 * k, 4))
    stop.record()
    torch.cuda.synchronize()
    total = start.elapsed_time(stop) / steps
    fwd = sum(ev.ms(4 * k, 4 * k + 1) for k in range(steps)) / steps
    bwd = sum(ev.ms(4 * k + 2, 4 * k + 3) for k in range(steps)) / steps
    ev.close()
    pl = rows * cols * q
    fwd_bytes, bwd_bytes = pl * 4, pl * 4 + rows * cols * 4
    return {"workload": f"dp_marginals{cols}x{rows}q{q}_i16", "pixel_labels_per_s": pl / (total / 1e3),
            "ms_per_step": total, "forward_ms": fwd, "backward_ms": bwd,
            "forward_GBps": fwd_bytes / (fwd / 1e3) / 1e9, "backward_GBps": bwd_bytes / (bwd / 1e3) / 1e9,
            "backward_frac_of_hbm": bwd_bytes / (bwd / 1e3) / 1e9 / HBM_PEAK_GBS}


def bench_dsi(edp, torch, steps, warmup):
    """Data cost formation (edp_dsi): the 961-label motion volume of the learned-window workload
    (640x480, int32, 1.18 GB written) and a three-view stereo volume of the paper's setup-2 shape
    (450x375, 60 disparities, composite cost, int32).  Algorithmic bytes: the volume written
    (the images are read from cache)."""
    import synth
    dev = torch.device("cuda:0")
    i0, i1, _, _ = synth.motion_frames(0, 640, 480, 15)
    rng = __import__("numpy").random.default_rng(7)
    j0, j1, j2 = (torch.from_numpy(rng.integers(0, 256, (375, 450), dtype="uint8")).to(dev) for _ in range(3))
    a0, a1 = torch.from_numpy(i0).to(dev), torch.from_numpy(i1).to(dev)
    runs = {"motion640x480_q961_i32": (lambda o: edp.dsi(a0, a1, 31, 31, -15, -15, 1, 1, 2, 2500, out=o),
                                       (480, 640, 961)),
            "stereo3view450x375_q60_i32": (lambda o: edp.dsi(j0, j1, 60, 1, 0, 0, -1, 1, 2, 10000, i2=j2, out=o),
                                           (375, 450, 60))}
    out = {}
    for name, (fn, shape) in runs.items():
        o = torch.empty(shape, dtype=torch.int32, device=dev)
        for _ in range(warmup):
            fn(o)
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(steps):
            fn(o)
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / steps
        nbytes = o.numel() * 4
        gbps = nbytes / (ms / 1e3) / 1e9
        out[name] = {"ms": ms, "GBps": gbps, "frac_of_hbm": gbps / HBM_PEAK_GBS}
        del o
    return out


def bench_dp(edp, torch, steps, warmup, rows=8192, cols=1024, q=64, seed=0, prior=0):
    """Scanline DP sweep on uniform int16 costs in [0, 50]: 8192 independent scanlines of 1024
    columns and 64 labels (16 stereo frames of 1024 x 512 with 64 disparities), a bandwidth
    workload of 1 GiB of costs.  prior 0: truncated linear, lambda 20, T 2; prior 1: truncated
    squared, lambda 5, T 3."""
    lam, trunc = (20, 2) if prior == 0 else (5, 3)
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    cost = torch.randint(0, 51, (rows, cols, q), generator=g, device=dev, dtype=torch.int16)
    ws = edp.Workspace()
    ev = HipEvents(4 * steps)
    for _ in range(warmup):
        edp.dp_scanline(cost, q, 1, lam, trunc, cost_bound=51, ws=ws, prior=prior)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for k in range(steps):
        edp.dp_scanline(cost, q, 1, lam, trunc, cost_bound=51, ws=ws, events=ev.view(4 * k, 4), prior=prior)
    stop.record()
    torch.cuda.synchronize()
    total = start.elapsed_time(stop) / steps
    fwd = sum(ev.ms(4 * k, 4 * k + 1) for k in range(steps)) / steps
    bt = sum(ev.ms(4 * k + 2, 4 * k + 3) for k in range(steps)) / steps
    ev.close()
    pl = rows * cols * q
    fwd_bytes = pl * (2 + 1)          # int16 cost read + one-byte choice index written
    return {"workload": f"dp_sweep{cols}x{rows}q{q}_i16" + ("_sq" if prior else ""),
            "pixel_labels_per_s": pl / (total / 1e3),
            "ms_per_step": total, "forward_ms": fwd, "backtrack_ms": bt,
            "forward_GBps": fwd_bytes / (fwd / 1e3) / 1e9,
            "forward_frac_of_hbm": fwd_bytes / (fwd / 1e3) / 1e9 / HBM_PEAK_GBS}


def bench_learned(torch, n, refine):
    """Plain against learned-window EDP on n held-out 640 x 480 motion instances, 31 x 31 labels."""
    import synth
    from paper_1410_7922_amd.learned import LearnedWindowEDP, evaluate, summarize
    frames = [synth.motion_frames(seed=s, W=640, H=480, r=15)[:2] for s in range(n)]
    solver = LearnedWindowEDP.pretrained(torch.device("cuda:0"))
    evaluate(solver, frames[:1], refine)                           # warm-up
    rows = evaluate(solver, frames, refine, log=log)
    out = summarize(rows, 480, 640, 961)
    out.update({"workload": "learned-window EDP, motion 640x480, 31x31 labels, int32 costs, window 7x7",
                "refinement_rounds": refine, "gap_bound": solver.max_gap,
                "seeds": f"0..{n - 1} (frames of the motion generator; training used seeds 1000..)"})
    return out


def window_study(torch, n, wins=(7, 11, 15, 21), rounds=3, big=40000):
    """Energy gap of the label-window EDP over the plain EDP for several window sizes on n
    held-out 640 x 480 motion instances (31 x 31 labels), with 0 .. rounds-1 re-centring rounds,
    for two proposals: the trained network's centres, and centres on the plain EDP's own labels
    (the best a proposal aiming at the plain solution can do).  The windowed problem is solved, for
    any window size, as the plain EDP on the cost volume with every label outside the pixel's
    window given cost `big` (the definition the windowed solve implements; big exceeds every
    in-window cost plus four sums' spreads of lambda * 2T), so no window-size-specific kernel is
    needed."""
    import numpy as np
    import synth
    import paper_1410_7922_amd as edp
    from paper_1410_7922_amd import binding as B
    from paper_1410_7922_amd.learned import LearnedWindowEDP
    dev = torch.device("cuda:0")
    solver = LearnedWindowEDP.pretrained(dev)
    Q = 31
    lx = (torch.arange(Q * Q, device=dev) % Q).view(1, 1, -1)
    ly = (torch.arange(Q * Q, device=dev) // Q).view(1, 1, -1)
    ws = edp.Workspace()
    props = ("network", "plain_labels")
    gaps = {(pr, w): [] for pr in props for w in wins}
    hits = {(pr, w): [] for pr in props for w in wins}
    for k in range(n):
        i0, i1 = synth.motion_frames(seed=k, W=640, H=480, r=15)[:2]
        cost = B.dsi_motion(torch.from_numpy(i0).to(dev), torch.from_numpy(i1).to(dev), 15, 2500)
        lp, ep = edp.solve(cost, Q, Q, 15, 3, 0, 1, cost_bound=2500, ws=ws)
        ep = int(ep.item())
        starts = {"network": solver.windows(cost),
                  "plain_labels": torch.stack([lp % Q, lp // Q], -1).to(torch.int32)}
        for pr in props:
            for win in wins:
                r = win // 2
                cen = starts[pr].clone()
                cen[..., 0].clamp_(r, Q - 1 - r)
                cen[..., 1].clamp_(r, Q - 1 - r)
                hit = (((lp % Q) - cen[..., 0]).abs() <= r) & (((lp // Q) - cen[..., 1]).abs() <= r)
                hits[(pr, win)].append(float(hit.float().mean()))
                row = []
                for _ in range(rounds):
                    inside = ((lx - cen[..., 0:1]).abs() <= r) & ((ly - cen[..., 1:2]).abs() <= r)
                    masked = torch.where(inside, cost, torch.full_like(cost, big))
                    lw, ew = edp.solve(masked, Q, Q, 15, 3, 0, 1, cost_bound=big, ws=ws)
                    row.append((int(ew.item()) - ep) / ep)
                    cen = torch.stack([(lw % Q).clamp(r, Q - 1 - r), (lw // Q).clamp(r, Q - 1 - r)],
                                      -1).to(torch.int32)
                    del inside, masked
                gaps[(pr, win)].append(row)
                log(f"window study instance {k} {pr} window {win}: gaps {[round(100 * g, 3) for g in row]} %")
        del cost
        torch.cuda.empty_cache()
    out = {}
    for pr in props:
        out[pr] = {}
        for win in wins:
            g = np.array(gaps[(pr, win)])
            out[pr][f"{win}x{win}"] = {
                "mean_gap_by_round": g.mean(axis=0).tolist(), "max_gap_by_round": g.max(axis=0).tolist(),
                "fraction_within_0.5pct_by_round": (g <= 0.005).mean(axis=0).tolist(),
                "window_hit_rate": float(np.mean(hits[(pr, win)]))}
    return {"workload": "label-window study, motion 640x480, 31x31 labels",
            "instances": n, "rounds": rounds, "outside_cost": big, "proposals": out}


def bench_paper_shapes(edp, torch, steps, warmup):
    """The shapes of the paper's timed setups (Sec. 5.1, Table 2), with synthetic images in place of
    the Middlebury pairs: setup 1, stereo 450x375 with 60 disparities and the truncated linear prior
    g = 5 (linear RMS), and setup 3, motion 320x265 with 15x27 labels, g = 3.  The paper's sequential
    CPU times per EDP iteration are quoted beside them for context (other hardware)."""
    import synth
    out = {}
    for key, prob, paper_s in (
            ("S1_stereo450x375q60_g5", synth.stereo_problem(seed=0, W=450, H=375, Q=60, lam=20, trunc=5), 2.3),
            ("S3_motion320x265q15x27_g3", synth.motion_problem(seed=0, W=320, H=265, r=7, ry=13, lam=15, trunc=3),
             10.8)):
        r = bench_edp(edp, torch, prob, steps, warmup, -1, 0)
        H, W, Q = prob.cost.shape
        out[key] = {"ms_per_step": r["ms_per_step"], "pixel_labels_per_s": W * H * Q / (r["ms_per_step"] / 1e3),
                    "energy": r["energy"], "labels": [prob.qx, prob.qy],
                    "paper_lrms_s_per_iteration_core_duo_3_16ghz": paper_s}
        del r
    return out


def bench_iterations(edp, torch, prob, iters=(1, 2, 4, 8, 16)):
    """Energy and time of the solve for several EDP iteration counts j (the paper's energy-versus-
    iteration experiments, Sec. 5.1)."""
    import numpy as np
    out = []
    for j in iters:
        r = bench_edp(edp, torch, prob, 2, 1, -1, 0, iterations=j)
        out.append({"iterations": j, "energy": r["energy"], "ms_per_solve": r["ms_per_step"]})
        del r
    return out


def cpu_baseline(prob, rows=None, budget_s=10.0):
    """The C oracle (one thread, general RMS minimum search) timed on the first `rows` rows of the
    workload's cost volume (all rows if None), repeated until budget_s has passed."""
    from oracle import cref
    cost = prob.cost if rows is None else prob.cost[:rows]
    H, W, Q = cost.shape
    t0 = time.perf_counter()
    reps, ref = 0, None
    while True:
        ref = cref.edp(cost, prob.qx, prob.qy, prob.lam, prob.trunc, prob.mode, 1, "grms", prior=prob.prior)
        reps += 1
        if time.perf_counter() - t0 >= budget_s or reps >= 30:
            break
    dt = (time.perf_counter() - t0) / reps
    what = "full" if rows is None else f"rows 0..{H - 1} ({W}x{H}x{Q}) of the"
    return {"value": W * H * Q / dt, "unit": "pixel-labels/s", "cores": 1, "kind": "oracle",
            "sample": f"C oracle (general RMS minimum search, single thread) on {what} {prob.name} cost volume, "
                      f"plain EDP j=1, x{reps} ({dt:.2f} s each); {os.cpu_count()} host cores available"}, ref


def bench_r3(edp, torch, steps, warmup):
    """EDP over a three-dimensional label space: the 640 x 480 motion-with-brightness-offset
    workload, 7 x 7 motion labels and 7 offset levels (343 labels, padded to 8 x 8 x 8 on the
    built-in wide tile 25: 8 x 8 lanes, two offset levels per lane on each of four wavefronts),
    lambda 40, T 3 per dimension, j = 1."""
    import numpy as np
    import synth
    prob = synth.workload("motion_offset640x480")
    H, W, Q = prob.cost.shape
    pl = H * W * Q
    r = bench_edp(edp, torch, prob, steps, warmup, -1, 0)
    roof = scan_roofline(prob, r, "edp_pass_motionoffset640x480q343", kernel="edp_pass_mv_kernel",
                         note=", tile 25 (8x8x8 labels over four wavefronts)")
    return {"workload": "plain EDP, motion with a brightness offset 640x480, 7x7x7 labels (dx, dy in [-3, 3], "
                        "7 offset levels of 6 grey levels), int32 truncated squared-difference costs (cmax 2500), "
                        "lambda 40, T 3 per dimension, j=1",
            "data": "synthetic (seeded frame pair with 8 affine-motion segments, per-segment brightness offset)",
            "pixel_labels_per_s": pl / (r["ms_per_step"] / 1e3), "ms_per_step": r["ms_per_step"],
            "energy": r["energy"], "labels": Q, "padded_labels": 512, "roofline": roof,
            "labels_sha256": hashlib.sha256(np.ascontiguousarray(r["labels"], np.int32).tobytes()).hexdigest()}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tile", type=int, default=-1)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--fuse", type=int, default=0, help="EDP scans per launch (1 or 2; 0 = built-in)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-instance batch")
    ap.add_argument("--learned", type=int, default=20, metavar="N",
                    help="held-out instances of the learned-window comparison (0 skips it)")
    ap.add_argument("--refine", type=int, default=0, help="window refinement rounds of the learned path")
    ap.add_argument("--window-study", type=int, default=0, metavar="N",
                    help="only the window-size study of the learned path on N instances")
    ap.add_argument("--r3-only", action="store_true",
                    help="only the EDP solve over three label dimensions (640x480, 7x7x7 labels)")
    ap.add_argument("--dp-only", action="store_true",
                    help="run only the scanline DP sweep (for hardware-counter profiles of its kernels)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the DP sweep and motion workloads")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: the library runs on one GPU (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE {world}); it has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1410_7922_amd as edp
    import synth

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    edp.load()

    if args.calibrate_copy > 0:
        n = args.calibrate_copy << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calibrate_copy} MiB done")
        del src, dst
    if args.window_study:
        r = window_study(torch, args.window_study)
        print(json.dumps({"metric": "energy gap of the label-window EDP over plain EDP", "value": None,
                          "unit": "fraction", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
                          "config": {"workload": r["workload"]}, "window_study": r}), flush=True)
        return
    if args.r3_only:
        r3 = bench_r3(edp, torch, args.steps, args.warmup)
        print(json.dumps({"metric": "pixel-labels/sec (EDP, three label dimensions)", "value": r3["pixel_labels_per_s"],
                          "unit": "pixel-labels/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": r3["ms_per_step"], "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "int32", "data": r3["data"],
                          "config": {"workload": r3["workload"]}, "roofline": r3["roofline"],
                          "r3": r3}), flush=True)
        return
    if args.dp_only:
        r = bench_dp(edp, torch, args.steps, args.warmup)
        print(json.dumps({"metric": "pixel-labels/sec (scanline DP sweep)", "value": r["pixel_labels_per_s"],
                          "unit": "pixel-labels/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "int32 (int16 costs)", "data": "synthetic uniform costs",
                          "config": {"workload": r["workload"]}, "dp_sweep": r}), flush=True)
        return
    prob = synth.workload("motion640x480")
    H, W, Q = prob.cost.shape
    pl = H * W * Q
    log(f"workload {prob.name} ({W}x{H}, {prob.qx}x{prob.qy} labels, int32), {args.warmup} warmup + "
        f"{args.steps} timed steps")
    r = bench_edp(edp, torch, prob, args.steps, args.warmup, args.tile, args.chunk, fuse=args.fuse)
    ms = r["ms_per_step"]
    roof = scan_roofline(prob, r, "edp_pass_motion640x480q961", kernel="edp_pass_mv_kernel")
    log(f"step {ms:.3f} ms, scan launches {[round(x, 4) for x in roof['mean_launch_ms']]} ms")
    golden = os.path.join(ROOT, "tests", "golden", "edp_motion640x480_q961.json")
    with open(golden) as f:
        g = json.load(f)
    lab_sha = hashlib.sha256(np.ascontiguousarray(r["labels"], np.int32).tobytes()).hexdigest()

    out = {
        "metric": "pixel-labels/sec (plain vs learned-window EDP) at <=0.5% energy gap; HBM GB/s",
        "value": pl / (ms / 1e3),
        "unit": "pixel-labels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded frame pair with 8 affine-motion segments, sigma 4)",
        "config": {"workload": "plain EDP motion 640x480, 31x31 labels (dx, dy in [-15, 15]), int32 truncated "
                               "squared-difference costs (cmax 2500), lambda 15, T 3 per dimension, j=1",
                   "width": W, "height": H, "labels": Q, "iterations": 1, "tile": args.tile, "chunk": args.chunk,
                   "fuse": args.fuse},
        "roofline": roof,
        "energy": r["energy"],
        "hbm_GBps_solve": solve_bytes_per_pl(4) * pl / (ms / 1e3) / 1e9,
        "parity_vs_oracle": bool(r["energy"] == g["energy"] and lab_sha == g["labels_sha256"]
                                 and g["cost_sha256"] == prob.sha256()),
    }
    extra = {}
    if not args.no_extra:
        log("stereo 384x288 (32 disparities, int16)")
        sp0 = synth.workload("stereo384x288")
        sr0 = bench_edp(edp, torch, sp0, args.steps, 1, -1, args.chunk, fuse=args.fuse)
        spl0 = sp0.cost.shape[0] * sp0.cost.shape[1] * sp0.cost.shape[2]
        extra["stereo384x288"] = {"pixel_labels_per_s": spl0 / (sr0["ms_per_step"] / 1e3),
                                  "ms_per_step": sr0["ms_per_step"], "energy": sr0["energy"],
                                  "roofline": scan_roofline(sp0, sr0, "edp_pass_stereo384x288")}
        del sr0
        log("motion 320x240 (15x15 labels, int32)")
        mp = synth.workload("motion320x240")
        mr = bench_edp(edp, torch, mp, max(3, args.steps // 4), 1, -1, args.chunk, fuse=args.fuse)
        mpl = mp.cost.shape[0] * mp.cost.shape[1] * mp.cost.shape[2]
        extra["motion320x240"] = {"pixel_labels_per_s": mpl / (mr["ms_per_step"] / 1e3),
                                  "ms_per_step": mr["ms_per_step"], "energy": mr["energy"],
                                  "mean_launch_ms": np.array(mr["launch_ms"]).mean(axis=0).tolist()}
        del mr
        log("scanline DP sweep 8192 rows x 1024 columns, Q=64 int16")
        extra["dp_sweep"] = bench_dp(edp, torch, max(3, args.steps // 4), 1)
        # the truncated squared prior (general RMS, window 2T - 1 = 5 per label)
        for name in ("stereo384x288_sq", "motion320x240_sq"):
            log(f"{name} (truncated squared prior, lambda 5, T 3)")
            sp = synth.workload(name)
            sr = bench_edp(edp, torch, sp, max(3, args.steps // 4), 1, -1, args.chunk, fuse=args.fuse)
            spl = sp.cost.shape[0] * sp.cost.shape[1] * sp.cost.shape[2]
            extra[name] = {"pixel_labels_per_s": spl / (sr["ms_per_step"] / 1e3), "ms_per_step": sr["ms_per_step"],
                           "energy": sr["energy"], "mean_launch_ms": np.array(sr["launch_ms"]).mean(axis=0).tolist()}
            del sr
        extra["dp_sweep_sq"] = bench_dp(edp, torch, max(3, args.steps // 4), 1, prior=1)
        log("data cost formation")
        extra["dsi"] = bench_dsi(edp, torch, max(3, args.steps // 4), 1)
        log("min-marginal scanline DP on the same sweep")
        extra["dp_marginals"] = bench_dp_marginals(edp, torch, max(3, args.steps // 4), 1)
        log("the paper's setup shapes (stereo 450x375x60 g=5, motion 320x265 with 15x27 labels g=3)")
        extra["paper_shapes"] = bench_paper_shapes(edp, torch, max(3, args.steps // 4), 1)
        log("energy against the number of EDP iterations (motion 640x480, 961 labels)")
        extra["energy_vs_iterations"] = bench_iterations(edp, torch, prob)
        log("three label dimensions: motion with a brightness offset 640x480, 7x7x7 labels")
        extra["motion_offset640x480"] = bench_r3(edp, torch, max(3, args.steps // 4), 1)
    if not args.no_batch:
        log("batch of 64 uneven instances (hipGraph replay)")
        extra["batch64"] = bench_batch(edp, torch, max(3, args.steps // 4), 1)
    if args.learned > 0:
        log(f"learned-window EDP against plain EDP on {args.learned} instances 640x480, 31x31 labels")
        extra["learned_window_640x480"] = bench_learned(torch, args.learned, args.refine)
    out["extra"] = extra
    if not args.no_cpu:
        rows = 96
        log(f"CPU oracle baseline (rows 0..{rows - 1} of the volume, about 20 s)")
        cb, _ = cpu_baseline(prob, rows=rows, budget_s=1.0)
        out["cpu_baseline"] = cb
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
