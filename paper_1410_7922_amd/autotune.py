"""Launch-shape autotuner for the EDP solver (tile, split, waves, chunk, fuse).

The library's results never depend on the launch shape; only its speed does.
For a label space (qx, qy, qz), a prior, a cost dtype and a grid size, the tuner
times candidate shapes of ``edp_solve`` on the caller's own cost volume and keeps
the fastest, checking that every candidate returns the same labels and energy as
the built-in shape.  Choices are cached in a JSON file keyed by
``qx x qy : dtype : mode : W x H : iterations``, with ``:z<qz>`` for three label
dimensions and ``:p<prior>`` for the squared prior appended.

Search (staged, so a key costs a few dozen solves):
  1. every single-wavefront tile that holds the label space with at most 4x padding, each
     split the tile allows, with 4 wavefronts per workgroup; and every wide tile (a vertex on
     several wavefronts; two or three label dimensions with a window search) with its
     built-in scanlines per workgroup;
  2. the best (tile, split) with 1, 2, 4 and 6 wavefronts (wide tiles: 1 up to 8 scanlines
     per workgroup, as many as the tile takes), one or two scans per launch;
  3. the best so far with progress published every 1, 2, 4, 8 or 16 columns (single-wavefront
     tiles).
"""
from __future__ import annotations

import json
import os

import torch

from . import binding as B

SHAPE_KEYS = ("tile", "split", "waves", "chunk", "fuse")


def key_of(qx, qy, dtype, mode, W, H, iterations=1, qz=1, prior=0) -> str:
    d = "i16" if dtype in (torch.int16, "i16", 1) else "i32"
    k = f"{qx}x{qy}:{d}:{mode}:{W}x{H}:{iterations}"
    if qz > 1:
        k += f":z{qz}"
    if prior:
        k += f":p{prior}"
    return k


class TuneCache:
    """JSON file of tuned launch shapes (read at start, written after each new key)."""

    def __init__(self, path: str | None = None):
        self.path = path
        self.table = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.table = json.load(f)

    def get(self, key):
        return self.table.get(key)

    def put(self, key, shape):
        self.table[key] = shape
        if self.path:
            os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.table, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def _time_solve(cost, p, shape, reps, ws, labels, energy):
    status = torch.empty(1, dtype=torch.int32, device=cost.device)
    kw = dict(mode=p["mode"], iterations=p.get("iterations", 1), cost_bound=p["cost_bound"], ws=ws,
              labels=labels, energy=energy, status=status, qz=p["qz"], prior=p["prior"],
              **{k: shape[k] for k in SHAPE_KEYS})
    B.solve(cost, p["qx"], p["qy"], p["lam"], p["trunc"], **kw)      # warm-up (waits, checks the status)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        B.solve(cost, p["qx"], p["qy"], p["lam"], p["trunc"], check=False, **kw)
    stop.record()
    torch.cuda.synchronize()
    B.check_status(status, "edp_solve")
    return start.elapsed_time(stop) / reps


def tune(cost: torch.Tensor, params: dict, reps: int = 3, verbose=False) -> dict:
    """Fastest launch shape for one instance (cost on the GPU, params as for BatchPlan)."""
    qx, qy = params["qx"], params.get("qy", 1)
    qz = max(params.get("qz", 1), 1)
    p = dict(params, qy=qy, qz=qz, mode=params.get("mode", B.TRUNC_PER_DIM), prior=params.get("prior", B.PRIOR_LINEAR))
    ws = B.Workspace()
    H, W = cost.shape[:2]
    labels = torch.empty((H, W), dtype=torch.int32, device=cost.device)
    energy = torch.empty(1, dtype=torch.int64, device=cost.device)
    ref_l, ref_e = B.solve(cost, qx, qy, p["lam"], p["trunc"], p["mode"], p.get("iterations", 1),
                           cost_bound=p["cost_bound"], qz=qz, prior=p["prior"])
    torch.cuda.synchronize()
    seen = {}

    def trial(shape):
        k = tuple(shape[x] for x in SHAPE_KEYS)
        if k in seen:
            return seen[k]
        try:
            ms = _time_solve(cost, p, shape, reps, ws, labels, energy)
        except B.EdpError:
            seen[k] = None
            return None
        if not (torch.equal(labels, ref_l) and torch.equal(energy, ref_e)):
            raise RuntimeError(f"launch shape {shape} changed the result")
        seen[k] = ms
        if verbose:
            print(f"[tune] {key_of(qx, qy, cost.dtype, p['mode'], W, H, 1, qz, p['prior'])} {shape} {ms:.3f} ms",
                  flush=True)
        return ms

    q = qx * qy * qz
    if qz > 1:
        tiles = B.tiles_3d(qx, qy, qz)
        wide = B.wide_tiles_3d(qx, qy, qz) if p["trunc"] <= 3 else []
    else:
        tiles = B.tiles(qx, qy)
        wide = B.wide_tiles(qx, qy) if qy > 1 and p["trunc"] <= 3 else []
    qts = {t: _qt(t) for t in tiles + wide}
    small = min(qts.values())
    tiles = [t for t in tiles if qts[t] <= max(4 * q, small)]
    wide = [t for t in wide if qts[t] <= max(4 * q, small)]
    best, best_ms = None, float("inf")

    def consider(shape):
        nonlocal best, best_ms
        ms = trial(shape)
        if ms is not None and ms < best_ms:
            best, best_ms = dict(shape), ms

    for t in tiles:
        px, kx, py, ky = B.tile_info(t)
        for split in (1, 2) if 2 * px * py <= 64 else (1,):
            consider(dict(tile=t, split=split, waves=4, chunk=4, fuse=2))
    for t in wide:
        consider(dict(tile=t, split=1, waves=0, chunk=0, fuse=2))
    if best is None:
        # no shape ran (the built-in shape is the only one for this problem)
        return dict(tile=-1, split=0, waves=0, chunk=0, fuse=0, ms=None)
    base = dict(best)
    if base["tile"] in wide:
        # scanlines per workgroup: the library refuses more than the tile's wavefronts allow
        for waves in range(1, 9):
            for fuse in (1, 2):
                consider(dict(base, waves=waves, fuse=fuse))
        return dict(best, ms=best_ms)
    for waves in (1, 2, 4, 6):
        for fuse in (1, 2):
            consider(dict(base, waves=waves, fuse=fuse))
    base = dict(best)
    for chunk in (1, 2, 4, 8, 16):
        consider(dict(base, chunk=chunk))
    return dict(best, ms=best_ms)


def _qt(tile):
    px, kx, py, ky = B.tile_info(tile)
    return px * kx * py * ky * B.tile_depth(tile)


def tune_batch(costs, params, cache: TuneCache | None = None, reps: int = 3, verbose=False,
               merge: bool = True) -> list:
    """Launch shape for every instance of a batch.  Instances sharing a label space, dtype, mode
    and iteration count are tuned once, on the largest of them (cached per instance key).  With
    merge, instances that chose the same tile share one shape (that of the tile's largest
    instance), so the batch keeps one launch class per tile instead of one per tuned key."""
    cache = cache or TuneCache(None)
    keys, groups = [], {}
    for i, (c, p) in enumerate(zip(costs, params)):
        H, W = c.shape[:2]
        qz, prior = max(p.get("qz", 1), 1), p.get("prior", 0)
        keys.append(key_of(p["qx"], p.get("qy", 1), c.dtype, p.get("mode", 0), W, H, p.get("iterations", 1), qz, prior))
        gk = (p["qx"], p.get("qy", 1), qz, prior, str(c.dtype), p.get("mode", 0), p.get("iterations", 1))
        groups.setdefault(gk, []).append(i)
    shapes = [None] * len(costs)
    for members in groups.values():
        if all(cache.get(keys[i]) is not None for i in members):
            for i in members:
                shapes[i] = cache.get(keys[i])
            continue
        big = max(members, key=lambda i: costs[i].numel())
        shape = tune(costs[big], params[big], reps, verbose)
        for i in members:
            cache.put(keys[i], shape)
            shapes[i] = shape
    if merge:
        by_tile = {}
        for i, sh in enumerate(shapes):
            by_tile.setdefault(sh["tile"], []).append(i)
        for members in by_tile.values():
            big = max(members, key=lambda i: costs[i].numel())
            for i in members:
                shapes[i] = shapes[big]
    return [{x: sh[x] for x in SHAPE_KEYS} for sh in shapes]
