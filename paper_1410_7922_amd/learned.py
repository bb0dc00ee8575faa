"""Learned-window EDP: the window network proposes a label window per pixel, the
EDP runs over the windows only (edp_solve_windowed), and the plain EDP remains
the fallback and the judge: an instance whose windowed energy exceeds the plain
energy by more than ``max_gap`` takes the plain EDP's result.

The judge needs the plain energy, so a solve that judges every instance pays the
plain EDP as well ("judge online"); the times are also reported with the judge
taken offline (the plain EDP paid only by instances that fall back), which is
what a deployment that trusts the proposal on instances like those judged would pay.

All steps run in the library's kernels; this module sequences them.
"""
from __future__ import annotations

import os

import numpy as np
import torch

from . import binding as B
from .window import WindowNet

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "window_net_31x31.npz")


class LearnedWindowEDP:
    def __init__(self, net: WindowNet, qx=31, qy=31, lam=15, trunc=3, mode=B.TRUNC_PER_DIM, cmax=2500, win=7,
                 max_gap=0.005, scale=250):
        self.net = net
        self.qx, self.qy, self.lam, self.trunc, self.mode = qx, qy, lam, trunc, mode
        self.cmax, self.win, self.max_gap, self.scale = cmax, win, max_gap, scale
        self.ws_win = B.Workspace()
        self.ws_plain = B.Workspace()

    @classmethod
    def pretrained(cls, device, path: str = DEFAULT_WEIGHTS, **kw):
        return cls(WindowNet.load(path, device), **kw)

    def windows(self, cost):
        return self.net.windows(cost, self.qx, self.qy, self.scale, self.win)

    def solve_windowed(self, cost, centers=None):
        """Window proposal and windowed EDP.  Returns (labels, energy tensor, centres)."""
        if centers is None:
            centers = self.windows(cost)
        lab, e = B.solve_windowed(cost, centers, self.win, self.qx, self.qy, self.lam, self.trunc, self.mode, 1,
                                  cost_bound=self.cmax, ws=self.ws_win)
        return lab, e, centers

    def solve_plain(self, cost):
        return B.solve(cost, self.qx, self.qy, self.lam, self.trunc, self.mode, 1, cost_bound=self.cmax,
                       ws=self.ws_plain)

    def judge(self, e_window: int, e_plain: int) -> float:
        """Relative energy gap of the windowed result over the plain EDP's."""
        return (e_window - e_plain) / max(abs(e_plain), 1)

    def solve_refined(self, cost, refine: int = 0):
        """Windowed solve, then `refine` rounds of re-centring the windows on the labels found and
        solving again.  Returns (labels, energy tensor, centres of the last round)."""
        lab, e, cen = self.solve_windowed(cost)
        for _ in range(refine):
            cen = B.window_recenter(lab, self.qx, self.qy, self.win, torch.empty_like(cen))
            lab, e, _ = self.solve_windowed(cost, cen)
        return lab, e, cen

    def solve(self, cost, e_plain: int | None = None, refine: int = 0):
        """Windowed solve (with refinement rounds), judged against the plain energy (computed here
        when not given); falls back to the plain EDP above max_gap, and when a windowed solve's
        scans gave up waiting (its result is invalid).  Returns a dict."""
        try:
            lab, e, centers = self.solve_refined(cost, refine)
            ew = int(e.item())
        except B.EdpError as err:
            if err.status != B.EDP_E_TIMEOUT:
                raise
            lab2, e2 = self.solve_plain(cost)
            e2 = int(e2.item())
            return {"labels": lab2, "energy": e2, "gap": float("inf"), "fallback": True, "centers": None,
                    "plain_energy": e2}
        lab_p = None
        if e_plain is None:
            lab_p, ep = self.solve_plain(cost)
            e_plain = int(ep.item())
        gap = self.judge(ew, e_plain)
        out = {"labels": lab, "energy": ew, "gap": gap, "fallback": gap > self.max_gap, "centers": centers,
               "plain_energy": e_plain}
        if out["fallback"]:
            if lab_p is None:
                lab_p, _ = self.solve_plain(cost)
            out["labels"], out["energy"] = lab_p, e_plain
        return out


def _timed(fn, reps=1):
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        out = fn()
    stop.record()
    torch.cuda.synchronize()
    return out, start.elapsed_time(stop) / reps


def evaluate(solver: "LearnedWindowEDP", frames, refine: int = 0, reps: int = 1, log=None):
    """Plain against learned-window EDP on motion frame pairs [(i0, i1), ...] (uint8): per instance
    the plain time and energy, the learned stages' times, the energy gap and the fallback.  The
    learned time with the judge online counts the plain EDP on every instance (the judge needs its
    energy; an instance that falls back takes its labels, so nothing is solved twice); with the
    judge offline only on the instances whose gap exceeds max_gap."""
    dev = solver.net.device
    rows = []
    r = (solver.qx - 1) // 2
    for k, (i0, i1) in enumerate(frames):
        cost = B.dsi_motion(torch.from_numpy(i0).to(dev), torch.from_numpy(i1).to(dev), r, solver.cmax)
        (lab_p, e_p), t_plain = _timed(lambda: solver.solve_plain(cost), reps)
        ep = int(e_p.item())
        cen, t_win = _timed(lambda: solver.windows(cost), reps)
        (lab_w, e_w, _), t_solve = _timed(lambda: solver.solve_refined(cost, refine), reps)
        ew = int(e_w.item())
        gap = solver.judge(ew, ep)
        fb = gap > solver.max_gap
        rows.append({"plain_ms": t_plain, "proposal_ms": t_win, "windowed_ms": t_solve,
                     "learned_ms_judge_online": t_win + t_solve + t_plain,
                     "learned_ms_judge_offline": t_win + t_solve + (t_plain if fb else 0.0), "gap": gap, "fallback": fb,
                     "plain_energy": ep, "windowed_energy": ew,
                     "hit_rate": window_hit_rate(cen, lab_p, solver.qx, solver.win)})
        if log:
            log(f"instance {k}: plain {t_plain:.2f} ms, proposal {t_win:.2f} ms, windowed x{refine + 1} "
                f"{t_solve:.2f} ms, gap {gap * 100:.3f}%{' (fallback)' if fb else ''}")
        del cost
    return rows


def summarize(rows, H, W, Q):
    pl = H * W * Q
    plain = float(np.mean([r["plain_ms"] for r in rows]))
    online = float(np.mean([r["learned_ms_judge_online"] for r in rows]))
    offline = float(np.mean([r["learned_ms_judge_offline"] for r in rows]))
    raw = float(np.mean([r["proposal_ms"] + r["windowed_ms"] for r in rows]))
    gaps = np.array([r["gap"] for r in rows])
    return {"instances": len(rows), "plain_ms": plain, "learned_ms_judge_online": online,
            "learned_ms_judge_offline": offline, "learned_ms_without_fallback": raw,
            "proposal_ms": float(np.mean([r["proposal_ms"] for r in rows])),
            "windowed_ms": float(np.mean([r["windowed_ms"] for r in rows])),
            "plain_pixel_labels_per_s": pl / (plain / 1e3),
            "learned_pixel_labels_per_s_judge_online": pl / (online / 1e3),
            "learned_pixel_labels_per_s_judge_offline": pl / (offline / 1e3),
            "raw_windowed_pixel_labels_per_s": pl / (raw / 1e3),
            "speedup_at_gap_bound_judge_online": plain / online,
            "speedup_at_gap_bound_judge_offline": plain / offline, "raw_speedup": plain / raw,
            "gap_mean": float(gaps.mean()), "gap_median": float(np.median(gaps)), "gap_max": float(gaps.max()),
            "fraction_within_gap": float(np.mean([not r["fallback"] for r in rows])),
            "window_hit_rate": float(np.mean([r["hit_rate"] for r in rows]))}


def window_hit_rate(centers: torch.Tensor, labels: torch.Tensor, qx: int, win: int) -> float:
    """Fraction of pixels whose label lies inside their window."""
    r = win // 2
    lx, ly = labels % qx, labels // qx
    inside = ((lx - centers[..., 0]).abs() <= r) & ((ly - centers[..., 1]).abs() <= r)
    return float(inside.float().mean().item())
