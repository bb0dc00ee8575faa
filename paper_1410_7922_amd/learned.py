"""Learned-window EDP: the window network proposes a label window per pixel, the
EDP runs over the windows only (edp_solve_windowed), and the plain EDP remains
the fallback and the judge: an instance whose windowed energy exceeds the
plain energy by more than ``max_gap`` is solved again by the plain EDP.

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

    def solve(self, cost, e_plain: int | None = None):
        """Windowed solve, judged against the plain energy (computed here when not given);
        falls back to the plain EDP above max_gap.  Returns a dict."""
        lab, e, centers = self.solve_windowed(cost)
        ew = int(e.item())
        if e_plain is None:
            _, ep = self.solve_plain(cost)
            e_plain = int(ep.item())
        gap = self.judge(ew, e_plain)
        out = {"labels": lab, "energy": ew, "gap": gap, "fallback": gap > self.max_gap, "centers": centers,
               "plain_energy": e_plain}
        if out["fallback"]:
            lab2, e2 = self.solve_plain(cost)
            out["labels"], out["energy"] = lab2, int(e2.item())
        return out


def window_hit_rate(centers: torch.Tensor, labels: torch.Tensor, qx: int, win: int) -> float:
    """Fraction of pixels whose label lies inside their window."""
    r = win // 2
    lx, ly = labels % qx, labels // qx
    inside = ((lx - centers[..., 0]).abs() <= r) & ((ly - centers[..., 1]).abs() <= r)
    return float(inside.float().mean().item())
