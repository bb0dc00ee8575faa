"""Python binding of ``libedp.so`` (include/edp.h): argument marshalling only.

Torch provides device memory and the current HIP stream; every step of the
solvers runs in the library's HIP kernels.  There is no CPU fallback: if the
library is missing or no GPU is visible, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libedp.so")

EDP_OK = 0
EDP_E_TIMEOUT = -6    # status word of a solve whose scans gave up waiting (results invalid)
EDP_I16 = 1
EDP_I32 = 2
TRUNC_PER_DIM = 0
TRUNC_JOINT = 1
PRIOR_LINEAR = 0      # f(a) = |a|
PRIOR_SQUARED = 1     # f(a) = a^2
OP_DP = 0
OP_EDP = 1
OP_DP_MARGINALS = 2

EXPORTS = ("edp_workspace_size", "edp_dp_scanline", "edp_solve", "edp_energy", "edp_tiles",
           "edp_tile_info", "edp_status_string", "edp_batch_workspace_size", "edp_batch_plan_create",
           "edp_batch_solve", "edp_batch_plan_info", "edp_batch_plan_destroy", "edp_window_workspace_size",
           "edp_solve_windowed", "edp_dp_marginals", "edp_dsi", "edp_solve_static", "edp_wide_tiles",
           "edp_tiles_3d", "edp_wide_tiles_3d", "edp_tile_depth")


class Problem(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "width", "height", "qx", "qy", "dtype", "trunc_mode", "lam", "trunc", "iterations", "cost_bound", "prior",
        "qz")]


class Tuning(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("chunk", ctypes.c_int32), ("split", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("fuse", ctypes.c_int32), ("events", ctypes.POINTER(ctypes.c_void_p)),
                ("n_events", ctypes.c_int32)]


class BatchItem(ctypes.Structure):
    _fields_ = [("problem", Problem), ("d_cost", ctypes.c_void_p), ("d_labels", ctypes.c_void_p),
                ("d_energy", ctypes.c_void_p), ("d_status", ctypes.c_void_p), ("tuning", Tuning)]


class EdpError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(path)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    pprob, ptun = ctypes.POINTER(Problem), ctypes.POINTER(Tuning)
    L.edp_workspace_size.argtypes = [pprob, ctypes.c_int32, ptun, ctypes.POINTER(sz)]
    L.edp_dp_scanline.argtypes = [pprob, ptun, vp, vp, vp, vp, vp, sz, vp]
    L.edp_solve.argtypes = [pprob, ptun, vp, vp, vp, vp, vp, sz, vp]
    L.edp_solve_static.argtypes = [pprob, ptun, vp, vp, vp, vp, vp]
    L.edp_dp_marginals.argtypes = [pprob, ptun, vp, vp, vp, vp, vp, vp, sz, vp]
    L.edp_dsi.argtypes = [vp, vp, vp] + [ctypes.c_int32] * 11 + [vp, vp]
    L.edp_energy.argtypes = [pprob, vp, vp, ctypes.c_int32, vp, vp, vp]
    L.edp_tiles.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
    L.edp_wide_tiles.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
    L.edp_tile_info.argtypes = [ctypes.c_int32] + [ctypes.POINTER(ctypes.c_int32)] * 4
    L.edp_tiles_3d.argtypes = [ctypes.c_int32] * 3 + [ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
    L.edp_wide_tiles_3d.argtypes = [ctypes.c_int32] * 3 + [ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
    L.edp_tile_depth.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.edp_status_string.argtypes = [ctypes.c_int32]
    L.edp_status_string.restype = ctypes.c_char_p
    pitem = ctypes.POINTER(BatchItem)
    L.edp_batch_workspace_size.argtypes = [ctypes.c_int32, pitem, ctypes.POINTER(sz)]
    L.edp_batch_plan_create.argtypes = [ctypes.c_int32, pitem, vp, sz, vp, ctypes.POINTER(vp)]
    L.edp_batch_solve.argtypes = [vp, vp]
    L.edp_batch_plan_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    L.edp_batch_plan_destroy.argtypes = [vp]
    L.edp_batch_plan_destroy.restype = None
    L.edp_window_workspace_size.argtypes = [pprob, ctypes.c_int32, ptun, ctypes.POINTER(sz)]
    L.edp_solve_windowed.argtypes = [pprob, ptun, vp, vp, ctypes.c_int32, vp, vp, vp, vp, sz, vp]
    for name in ("edp_workspace_size", "edp_dp_scanline", "edp_solve", "edp_energy", "edp_tiles",
                 "edp_tile_info", "edp_batch_workspace_size", "edp_batch_plan_create", "edp_batch_solve",
                 "edp_batch_plan_info", "edp_window_workspace_size", "edp_solve_windowed", "edp_dp_marginals",
                 "edp_dsi", "edp_solve_static", "edp_wide_tiles", "edp_tiles_3d", "edp_wide_tiles_3d",
                 "edp_tile_depth"):
        getattr(L, name).restype = ctypes.c_int32
    _lib = L
    return L


def status_string(status: int) -> str:
    return load().edp_status_string(int(status)).decode()


def _check(status: int, where: str):
    if status != EDP_OK:
        raise EdpError(status, where)


def check_status(status, where: str = "solve"):
    """Raise EdpError if a solve's device status word (a tensor, or its value) is not EDP_OK.
    Reading a device tensor waits for the solve."""
    values = status.flatten().tolist() if isinstance(status, torch.Tensor) else [int(status)]
    for v in values:
        if int(v) != EDP_OK:
            raise EdpError(int(v), where)


def make_problem(cost: torch.Tensor, qx: int, qy: int, lam: int, trunc: int, mode: int = TRUNC_PER_DIM,
                 iterations: int = 1, cost_bound: int = 0, prior: int = PRIOR_LINEAR, qz: int = 1) -> Problem:
    if cost.dim() != 3:
        raise ValueError("cost must be [H][W][Q]")
    if cost.dtype not in (torch.int16, torch.int32):
        raise ValueError("cost must be int16 or int32")
    H, W, Q = cost.shape
    if Q != qx * qy * qz:
        raise ValueError(f"cost has {Q} labels, qx*qy*qz = {qx * qy * qz}")
    return Problem(W, H, qx, qy, EDP_I16 if cost.dtype == torch.int16 else EDP_I32, mode, lam, trunc,
                   iterations, cost_bound, prior, qz)


def _tuning(tile: int, chunk: int, events=None, split: int = 0, waves: int = 0, fuse: int = 0):
    if tile < 0 and chunk <= 0 and split <= 0 and waves <= 0 and fuse <= 0 and events is None:
        return None
    t = Tuning(tile, chunk, split, waves, fuse, None, 0)
    if events is not None:
        t.events = ctypes.cast(events, ctypes.POINTER(ctypes.c_void_p))
        t.n_events = len(events)
    return ctypes.byref(t)


def _device_tensor(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(dev) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def workspace_size(prob: Problem, op: int, tile: int = -1, chunk: int = 0, split: int = 0, waves: int = 0,
                   fuse: int = 0) -> int:
    n = ctypes.c_size_t(0)
    _check(load().edp_workspace_size(ctypes.byref(prob), op, _tuning(tile, chunk, None, split, waves, fuse),
                                     ctypes.byref(n)),
           "edp_workspace_size")
    return int(n.value)


def tiles(qx: int, qy: int = 1) -> list:
    L = load()
    n = L.edp_tiles(qx, qy, None, 0)
    if n < 0:
        raise EdpError(n, "edp_tiles")
    ids = (ctypes.c_int32 * max(n, 1))()
    L.edp_tiles(qx, qy, ids, n)
    return list(ids[:n])


def wide_tiles(qx: int, qy: int) -> list:
    """Wide-vertex tiles (a vertex on several wavefronts) of the EDP scans for a label space."""
    L = load()
    n = L.edp_wide_tiles(qx, qy, None, 0)
    if n < 0:
        raise EdpError(n, "edp_wide_tiles")
    ids = (ctypes.c_int32 * max(n, 1))()
    L.edp_wide_tiles(qx, qy, ids, n)
    return list(ids[:n])


def tiles_3d(qx: int, qy: int, qz: int) -> list:
    """Lane tiles of the EDP scans for a label space with three label dimensions."""
    L = load()
    n = L.edp_tiles_3d(qx, qy, qz, None, 0)
    if n < 0:
        raise EdpError(n, "edp_tiles_3d")
    ids = (ctypes.c_int32 * max(n, 1))()
    L.edp_tiles_3d(qx, qy, qz, ids, n)
    return list(ids[:n])


def tile_info(tile: int) -> tuple:
    v = [ctypes.c_int32() for _ in range(4)]
    _check(load().edp_tile_info(tile, *[ctypes.byref(x) for x in v]), "edp_tile_info")
    return tuple(x.value for x in v)


def wide_tiles_3d(qx: int, qy: int, qz: int) -> list:
    """Wide-vertex tiles of the EDP scans for a label space with three label dimensions."""
    L = load()
    n = L.edp_wide_tiles_3d(qx, qy, qz, None, 0)
    if n < 0:
        raise EdpError(n, "edp_wide_tiles_3d")
    ids = (ctypes.c_int32 * max(n, 1))()
    L.edp_wide_tiles_3d(qx, qy, qz, ids, n)
    return list(ids[:n])


def tile_depth(tile: int) -> int:
    """Labels along the third label dimension that a tile holds (1 below three dimensions)."""
    kz = ctypes.c_int32()
    _check(load().edp_tile_depth(tile, ctypes.byref(kz)), "edp_tile_depth")
    return kz.value


class Workspace:
    """Reusable device workspace (grows on demand, never shrinks)."""

    def __init__(self, device=None):
        self.device = device
        self.buf = None

    def get(self, nbytes: int, device) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        return self.buf


_default_ws = Workspace()


def dp_scanline(cost: torch.Tensor, qx: int, qy: int = 1, lam: int = 20, trunc: int = 2,
                mode: int = TRUNC_PER_DIM, cost_bound: int = 0, tile: int = -1, ws: Workspace | None = None,
                events=None, prior: int = PRIOR_LINEAR):
    """Independent scanline DP (edp_dp_scanline).  Returns (labels [H][W] int32,
    row energies [H] int64, total energy [1] int64) as device tensors."""
    _device_tensor(cost, "cost")
    prob = make_problem(cost, qx, qy, lam, trunc, mode, 1, cost_bound, prior)
    nbytes = workspace_size(prob, OP_DP, tile)
    w = (ws or _default_ws).get(nbytes, cost.device)
    H, W, _ = cost.shape
    labels = torch.empty((H, W), dtype=torch.int32, device=cost.device)
    row_e = torch.empty(H, dtype=torch.int64, device=cost.device)
    tot = torch.empty(1, dtype=torch.int64, device=cost.device)
    _check(load().edp_dp_scanline(ctypes.byref(prob), _tuning(tile, 0, events), cost.data_ptr(), labels.data_ptr(),
                                  row_e.data_ptr(), tot.data_ptr(), w.data_ptr(), w.numel(),
                                  _stream(cost.device)), "edp_dp_scanline")
    return labels, row_e, tot


def dp_marginals(cost: torch.Tensor, qx: int, qy: int = 1, lam: int = 20, trunc: int = 2,
                 mode: int = TRUNC_PER_DIM, cost_bound: int = 0, tile: int = -1, ws: Workspace | None = None,
                 events=None, prior: int = PRIOR_LINEAR, marginal: bool = False):
    """Scanline DP by min-marginals (edp_dp_marginals).  Returns (labels [H][W] int32,
    marginal excess [H][W][Q] int32 or None, row optima [H] int64, their sum [1] int64)."""
    _device_tensor(cost, "cost")
    prob = make_problem(cost, qx, qy, lam, trunc, mode, 1, cost_bound, prior)
    nbytes = workspace_size(prob, OP_DP_MARGINALS, tile)
    w = (ws or _default_ws).get(nbytes, cost.device)
    H, W, Q = cost.shape
    labels = torch.empty((H, W), dtype=torch.int32, device=cost.device)
    marg = torch.empty((H, W, Q), dtype=torch.int32, device=cost.device) if marginal else None
    row_e = torch.empty(H, dtype=torch.int64, device=cost.device)
    tot = torch.empty(1, dtype=torch.int64, device=cost.device)
    _check(load().edp_dp_marginals(ctypes.byref(prob), _tuning(tile, 0, events), cost.data_ptr(), labels.data_ptr(),
                                   marg.data_ptr() if marg is not None else None, row_e.data_ptr(), tot.data_ptr(),
                                   w.data_ptr(), w.numel(), _stream(cost.device)), "edp_dp_marginals")
    return labels, marg, row_e, tot


def dsi(i0: torch.Tensor, i1: torch.Tensor, qx: int, qy: int = 1, ox: int = 0, oy: int = 0, sx: int = -1,
        sy: int = 1, l2: int = 1, cmax: int = 50, dtype=torch.int16, i2: torch.Tensor | None = None,
        out: torch.Tensor | None = None) -> torch.Tensor:
    """Data cost volume [H][W][qx*qy] (edp_dsi) of uint8 images; with i2 the composite three-view cost."""
    for t, nm in ((i0, "i0"), (i1, "i1")) + (((i2, "i2"),) if i2 is not None else ()):
        _device_tensor(t, nm)
        if t.dtype != torch.uint8 or t.shape != i0.shape or t.dim() != 2:
            raise ValueError(f"{nm} must be uint8 [H][W] like i0")
    H, W = i0.shape
    if out is None:
        out = torch.empty((H, W, qx * qy), dtype=dtype, device=i0.device)
    _device_tensor(out, "out")
    code = EDP_I16 if out.dtype == torch.int16 else EDP_I32 if out.dtype == torch.int32 else 0
    if code == 0 or tuple(out.shape) != (H, W, qx * qy):
        raise ValueError("out must be int16 or int32 [H][W][qx*qy]")
    _check(load().edp_dsi(i0.data_ptr(), i1.data_ptr(), i2.data_ptr() if i2 is not None else None, W, H, qx, qy,
                          ox, oy, sx, sy, l2, cmax, code, out.data_ptr(), _stream(i0.device)), "edp_dsi")
    return out


def solve(cost: torch.Tensor, qx: int, qy: int = 1, lam: int = 20, trunc: int = 2, mode: int = TRUNC_PER_DIM,
          iterations: int = 1, cost_bound: int = 0, tile: int = -1, chunk: int = 0,
          ws: Workspace | None = None, labels: torch.Tensor | None = None, energy: torch.Tensor | None = None,
          events=None, split: int = 0, waves: int = 0, fuse: int = 0, prior: int = PRIOR_LINEAR,
          status: torch.Tensor | None = None, check: bool = True, qz: int = 1):
    """EDP (edp_solve).  Returns (labels [H][W] int32, energy [1] int64) as device tensors.
    ``qz``: labels along a third label dimension (cost [H][W][qx*qy*qz]).

    ``events``: optional ctypes array of hipEvent_t handles recorded around the scan launches.
    ``status``: optional [1] int32 device tensor receiving the solve's status word.  ``check``:
    wait for the solve and raise EdpError if its scans gave up waiting (EDP_E_TIMEOUT); with
    check=False the call only enqueues and the caller reads ``status`` (check_status) later."""
    _device_tensor(cost, "cost")
    prob = make_problem(cost, qx, qy, lam, trunc, mode, iterations, cost_bound, prior, qz)
    nbytes = workspace_size(prob, OP_EDP, tile, chunk, split, waves, fuse)
    w = (ws or _default_ws).get(nbytes, cost.device)
    H, W, _ = cost.shape
    if labels is None:
        labels = torch.empty((H, W), dtype=torch.int32, device=cost.device)
    if energy is None:
        energy = torch.empty(1, dtype=torch.int64, device=cost.device)
    if status is None and check:
        status = torch.empty(1, dtype=torch.int32, device=cost.device)
    _check(load().edp_solve(ctypes.byref(prob), _tuning(tile, chunk, events, split, waves, fuse), cost.data_ptr(),
                            labels.data_ptr(), energy.data_ptr(), _ptr(status), w.data_ptr(), w.numel(),
                            _stream(cost.device)), "edp_solve")
    if check:
        check_status(status, "edp_solve")
    return labels, energy


def solve_static(cost: torch.Tensor, qx: int, qy: int = 1, lam: int = 20, trunc: int = 2, mode: int = TRUNC_PER_DIM,
                 iterations: int = 1, cost_bound: int = 0, labels: torch.Tensor | None = None,
                 energy: torch.Tensor | None = None, status: torch.Tensor | None = None, check: bool = True,
                 prior: int = PRIOR_LINEAR, tile: int = -1, chunk: int = 0, split: int = 0, waves: int = 0,
                 fuse: int = 0, qz: int = 1):
    """EDP with the library's static workspace (edp_solve_static): the library allocates nothing;
    pass ``labels``, ``energy`` and ``status`` to allocate nothing here either.  Returns (labels, energy)
    as solve()."""
    _device_tensor(cost, "cost")
    prob = make_problem(cost, qx, qy, lam, trunc, mode, iterations, cost_bound, prior, qz)
    H, W, _ = cost.shape
    if labels is None:
        labels = torch.empty((H, W), dtype=torch.int32, device=cost.device)
    if energy is None:
        energy = torch.empty(1, dtype=torch.int64, device=cost.device)
    if status is None and check:
        status = torch.empty(1, dtype=torch.int32, device=cost.device)
    _check(load().edp_solve_static(ctypes.byref(prob), _tuning(tile, chunk, None, split, waves, fuse), cost.data_ptr(),
                                   labels.data_ptr(), energy.data_ptr(), _ptr(status), _stream(cost.device)),
           "edp_solve_static")
    if check:
        check_status(status, "edp_solve_static")
    return labels, energy


def solve_windowed(cost: torch.Tensor, centers: torch.Tensor, win: int, qx: int, qy: int, lam: int = 15,
                   trunc: int = 3, mode: int = TRUNC_PER_DIM, iterations: int = 1, cost_bound: int = 0,
                   ws: Workspace | None = None, labels: torch.Tensor | None = None,
                   energy: torch.Tensor | None = None, events=None, waves: int = 0, chunk: int = 0, fuse: int = 0,
                   status: torch.Tensor | None = None, check: bool = True):
    """Label-window EDP (edp_solve_windowed).  Returns (labels [H][W] int32, energy [1] int64);
    ``status`` and ``check`` as for solve()."""
    _device_tensor(cost, "cost")
    _device_tensor(centers, "centers")
    prob = make_problem(cost, qx, qy, lam, trunc, mode, iterations, cost_bound)
    tu = _tuning(-1, chunk, events, 0, waves, fuse)
    n = ctypes.c_size_t(0)
    _check(load().edp_window_workspace_size(ctypes.byref(prob), win, tu, ctypes.byref(n)),
           "edp_window_workspace_size")
    w = (ws or _default_ws).get(int(n.value), cost.device)
    H, W, _ = cost.shape
    if labels is None:
        labels = torch.empty((H, W), dtype=torch.int32, device=cost.device)
    if energy is None:
        energy = torch.empty(1, dtype=torch.int64, device=cost.device)
    if status is None and check:
        status = torch.empty(1, dtype=torch.int32, device=cost.device)
    _check(load().edp_solve_windowed(ctypes.byref(prob), tu, cost.data_ptr(), centers.data_ptr(), win,
                                     labels.data_ptr(), energy.data_ptr(), _ptr(status), w.data_ptr(), w.numel(),
                                     _stream(cost.device)), "edp_solve_windowed")
    if check:
        check_status(status, "edp_solve_windowed")
    return labels, energy


def energy(cost: torch.Tensor, labels: torch.Tensor, qx: int, qy: int = 1, lam: int = 20, trunc: int = 2,
           mode: int = TRUNC_PER_DIM, grid4: bool = True, cost_bound: int = 0, prior: int = PRIOR_LINEAR,
           qz: int = 1):
    """Energy of a labelling (edp_energy).  Returns (energy [1] int64, invalid-label count [1] int64)."""
    _device_tensor(cost, "cost")
    _device_tensor(labels, "labels")
    if labels.dtype != torch.int32 or tuple(labels.shape) != tuple(cost.shape[:2]):
        raise ValueError("labels must be int32 [H][W]")
    prob = make_problem(cost, qx, qy, lam, trunc, mode, 1, cost_bound, prior, qz)
    e = torch.empty(1, dtype=torch.int64, device=cost.device)
    bad = torch.empty(1, dtype=torch.int64, device=cost.device)
    _check(load().edp_energy(ctypes.byref(prob), cost.data_ptr(), labels.data_ptr(), int(bool(grid4)),
                             e.data_ptr(), bad.data_ptr(), _stream(cost.device)), "edp_energy")
    return e, bad


def batch_items(costs, params, labels, energies, tunings=None, statuses=None):
    """ctypes array of edp_batch_item for device tensors: params[i] holds qx, qy, lam, trunc, mode,
    iterations, cost_bound, prior, qz; tunings[i] (optional) holds tile, chunk, split, waves, fuse."""
    n = len(costs)
    items = (BatchItem * n)()
    for i in range(n):
        _device_tensor(costs[i], f"costs[{i}]")
        _device_tensor(labels[i], f"labels[{i}]")
        pr = params[i]
        items[i].problem = make_problem(costs[i], pr["qx"], pr.get("qy", 1), pr["lam"], pr["trunc"],
                                        pr.get("mode", TRUNC_PER_DIM), pr.get("iterations", 1),
                                        pr.get("cost_bound", 0), pr.get("prior", PRIOR_LINEAR), pr.get("qz", 1))
        items[i].d_cost = costs[i].data_ptr()
        items[i].d_labels = labels[i].data_ptr()
        items[i].d_energy = energies.data_ptr() + 8 * i if energies is not None else None
        items[i].d_status = statuses.data_ptr() + 4 * i if statuses is not None else None
        tu = (tunings[i] if tunings else None) or {}
        items[i].tuning = Tuning(tu.get("tile", -1), tu.get("chunk", 0), tu.get("split", 0), tu.get("waves", 0),
                                 tu.get("fuse", 0), None, 0)
    return items


def batch_workspace_size(items) -> int:
    n = ctypes.c_size_t(0)
    _check(load().edp_batch_workspace_size(len(items), items, ctypes.byref(n)), "edp_batch_workspace_size")
    return int(n.value)


class BatchPlan:
    """A batch of EDP instances bound to their device tensors (edp_batch_plan_create).

    ``solve()`` enqueues kernels only, so it may be captured into a hipGraph
    (torch.cuda.graph) and replayed; outputs land in ``labels[i]``, ``energies[i]`` and the status
    words ``statuses[i]`` (``check()`` raises if a solve's scans gave up waiting)."""

    def __init__(self, costs, params, tunings=None, device=None):
        self.device = device or costs[0].device
        self.costs = list(costs)
        self.labels = [torch.empty(tuple(c.shape[:2]), dtype=torch.int32, device=self.device) for c in costs]
        self.energies = torch.empty(len(costs), dtype=torch.int64, device=self.device)
        self.statuses = torch.empty(len(costs), dtype=torch.int32, device=self.device)
        self.items = batch_items(self.costs, params, self.labels, self.energies, tunings, self.statuses)
        nbytes = batch_workspace_size(self.items)
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p(None)
        _check(load().edp_batch_plan_create(len(self.items), self.items, self.ws.data_ptr(), self.ws.numel(),
                                            _stream(self.device), ctypes.byref(h)), "edp_batch_plan_create")
        self.handle = h

    def solve(self):
        _check(load().edp_batch_solve(self.handle, _stream(self.device)), "edp_batch_solve")
        return self.labels, self.energies

    def check(self):
        """Wait for the last solve and raise EdpError if any instance's scans gave up waiting."""
        check_status(self.statuses, "edp_batch_solve")

    def info(self) -> tuple:
        c, l = ctypes.c_int32(), ctypes.c_int32()
        _check(load().edp_batch_plan_info(self.handle, ctypes.byref(c), ctypes.byref(l)), "edp_batch_plan_info")
        return c.value, l.value

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            torch.cuda.synchronize(self.device)
            load().edp_batch_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# label-window network (include/edp_learn.h)
# ---------------------------------------------------------------------------

LEARN_EXPORTS = ("edp_dsi_motion", "edp_pool_cost", "edp_conv3x3_forward", "edp_conv3x3_dgrad",
                 "edp_conv3x3_wgrad", "edp_colsum", "edp_ce_loss", "edp_adam", "edp_decode_windows",
                 "edp_window_targets", "edp_window_recenter")


def _learn_lib():
    L = load()
    if getattr(L, "_learn_ready", False):
        return L
    vp, i32, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
    sig = {
        "edp_dsi_motion": [vp, vp, i32, i32, i32, i32, vp, vp],
        "edp_pool_cost": [vp, i32, i32, i32, i32, i32, i32, vp, vp],
        "edp_conv3x3_forward": [vp, vp, vp, i32, i32, i32, i32, i32, i32, vp, vp, vp],
        "edp_conv3x3_dgrad": [vp, vp, vp, i32, i32, i32, i32, i32, vp, vp, vp, vp],
        "edp_conv3x3_wgrad": [vp, vp, i32, i32, i32, i32, i32, vp, vp],
        "edp_colsum": [vp, i32, i32, i32, vp, vp],
        "edp_ce_loss": [vp, i32, i32, vp, vp, i32, i32, vp, vp, vp, vp],
        "edp_adam": [vp, vp, vp, vp, vp, i32, f32, f32, f32, f32, f32, i32, vp],
        "edp_decode_windows": [vp, i32, i32, i32, i32, i32, i32, i32, vp, vp],
        "edp_window_targets": [vp, i32, i32, i32, vp, vp, vp],
        "edp_window_recenter": [vp, i32, i32, i32, i32, i32, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    L._learn_ready = True
    return L


def dsi_motion(i0: torch.Tensor, i1: torch.Tensor, r: int, cmax: int, out: torch.Tensor | None = None):
    """Motion cost volume [H][W][(2r+1)^2] int32 from two uint8 frames (edp_dsi_motion)."""
    _device_tensor(i0, "i0")
    _device_tensor(i1, "i1")
    H, W = i0.shape
    n = 2 * r + 1
    if out is None:
        out = torch.empty((H, W, n * n), dtype=torch.int32, device=i0.device)
    _check(_learn_lib().edp_dsi_motion(i0.data_ptr(), i1.data_ptr(), W, H, r, cmax, out.data_ptr(),
                                       _stream(i0.device)), "edp_dsi_motion")
    return out


def pool_cost(cost: torch.Tensor, qx: int, qy: int, scale: int, out: torch.Tensor | None = None, mode: int = 0):
    """Network input [H/2][W/2][C] bf16 (as int16 storage) from an int32 cost volume (edp_pool_cost):
    mode 0 minima over 4 x 4 label blocks, mode 1 minima over label columns and rows (64 channels)."""
    _device_tensor(cost, "cost")
    H, W, _ = cost.shape
    nch = ((qx + 3) // 4) * ((qy + 3) // 4) if mode == 0 else 64
    if out is None:
        out = torch.empty((H // 2, W // 2, nch), dtype=torch.int16, device=cost.device)
    _check(_learn_lib().edp_pool_cost(cost.data_ptr(), W, H, qx, qy, scale, mode, out.data_ptr(),
                                      _stream(cost.device)), "edp_pool_cost")
    return out


def conv3x3_forward(x, w, b, h, wd, cin, cout, relu, y_bf16=None, y_f32=None, dilation=1):
    _check(_learn_lib().edp_conv3x3_forward(_ptr(x), _ptr(w), _ptr(b), h, wd, cin, cout, dilation, int(bool(relu)),
                                            _ptr(y_bf16), _ptr(y_f32), _stream(x.device)), "edp_conv3x3_forward")


def conv3x3_dgrad(dy, w, x, h, wd, cin, cout, wt, dx_f32, dx_bf16, dilation=1):
    _check(_learn_lib().edp_conv3x3_dgrad(_ptr(dy), _ptr(w), _ptr(x), h, wd, cin, cout, dilation, _ptr(wt),
                                          _ptr(dx_f32), _ptr(dx_bf16), _stream(dy.device)), "edp_conv3x3_dgrad")


def conv3x3_wgrad(dy, x, h, wd, cin, cout, dw, dilation=1):
    _check(_learn_lib().edp_conv3x3_wgrad(_ptr(dy), _ptr(x), h, wd, cin, cout, dilation, _ptr(dw),
                                          _stream(dy.device)), "edp_conv3x3_wgrad")


def colsum(a, rows, cols, ld, out):
    _check(_learn_lib().edp_colsum(_ptr(a), rows, cols, ld, _ptr(out), _stream(a.device)), "edp_colsum")


def ce_loss(logits, n, ld, tx, ty, nclass, grad_f32, grad_bf16, loss, win=1):
    _check(_learn_lib().edp_ce_loss(_ptr(logits), n, ld, _ptr(tx), _ptr(ty), nclass, win, _ptr(grad_f32),
                                    _ptr(grad_bf16), _ptr(loss), _stream(logits.device)), "edp_ce_loss")


def adam(p, g, m, v, p_bf16, lr, t, beta1=0.9, beta2=0.999, eps=1e-8, clip=0.0):
    _check(_learn_lib().edp_adam(_ptr(p), _ptr(g), _ptr(m), _ptr(v), _ptr(p_bf16), p.numel(), lr, beta1, beta2,
                                 eps, clip, t, _stream(p.device)), "edp_adam")


def decode_windows(logits, h, wd, ld, qx, qy, win, nclass, centers):
    _check(_learn_lib().edp_decode_windows(_ptr(logits), h, wd, ld, qx, qy, win, nclass, _ptr(centers),
                                           _stream(logits.device)), "edp_decode_windows")


def window_targets(labels, W, H, qx, tx, ty):
    _check(_learn_lib().edp_window_targets(_ptr(labels), W, H, qx, _ptr(tx), _ptr(ty), _stream(labels.device)),
           "edp_window_targets")


def window_recenter(labels, qx, qy, win, centers):
    H, W = labels.shape
    _check(_learn_lib().edp_window_recenter(_ptr(labels), W, H, qx, qy, win, _ptr(centers), _stream(labels.device)),
           "edp_window_recenter")
    return centers
