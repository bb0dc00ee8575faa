"""ctypes wrapper of the plain C oracle -- TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "edp_oracle.c")
LIB = os.path.join(HERE, "libedp_oracle.so")

SEARCH = {"sfms": 0, "lrms": 1, "grms": 2}
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no target-specific tuning)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        i32, i64p, i32p = ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)
        L.oracle_energy.restype = ctypes.c_int64
        L.oracle_energy.argtypes = [i32] * 10 + [i32p, i32p]
        L.oracle_dp_scanline.restype = ctypes.c_int
        L.oracle_dp_scanline.argtypes = [i32] * 10 + [i32p, i32p, i64p, i64p]
        L.oracle_edp.restype = ctypes.c_int
        L.oracle_edp.argtypes = [i32] * 11 + [i32p, i32p, i64p, i64p, i64p]
        L.oracle_edp_window.restype = ctypes.c_int
        L.oracle_edp_window.argtypes = [i32] * 10 + [i32p, i32p, i32, i32p, i64p, i64p]
        L.oracle_min_search.restype = ctypes.c_int
        L.oracle_min_search.argtypes = [i32] * 9 + [i64p, i64p, i32p]
        L.oracle_energy_volume.restype = ctypes.c_int64
        L.oracle_energy_volume.argtypes = [i32] * 9 + [i32p, i32p]
        L.oracle_edp_volume.restype = ctypes.c_int
        L.oracle_edp_volume.argtypes = [i32] * 11 + [i32p, i32p, i64p, i64p, i64p]
        _lib = L
    return _lib


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _p64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _cost32(cost):
    return np.ascontiguousarray(cost, dtype=np.int32)


def min_search(h, qx, qy, lam, trunc, mode, search: str = "sfms", prior: int = 0, qz: int = 1):
    """M over the last axis of ``h``; returns (values int64, argmin int32 or None).
    ``prior`` 0: truncated linear, 1: truncated squared; ``qz`` labels along a third dimension."""
    hh = np.ascontiguousarray(h, dtype=np.int64)
    flat = hh.reshape(-1, qx * qy * qz)
    out = np.zeros_like(flat)
    arg = np.zeros(flat.shape, np.int32) if search == "sfms" else None
    rc = lib().oracle_min_search(qx, qy, qz, lam, trunc, mode, prior, SEARCH[search], flat.shape[0], _p64(flat),
                                 _p64(out), _p32(arg) if arg is not None else ctypes.POINTER(ctypes.c_int32)())
    if rc != 0:
        raise RuntimeError(f"oracle_min_search failed: {rc}")
    return out.reshape(hh.shape), (arg.reshape(hh.shape) if arg is not None else None)


def energy(cost, labels, qx, qy, lam, trunc, mode, grid4, prior: int = 0, qz: int = 1) -> int:
    c = _cost32(cost)
    H, W, _ = c.shape
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    return int(lib().oracle_energy(W, H, qx, qy, qz, lam, trunc, mode, prior, int(bool(grid4)), _p32(c),
                                   _p32(lab)))


def dp_scanline(cost, qx, qy, lam, trunc, mode, search: str = "sfms", prior: int = 0, qz: int = 1):
    """Returns (labels [H][W] int32, row energies [H] int64, total)."""
    c = _cost32(cost)
    H, W, _ = c.shape
    labels = np.zeros((H, W), np.int32)
    row_e = np.zeros(H, np.int64)
    tot = np.zeros(1, np.int64)
    rc = lib().oracle_dp_scanline(W, H, qx, qy, qz, lam, trunc, mode, prior, SEARCH[search], _p32(c),
                                  _p32(labels), _p64(row_e), _p64(tot))
    if rc != 0:
        raise RuntimeError(f"oracle_dp_scanline failed: {rc}")
    return labels, row_e, int(tot[0])


def edp(cost, qx, qy, lam, trunc, mode, iterations=1, search: str = "lrms", marginal=False, prior: int = 0,
        qz: int = 1):
    """Returns dict(labels int32 [H][W], energy, max_abs_sum, marginal (optional int64 [H][W][Q]))."""
    c = _cost32(cost)
    H, W, Q = c.shape
    labels = np.zeros((H, W), np.int32)
    e = np.zeros(1, np.int64)
    mx = np.zeros(1, np.int64)
    marg = np.zeros((H, W, Q), np.int64) if marginal else None
    rc = lib().oracle_edp(W, H, qx, qy, qz, lam, trunc, mode, prior, iterations, SEARCH[search], _p32(c),
                          _p32(labels), _p64(e), _p64(mx),
                          _p64(marg) if marginal else ctypes.POINTER(ctypes.c_int64)())
    if rc == -2:
        raise OverflowError("EDP sum exceeds int32")
    if rc != 0:
        raise RuntimeError(f"oracle_edp failed: {rc}")
    out = {"labels": labels, "energy": int(e[0]), "max_abs_sum": int(mx[0])}
    if marginal:
        out["marginal"] = marg
    return out


def edp_window(cost, centers, win, qx, qy, lam, trunc, mode, iterations=1, search: str = "lrms"):
    """Windowed EDP: the plain EDP on the cost masked outside each vertex's win x win box
    centred on centers[y][x] = (cx, cy).  Returns dict(labels, energy (unmasked cost), max_abs_sum)."""
    c = _cost32(cost)
    H, W, Q = c.shape
    cen = np.ascontiguousarray(centers, dtype=np.int32)
    assert cen.shape == (H, W, 2)
    labels = np.zeros((H, W), np.int32)
    e = np.zeros(1, np.int64)
    mx = np.zeros(1, np.int64)
    rc = lib().oracle_edp_window(W, H, qx, qy, lam, trunc, mode, 0, iterations, SEARCH[search], _p32(c), _p32(cen),
                                 int(win), _p32(labels), _p64(e), _p64(mx))
    if rc == -2:
        raise OverflowError("EDP sum exceeds int32")
    if rc != 0:
        raise RuntimeError(f"oracle_edp_window failed: {rc}")
    return {"labels": labels, "energy": int(e[0]), "max_abs_sum": int(mx[0])}


def energy_volume(cost, labels, qx, qy, lam, trunc, mode, prior: int = 0) -> int:
    """6-connected energy of labels [Z][H][W] on cost [Z][H][W][Q]."""
    c = _cost32(cost)
    Z, H, W, _ = c.shape
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    return int(lib().oracle_energy_volume(W, H, Z, qx, qy, lam, trunc, mode, prior, _p32(c), _p32(lab)))


def edp_volume(cost, qx, qy, lam, trunc, mode, iterations=1, search: str = "lrms", marginal=False, prior: int = 0):
    """EDP on a volume cost [Z][H][W][Q] (D = 3).  Returns dict(labels int32 [Z][H][W], energy,
    max_abs_sum, marginal (optional int64 [Z][H][W][Q]))."""
    c = _cost32(cost)
    Z, H, W, Q = c.shape
    labels = np.zeros((Z, H, W), np.int32)
    e = np.zeros(1, np.int64)
    mx = np.zeros(1, np.int64)
    marg = np.zeros((Z, H, W, Q), np.int64) if marginal else None
    rc = lib().oracle_edp_volume(W, H, Z, qx, qy, lam, trunc, mode, prior, iterations, SEARCH[search], _p32(c),
                                 _p32(labels), _p64(e), _p64(mx),
                                 _p64(marg) if marginal else ctypes.POINTER(ctypes.c_int64)())
    if rc == -2:
        raise OverflowError("EDP sum exceeds int32")
    if rc != 0:
        raise RuntimeError(f"oracle_edp_volume failed: {rc}")
    out = {"labels": labels, "energy": int(e[0]), "max_abs_sum": int(mx[0])}
    if marginal:
        out["marginal"] = marg
    return out
