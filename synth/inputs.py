"""Seeded synthetic workloads for the scanline-DP / EDP solvers.

Every generator is a pure function of its seed (numpy ``default_rng``).  The
outputs are integer cost volumes ``C[y][x][q]`` (the disparity space image of
Sec. 2) with the flat label ``q = (vz * qy + vy) * qx + vx`` (qz = 1 below three
label dimensions), plus the smoothness parameters of the workload.  Nothing here
minimises an energy.

Workload recipes (shapes and value distributions follow the paper's stereo
and motion experiments of Sec. 5.1; the Middlebury images themselves are not
used, textured synthetic pairs stand in for them):

* ``chain_problem``   -- 1D scanline DP: uniform costs in [0, 255] with planted
  piecewise-constant labels whose cost is lowered by 60 (costs may go negative).
* ``stereo_problem``  -- 1D disparity space: a textured left image, a
  piecewise-planar disparity field over Voronoi segments, a right image made by
  a z-ordered forward splat, Gaussian noise, truncated absolute difference cost
  (eq. Cost_value with l2 = 1).
* ``motion_problem``  -- 2D disparity space (dx, dy in [-r, r]): affine motion
  over Voronoi segments, truncated squared difference cost (l2 = 2).
* ``motion_offset_problem`` -- 3D disparity space (dx, dy, b): the motion frames
  with a brightness offset per segment, b one of ``levels`` offset steps; the
  cost compares I0 + offset with the displaced I1 (truncated squared difference).
* ``random_problem``  -- uniform random costs of any shape, for parity sweeps.
* ``volume_problem``  -- a three-dimensional grid (D = 3): a noisy volume over
  3D Voronoi cells of constant intensity level, truncated squared difference
  cost to each of Q levels (denoising of a tomography-like volume).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

# Truncation modes of the smoothness prior (meaning is fixed by the solvers):
#   0: per label dimension  lambda * (min(f(|dx|), f(T)) + min(f(|dy|), f(T)) [+ min(f(|dz|), f(T))])
#   1: joint                lambda * min(f(|dx|) + f(|dy|) [+ f(|dz|)], f(T))
TRUNC_PER_DIM = 0
TRUNC_JOINT = 1
# Prior functions f: 0 truncated linear f(a) = a, 1 truncated squared f(a) = a^2.
PRIOR_LINEAR = 0
PRIOR_QUAD = 1


@dataclass
class Problem:
    """One energy-minimisation instance: cost volume plus prior parameters."""

    cost: np.ndarray            # [H][W][Q], int16 or int32, C-contiguous
    qx: int
    qy: int
    lam: int
    trunc: int
    mode: int = TRUNC_PER_DIM
    name: str = ""
    meta: dict = field(default_factory=dict)
    prior: int = PRIOR_LINEAR
    qz: int = 1                 # labels along a third label dimension
    # cost [Z][H][W][Q] for a volume (D = 3): height and width read the last grid axes

    @property
    def height(self) -> int:
        return int(self.cost.shape[-3])

    @property
    def width(self) -> int:
        return int(self.cost.shape[-2])

    @property
    def depth(self) -> int:
        return int(self.cost.shape[0]) if self.cost.ndim == 4 else 1

    @property
    def q(self) -> int:
        return self.qx * self.qy * self.qz

    @property
    def pixel_labels(self) -> int:
        return self.depth * self.height * self.width * self.q

    def sha256(self) -> str:
        return hashlib.sha256(np.ascontiguousarray(self.cost).tobytes()).hexdigest()


# --------------------------------------------------------------------------
# image synthesis helpers
# --------------------------------------------------------------------------

def _bilinear_up(grid: np.ndarray, cell: int, W: int, H: int) -> np.ndarray:
    ys = np.arange(H) / cell
    xs = np.arange(W) / cell
    y0 = ys.astype(np.int64)
    x0 = xs.astype(np.int64)
    fy = (ys - y0)[:, None]
    fx = (xs - x0)[None, :]
    g00 = grid[y0][:, x0]
    g01 = grid[y0][:, x0 + 1]
    g10 = grid[y0 + 1][:, x0]
    g11 = grid[y0 + 1][:, x0 + 1]
    return g00 * (1 - fy) * (1 - fx) + g01 * (1 - fy) * fx + g10 * fy * (1 - fx) + g11 * fy * fx


def textured_image(rng: np.random.Generator, W: int, H: int) -> np.ndarray:
    """Four octaves of bilinearly upsampled uniform noise plus random rectangles, in [0, 255]."""
    img = np.zeros((H, W), np.float64)
    amp = 1.0
    for octave in range(4):
        cell = 32 >> octave
        g = rng.uniform(0.0, 1.0, size=(H // cell + 2, W // cell + 2))
        img += amp * _bilinear_up(g, cell, W, H)
        amp *= 0.6
    lo, hi = img.min(), img.max()
    img = (img - lo) / max(hi - lo, 1e-9) * 200.0 + 20.0
    nrect = max(4, (W * H) // 6000)
    for _ in range(nrect):
        w = int(rng.integers(max(1, W // 16), max(2, W // 4)))
        h = int(rng.integers(max(1, H // 16), max(2, H // 4)))
        x0 = int(rng.integers(0, max(1, W - w)))
        y0 = int(rng.integers(0, max(1, H - h)))
        val = rng.uniform(0.0, 255.0)
        img[y0:y0 + h, x0:x0 + w] = 0.5 * img[y0:y0 + h, x0:x0 + w] + 0.5 * val
    return np.clip(img, 0.0, 255.0)


def voronoi_segments(rng: np.random.Generator, W: int, H: int, n: int):
    sx = rng.uniform(0, W, n)
    sy = rng.uniform(0, H, n)
    yy, xx = np.mgrid[0:H, 0:W]
    seg = np.zeros((H, W), np.int64)
    best = np.full((H, W), np.inf)
    for s in range(n):
        d2 = (xx - sx[s]) ** 2 + (yy - sy[s]) ** 2
        closer = d2 < best
        seg[closer] = s
        best[closer] = d2[closer]
    return seg, sx, sy


def _forward_splat(src: np.ndarray, tx: np.ndarray, ty: np.ndarray, depth: np.ndarray,
                   rng: np.random.Generator) -> np.ndarray:
    """dst[ty, tx] = src, nearest (largest depth, then largest source index) wins; holes get noise."""
    H, W = src.shape
    n = H * W
    idx = np.arange(n, dtype=np.int64)
    ok = (tx >= 0) & (tx < W) & (ty >= 0) & (ty < H)
    key = depth.astype(np.int64).ravel() * n + idx
    tgt = (ty * W + tx).ravel()
    okr = ok.ravel()
    zbuf = np.full(n, -1, np.int64)
    np.maximum.at(zbuf, tgt[okr], key[okr])
    dst = rng.uniform(0.0, 255.0, size=n)
    hit = zbuf >= 0
    dst[hit] = src.ravel()[zbuf[hit] % n]
    return dst.reshape(H, W)


def _noisy_u8(rng: np.random.Generator, img: np.ndarray, sigma: float) -> np.ndarray:
    return np.clip(np.rint(img + rng.normal(0.0, sigma, size=img.shape)), 0, 255)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def chain_problem(seed: int = 0, W: int = 64, H: int = 48, Q: int = 16, lam: int = 20,
                  trunc: int = 2, lowered: int = 60) -> Problem:
    """Independent scanlines: uniform costs in [0,255], planted labels lowered by ``lowered``."""
    rng = np.random.default_rng(seed)
    cost = rng.integers(0, 256, size=(H, W, Q), dtype=np.int64)
    gt = np.zeros((H, W), np.int64)
    for y in range(H):
        x = 0
        while x < W:
            run = int(rng.integers(4, 17))
            gt[y, x:x + run] = int(rng.integers(0, Q))
            x += run
    yy, xx = np.mgrid[0:H, 0:W]
    cost[yy, xx, gt] -= lowered
    return Problem(cost.astype(np.int32), Q, 1, lam, trunc, TRUNC_PER_DIM,
                   name=f"chain{W}x{H}q{Q}s{seed}", meta={"gt": gt})


def stereo_problem(seed: int = 0, W: int = 384, H: int = 288, Q: int = 32, lam: int = 20,
                   trunc: int = 2, cmax: int = 50, segments: int = 6, sigma: float = 4.0,
                   dtype=np.int16) -> Problem:
    """Rectified stereo pair over piecewise-planar disparities, truncated |I_L - I_R| cost."""
    rng = np.random.default_rng(seed)
    left = textured_image(rng, W, H)
    seg, sx, sy = voronoi_segments(rng, W, H, segments)
    a = rng.uniform(0, Q - 1, segments)
    b = rng.uniform(-1, 1, segments) * (Q / 4.0) / W
    c = rng.uniform(-1, 1, segments) * (Q / 4.0) / H
    yy, xx = np.mgrid[0:H, 0:W]
    disp = a[seg] + b[seg] * (xx - sx[seg]) + c[seg] * (yy - sy[seg])
    disp = np.clip(np.rint(disp), 0, Q - 1).astype(np.int64)
    right = _forward_splat(left, xx - disp, yy, disp, rng)
    left_n = _noisy_u8(rng, left, sigma)
    right_n = _noisy_u8(rng, right, sigma)
    cost = np.full((H, W, Q), cmax, np.int64)
    for d in range(Q):
        if d >= W:
            break
        diff = np.abs(left_n[:, d:] - right_n[:, :W - d])
        cost[:, d:, d] = np.minimum(diff, cmax)
    return Problem(np.ascontiguousarray(cost.astype(dtype)), Q, 1, lam, trunc, TRUNC_PER_DIM,
                   name=f"stereo{W}x{H}q{Q}s{seed}",
                   meta={"gt": disp, "frames": (left_n.astype(np.uint8), right_n.astype(np.uint8))})


def motion_frames(seed: int = 0, W: int = 320, H: int = 240, r: int = 7, segments: int = 8,
                  sigma: float = 4.0, ry: int | None = None):
    """Two 8-bit frames with affine motion over Voronoi segments, and the planted flow.

    Returns (i0, i1, fu, fv): uint8 [H][W] frames where I1(x + fu, y + fv) shows I0(x, y),
    and the integer flow components in [-r, r] (fu) and [-ry, ry] (fv, ry = r by default).
    """
    return _motion_frames(seed, W, H, r, segments, sigma, ry, 1, 0)[:4]


def _motion_frames(seed, W, H, r, segments, sigma, ry, levels, step):
    """motion_frames with a brightness offset per segment when levels > 1: I1(x + fu, y + fv)
    shows I0(x, y) + (fb - levels // 2) step, fb in [0, levels).  Returns (i0, i1, fu, fv, fb)."""
    ry = r if ry is None else ry
    rng = np.random.default_rng(seed)
    img0 = textured_image(rng, W, H)
    seg, sx, sy = voronoi_segments(rng, W, H, segments)
    u0 = rng.uniform(-r, r, segments)
    v0 = rng.uniform(-ry, ry, segments)
    ux, uy = (rng.uniform(-1, 1, (2, segments)) * (r / 2.0) / np.array([[W], [H]]))
    vx, vy = (rng.uniform(-1, 1, (2, segments)) * (ry / 2.0) / np.array([[W], [H]]))
    depth = rng.permutation(segments)
    yy, xx = np.mgrid[0:H, 0:W]
    fu = np.clip(np.rint(u0[seg] + ux[seg] * (xx - sx[seg]) + uy[seg] * (yy - sy[seg])), -r, r)
    fv = np.clip(np.rint(v0[seg] + vx[seg] * (xx - sx[seg]) + vy[seg] * (yy - sy[seg])), -ry, ry)
    fu = fu.astype(np.int64)
    fv = fv.astype(np.int64)
    fb = np.full((H, W), levels // 2, np.int64)
    src = img0
    if levels > 1:
        fb = rng.integers(0, levels, segments)[seg]
        src = img0 + (fb - levels // 2) * float(step)
    img1 = _forward_splat(src, xx + fu, yy + fv, depth[seg], rng)
    i0 = _noisy_u8(rng, img0, sigma).astype(np.uint8)
    i1 = _noisy_u8(rng, img1, sigma).astype(np.uint8)
    return i0, i1, fu, fv, fb


def motion_cost(i0: np.ndarray, i1: np.ndarray, r: int, cmax: int, ry: int | None = None) -> np.ndarray:
    """Truncated squared difference cost [H][W][(2r+1)(2ry+1)] int64 (ry = r by default): label
    q = (dy + ry)(2r + 1) + (dx + r) compares I0(x, y) with I1(x + dx, y + dy); a displaced position
    outside the frame costs cmax."""
    ry = r if ry is None else ry
    H, W = i0.shape
    n = 2 * r + 1
    m = max(r, ry)
    a = i0.astype(np.float64)
    pad = np.full((H + 2 * m, W + 2 * m), np.nan)
    pad[m:m + H, m:m + W] = i1
    cost = np.empty((n * (2 * ry + 1), H, W), np.int64)
    for dy in range(-ry, ry + 1):
        for dx in range(-r, r + 1):
            sh = pad[m + dy:m + dy + H, m + dx:m + dx + W]
            d2 = (a - sh) ** 2
            cq = np.where(np.isnan(d2), cmax, np.minimum(np.nan_to_num(d2, nan=0.0), cmax))
            cost[(dy + ry) * n + (dx + r)] = cq.astype(np.int64)
    return np.ascontiguousarray(np.moveaxis(cost, 0, -1))


def motion_problem(seed: int = 0, W: int = 320, H: int = 240, r: int = 7, lam: int = 15,
                   trunc: int = 3, cmax: int = 2500, segments: int = 8, sigma: float = 4.0,
                   mode: int = TRUNC_PER_DIM, dtype=np.int32, ry: int | None = None) -> Problem:
    """Two frames with affine motion over Voronoi segments, truncated squared difference cost.

    Labels: q = (dy + ry) * (2r + 1) + (dx + r) (ry = r by default), the cost of q at pixel (x, y)
    compares I0(x, y) with I1(x + dx, y + dy).
    """
    ry_ = r if ry is None else ry
    n = 2 * r + 1
    i0, i1, fu, fv = motion_frames(seed, W, H, r, segments, sigma, ry=ry_)
    cost = np.ascontiguousarray(motion_cost(i0, i1, r, cmax, ry=ry_).astype(dtype))
    gt = (fv + ry_) * n + (fu + r)
    name = f"motion{W}x{H}r{r}s{seed}" if ry_ == r else f"motion{W}x{H}r{r}x{ry_}s{seed}"
    return Problem(cost, n, 2 * ry_ + 1, lam, trunc, mode, name=name, meta={"gt": gt, "frames": (i0, i1)})


def motion_offset_cost(i0: np.ndarray, i1: np.ndarray, r: int, levels: int, step: int, cmax: int) -> np.ndarray:
    """Truncated squared difference cost [H][W][(2r+1)^2 levels] int64 of a motion with a brightness
    offset: label q = (b (2r + 1) + dy + r)(2r + 1) + dx + r compares I0(x, y) + (b - levels // 2) step
    with I1(x + dx, y + dy); a displaced position outside the frame costs cmax."""
    H, W = i0.shape
    n = 2 * r + 1
    a = i0.astype(np.float64)
    pad = np.full((H + 2 * r, W + 2 * r), np.nan)
    pad[r:r + H, r:r + W] = i1
    cost = np.empty((levels * n * n, H, W), np.int64)
    for b in range(levels):
        ab = a + (b - levels // 2) * float(step)
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                sh = pad[r + dy:r + dy + H, r + dx:r + dx + W]
                d2 = (ab - sh) ** 2
                cq = np.where(np.isnan(d2), cmax, np.minimum(np.nan_to_num(d2, nan=0.0), cmax))
                cost[(b * n + dy + r) * n + dx + r] = cq.astype(np.int64)
    return np.ascontiguousarray(np.moveaxis(cost, 0, -1))


def motion_offset_problem(seed: int = 0, W: int = 320, H: int = 240, r: int = 3, levels: int = 7, step: int = 6,
                          lam: int = 40, trunc: int = 3, cmax: int = 2500, segments: int = 8, sigma: float = 4.0,
                          mode: int = TRUNC_PER_DIM, dtype=np.int32) -> Problem:
    """A three-dimensional disparity space: motion (dx, dy in [-r, r]) and a brightness offset
    (levels steps of ``step`` grey levels) over Voronoi segments, truncated squared difference cost.

    Labels: q = (b * (2r + 1) + dy + r) * (2r + 1) + dx + r, so qx = qy = 2r + 1 and qz = levels.
    """
    n = 2 * r + 1
    i0, i1, fu, fv, fb = _motion_frames(seed, W, H, r, segments, sigma, r, levels, step)
    cost = np.ascontiguousarray(motion_offset_cost(i0, i1, r, levels, step, cmax).astype(dtype))
    gt = (fb * n + fv + r) * n + fu + r
    return Problem(cost, n, n, lam, trunc, mode, name=f"motionoff{W}x{H}r{r}b{levels}s{seed}",
                   meta={"gt": gt, "frames": (i0, i1)}, qz=levels)


def random_volume(seed: int, W: int, H: int, Z: int, qx: int, qy: int = 1, lam: int = 7, trunc: int = 2,
                  mode: int = TRUNC_PER_DIM, lo: int = 0, hi: int = 100, dtype=np.int32) -> Problem:
    """Uniform random integer costs in [lo, hi] on a volume [Z][H][W][Q]."""
    rng = np.random.default_rng(seed)
    cost = rng.integers(lo, hi + 1, size=(Z, H, W, qx * qy), dtype=np.int64).astype(dtype)
    return Problem(np.ascontiguousarray(cost), qx, qy, lam, trunc, mode, name=f"vol{W}x{H}x{Z}q{qx}x{qy}s{seed}")


def volume_problem(seed: int = 0, W: int = 128, H: int = 128, Z: int = 128, Q: int = 32, cells: int = 24,
                   sigma: float = 10.0, lam: int = 60, trunc: int = 3, cmax: int = 2500, dtype=np.int16) -> Problem:
    """A noisy volume over 3D Voronoi cells, each of one of Q intensity levels (level q is grey
    value round(q * 255 / (Q - 1))), Gaussian noise sigma; label q costs
    min((I - level_q)^2, cmax).  Planted labels in meta["gt"]."""
    rng = np.random.default_rng(seed)
    cz, cy, cx = rng.uniform(0, Z, cells), rng.uniform(0, H, cells), rng.uniform(0, W, cells)
    lev = rng.integers(0, Q, cells)
    zz, yy, xx = np.mgrid[0:Z, 0:H, 0:W]
    best = np.full((Z, H, W), np.inf)
    gt = np.zeros((Z, H, W), np.int64)
    for k in range(cells):
        d2 = (xx - cx[k]) ** 2 + (yy - cy[k]) ** 2 + (zz - cz[k]) ** 2
        closer = d2 < best
        gt[closer] = lev[k]
        best[closer] = d2[closer]
    levels = np.rint(np.arange(Q) * 255.0 / (Q - 1))
    img = np.clip(np.rint(levels[gt] + rng.normal(0.0, sigma, size=gt.shape)), 0, 255)
    cost = np.minimum((img[..., None] - levels[None, None, None, :]) ** 2, cmax).astype(dtype)
    return Problem(np.ascontiguousarray(cost), Q, 1, lam, trunc, TRUNC_PER_DIM,
                   name=f"volume{W}x{H}x{Z}q{Q}s{seed}", meta={"gt": gt})


def random_problem(seed: int, W: int, H: int, qx: int, qy: int = 1, lam: int = 7, trunc: int = 2,
                   mode: int = TRUNC_PER_DIM, lo: int = 0, hi: int = 100,
                   dtype=np.int32, qz: int = 1) -> Problem:
    """Uniform random integer costs in [lo, hi] of any shape."""
    rng = np.random.default_rng(seed)
    cost = rng.integers(lo, hi + 1, size=(H, W, qx * qy * qz), dtype=np.int64).astype(dtype)
    name = f"rand{W}x{H}q{qx}x{qy}s{seed}" if qz == 1 else f"rand{W}x{H}q{qx}x{qy}x{qz}s{seed}"
    return Problem(np.ascontiguousarray(cost), qx, qy, lam, trunc, mode, name=name, qz=qz)


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------

def workload(name: str, seed: int = 0) -> Problem:
    """The named workloads: chain64x48, stereo384x288, motion320x240, motion640x480, and with
    the truncated squared prior (lambda 5, T 3, so the clip lambda T^2 = 45 is near the linear
    workloads' lambda T): stereo384x288_sq, motion320x240_sq; three label dimensions (7 x 7 motion
    and 7 brightness offsets, 343 labels): motion_offset320x240, motion_offset640x480."""
    if name == "chain64x48":
        return chain_problem(seed)
    if name == "stereo384x288":
        return stereo_problem(seed)
    if name == "motion320x240":
        return motion_problem(seed)
    if name in ("stereo384x288_sq", "motion320x240_sq"):
        p = stereo_problem(seed, lam=5, trunc=3) if name.startswith("stereo") else motion_problem(seed, lam=5, trunc=3)
        p.prior = PRIOR_QUAD
        p.name += "_sq"
        return p
    if name == "motion640x480":
        return motion_problem(seed, W=640, H=480, r=15)
    if name == "motion_offset320x240":
        return motion_offset_problem(seed)
    if name == "motion_offset640x480":
        return motion_offset_problem(seed, W=640, H=480)
    if name == "volume128q32":
        return volume_problem(seed)
    raise KeyError(name)


def batch_problems(n: int = 64, first_seed: int = 0) -> list:
    """Uneven mix for batched solving: even seeds stereo (int16), odd seeds 2D motion (int32).

    Stereo: (W, H) in {160x120, 320x240, 480x360, 640x480}, Q uniform in [16, 64],
    lambda 20, T 2.  Motion: s x s labels with s in {9, 11, ..., 21},
    (W, H) in {160x120, 240x180, 320x240}, lambda 15, T 3, per-dimension truncation.
    """
    out = []
    for i in range(first_seed, first_seed + n):
        rng = np.random.default_rng(10_000 + i)
        if i % 2 == 0:
            W, H = [(160, 120), (320, 240), (480, 360), (640, 480)][int(rng.integers(0, 4))]
            Q = int(rng.integers(16, 65))
            out.append(stereo_problem(seed=i, W=W, H=H, Q=Q))
        else:
            s = [9, 11, 13, 15, 17, 19, 21][int(rng.integers(0, 7))]
            W, H = [(160, 120), (240, 180), (320, 240)][int(rng.integers(0, 3))]
            out.append(motion_problem(seed=i, W=W, H=H, r=s // 2))
    return out
