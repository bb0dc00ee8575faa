"""Plain numpy / Python oracle -- TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Notation follows the paper (Mozerov, arXiv 1410.7922):

* ``C[y][x][q]``  data cost (disparity space image), Sec. 2;
  flat label ``q = (vz * qy + vy) * qx + vx``, 0-based (the paper counts from 1);
  the label space has R = 1, 2 or 3 dimensions (``qz`` = 1 unless R = 3: the
  paper defines the search for any R, Sec. 2 and Sec. 3 eq. M_decmp).
* ``V(u)``        truncated prior, Sec. 2 eq. Smooth_value_t with f(|a|) = |a|
  (``prior`` 0, truncated linear) or f(|a|) = a^2 (``prior`` 1, truncated
  squared, the paper's l_1 = 2); ``mode`` 1 truncates the summed distance over
  the label dimensions as the paper does, ``mode`` 0 truncates each dimension
  on its own.
* ``M(h)(v) = min_v' h(v') + V(v - v')``  the minimum search operator,
  Sec. 2 eq. M_strf; ``argM`` takes the smallest flat index among ties.
* scanline DP: Sec. 2 eq. base with the zero boundary of Sec. 4.1 eq. DP_1D_2;
* EDP: Sec. 4.2 eqs. DP_2D_1, DP_2D_base, DP_2D_2 and Algorithm 1; on a volume (D = 3) the same
  equations in their general form (2D directional sums, normalisation 1/D).

Readings where the paper is silent or garbled (each one is listed in the
design notes of the repository):

* the data cost C(x, v) is added in eqs. DP_2D_1 and DP_2D_base, as in the
  one-dimensional forms eq. base and eq. DP_1D_3 (without it every sum stays 0);
* ``S / D`` with D = 2 is floor division (``S // 2``), S can be negative;
* before the first pass every S_k is 0, and off the grid S_k and M(S_k) are 0;
* the four scans run P1, P2, P3, P4 in place; a scan reads the sums it does
  not write with the values they hold when the scan starts;
* every argmin returns the smallest flat label;
* eq. L_dec5 (backward pass of the linear RMS) is read as the mirror of
  eq. L_dec3: S^-(v) = min over v'' > v of S(v'') + lambda (v'' - v), with
  S^-(v_max) = +inf;
* eq. M_decmp1 (one operator of the general RMS) adds lambda f(|u_r|) inside
  the window minimum, not lambda f(g): with the constant the operator would be
  a plain window minimum and eq. derivation2, from which it is derived, would
  not hold;
* a volume (D = 3) is scanned by the eight raster scans with x innermost, the
  x order alternating fastest, then y, then z (the generalisation of P1..P4),
  each computing the sums of its three directions; S / 3 is floor division;
* with three label dimensions the recursive searches apply their operators in
  the order x, y, z (eq. M_decmp nests them for any R; every order gives the
  same values), each followed by its per-line clip under per-dimension
  truncation.

Every floating point question is absent: all arithmetic is on Python / int64
integers, and every EDP sum is checked to fit in int32 (the GPU's type).
"""
from __future__ import annotations

import itertools

import numpy as np

TRUNC_PER_DIM = 0
TRUNC_JOINT = 1
PRIOR_LINEAR = 0        # f(|a|) = |a|
PRIOR_QUAD = 1          # f(|a|) = a^2
INT32_MAX = 2**31 - 1


# ---------------------------------------------------------------------------
# prior and minimum search
# ---------------------------------------------------------------------------

def prior_f(a, prior: int = PRIOR_LINEAR):
    """The increasing function f of Sec. 2 eq. Smooth_value_t: |a|, or a^2 (Sec. 5.1, l_1 = 2)."""
    if prior == PRIOR_LINEAR:
        return abs(a)
    if prior == PRIOR_QUAD:
        return a * a
    raise ValueError(f"unknown prior {prior}")


def label_coords(q, qx: int, qy: int):
    """(vx, vy, vz) of flat labels q = (vz * qy + vy) * qx + vx."""
    return q % qx, (q // qx) % qy, q // (qx * qy)


def prior_matrix(qx: int, qy: int, lam: int, trunc: int, mode: int, prior: int = PRIOR_LINEAR,
                 qz: int = 1) -> np.ndarray:
    """Vm[v, v'] = V(v - v') over flat labels, int64 [Q, Q]."""
    q = np.arange(qx * qy * qz, dtype=np.int64)
    vx, vy, vz = label_coords(q, qx, qy)
    fx = prior_f(vx[:, None] - vx[None, :], prior)
    fy = prior_f(vy[:, None] - vy[None, :], prior)
    fz = prior_f(vz[:, None] - vz[None, :], prior)
    fg = prior_f(int(trunc), prior)
    if mode == TRUNC_PER_DIM:
        return (lam * (np.minimum(fx, fg) + np.minimum(fy, fg) + np.minimum(fz, fg))).astype(np.int64)
    return (lam * np.minimum(fx + fy + fz, fg)).astype(np.int64)


class OpCounter:
    """Counts candidate comparisons per output label (Sec. 5.2, Table 1)."""

    def __init__(self):
        self.ops = 0
        self.outputs = 0

    @property
    def per_vertex(self) -> float:
        return self.ops / max(self.outputs, 1)


def min_search_sfms(h: np.ndarray, qx: int, qy: int, lam: int, trunc: int, mode: int,
                    counter: OpCounter | None = None, prior: int = PRIOR_LINEAR, qz: int = 1):
    """Straightforward minimum search (SFMS, Sec. 3 end): the definition eq. M_strf.

    ``h`` has shape [..., Q].  Returns (M(h), argM(h)); argM is the smallest
    flat index v' attaining the minimum.
    """
    h = np.asarray(h, dtype=np.int64)
    vm = prior_matrix(qx, qy, lam, trunc, mode, prior, qz)
    tot = h[..., None, :] + vm                    # [..., v, v']
    arg = np.argmin(tot, axis=-1)                 # first minimum = smallest v'
    val = np.take_along_axis(tot, arg[..., None], axis=-1)[..., 0]
    if counter is not None:
        n_out = int(np.prod(h.shape))
        counter.outputs += n_out
        counter.ops += n_out * h.shape[-1]
    return val, arg


def _linear_rms_line(line: list, lam: int, counter: OpCounter | None):
    """Operator L_r of Sec. 3.2 on one line: eq. L_dec3, eq. L_dec5 (read as its mirror), eq. L_dec6."""
    n = len(line)
    plus = [0] * n
    plus[0] = line[0]                                  # S+(1) = S(1)
    for v in range(1, n):                              # S+(v+1) = (S+(v) + lam) ^ S(v+1)
        plus[v] = min(plus[v - 1] + lam, line[v])
    minus = [None] * n                                 # S-(v_max) = +inf
    for v in range(n - 2, -1, -1):                     # S-(v) = (S-(v+1) ^ S(v+1)) + lam
        nxt = line[v + 1] if minus[v + 1] is None else min(minus[v + 1], line[v + 1])
        minus[v] = nxt + lam
    out = [plus[v] if minus[v] is None else min(plus[v], minus[v]) for v in range(n)]
    if counter is not None:
        counter.ops += 3 * n                           # forward, backward, comparison
    return out


def _lines(g, dims, r):
    """Index lists of the lines of the label grid g along dimension r (0 x, 1 y, 2 z)."""
    qx, qy, qz = dims
    if r == 0:
        return [[(vz, vy, vx) for vx in range(qx)] for vz in range(qz) for vy in range(qy)]
    if r == 1:
        return [[(vz, vy, vx) for vy in range(qy)] for vz in range(qz) for vx in range(qx)]
    return [[(vz, vy, vx) for vz in range(qz)] for vy in range(qy) for vx in range(qx)]


def _separable_search(h, qx, qy, qz, lam, trunc, mode, clipd, line_op, counter):
    """Eq. M_decmp: the one-dimensional operator line_op along every label dimension r = 1..R in
    turn; per-dimension truncation clips each line at its own minimum + clipd after its operator
    (eq. derivation1 applied to that dimension), joint truncation clips once at min h + clipd."""
    h = np.asarray(h, dtype=np.int64)
    lead = h.shape[:-1]
    dims = (qx, qy, qz)
    flat = h.reshape(-1, qz, qy, qx)
    out = np.empty_like(flat)
    for n in range(flat.shape[0]):
        g = {(vz, vy, vx): int(flat[n, vz, vy, vx]) for vz in range(qz) for vy in range(qy) for vx in range(qx)}
        for r in range(3):
            if dims[r] == 1 and r > 0:
                continue                      # a dimension of one label has no operator
            for idx in _lines(g, dims, r):
                line = [g[i] for i in idx]
                res = line_op(line)
                if mode == TRUNC_PER_DIM:
                    clip = min(line) + clipd
                    res = [min(a, clip) for a in res]
                for i, a in zip(idx, res):
                    g[i] = a
        if mode == TRUNC_JOINT:
            clip = int(flat[n].min()) + clipd
            g = {i: min(a, clip) for i, a in g.items()}
        for (vz, vy, vx), a in g.items():
            out[n, vz, vy, vx] = a
        if counter is not None:
            counter.outputs += qx * qy * qz
    return out.reshape(*lead, qx * qy * qz)


def min_search_lrms(h: np.ndarray, qx: int, qy: int, lam: int, trunc: int, mode: int,
                    counter: OpCounter | None = None, qz: int = 1) -> np.ndarray:
    """Linear RMS (LRMS, Sec. 3.2): per-dimension L_r passes and the clip of eq. L_dec7.

    ``mode`` 1 (joint truncation, the paper's prior): M = L_y(L_x(h)) ^ (min h + lam*T),
    eq. L_dec7.  ``mode`` 0 (per-dimension truncation): each dimension's prior is a
    one-dimensional truncated linear prior, so the decomposition of eq. derivation2 applies
    per dimension with its own clip (eq. derivation1 applied to that dimension):
    M = clip_y(L_y(clip_x(L_x(h)))).  With a third label dimension (``qz`` > 1) L_z follows
    in the same way.  Only the values are returned.
    """
    return _separable_search(h, qx, qy, qz, lam, trunc, mode, lam * trunc,
                             lambda line: _linear_rms_line(line, lam, counter), counter)


def _general_rms_line(line: list, lam: int, trunc: int, prior: int, counter: OpCounter | None):
    """Operator M-bar_r of Sec. 3.1 eq. M_decmp1 on one line: the minimum over the window
    |u| < g of S(v - u) + lam f(|u|).  The line is extended by g - 1 infinite entries at
    each end, so every output label examines the whole window of 2g - 1 entries."""
    n = len(line)
    inf = None
    ext = [inf] * (trunc - 1) + list(line) + [inf] * (trunc - 1)
    out = []
    for v in range(n):
        best = None
        for u in range(-(trunc - 1), trunc):
            s = ext[v - u + trunc - 1]
            if s is inf:
                continue
            t = s + lam * prior_f(u, prior)
            best = t if best is None else min(best, t)
        out.append(best)
    if counter is not None:
        counter.ops += (2 * trunc - 1) * n
    return out


def min_search_grms(h: np.ndarray, qx: int, qy: int, lam: int, trunc: int, mode: int,
                    counter: OpCounter | None = None, prior: int = PRIOR_QUAD, qz: int = 1) -> np.ndarray:
    """General RMS (GRMS, Sec. 3.1) for any truncated prior f: one windowed operator per
    label dimension and the clip of eq. M_decmp.

    ``mode`` 1 (joint truncation): M = M-bar_y(M-bar_x(h)) ^ (min h + lam f(g)), eq. M_decmp
    (the product of the per-dimension windows holds every u with f(|u|) < f(g), eq. derivation2).
    ``mode`` 0 (per-dimension truncation): each dimension's operator is followed by the clip of
    its own line, min h_line + lam f(g) (eq. derivation1 applied to that dimension).
    The dimensions run x, y, then z (``qz`` > 1).  Only the values are returned.
    """
    return _separable_search(h, qx, qy, qz, lam, trunc, mode, lam * prior_f(trunc, prior),
                             lambda line: _general_rms_line(line, lam, trunc, prior, counter), counter)


# ---------------------------------------------------------------------------
# energy (Sec. 2 eq. GE_objective_function)
# ---------------------------------------------------------------------------

def energy(cost: np.ndarray, labels: np.ndarray, qx: int, qy: int, lam: int, trunc: int,
           mode: int, grid4: bool, prior: int = PRIOR_LINEAR, qz: int = 1) -> int:
    """E = sum_x C(x, v(x)) + sum over neighbour pairs of V(v(x') - v(x)).

    ``grid4`` False: horizontal pairs only (independent scanlines, eq. One_d);
    True: horizontal and vertical pairs (the 2D energy EDP approximates).
    """
    cost = np.asarray(cost)
    labels = np.asarray(labels, dtype=np.int64)
    H, W, _ = cost.shape
    yy, xx = np.mgrid[0:H, 0:W]
    e = int(cost[yy, xx, labels].astype(np.int64).sum())
    vx, vy, vz = label_coords(labels, qx, qy)

    def pair(ax, ay, az):
        fx, fy, fz, fg = prior_f(ax, prior), prior_f(ay, prior), prior_f(az, prior), prior_f(trunc, prior)
        if mode == TRUNC_PER_DIM:
            return lam * (np.minimum(fx, fg) + np.minimum(fy, fg) + np.minimum(fz, fg))
        return lam * np.minimum(fx + fy + fz, fg)

    e += int(pair(np.abs(vx[:, 1:] - vx[:, :-1]), np.abs(vy[:, 1:] - vy[:, :-1]),
                  np.abs(vz[:, 1:] - vz[:, :-1])).sum())
    if grid4:
        e += int(pair(np.abs(vx[1:, :] - vx[:-1, :]), np.abs(vy[1:, :] - vy[:-1, :]),
                      np.abs(vz[1:, :] - vz[:-1, :])).sum())
    return e


# ---------------------------------------------------------------------------
# scanline DP (Sec. 2 eq. One_d / eq. base, Sec. 4.1)
# ---------------------------------------------------------------------------

def dp_scanline(cost: np.ndarray, qx: int, qy: int, lam: int, trunc: int, mode: int,
                prior: int = PRIOR_LINEAR, qz: int = 1):
    """Brute-force scanline DP: every row is an independent chain.

    S(0, v) = C(0, v) (zero boundary, eq. DP_1D_2), S(x+1) = C(x+1) + M(S(x)) (eq. base)
    with M by straightforward search; E_row = min_v S(W-1, v); the labels are
    recovered backwards from the stored optimal choice indexes.
    Returns (labels [H][W] int64, row energies [H] int64, total energy int).
    """
    cost = np.asarray(cost, dtype=np.int64)
    H, W, Q = cost.shape
    ptr = np.zeros((H, W, Q), np.int64)
    s = cost[:, 0, :].copy()
    for x in range(1, W):
        m, a = min_search_sfms(s, qx, qy, lam, trunc, mode, prior=prior, qz=qz)
        ptr[:, x, :] = a
        s = cost[:, x, :] + m
    row_e = s.min(axis=1)
    labels = np.zeros((H, W), np.int64)
    labels[:, W - 1] = np.argmin(s, axis=1)
    rows = np.arange(H)
    for x in range(W - 1, 0, -1):
        labels[:, x - 1] = ptr[rows, x, labels[:, x]]
    return labels, row_e, int(row_e.sum())


def dp_min_marginals(cost_row: np.ndarray, qx: int, qy: int, lam: int, trunc: int, mode: int,
                     prior: int = PRIOR_LINEAR, qz: int = 1):
    """Modified DP of Sec. 4.1, eq. DP_1D_3: S_Omega(x) = M(S_1(x-1)) + C(x) + M(S_-1(x+1)).

    S_1 runs left to right, S_-1 right to left, both with the zero boundary.
    Returns S_Omega [W][Q].
    """
    c = np.asarray(cost_row, dtype=np.int64)
    W, Q = c.shape
    fwd = np.zeros((W, Q), np.int64)
    bwd = np.zeros((W, Q), np.int64)
    fwd[0] = c[0]
    for x in range(1, W):
        fwd[x] = c[x] + min_search_sfms(fwd[x - 1], qx, qy, lam, trunc, mode, prior=prior, qz=qz)[0]
    bwd[W - 1] = c[W - 1]
    for x in range(W - 2, -1, -1):
        bwd[x] = c[x] + min_search_sfms(bwd[x + 1], qx, qy, lam, trunc, mode, prior=prior, qz=qz)[0]
    marg = c.copy()
    for x in range(W):
        if x > 0:
            marg[x] += min_search_sfms(fwd[x - 1], qx, qy, lam, trunc, mode, prior=prior, qz=qz)[0]
        if x < W - 1:
            marg[x] += min_search_sfms(bwd[x + 1], qx, qy, lam, trunc, mode, prior=prior, qz=qz)[0]
    return marg


# ---------------------------------------------------------------------------
# exhaustive enumeration (tiny inputs)
# ---------------------------------------------------------------------------

def chain_exhaustive(cost_row: np.ndarray, qx: int, qy: int, lam: int, trunc: int, mode: int,
                     prior: int = PRIOR_LINEAR, qz: int = 1):
    """All Q^W labellings of one chain.  Returns (E_min, canonical optimal labelling).

    The canonical labelling is the reverse-lexicographic minimum among the optimal
    ones (smallest v(W-1), then smallest v(W-2), ...).
    """
    c = np.asarray(cost_row, dtype=np.int64)
    W, Q = c.shape
    labs = np.array(list(itertools.product(range(Q), repeat=W)), dtype=np.int64)
    e = c[np.arange(W)[None, :], labs].sum(axis=1)
    vm = prior_matrix(qx, qy, lam, trunc, mode, prior, qz)
    for x in range(W - 1):
        e += vm[labs[:, x + 1], labs[:, x]]
    best = e.min()
    opt = labs[e == best]
    order = np.lexsort(tuple(opt[:, x] for x in range(W)))   # last key (x = W-1) is primary
    return int(best), opt[order[0]]


def grid_exhaustive(cost: np.ndarray, qx: int, qy: int, lam: int, trunc: int, mode: int,
                    prior: int = PRIOR_LINEAR, qz: int = 1) -> int:
    """Minimum 4-connected energy over all Q^(W*H) labellings of a tiny grid."""
    c = np.asarray(cost, dtype=np.int64)
    H, W, Q = c.shape
    n = H * W
    labs = np.array(list(itertools.product(range(Q), repeat=n)), dtype=np.int64).reshape(-1, H, W)
    yy, xx = np.mgrid[0:H, 0:W]
    e = c[yy[None], xx[None], labs].reshape(labs.shape[0], -1).sum(axis=1)
    vm = prior_matrix(qx, qy, lam, trunc, mode, prior, qz)
    e += vm[labs[:, :, 1:], labs[:, :, :-1]].reshape(labs.shape[0], -1).sum(axis=1)
    e += vm[labs[:, 1:, :], labs[:, :-1, :]].reshape(labs.shape[0], -1).sum(axis=1)
    return int(e.min())


# ---------------------------------------------------------------------------
# EDP (Sec. 4.2, Algorithm 1)
# ---------------------------------------------------------------------------

# k in K = {+x, -x, +y, -y}: (axis step dx, dy) of sgn(k) along axis |k|.
DIRECTIONS = {"+x": (1, 0), "-x": (-1, 0), "+y": (0, 1), "-y": (0, -1)}
OPPOSITE = {"+x": "-x", "-x": "+x", "+y": "-y", "-y": "+y"}
# The four scans of Sec. 4.2: (x order, y order, sums computed).
SCANS = (
    ("inc", "inc", ("+x", "+y")),   # P1
    ("dec", "inc", ("-x", "+y")),   # P2
    ("inc", "dec", ("+x", "-y")),   # P3
    ("dec", "dec", ("-x", "-y")),   # P4
)


def edp(cost: np.ndarray, qx: int, qy: int, lam: int, trunc: int, mode: int,
        iterations: int = 1, search: str = "sfms", trace=None, prior: int = PRIOR_LINEAR, qz: int = 1,
        divisor: int = 2):
    """Literal EDP, Algorithm 1 steps 3-5 (the DSI and the prior are the inputs).

    For every scan P1..P4 and every vertex x in the scan's raster order, each sum
    k' the scan computes is updated by eq. DP_2D_base with the data cost added:
        S_k'(x) = C(x) + sum_{k != -k'} M(S_k(x_k) // 2) - M(S_-k'(x_-k') // 2),
    where x_k = x - sgn(k) e_|k| and M(.) is 0 off the grid.  After ``iterations``
    rounds of the four scans, S_Omega(x) = C(x) + sum_k M(S_k(x_k) // 2) (eq. DP_2D_1)
    and the label is its smallest argmin (eq. DP_2D_2).

    ``search`` selects M: "sfms" (definition), "lrms" (Sec. 3.2 passes, linear prior only)
    or "grms" (Sec. 3.1 windowed operators).
    ``trace`` (optional) is called after every scan as trace(iteration, scan, sums).
    ``divisor`` is the normalisation D of eq. DP_2D_1 (2 for an image; other values serve only to
    compare with the volume solve, whose D is 3).
    Returns dict(labels, energy, marginal, sums, max_abs_sum).
    """
    c = np.asarray(cost, dtype=np.int64)
    H, W, Q = c.shape
    if search == "lrms" and prior != PRIOR_LINEAR:
        raise ValueError("the linear RMS applies to the truncated linear prior only")
    msearch = {"sfms": lambda h: min_search_sfms(h, qx, qy, lam, trunc, mode, prior=prior, qz=qz)[0],
               "lrms": lambda h: min_search_lrms(h, qx, qy, lam, trunc, mode, qz=qz),
               "grms": lambda h: min_search_grms(h, qx, qy, lam, trunc, mode, prior=prior, qz=qz)}[search]
    sums = {k: np.zeros((H, W, Q), np.int64) for k in DIRECTIONS}
    max_abs = 0

    def m_term(k, x, y):
        dx, dy = DIRECTIONS[k]
        px, py = x - dx, y - dy
        if 0 <= px < W and 0 <= py < H:
            return msearch(sums[k][py, px] // divisor)
        return np.zeros(Q, np.int64)

    for it in range(iterations):
        for scan, (xo, yo, computed) in enumerate(SCANS):
            ys = range(H) if yo == "inc" else range(H - 1, -1, -1)
            xs = range(W) if xo == "inc" else range(W - 1, -1, -1)
            for y in ys:
                for x in xs:
                    m = {k: m_term(k, x, y) for k in DIRECTIONS}
                    new = {}
                    for kp in computed:
                        acc = c[y, x].copy()
                        for k in DIRECTIONS:
                            if k != OPPOSITE[kp]:
                                acc = acc + m[k]
                        new[kp] = acc - m[OPPOSITE[kp]]
                    for kp, val in new.items():
                        sums[kp][y, x] = val
                        max_abs = max(max_abs, int(np.abs(val).max()))
            if trace is not None:
                trace(it, scan, {k: v.copy() for k, v in sums.items()})
    marg = c.copy()
    for y in range(H):
        for x in range(W):
            for k in DIRECTIONS:
                marg[y, x] += m_term(k, x, y)
    labels = np.argmin(marg, axis=-1)
    if max_abs > INT32_MAX:
        raise OverflowError(f"EDP sum {max_abs} exceeds int32")
    e = energy(c, labels, qx, qy, lam, trunc, mode, grid4=True, prior=prior, qz=qz)
    return {"labels": labels, "energy": e, "marginal": marg, "sums": sums,
            "max_abs_sum": max_abs}


# ---------------------------------------------------------------------------
# EDP on a three-dimensional grid (D = 3; Sec. 4.2 in the general form)
# ---------------------------------------------------------------------------

# k in K = {+-1, +-2, +-3}: unit step (dx, dy, dz) of sgn(k) along axis |k|.
DIRECTIONS3 = {"+x": (1, 0, 0), "-x": (-1, 0, 0), "+y": (0, 1, 0), "-y": (0, -1, 0),
               "+z": (0, 0, 1), "-z": (0, 0, -1)}
OPPOSITE3 = {"+x": "-x", "-x": "+x", "+y": "-y", "-y": "+y", "+z": "-z", "-z": "+z"}


def volume_scans():
    """The eight raster scans of a volume: loops x (innermost), y, z, each incrementing or
    decrementing; the x order alternates fastest, then y, then z, as P1..P4 do for an image.
    A scan with directions (sx, sy, sz) computes the sums S_{sx x}, S_{sy y}, S_{sz z}."""
    out = []
    for sz in (1, -1):
        for sy in (1, -1):
            for sx in (1, -1):
                out.append((sx, sy, sz, ("+x" if sx > 0 else "-x", "+y" if sy > 0 else "-y",
                                         "+z" if sz > 0 else "-z")))
    return tuple(out)


def edp_volume(cost: np.ndarray, qx: int, qy: int, lam: int, trunc: int, mode: int,
               iterations: int = 1, search: str = "sfms", trace=None, prior: int = PRIOR_LINEAR):
    """Literal EDP on a volume C[z][y][x][q] (D = 3): eq. DP_2D_base with K = {+-x, +-y, +-z}
    and the normalisation 1/D = 1/3 (floor division), the data cost added, the eight scans of
    volume_scans() in place, then eq. DP_2D_1 and the smallest argmin of eq. DP_2D_2:
        S_k'(x) = C(x) + sum_{k != -k'} M(S_k(x_k) // 3) - M(S_-k'(x_-k') // 3),
    x_k = x - sgn(k) e_|k|, M(.) = 0 off the grid, every S_k = 0 before the first scan.
    ``trace`` (optional) is called after every scan as trace(iteration, scan, sums).
    Returns dict(labels [Z][H][W], energy (6-connected), marginal, sums, max_abs_sum)."""
    c = np.asarray(cost, dtype=np.int64)
    Z, H, W, Q = c.shape
    if search == "lrms" and prior != PRIOR_LINEAR:
        raise ValueError("the linear RMS applies to the truncated linear prior only")
    msearch = {"sfms": lambda h: min_search_sfms(h, qx, qy, lam, trunc, mode, prior=prior)[0],
               "lrms": lambda h: min_search_lrms(h, qx, qy, lam, trunc, mode),
               "grms": lambda h: min_search_grms(h, qx, qy, lam, trunc, mode, prior=prior)}[search]
    sums = {k: np.zeros((Z, H, W, Q), np.int64) for k in DIRECTIONS3}
    max_abs = 0

    def m_term(k, x, y, z):
        dx, dy, dz = DIRECTIONS3[k]
        px, py, pz = x - dx, y - dy, z - dz
        if 0 <= px < W and 0 <= py < H and 0 <= pz < Z:
            return msearch(sums[k][pz, py, px] // 3)
        return np.zeros(Q, np.int64)

    for it in range(iterations):
        for scan, (sx, sy, sz, computed) in enumerate(volume_scans()):
            for z in (range(Z) if sz > 0 else range(Z - 1, -1, -1)):
                for y in (range(H) if sy > 0 else range(H - 1, -1, -1)):
                    for x in (range(W) if sx > 0 else range(W - 1, -1, -1)):
                        m = {k: m_term(k, x, y, z) for k in DIRECTIONS3}
                        new = {}
                        for kp in computed:
                            acc = c[z, y, x].copy()
                            for k in DIRECTIONS3:
                                if k != OPPOSITE3[kp]:
                                    acc = acc + m[k]
                            new[kp] = acc - m[OPPOSITE3[kp]]
                        for kp, val in new.items():
                            sums[kp][z, y, x] = val
                            max_abs = max(max_abs, int(np.abs(val).max()))
            if trace is not None:
                trace(it, scan, {k: v.copy() for k, v in sums.items()})
    marg = c.copy()
    for z in range(Z):
        for y in range(H):
            for x in range(W):
                for k in DIRECTIONS3:
                    marg[z, y, x] += m_term(k, x, y, z)
    labels = np.argmin(marg, axis=-1)
    if max_abs > INT32_MAX:
        raise OverflowError(f"EDP sum {max_abs} exceeds int32")
    e = energy_volume(c, labels, qx, qy, lam, trunc, mode, prior=prior)
    return {"labels": labels, "energy": e, "marginal": marg, "sums": sums, "max_abs_sum": max_abs}


def energy_volume(cost: np.ndarray, labels: np.ndarray, qx: int, qy: int, lam: int, trunc: int, mode: int,
                  prior: int = PRIOR_LINEAR) -> int:
    """Energy of eq. GE_objective_function on a 6-connected volume: data costs plus V over every
    pair of voxels one step apart along x, y or z."""
    c = np.asarray(cost, dtype=np.int64)
    labels = np.asarray(labels, dtype=np.int64)
    Z, H, W, Q = c.shape
    zz, yy, xx = np.mgrid[0:Z, 0:H, 0:W]
    e = int(c[zz, yy, xx, labels].sum())
    vm = prior_matrix(qx, qy, lam, trunc, mode, prior)
    e += int(vm[labels[:, :, 1:], labels[:, :, :-1]].sum())
    e += int(vm[labels[:, 1:, :], labels[:, :-1, :]].sum())
    e += int(vm[labels[1:, :, :], labels[:-1, :, :]].sum())
    return e


def volume_exhaustive(cost: np.ndarray, qx: int, qy: int, lam: int, trunc: int, mode: int,
                      prior: int = PRIOR_LINEAR) -> int:
    """Minimum 6-connected energy over all Q^(W*H*Z) labellings of a tiny volume."""
    c = np.asarray(cost, dtype=np.int64)
    Z, H, W, Q = c.shape
    best = None
    for lab in itertools.product(range(Q), repeat=Z * H * W):
        e = energy_volume(c, np.array(lab).reshape(Z, H, W), qx, qy, lam, trunc, mode, prior)
        best = e if best is None else min(best, e)
    return best


def wta(cost: np.ndarray) -> np.ndarray:
    """Winner-take-all labels: per-pixel smallest argmin of C."""
    return np.argmin(np.asarray(cost), axis=-1)
