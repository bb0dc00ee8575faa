"""C ABI checks that need no GPU: the library loads, exports every declared entry point, and
rejects bad arguments on the host before anything is enqueued."""
import ctypes
import os
import re

import pytest

from paper_1410_7922_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", n) for n in ("edp.h", "edp_learn.h")]


def declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"^\s*(?:edp_status|int32_t|const char\*|void)\s+(edp_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = B.load()
    names = declared_functions()
    assert len(names) >= 7
    for n in names:
        assert hasattr(lib, n), n
    assert set(B.EXPORTS) | set(B.LEARN_EXPORTS) <= set(names)


def test_status_strings():
    assert B.status_string(0) == "ok"
    for s in (-1, -2, -3, -4, -5, -6):
        assert B.status_string(s) != "unknown status"
    assert B.status_string(42) == "unknown status"


def _prob(**kw):
    d = dict(width=384, height=288, qx=32, qy=1, dtype=1, trunc_mode=0, lam=20, trunc=2, iterations=1,
             cost_bound=50, prior=0, qz=1)
    d.update(kw)
    return B.Problem(*[d[f] for f, _ in B.Problem._fields_])


def _ws(prob, op, tile=-1):
    n = ctypes.c_size_t(0)
    tu = ctypes.byref(B.Tuning(tile, 0, 0, 0, 0, None, 0)) if tile >= 0 else None
    st = B.load().edp_workspace_size(ctypes.byref(prob), op, tu, ctypes.byref(n))
    return st, n.value


@pytest.mark.parametrize("field,value", [("width", 0), ("height", -1), ("qx", 0), ("qy", 0), ("dtype", 3),
                                         ("trunc_mode", 2), ("lam", -1), ("lam", 70000), ("trunc", 0),
                                         ("iterations", 0), ("cost_bound", -5), ("qx", 4097), ("prior", 2),
                                         ("prior", -1), ("qz", -1), ("qz", 129)])
def test_invalid_problems_rejected(field, value):
    st, _ = _ws(_prob(**{field: value}), B.OP_EDP)
    assert st == -1


def test_int32_costs_need_a_bound_and_range_guard():
    assert _ws(_prob(dtype=2, cost_bound=0), B.OP_EDP)[0] == -1
    assert _ws(_prob(dtype=2, cost_bound=2500), B.OP_EDP)[0] == 0
    # a cost bound too large for the int32 EDP sums on this grid
    assert _ws(_prob(dtype=2, cost_bound=10**6), B.OP_EDP)[0] == -2
    # the DP packs the label index under the value: a huge lambda trips its guard
    assert _ws(_prob(lam=60000, trunc=4000, qx=64), B.OP_DP)[0] == -2


def test_dsi_rejects_bad_arguments_on_the_host():
    L = B.load()
    ok = dict(i0=16, i1=16, i2=None, w=8, h=4, qx=4, qy=1, ox=0, oy=0, sx=-1, sy=1, l2=1, cmax=50, dt=1, out=256)

    def call(**kw):
        d = dict(ok)
        d.update(kw)
        return L.edp_dsi(d["i0"], d["i1"], d["i2"], d["w"], d["h"], d["qx"], d["qy"], d["ox"], d["oy"], d["sx"],
                         d["sy"], d["l2"], d["cmax"], d["dt"], d["out"], None)

    for bad in (dict(i0=None), dict(out=None), dict(w=0), dict(qx=0), dict(qx=65, qy=65), dict(sx=2), dict(sy=0),
                dict(l2=3), dict(cmax=-1), dict(cmax=40000), dict(dt=3), dict(out=257), dict(ox=16385),
                dict(oy=-20000)):
        assert call(**bad) == -1, bad


def test_min_marginal_dp_workspace_and_term_range():
    """The min-marginal DP stores its forward terms in 16 bits: a clip distance above 65535 is refused."""
    st, n = _ws(_prob(), 2)
    assert st == 0 and n >= 384 * 288 * 32 * 2
    assert _ws(_prob(lam=20, trunc=3000, qx=2), 2)[0] == 0      # lambda T = 60000 fits
    assert _ws(_prob(prior=1, lam=10, trunc=100, qx=4), 2)[0] == -2    # lambda T^2 = 100000
    assert _ws(_prob(prior=1, lam=10, trunc=50, qx=4), 2)[0] == 0      # lambda T^2 = 25000
    assert _ws(_prob(), 3)[0] == -1


def test_squared_prior_range_guard_and_window_solve():
    """The squared prior's clip lambda T^2 enters both guards; the label-window solve is linear only."""
    assert _ws(_prob(prior=1, lam=5, trunc=3), B.OP_EDP)[0] == 0
    assert _ws(_prob(prior=1, lam=5, trunc=3), B.OP_DP)[0] == 0
    # lambda T = 4000 passes with the linear prior, lambda T^2 = 800000 does not
    assert _ws(_prob(prior=0, lam=20, trunc=200), B.OP_EDP)[0] == 0
    assert _ws(_prob(prior=1, lam=20, trunc=200), B.OP_EDP)[0] == -2
    assert _ws(_prob(prior=1, lam=65535, trunc=4096), B.OP_DP)[0] == -2
    n = ctypes.c_size_t(0)
    p = _prob(prior=1, dtype=2, qx=15, qy=15, lam=15, trunc=3, cost_bound=2500)
    assert B.load().edp_window_workspace_size(ctypes.byref(p), 7, None, ctypes.byref(n)) == -5
    p.prior = 0
    assert B.load().edp_window_workspace_size(ctypes.byref(p), 7, None, ctypes.byref(n)) == 0


def test_tiles_and_workspace_sizes():
    assert B.tiles(32) == [1, 2, 3, 4, 5, 6, 7, 8, 12, 15]
    assert 10 in B.tiles(15, 15) and 0 not in B.tiles(15, 15)
    assert B.tiles(65, 65) == []
    st, n = _ws(_prob(qx=65, qy=65), B.OP_EDP)
    assert st == -1                                  # more than 4096 labels
    st, n = _ws(_prob(qx=200, qy=1), B.OP_EDP)
    assert st == 0
    st, n = _ws(_prob(qx=40, qy=40), B.OP_EDP)
    assert st == 0                                   # 1600 labels: the 64 x 64 wide tile (T = 2)
    assert _ws(_prob(qx=40, qy=40, trunc=5), B.OP_EDP)[0] == -5   # the linear RMS: no tile beyond 32 x 32
    assert _ws(_prob(qx=64, qy=64, dtype=2, cost_bound=100), B.OP_EDP)[0] == 0
    assert B.wide_tiles(64, 64) == [22] and B.wide_tiles(33, 20) == [22, 23] and B.wide_tiles(20, 33) == [22, 24]
    assert B.tile_info(22) == (16, 4, 32, 2) and B.tile_depth(22) == 1
    for tile in B.tiles(32):
        st, n = _ws(_prob(), B.OP_EDP, tile)
        px, kx, py, ky = B.tile_info(tile)
        qt = px * kx * py * ky
        assert st == 0 and n >= 4 * 384 * 288 * qt * 4
    assert _ws(_prob(), B.OP_EDP, 0)[0] == -1        # tile 0 holds 16 labels only
    lib = B.load()
    n = ctypes.c_size_t(0)
    p = _prob()
    bad_split = B.Tuning(2, 0, 2, 0, 0, None, 0)          # tile 2 spans 64 lanes: no room for two halves
    assert lib.edp_workspace_size(ctypes.byref(p), B.OP_EDP, ctypes.byref(bad_split), ctypes.byref(n)) == -1
    bad_waves = B.Tuning(-1, 0, 0, 7, 0, None, 0)
    assert lib.edp_workspace_size(ctypes.byref(p), B.OP_EDP, ctypes.byref(bad_waves), ctypes.byref(n)) == -1
    bad_fuse = B.Tuning(-1, 0, 0, 0, 3, None, 0)
    assert lib.edp_workspace_size(ctypes.byref(p), B.OP_EDP, ctypes.byref(bad_fuse), ctypes.byref(n)) == -1
    # one scan per launch needs fewer ticket counters than the fused pairs, never more memory
    one = B.Tuning(-1, 0, 0, 0, 1, None, 0)
    n1 = ctypes.c_size_t(0)
    assert lib.edp_workspace_size(ctypes.byref(p), B.OP_EDP, ctypes.byref(one), ctypes.byref(n1)) == 0
    assert n1.value <= _ws(p, B.OP_EDP)[1]


def test_workspace_and_pointer_errors_are_host_side():
    lib = B.load()
    p = _prob()
    fake = ctypes.c_void_p(1 << 40)
    st, need = _ws(p, B.OP_EDP)
    assert st == 0
    # too small, misaligned, null: rejected before any launch
    assert lib.edp_solve(ctypes.byref(p), None, fake, fake, fake, fake, fake, need - 1, None) == -3
    assert lib.edp_solve(ctypes.byref(p), None, fake, fake, fake, fake, ctypes.c_void_p((1 << 40) + 8), need,
                         None) == -3
    assert lib.edp_solve(ctypes.byref(p), None, fake, fake, fake, None, None, need, None) == -3
    assert lib.edp_solve(ctypes.byref(p), None, None, fake, fake, fake, fake, need, None) == -1
    assert lib.edp_dp_scanline(ctypes.byref(p), None, fake, None, None, None, fake, 1 << 30, None) == -1
    assert lib.edp_energy(ctypes.byref(p), fake, fake, 2, fake, None, None) == -1
    assert lib.edp_solve(None, None, fake, fake, fake, fake, fake, need, None) == -1


def test_window_shift_codes_fit_eight_bits():
    # neighbouring window centres differ by up to q - win labels, kept as int8 frame shifts
    lib = B.load()
    n = ctypes.c_size_t(0)
    ok = _prob(width=12, height=10, qx=134, qy=9, dtype=2, cost_bound=100, lam=5, trunc=3)
    assert lib.edp_window_workspace_size(ctypes.byref(ok), 7, None, ctypes.byref(n)) == 0
    wide = _prob(width=12, height=10, qx=135, qy=9, dtype=2, cost_bound=100, lam=5, trunc=3)
    assert lib.edp_window_workspace_size(ctypes.byref(wide), 7, None, ctypes.byref(n)) == -5
    tall = _prob(width=12, height=10, qx=9, qy=135, dtype=2, cost_bound=100, lam=5, trunc=3)
    assert lib.edp_window_workspace_size(ctypes.byref(tall), 7, None, ctypes.byref(n)) == -5


def test_status_word_check_raises_on_timeout():
    import torch
    B.check_status(torch.zeros(3, dtype=torch.int32))
    B.check_status(0)
    with pytest.raises(B.EdpError) as e:
        B.check_status(torch.tensor([0, B.EDP_E_TIMEOUT, 0], dtype=torch.int32), "batch")
    assert e.value.status == B.EDP_E_TIMEOUT and "gave up" in str(e.value)
    with pytest.raises(B.EdpError):
        B.check_status(B.EDP_E_TIMEOUT)


def _items(probs, fake=1 << 40):
    items = (B.BatchItem * len(probs))()
    for i, p in enumerate(probs):
        items[i].problem = p
        items[i].d_cost = fake
        items[i].d_labels = fake + (1 << 30)
        items[i].d_energy = None
        items[i].d_status = None
        items[i].tuning = B.Tuning(-1, 0, 0, 0, 0, None, 0)
    return items


def test_batch_workspace_and_host_side_errors():
    lib = B.load()
    n = ctypes.c_size_t(0)
    probs = [_prob(width=160, height=120, qx=16), _prob(width=640, height=480, qx=64),
             _prob(width=320, height=240, qx=15, qy=15, dtype=2, cost_bound=2500, lam=15, trunc=3)]
    items = _items(probs)
    assert lib.edp_batch_workspace_size(3, items, ctypes.byref(n)) == 0
    single = sum(_ws(p, B.OP_EDP)[1] for p in probs)
    # every instance's arrays plus a descriptor table; only the control words are shared differently
    assert n.value >= single - 3 * 4096
    assert lib.edp_batch_workspace_size(0, items, ctypes.byref(n)) == -1
    assert lib.edp_batch_workspace_size(3, None, ctypes.byref(n)) == -1
    assert lib.edp_batch_workspace_size(3, items, None) == -1
    bad = _items(probs[:1] + [_prob(trunc=0)])
    assert lib.edp_batch_workspace_size(2, bad, ctypes.byref(n)) == -1
    nocost = _items(probs)
    nocost[1].d_cost = None
    assert lib.edp_batch_workspace_size(3, nocost, ctypes.byref(n)) == -1
    wide = _items([_prob(qx=40, qy=40, trunc=5)])          # no tile for the linear RMS at 40 x 40
    assert lib.edp_batch_workspace_size(1, wide, ctypes.byref(n)) == -5
    plan = ctypes.c_void_p(None)
    assert lib.edp_batch_workspace_size(3, items, ctypes.byref(n)) == 0
    fake = ctypes.c_void_p(1 << 40)
    assert lib.edp_batch_plan_create(3, items, None, n.value, None, ctypes.byref(plan)) == -3
    assert lib.edp_batch_plan_create(3, items, fake, n.value - 1, None, ctypes.byref(plan)) == -3
    assert lib.edp_batch_plan_create(3, items, fake, n.value, None, None) == -1
    assert plan.value is None
    assert lib.edp_batch_solve(None, None) == -1
    assert lib.edp_batch_plan_info(None, None, None) == -1
    lib.edp_batch_plan_destroy(None)


def test_static_workspace_solve_refuses_problems_beyond_its_array():
    # the 961-label motion workload needs gigabytes of workspace: refused on the host, before any
    # device work (no GPU needed)
    lib = B.load()
    fake = ctypes.c_void_p(1 << 40)
    big = _prob(width=640, height=480, qx=31, qy=31, dtype=2, cost_bound=2500, lam=15, trunc=3)
    assert lib.edp_solve_static(ctypes.byref(big), None, fake, fake, None, None, None) == -3
    assert lib.edp_solve_static(None, None, fake, fake, None, None, None) == -1
    bad = _prob(trunc=0)
    assert lib.edp_solve_static(ctypes.byref(bad), None, fake, fake, None, None, None) == -1


def test_three_label_dimensions_on_the_host():
    """qz > 1: the EDP solve takes 3D label spaces on the tiles of edp_tiles_3d (z inside a lane) and
    of edp_wide_tiles_3d (z across the wavefronts of a vertex);
    the DP calls and the label-window solve refuse them; qz = 0 means one or two dimensions."""
    assert B.tiles_3d(7, 7, 7) == [19]
    assert B.tiles_3d(4, 4, 4) == [19, 20, 21] and B.tiles_3d(8, 8, 4) == [19, 21]
    assert B.tiles_3d(9, 2, 2) == [] and B.tiles_3d(2, 2, 9) == []
    assert B.tile_info(19) == (8, 1, 8, 1) and B.tile_depth(19) == 8
    assert B.tile_depth(21) == 4 and B.tile_depth(16) == 1 and B.tile_depth(0) == 1
    # the wide-vertex tile of three label dimensions: 8 x 8 lanes, z over four wavefronts
    assert B.wide_tiles_3d(7, 7, 7) == [25] and B.wide_tiles_3d(8, 8, 8) == [25] and B.wide_tiles_3d(2, 2, 2) == [25]
    assert B.wide_tiles_3d(9, 1, 2) == [] and B.wide_tiles_3d(1, 1, 9) == []
    assert B.tile_info(25) == (8, 1, 8, 1) and B.tile_depth(25) == 8
    assert 25 not in B.wide_tiles(8, 8) and 25 not in B.tiles_3d(7, 7, 7)
    p3 = dict(qx=7, qy=7, qz=7, dtype=2, cost_bound=2500, lam=40, trunc=3)
    assert _ws(_prob(**p3), B.OP_EDP, 25)[0] == 0
    assert _ws(_prob(**{**p3, "trunc": 5}), B.OP_EDP, 25)[0] == -5   # wide tiles: window search, T <= 3
    st, n = _ws(_prob(**p3), B.OP_EDP)
    assert st == 0 and n >= 4 * 384 * 288 * 512 * 4
    assert _ws(_prob(**p3), B.OP_EDP, 19)[0] == 0
    assert _ws(_prob(**p3), B.OP_EDP, 21)[0] == -1        # 8 x 8 x 4 labels: qz = 7 does not fit
    assert _ws(_prob(**p3), B.OP_EDP, 13)[0] == -1        # a two-dimensional tile
    assert _ws(_prob(**p3), B.OP_EDP, 16)[0] == -1        # a wide tile
    assert _ws(_prob(**p3), B.OP_DP)[0] == -5
    assert _ws(_prob(**p3), 2)[0] == -5
    assert _ws(_prob(qx=9, qy=9, qz=5, dtype=2, cost_bound=2500), B.OP_EDP)[0] == -5   # no tile holds 9 x 9 x 5
    assert _ws(_prob(qx=16, qy=16, qz=17), B.OP_EDP)[0] == -1                          # 4352 labels
    # qz = 0 and qz = 1 are the same problem
    assert _ws(_prob(qz=0), B.OP_EDP) == _ws(_prob(qz=1), B.OP_EDP)
    n = ctypes.c_size_t(0)
    pw = _prob(prior=0, dtype=2, qx=15, qy=15, lam=15, trunc=3, cost_bound=2500, qz=2)
    assert B.load().edp_window_workspace_size(ctypes.byref(pw), 7, None, ctypes.byref(n)) == -5
