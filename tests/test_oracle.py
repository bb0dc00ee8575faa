"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test names the passage it rests on.  The expected values are closed forms,
hand-worked examples (tests/golden), exhaustive enumeration or properties of
the definitions -- never the oracle's own formula retyped.
"""
import itertools
import json
import os

import numpy as np
import pytest

import synth
from oracle import cref
from oracle import edp_ref as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
BIG = 10**6


# ---------------------------------------------------------------------------
# the minimum search operator M (Sec. 2 eq. M_strf; Sec. 3)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("impl", ["py_sfms", "py_lrms", "c_sfms", "c_lrms"])
def test_min_search_impulse_response_is_the_prior(impl):
    """M of an impulse at v0 is V(v - v0): hand-written tables for both truncation modes.

    qx = 4, qy = 3, v0 = (vx, vy) = (1, 1), lambda = 2, T = 2 (Sec. 2 eq. Smooth_value_t).
    """
    h = np.full(12, BIG, np.int64)
    h[1 * 4 + 1] = 0
    per_dim = [4, 2, 4, 6,
               2, 0, 2, 4,
               4, 2, 4, 6]
    joint = [4, 2, 4, 4,
             2, 0, 2, 4,
             4, 2, 4, 4]
    for mode, expect in ((0, per_dim), (1, joint)):
        if impl == "py_sfms":
            got = R.min_search_sfms(h, 4, 3, 2, 2, mode)[0]
        elif impl == "py_lrms":
            got = R.min_search_lrms(h, 4, 3, 2, 2, mode)
        else:
            got = cref.min_search(h, 4, 3, 2, 2, mode, impl[2:])[0]
        assert list(got) == expect, (impl, mode)


def _random_vectors(rng, n, q, lo, hi):
    return rng.integers(lo, hi + 1, size=(n, q), dtype=np.int64)


SHAPES = [(1, 1), (2, 1), (5, 1), (16, 1), (33, 1), (3, 3), (4, 2), (2, 5), (7, 5), (9, 9)]


@pytest.mark.parametrize("qx,qy", SHAPES)
@pytest.mark.parametrize("mode", [0, 1])
def test_lrms_equals_straightforward_search(qx, qy, mode):
    """Sec. 1 / Sec. 3: the fast RMS gives the same result as the straightforward search.

    Covers negative entries, heavy ties, lambda = 0, T >= Q and Qx != Qy.
    """
    rng = np.random.default_rng(qx * 100 + qy * 10 + mode)
    cases = []
    for lam, trunc, lo, hi in [(3, 2, -50, 50), (0, 1, -5, 5), (7, 40, 0, 3), (1, 1, 0, 1),
                               (20, 3, -1000, 1000)]:
        cases.append((lam, trunc, _random_vectors(rng, 40, qx * qy, lo, hi)))
    for lam, trunc, h in cases:
        ref, _ = R.min_search_sfms(h, qx, qy, lam, trunc, mode)
        assert np.array_equal(R.min_search_lrms(h, qx, qy, lam, trunc, mode), ref)
        assert np.array_equal(cref.min_search(h, qx, qy, lam, trunc, mode, "lrms")[0], ref)
        cv, ca = cref.min_search(h, qx, qy, lam, trunc, mode, "sfms")
        assert np.array_equal(cv, ref)
        assert np.array_equal(ca, R.min_search_sfms(h, qx, qy, lam, trunc, mode)[1])


@pytest.mark.parametrize("mode", [0, 1])
def test_min_search_invariants(mode):
    """Properties fixed by the definition M(h)(v) = min_v' h(v') + V(v - v'), V >= 0, V(0) = 0.

    min h <= M(h) <= h;  M(h) <= min h + lambda * f(T) (the clip, Sec. 3.1 eq. derivation1);
    M(h + c) = M(h) + c;  h <= g elementwise implies M(h) <= M(g).
    """
    rng = np.random.default_rng(5 + mode)
    qx, qy, lam, trunc = 6, 4, 5, 2
    h = _random_vectors(rng, 200, qx * qy, -300, 300)
    m = R.min_search_sfms(h, qx, qy, lam, trunc, mode)[0]
    hmin = h.min(axis=1, keepdims=True)
    cap = lam * trunc * (2 if mode == 0 else 1)
    assert (m <= h).all() and (m >= hmin).all() and (m <= hmin + cap).all()
    assert np.array_equal(R.min_search_sfms(h + 17, qx, qy, lam, trunc, mode)[0], m + 17)
    g = h + rng.integers(0, 20, size=h.shape)
    assert (R.min_search_sfms(g, qx, qy, lam, trunc, mode)[0] >= m).all()


def test_min_search_ties_take_smallest_index():
    """Tie-break reading: argM takes the smallest flat v' (lambda = 0: everything ties)."""
    h = np.zeros(6, np.int64)
    _, arg = R.min_search_sfms(h, 6, 1, 0, 1, 0)
    assert list(arg) == [0] * 6
    _, arg = R.min_search_sfms(h, 6, 1, 3, 2, 0)       # lambda > 0: v' = v is the unique best
    assert list(arg) == list(range(6))
    h = np.array([4, 1, 9, 1, 5], np.int64)             # lambda = 1: ties at distance
    _, arg = R.min_search_sfms(h, 5, 1, 1, 5, 0)
    # v = 2: candidates 1 + 1 (v'=1), 1 + 1 (v'=3) -> smallest index 1
    assert list(arg) == [1, 1, 1, 3, 3]


def test_table1_operation_counts():
    """Sec. 5.2 Table 1: ops per DSI vertex -- SFMS 60 / 405, LRMS 3 (R = 1) / 6 (R = 2).

    Setup 1: 60 stereo labels.  Setup 3: +-13 x +-7 motion = 27 x 15 = 405 labels.
    """
    rng = np.random.default_rng(0)
    for (qx, qy), sfms, lrms in (((60, 1), 60, 3), ((27, 15), 405, 6)):
        h = _random_vectors(rng, 3, qx * qy, 0, 100)
        c1, c2 = R.OpCounter(), R.OpCounter()
        R.min_search_sfms(h, qx, qy, 4, 3, 1, counter=c1)
        R.min_search_lrms(h, qx, qy, 4, 3, 1, counter=c2)
        assert c1.per_vertex == sfms
        assert c2.per_vertex == lrms


# ---------------------------------------------------------------------------
# energy (Sec. 2 eq. GE_objective_function)
# ---------------------------------------------------------------------------

def test_energy_hand_examples():
    """Energies worked by hand for per-dimension and joint truncation."""
    # 1 x 2 grid, 3 x 3 labels; labels (vx,vy) = (0,0) and (2,2) -> q = 0 and 8.
    cost = np.zeros((1, 2, 9), np.int32)
    cost[0, 0, 0] = 5
    cost[0, 1, 8] = -2
    lab = np.array([[0, 8]])
    # per-dim lambda=2, T=1: 5 - 2 + 2*(min(2,1)+min(2,1)) = 7
    assert R.energy(cost, lab, 3, 3, 2, 1, 0, False) == 7
    assert cref.energy(cost, lab, 3, 3, 2, 1, 0, False) == 7
    # joint lambda=2, T=3: 5 - 2 + 2*min(4,3) = 9
    assert R.energy(cost, lab, 3, 3, 2, 3, 1, False) == 9
    assert cref.energy(cost, lab, 3, 3, 2, 3, 1, False) == 9
    # 2 x 2 grid of the worked EDP example, labels [[0,1],[1,1]]: 3 (data) + 1 + 1 = 5
    g = json.load(open(os.path.join(GOLDEN, "edp_worked_2x2_q2.json")))
    c = np.array(g["cost_yxq"])
    assert R.energy(c, np.array(g["labels_yx"]), 2, 1, 1, 1, 0, True) == 5
    assert R.energy(c, np.array(g["labels_yx"]), 2, 1, 1, 1, 0, False) == 4


# ---------------------------------------------------------------------------
# scanline DP (Sec. 2 eq. One_d, eq. base; Sec. 4.1)
# ---------------------------------------------------------------------------

CHAIN_CASES = [
    # W, qx, qy, lam, T, mode, lo, hi
    (1, 3, 1, 5, 1, 0, -10, 10),
    (2, 2, 1, 3, 1, 0, 0, 9),
    (5, 3, 1, 4, 2, 0, -20, 20),
    (6, 4, 1, 7, 2, 0, 0, 30),
    (7, 4, 1, 2, 5, 0, 0, 3),      # heavy ties
    (7, 2, 1, 0, 1, 0, 0, 5),      # lambda = 0
    (5, 2, 2, 3, 1, 0, -9, 9),     # 2D label space, per dimension
    (5, 2, 2, 3, 2, 1, -9, 9),     # 2D label space, joint
    (4, 3, 1, 6, 9, 0, 0, 40),     # T beyond the label range
]


@pytest.mark.parametrize("case", CHAIN_CASES)
def test_dp_matches_exhaustive_enumeration(case):
    """The DP optimum equals the minimum over all Q^W labellings (Sec. 4.1 eq. DP_1D_2), and the
    backtracked labels are the reverse-lexicographically smallest optimal labelling."""
    W, qx, qy, lam, trunc, mode, lo, hi = case
    for seed in range(6):
        p = synth.random_problem(seed, W, 3, qx, qy, lam, trunc, mode, lo, hi)
        labels, row_e, tot = R.dp_scanline(p.cost, qx, qy, lam, trunc, mode)
        clab, crow, ctot = cref.dp_scanline(p.cost, qx, qy, lam, trunc, mode, "sfms")
        llab, lrow, ltot = cref.dp_scanline(p.cost, qx, qy, lam, trunc, mode, "lrms")
        for y in range(3):
            best, canon = R.chain_exhaustive(p.cost[y], qx, qy, lam, trunc, mode)
            assert row_e[y] == best
            assert list(labels[y]) == list(canon)
        assert ctot == tot and ltot == tot
        assert np.array_equal(clab, labels) and np.array_equal(llab, labels)
        assert R.energy(p.cost, labels, qx, qy, lam, trunc, mode, False) == tot


def test_dp_min_marginal_invariant():
    """Sec. 4.1 eq. DP_1D_3: min_v S_Omega(x, v) equals the chain optimum at every x, and at a
    unique optimum its argmin is the optimal label (eq. DP_1D_5)."""
    p = synth.chain_problem(3, W=20, H=6, Q=6)
    labels, row_e, _ = R.dp_scanline(p.cost, p.qx, 1, p.lam, p.trunc, 0)
    for y in range(p.height):
        marg = R.dp_min_marginals(p.cost[y], p.qx, 1, p.lam, p.trunc, 0)
        assert (marg.min(axis=1) == row_e[y]).all()
        srt = np.sort(marg, axis=1)
        uniq = srt[:, 0] < srt[:, 1]
        if uniq.all():
            assert np.array_equal(np.argmin(marg, axis=1), labels[y])


def test_dp_chain_workload_c_matches_python():
    p = synth.workload("chain64x48")
    a = R.dp_scanline(p.cost, p.qx, p.qy, p.lam, p.trunc, p.mode)
    b = cref.dp_scanline(p.cost, p.qx, p.qy, p.lam, p.trunc, p.mode, "lrms")
    assert a[2] == b[2] and np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ---------------------------------------------------------------------------
# EDP (Sec. 4.2, Algorithm 1)
# ---------------------------------------------------------------------------

def test_edp_hand_worked_example():
    """Every sum after every scan, the marginal, the labels and the energy of a 2 x 2 example
    worked by hand from eq. DP_2D_base / DP_2D_1 / DP_2D_2 (tests/golden/edp_worked_2x2_q2.json)."""
    g = json.load(open(os.path.join(GOLDEN, "edp_worked_2x2_q2.json")))
    p = g["grid"]
    cost = np.array(g["cost_yxq"], np.int64)
    seen = {}

    def trace(it, scan, sums):
        seen["P%d" % (scan + 1)] = {k: v.reshape(4, 2).tolist() for k, v in sums.items()}

    for search in ("sfms", "lrms"):
        seen.clear()
        r = R.edp(cost, p["qx"], p["qy"], p["lambda"], p["trunc"], p["mode"], 1, search, trace)
        assert seen == g["after_scan"]
        assert r["marginal"].reshape(4, 2).tolist() == g["marginal"]
        assert r["labels"].tolist() == g["labels_yx"]
        assert r["energy"] == g["energy"]
    for search in ("sfms", "lrms"):
        c = cref.edp(cost, p["qx"], p["qy"], p["lambda"], p["trunc"], p["mode"], 1, search, True)
        assert c["marginal"].reshape(4, 2).tolist() == g["marginal"]
        assert c["labels"].tolist() == g["labels_yx"] and c["energy"] == g["energy"]
    assert R.grid_exhaustive(cost, 2, 1, 1, 1, 0) == g["exhaustive_min_energy"]


@pytest.mark.parametrize("qx,qy,mode", [(5, 1, 0), (3, 3, 0), (3, 3, 1), (4, 2, 0)])
def test_edp_lambda_zero_is_winner_take_all(qx, qy, mode):
    """lambda = 0 makes M(h) the constant min h, so S_Omega = C + const per pixel and the
    EDP labels are the per-pixel smallest argmin of C (eq. DP_2D_1, eq. DP_2D_2)."""
    p = synth.random_problem(11, 7, 6, qx, qy, lam=0, trunc=2, mode=mode, lo=-40, hi=40)
    for j in (1, 2):
        r = R.edp(p.cost, qx, qy, 0, 2, mode, j)
        assert np.array_equal(r["labels"], R.wta(p.cost))
        c = cref.edp(p.cost, qx, qy, 0, 2, mode, j, "lrms")
        assert np.array_equal(c["labels"], R.wta(p.cost))


def test_edp_planted_constant_label():
    """A cost of 0 at one label everywhere and 500 elsewhere: the constant labelling has
    energy 0, the global minimum; EDP must return it."""
    H, W, qx, qy = 5, 6, 3, 3
    cost = np.full((H, W, qx * qy), 500, np.int32)
    cost[:, :, 4] = 0
    for mode in (0, 1):
        r = R.edp(cost, qx, qy, 9, 2, mode, 1)
        assert (r["labels"] == 4).all() and r["energy"] == 0
        c = cref.edp(cost, qx, qy, 9, 2, mode, 1, "lrms")
        assert (c["labels"] == 4).all() and c["energy"] == 0


def test_edp_single_pixel_is_winner_take_all():
    """One pixel: every neighbour is off the grid, so S_Omega = C."""
    cost = np.array([[[5, -3, 2, -3]]], np.int32)
    r = R.edp(cost, 4, 1, 3, 1, 0, 3)
    assert r["labels"].tolist() == [[1]] and r["energy"] == -3


@pytest.mark.parametrize("H,W,qx,qy,mode", [(2, 3, 3, 1, 0), (3, 3, 3, 1, 0), (2, 2, 2, 2, 0),
                                            (2, 2, 2, 2, 1), (3, 2, 2, 1, 0)])
def test_edp_energy_not_below_exhaustive_minimum(H, W, qx, qy, mode):
    """EDP is a heuristic (Sec. 4.2): its energy can never be below the exact 4-connected minimum."""
    for seed in range(4):
        p = synth.random_problem(seed, W, H, qx, qy, lam=6, trunc=2, mode=mode, lo=0, hi=30)
        e_star = R.grid_exhaustive(p.cost, qx, qy, 6, 2, mode)
        r = R.edp(p.cost, qx, qy, 6, 2, mode, 2)
        assert r["energy"] >= e_star


@pytest.mark.parametrize("qx,qy,mode,j", [(4, 1, 0, 1), (6, 1, 0, 2), (3, 3, 0, 1), (3, 3, 1, 2),
                                          (4, 3, 0, 1)])
def test_edp_python_and_c_agree(qx, qy, mode, j):
    """Two independently written literal EDPs (numpy and C), with both M implementations."""
    p = synth.random_problem(qx + 7 * qy + j, 9, 7, qx, qy, lam=8, trunc=2, mode=mode, lo=-20, hi=60)
    r = R.edp(p.cost, qx, qy, 8, 2, mode, j, "sfms")
    for search in ("sfms", "lrms"):
        c = cref.edp(p.cost, qx, qy, 8, 2, mode, j, search, marginal=True)
        assert np.array_equal(c["marginal"], r["marginal"])
        assert np.array_equal(c["labels"], r["labels"]) and c["energy"] == r["energy"]


def test_edp_beats_winner_take_all_and_improves_with_iterations():
    """Sec. 5.1: EDP lowers the energy far below the unsmoothed solution and further iterations
    keep lowering it on these seeded chain-like volumes (soft check on fixed seeds)."""
    p = synth.chain_problem(0, W=32, H=24, Q=16)
    e_wta = R.energy(p.cost, R.wta(p.cost), 16, 1, 20, 2, 0, True)
    es = [cref.edp(p.cost, 16, 1, 20, 2, 0, j, "lrms")["energy"] for j in (1, 2, 4)]
    assert es[0] < 0.9 * e_wta
    assert es[2] <= es[0]


def test_edp_sums_fit_int32_on_workloads():
    """The GPU keeps EDP sums in int32; the oracle checks the range on the stereo workload."""
    p = synth.workload("stereo384x288")
    c = cref.edp(p.cost, p.qx, p.qy, p.lam, p.trunc, p.mode, 2, "lrms")
    assert c["max_abs_sum"] < 2**31 // 16
