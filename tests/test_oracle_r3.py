"""Pins of the oracle over three label dimensions (no GPU).

Sec. 2 defines the energy for a disparity vector of any dimension R, and the
recursive searches of Sec. 3 apply one one-dimensional operator per label
dimension: the general RMS costs R(2g - 1) operations per vertex (Sec. 3.1),
the linear RMS 3R (Sec. 3.2, Sec. 5.2).  Here R = 3, labels flat as
q = (vz * qy + vy) * qx + vx.  Expected values are hand-worked tables, scipy's
distance transforms, the straightforward search (the definition), exhaustive
enumeration, the already pinned one- and two-dimensional searches (a label
space with a dimension of one label is a smaller one relabelled) and the
operation counts of Sec. 3 and Sec. 5.2.
"""
import numpy as np
import pytest
from scipy import ndimage

import synth
from oracle import cref
from oracle import edp_ref as R

BIG = 10**6
QUAD = R.PRIOR_QUAD

IMPLS = ["py_sfms", "py_lrms", "py_grms", "c_sfms", "c_lrms", "c_grms"]


def _search(impl, h, qx, qy, qz, lam, trunc, mode, prior=R.PRIOR_LINEAR):
    if impl == "py_sfms":
        return R.min_search_sfms(h, qx, qy, lam, trunc, mode, prior=prior, qz=qz)[0]
    if impl == "py_lrms":
        return R.min_search_lrms(h, qx, qy, lam, trunc, mode, qz=qz)
    if impl == "py_grms":
        return R.min_search_grms(h, qx, qy, lam, trunc, mode, prior=prior, qz=qz)
    return cref.min_search(h, qx, qy, lam, trunc, mode, impl[2:], prior=prior, qz=qz)[0]


@pytest.mark.parametrize("impl", IMPLS)
def test_impulse_response_by_hand(impl):
    """M of an impulse at (vx, vy, vz) = (1, 1, 0) in a 4 x 3 x 2 label space, lambda 2, T 2
    (Sec. 2 eq. Smooth_value_t), both truncation modes; tables worked by hand, slice vz = 0 first."""
    h = np.full(24, BIG, np.int64)
    h[(0 * 3 + 1) * 4 + 1] = 0
    per_dim = [4, 2, 4, 6,
               2, 0, 2, 4,
               4, 2, 4, 6,
               # vz = 1: one more step along z, 2 more
               6, 4, 6, 8,
               4, 2, 4, 6,
               6, 4, 6, 8]
    joint = [4, 2, 4, 4,
             2, 0, 2, 4,
             4, 2, 4, 4,
             # vz = 1: 2 min(|dx| + |dy| + 1, 2)
             4, 4, 4, 4,
             4, 2, 4, 4,
             4, 4, 4, 4]
    for mode, expect in ((0, per_dim), (1, joint)):
        assert list(_search(impl, h, 4, 3, 2, 2, 2, mode)) == expect, (impl, mode)


@pytest.mark.parametrize("impl", IMPLS)
def test_cube_impulse_by_hand(impl):
    """3 x 3 x 3 labels, impulse at the centre, lambda 3, T 2: a face neighbour is 1 step away,
    an edge neighbour 2, a corner 3.  Per dimension every step costs 3 (each |d| <= 1 < T);
    joint truncation caps the summed distance at 2."""
    h = np.full(27, BIG, np.int64)
    h[13] = 0
    out = np.asarray(_search(impl, h, 3, 3, 3, 3, 2, 0)).reshape(3, 3, 3)
    outj = np.asarray(_search(impl, h, 3, 3, 3, 3, 2, 1)).reshape(3, 3, 3)
    assert out[1, 1, 1] == 0 and outj[1, 1, 1] == 0
    for (z, y, x), steps in (((1, 1, 0), 1), ((0, 1, 1), 1), ((1, 0, 1), 1), ((0, 0, 1), 2), ((2, 1, 2), 2),
                             ((0, 0, 0), 3), ((2, 2, 2), 3), ((2, 0, 2), 3)):
        assert out[z, y, x] == 3 * steps, (impl, z, y, x)
        assert outj[z, y, x] == 3 * min(steps, 2), (impl, z, y, x)


def _random_vectors(rng, n, q, lo, hi):
    return rng.integers(lo, hi + 1, size=(n, q), dtype=np.int64)


SHAPES3 = [(2, 2, 2), (3, 4, 5), (1, 3, 4), (4, 1, 3), (1, 1, 6), (5, 2, 1), (7, 7, 7), (2, 9, 3)]


@pytest.mark.parametrize("qx,qy,qz", SHAPES3)
@pytest.mark.parametrize("mode", [0, 1])
def test_linear_rms_equals_straightforward_search(qx, qy, qz, mode):
    """Sec. 3.2: the linear RMS over three label dimensions gives the definition's values (Python
    and C), including lambda = 0, T beyond the label range, heavy ties and negative entries."""
    rng = np.random.default_rng(qx * 100 + qy * 10 + qz + 1000 * mode)
    for lam, trunc, lo, hi in [(3, 2, -50, 50), (0, 1, -5, 5), (7, 40, 0, 3), (1, 1, 0, 1), (20, 3, -1000, 1000)]:
        h = _random_vectors(rng, 12, qx * qy * qz, lo, hi)
        ref = R.min_search_sfms(h, qx, qy, lam, trunc, mode, qz=qz)[0]
        assert np.array_equal(R.min_search_lrms(h, qx, qy, lam, trunc, mode, qz=qz), ref)
        assert np.array_equal(cref.min_search(h, qx, qy, lam, trunc, mode, "lrms", qz=qz)[0], ref)
        cv, ca = cref.min_search(h, qx, qy, lam, trunc, mode, "sfms", qz=qz)
        assert np.array_equal(cv, ref)
        assert np.array_equal(ca, R.min_search_sfms(h, qx, qy, lam, trunc, mode, qz=qz)[1])


@pytest.mark.parametrize("qx,qy,qz", SHAPES3)
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("prior", [0, 1])
def test_general_rms_equals_straightforward_search(qx, qy, qz, mode, prior):
    """Sec. 3.1: one window operator per label dimension and the clip of eq. M_decmp give the
    definition's values for R = 3, with both priors."""
    rng = np.random.default_rng(7 + qx * 100 + qy * 10 + qz + 1000 * mode + 5000 * prior)
    for lam, g, lo, hi in [(3, 2, -50, 50), (5, 3, -200, 200), (2, 5, 0, 100), (0, 2, -5, 5), (4, 1, 0, 30)]:
        h = _random_vectors(rng, 10, qx * qy * qz, lo, hi)
        ref = R.min_search_sfms(h, qx, qy, lam, g, mode, prior=prior, qz=qz)[0]
        assert np.array_equal(R.min_search_grms(h, qx, qy, lam, g, mode, prior=prior, qz=qz), ref)
        assert np.array_equal(cref.min_search(h, qx, qy, lam, g, mode, "grms", prior=prior, qz=qz)[0], ref)


def test_untruncated_linear_prior_is_the_taxicab_distance_transform():
    """With T beyond the label space the joint linear prior is lambda |u|_1: M of a 0 / +inf
    indicator is lambda times scipy's exact 3D taxicab distance to the nearest zero, and with
    a T inside the range it is lambda min(distance, T)."""
    rng = np.random.default_rng(3)
    for qx, qy, qz in ((7, 5, 4), (3, 8, 6), (9, 1, 5)):
        for _ in range(3):
            mask = rng.random((qz, qy, qx)) < 0.1
            mask[rng.integers(0, qz), rng.integers(0, qy), rng.integers(0, qx)] = True
            h = np.where(mask, 0, BIG).astype(np.int64).reshape(-1)
            d = ndimage.distance_transform_cdt(~mask, metric="taxicab").astype(np.int64).reshape(-1)
            for trunc in (qx + qy + qz, 2):
                lam = 5
                expect = lam * np.minimum(d, trunc)
                assert np.array_equal(R.min_search_lrms(h, qx, qy, lam, trunc, 1, qz=qz), expect)
                assert np.array_equal(cref.min_search(h, qx, qy, lam, trunc, 1, "lrms", qz=qz)[0], expect)
                assert np.array_equal(cref.min_search(h, qx, qy, lam, trunc, 1, "grms", qz=qz)[0], expect)


def test_untruncated_squared_prior_is_the_euclidean_distance_transform():
    """With g beyond the label space the joint squared prior is lambda |u|^2: scipy's exact 3D
    Euclidean distance transform, squared."""
    rng = np.random.default_rng(4)
    for qx, qy, qz in ((6, 5, 4), (4, 7, 7)):
        for _ in range(3):
            mask = rng.random((qz, qy, qx)) < 0.12
            mask[rng.integers(0, qz), rng.integers(0, qy), rng.integers(0, qx)] = True
            h = np.where(mask, 0, BIG).astype(np.int64).reshape(-1)
            d2 = np.rint(ndimage.distance_transform_edt(~mask) ** 2).astype(np.int64).reshape(-1)
            g = qx + qy + qz
            assert np.array_equal(R.min_search_grms(h, qx, qy, 3, g, 1, prior=QUAD, qz=qz), 3 * d2)
            assert np.array_equal(cref.min_search(h, qx, qy, 3, g, 1, "grms", prior=QUAD, qz=qz)[0], 3 * d2)


def test_operation_counts_three_dimensions():
    """Sec. 3.1 and Sec. 3.2 (the counts of Table 1 for R = 3): SFMS Q, linear RMS 3R = 9, general
    RMS R(2g - 1) = 15 for g = 3 and 27 for g = 5, per DSI vertex."""
    rng = np.random.default_rng(0)
    for qx, qy, qz in ((7, 7, 7), (9, 9, 5)):
        h = _random_vectors(rng, 2, qx * qy * qz, 0, 100)
        c0, c1 = R.OpCounter(), R.OpCounter()
        R.min_search_sfms(h, qx, qy, 4, 3, 1, counter=c0, qz=qz)
        R.min_search_lrms(h, qx, qy, 4, 3, 1, counter=c1, qz=qz)
        assert c0.per_vertex == qx * qy * qz
        assert c1.per_vertex == 9
        for g, ops in ((3, 15), (5, 27)):
            c2 = R.OpCounter()
            R.min_search_grms(h, qx, qy, 4, g, 1, counter=c2, prior=QUAD, qz=qz)
            assert c2.per_vertex == ops


@pytest.mark.parametrize("mode", [0, 1])
def test_a_dimension_of_one_label_reduces_to_the_smaller_space(mode):
    """A label space (qx, 1, qz) is the two-dimensional (qx, qz) space under the same flat index,
    and (1, 1, qz) the one-dimensional (qz): the searches must agree with the pinned ones there."""
    rng = np.random.default_rng(21 + mode)
    h = _random_vectors(rng, 30, 5 * 4, -60, 60)
    for search in ("sfms", "lrms", "grms"):
        a = cref.min_search(h, 5, 1, 3, 2, mode, search, qz=4)[0]
        b = cref.min_search(h, 5, 4, 3, 2, mode, search)[0]
        assert np.array_equal(a, b), search
    h1 = _random_vectors(rng, 30, 6, -60, 60)
    assert np.array_equal(R.min_search_lrms(h1, 1, 1, 4, 2, mode, qz=6), R.min_search_lrms(h1, 6, 1, 4, 2, mode))
    assert np.array_equal(R.min_search_grms(h1, 1, 1, 4, 2, mode, prior=QUAD, qz=6),
                          R.min_search_grms(h1, 6, 1, 4, 2, mode, prior=QUAD))


@pytest.mark.parametrize("mode", [0, 1])
def test_searches_commute_with_label_axis_permutations(mode):
    """V is symmetric in the label dimensions, so relabelling the axes (x <-> z, y <-> z) of the
    input relabels the output.  A wrong stride or a dropped pass along one dimension breaks it."""
    rng = np.random.default_rng(31 + mode)
    qx, qy, qz = 4, 3, 5
    h = _random_vectors(rng, 8, qx * qy * qz, -80, 80)
    g = h.reshape(-1, qz, qy, qx)
    for search in ("lrms", "grms"):
        m = cref.min_search(h, qx, qy, 3, 2, mode, search, qz=qz)[0].reshape(-1, qz, qy, qx)
        hz = np.ascontiguousarray(np.transpose(g, (0, 3, 2, 1)))        # axes (vx, vy, vz) -> (z, y, x)
        mz = cref.min_search(hz.reshape(8, -1), qz, qy, 3, 2, mode, search, qz=qx)[0].reshape(-1, qx, qy, qz)
        assert np.array_equal(np.transpose(mz, (0, 3, 2, 1)), m), search
        hy = np.ascontiguousarray(np.transpose(g, (0, 2, 1, 3)))        # swap z and y
        my = cref.min_search(hy.reshape(8, -1), qx, qz, 3, 2, mode, search, qz=qy)[0].reshape(-1, qy, qz, qx)
        assert np.array_equal(np.transpose(my, (0, 2, 1, 3)), m), search


def test_energy_by_hand():
    """1 x 2 grid, 3 x 2 x 2 labels: (0, 0, 0) -> q = 0 and (2, 1, 1) -> q = (1 * 2 + 1) * 3 + 2 = 11,
    costs 5 and -2 (Sec. 2 eq. GE_objective_function)."""
    cost = np.zeros((1, 2, 12), np.int32)
    cost[0, 0, 0], cost[0, 1, 11] = 5, -2
    lab = np.array([[0, 11]])
    # per dimension, lambda 2, T 1: 2 (1 + 1 + 1) = 6
    assert R.energy(cost, lab, 3, 2, 2, 1, 0, False, qz=2) == 9
    assert cref.energy(cost, lab, 3, 2, 2, 1, 0, False, qz=2) == 9
    # joint, lambda 2, T 5: 2 min(2 + 1 + 1, 5) = 8; T 3: 2 * 3 = 6
    assert R.energy(cost, lab, 3, 2, 2, 5, 1, False, qz=2) == 11
    assert cref.energy(cost, lab, 3, 2, 2, 5, 1, False, qz=2) == 11
    assert cref.energy(cost, lab, 3, 2, 2, 3, 1, False, qz=2) == 9
    # squared prior, per dimension, lambda 1, g 2: min(4, 4) + 1 + 1 = 6
    assert R.energy(cost, lab, 3, 2, 1, 2, 0, False, prior=QUAD, qz=2) == 9
    assert cref.energy(cost, lab, 3, 2, 1, 2, 0, False, prior=QUAD, qz=2) == 9


CHAIN3 = [
    # W, qx, qy, qz, lam, T, mode, prior
    (4, 2, 2, 2, 3, 1, 0, 0),
    (4, 2, 2, 2, 3, 2, 1, 0),
    (3, 3, 1, 3, 4, 2, 0, 1),
    (5, 1, 2, 3, 2, 2, 1, 1),
]


@pytest.mark.parametrize("case", CHAIN3)
def test_dp_matches_exhaustive_enumeration(case):
    """Scanline DP over a three-dimensional label space equals the minimum over all Q^W labellings
    (Sec. 4.1), and its labels are the canonical optimal labelling."""
    W, qx, qy, qz, lam, trunc, mode, prior = case
    for seed in range(3):
        p = synth.random_problem(seed, W, 2, qx, qy, lam, trunc, mode, -9, 9, qz=qz)
        labels, row_e, tot = R.dp_scanline(p.cost, qx, qy, lam, trunc, mode, prior=prior, qz=qz)
        for search in (("sfms", "grms") if prior else ("sfms", "lrms", "grms")):
            cl, cr, ct = cref.dp_scanline(p.cost, qx, qy, lam, trunc, mode, search, prior=prior, qz=qz)
            assert ct == tot and np.array_equal(cl, labels), search
        for y in range(2):
            best, canon = R.chain_exhaustive(p.cost[y], qx, qy, lam, trunc, mode, prior=prior, qz=qz)
            assert row_e[y] == best and list(labels[y]) == list(canon)
        assert R.energy(p.cost, labels, qx, qy, lam, trunc, mode, False, prior=prior, qz=qz) == tot


@pytest.mark.parametrize("mode", [0, 1])
def test_edp_lambda_zero_is_winner_take_all(mode):
    """lambda = 0: M(h) is the constant min h, so EDP returns the per-pixel argmin (eq. DP_2D_2)."""
    p = synth.random_problem(5, 6, 5, 3, 2, lam=0, trunc=2, mode=mode, lo=-40, hi=40, qz=3)
    r = R.edp(p.cost, 3, 2, 0, 2, mode, 1, qz=3)
    assert np.array_equal(r["labels"], R.wta(p.cost))
    c = cref.edp(p.cost, 3, 2, 0, 2, mode, 2, "lrms", qz=3)
    assert np.array_equal(c["labels"], R.wta(p.cost))


def test_edp_planted_constant_label():
    """Cost 0 at one label everywhere, 500 elsewhere: the constant labelling (energy 0) is the
    global minimum and EDP returns it."""
    cost = np.full((4, 5, 3 * 3 * 3), 500, np.int32)
    cost[:, :, 14] = 0
    for mode in (0, 1):
        r = R.edp(cost, 3, 3, 9, 2, mode, 1, qz=3)
        assert (r["labels"] == 14).all() and r["energy"] == 0
        for search in ("lrms", "grms"):
            c = cref.edp(cost, 3, 3, 9, 2, mode, 1, search, qz=3)
            assert (c["labels"] == 14).all() and c["energy"] == 0


@pytest.mark.parametrize("mode", [0, 1])
def test_edp_energy_not_below_exhaustive_minimum(mode):
    """EDP is a heuristic (Sec. 4.2): its energy is never below the exact 4-connected minimum
    (2 x 2 grid, 2 x 1 x 2 labels: 256 labellings)."""
    for seed in range(4):
        p = synth.random_problem(seed, 2, 2, 2, 1, lam=6, trunc=2, mode=mode, lo=0, hi=30, qz=2)
        e_star = R.grid_exhaustive(p.cost, 2, 1, 6, 2, mode, qz=2)
        r = R.edp(p.cost, 2, 1, 6, 2, mode, 2, qz=2)
        assert r["energy"] >= e_star


@pytest.mark.parametrize("mode,prior,j", [(0, 0, 1), (1, 0, 2), (0, 1, 1), (1, 1, 2)])
def test_edp_python_and_c_agree(mode, prior, j):
    """Two independently written literal EDPs (numpy and C) with every search, R = 3."""
    qx, qy, qz = 3, 2, 4
    p = synth.random_problem(mode + 2 * prior + 4 * j, 6, 5, qx, qy, lam=8, trunc=2, mode=mode, lo=-20, hi=60, qz=qz)
    r = R.edp(p.cost, qx, qy, 8, 2, mode, j, "sfms", prior=prior, qz=qz)
    for search in (("sfms", "grms") if prior else ("sfms", "lrms", "grms")):
        c = cref.edp(p.cost, qx, qy, 8, 2, mode, j, search, marginal=True, prior=prior, qz=qz)
        assert np.array_equal(c["marginal"], r["marginal"]), search
        assert np.array_equal(c["labels"], r["labels"]) and c["energy"] == r["energy"]


def test_edp_one_label_along_y_is_the_two_dimensional_solve():
    """(qx, 1, qz) labels are the (qx, qz) space relabelled: the whole EDP solve must agree."""
    p = synth.random_problem(9, 7, 6, 4, 1, lam=6, trunc=2, mode=0, lo=-20, hi=40, qz=3)
    a = cref.edp(p.cost, 4, 1, 6, 2, 0, 2, "lrms", marginal=True, qz=3)
    b = cref.edp(p.cost, 4, 3, 6, 2, 0, 2, "lrms", marginal=True)
    assert np.array_equal(a["marginal"], b["marginal"]) and a["energy"] == b["energy"]


def test_offset_workload_labels_and_solve():
    """The three-dimensional workload: its planted labels lie in range, the oracle's EDP on a crop
    beats winner-take-all in energy by far and recovers most planted labels (soft check, fixed seed)."""
    p = synth.motion_offset_problem(0, W=96, H=64)
    assert p.q == 343 and p.cost.shape == (64, 96, 343)
    assert p.meta["gt"].min() >= 0 and p.meta["gt"].max() < 343
    c = p.cost[8:40, 8:56]
    gt = p.meta["gt"][8:40, 8:56]
    r = cref.edp(c, 7, 7, p.lam, p.trunc, p.mode, 2, "lrms", qz=7)
    e_wta = cref.energy(c, R.wta(c), 7, 7, p.lam, p.trunc, p.mode, True, qz=7)
    assert r["energy"] < 0.5 * e_wta
    assert (r["labels"] == gt).mean() > 0.5
