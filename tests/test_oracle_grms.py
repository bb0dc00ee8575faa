"""Pins of the oracle's truncated squared prior and general RMS (no GPU).

The general recursive minimum search (GRMS, Sec. 3.1, eqs. derivation1,
derivation2, M_decmp1, M_decmp) replaces the search over all labels by one
window minimum of 2g - 1 entries per label dimension plus a clip.  It holds for
any increasing prior f; the paper runs it with the truncated squared prior
f(a) = a^2 (l_1 = 2 in Sec. 5.1, setups 2 and 4).  Expected values here are
hand-worked tables, a library distance transform, the straightforward search
(the definition), exhaustive enumeration and the operation counts of Table 1.
"""
import numpy as np
import pytest
from scipy import ndimage

import synth
from oracle import cref
from oracle import edp_ref as R

BIG = 10**6
QUAD = R.PRIOR_QUAD


def _impulse(qx, qy, vx, vy):
    h = np.full(qx * qy, BIG, np.int64)
    h[vy * qx + vx] = 0
    return h


@pytest.mark.parametrize("impl", ["py_sfms", "py_grms", "c_sfms", "c_grms"])
def test_squared_prior_impulse_response(impl):
    """M of an impulse is the prior itself, worked by hand from eq. Smooth_value_t with f(a) = a^2.

    qx = 4, qy = 3, impulse at (vx, vy) = (1, 1), lambda = 2, g = 2, so lambda f(g) = 8:
    per dimension 2 (min(ux^2, 4) + min(uy^2, 4)); joint 2 min(ux^2 + uy^2, 4).
    """
    h = _impulse(4, 3, 1, 1)
    per_dim = [4, 2, 4, 10,
               2, 0, 2, 8,
               4, 2, 4, 10]
    joint = [4, 2, 4, 8,
             2, 0, 2, 8,
             4, 2, 4, 8]
    for mode, expect in ((0, per_dim), (1, joint)):
        if impl == "py_sfms":
            got = R.min_search_sfms(h, 4, 3, 2, 2, mode, prior=QUAD)[0]
        elif impl == "py_grms":
            got = R.min_search_grms(h, 4, 3, 2, 2, mode, prior=QUAD)
        else:
            got = cref.min_search(h, 4, 3, 2, 2, mode, impl[2:], prior=QUAD)[0]
        assert list(got) == expect, (impl, mode)


def test_squared_prior_one_dimension_by_hand():
    """Stereo line of 7 labels, impulse at 3, lambda = 3, g = 3: 3 min(u^2, 9)."""
    h = _impulse(7, 1, 3, 0)
    expect = [27, 12, 3, 0, 3, 12, 27]
    assert list(R.min_search_grms(h, 7, 1, 3, 3, 1, prior=QUAD)) == expect
    assert list(cref.min_search(h, 7, 1, 3, 3, 0, "grms", prior=QUAD)[0]) == expect


def test_untruncated_squared_prior_is_the_euclidean_distance_transform():
    """With g beyond the label space the joint squared prior is lambda |u|^2, so M of a 0 / +inf
    indicator is lambda times the squared Euclidean distance to the nearest zero: scipy's exact
    distance transform, an implementation independent of the oracle."""
    rng = np.random.default_rng(5)
    for qx, qy in ((9, 7), (16, 1), (5, 12)):
        for _ in range(4):
            mask = rng.random((qy, qx)) < 0.15
            mask[rng.integers(0, qy), rng.integers(0, qx)] = True
            h = np.where(mask, 0, BIG).astype(np.int64).reshape(-1)
            d2 = np.rint(ndimage.distance_transform_edt(~mask) ** 2).astype(np.int64).reshape(-1)
            g = qx + qy
            lam = 3
            assert np.array_equal(R.min_search_grms(h, qx, qy, lam, g, 1, prior=QUAD), lam * d2)
            assert np.array_equal(cref.min_search(h, qx, qy, lam, g, 1, "grms", prior=QUAD)[0], lam * d2)


SHAPES = [(1, 1), (2, 1), (5, 1), (16, 1), (33, 1), (3, 3), (4, 2), (2, 5), (7, 5), (9, 9), (15, 15)]


@pytest.mark.parametrize("qx,qy", SHAPES)
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("prior", [0, 1])
def test_grms_equals_straightforward_search(qx, qy, mode, prior):
    """Sec. 3.1: the windowed per-dimension search gives the straightforward search's values,
    for the squared prior and (GRMS holds for any increasing f) the linear one; windows wider
    than the label space and g = 1 included."""
    rng = np.random.default_rng(qx * 100 + qy + 7 * mode + 31 * prior)
    for g in (1, 2, 3, 5, 40):
        for lam in (0, 1, 6):
            h = rng.integers(-80, 300, size=(3, qx * qy), dtype=np.int64)
            ref = R.min_search_sfms(h, qx, qy, lam, g, mode, prior=prior)[0]
            assert np.array_equal(R.min_search_grms(h, qx, qy, lam, g, mode, prior=prior), ref)
            assert np.array_equal(cref.min_search(h, qx, qy, lam, g, mode, "grms", prior=prior)[0], ref)
            assert np.array_equal(cref.min_search(h, qx, qy, lam, g, mode, "sfms", prior=prior)[0], ref)


def test_squared_prior_with_threshold_one_is_the_linear_one():
    """For g = 1 every nonzero label change costs lambda f(1) = lambda under both priors (a Potts
    prior), so the squared-prior GRMS equals the linear RMS with T = 1."""
    rng = np.random.default_rng(11)
    for qx, qy in ((6, 1), (4, 5)):
        for mode in (0, 1):
            h = rng.integers(0, 50, size=(5, qx * qy), dtype=np.int64)
            assert np.array_equal(R.min_search_grms(h, qx, qy, 7, 1, mode, prior=QUAD),
                                  R.min_search_lrms(h, qx, qy, 7, 1, mode))


def test_table1_general_rms_operation_counts():
    """Sec. 5.2 Table 1: GRMS costs R(2g - 1) operations per DSI vertex.

    Setup 4: 27 x 15 = 405 motion labels, g = 3, R = 2 -> 10 (printed 10).  Setup 2: 60 stereo
    labels, g = 3, R = 1 -> 5; the table prints 9 there, which R(2g - 1) gives only for g = 5
    (a misprint: the text of setup 2 states g = 3).  SFMS costs Q on both.
    """
    rng = np.random.default_rng(0)
    for (qx, qy), g, grms, sfms in (((27, 15), 3, 10, 405), ((60, 1), 3, 5, 60), ((60, 1), 5, 9, 60)):
        h = rng.integers(0, 100, size=(2, qx * qy), dtype=np.int64)
        c1, c2 = R.OpCounter(), R.OpCounter()
        R.min_search_sfms(h, qx, qy, 4, g, 1, counter=c1, prior=QUAD)
        R.min_search_grms(h, qx, qy, 4, g, 1, counter=c2, prior=QUAD)
        assert c1.per_vertex == sfms
        assert c2.per_vertex == grms


def test_squared_prior_energy_by_hand():
    """1 x 3 grid, 3 x 3 labels (vx, vy): (0,0), (2,1), (2,2) -> q = 0, 5, 8; costs 4, -1, 2."""
    cost = np.zeros((1, 3, 9), np.int32)
    cost[0, 0, 0], cost[0, 1, 5], cost[0, 2, 8] = 4, -1, 2
    lab = np.array([[0, 5, 8]])
    # per dimension, lambda 3, g 2 (f(g) = 4): pairs (2,1): 3(4 + 1) = 15, (0,1): 3(0 + 1) = 3
    assert R.energy(cost, lab, 3, 3, 3, 2, 0, False, prior=QUAD) == 5 + 15 + 3
    assert cref.energy(cost, lab, 3, 3, 3, 2, 0, False, prior=QUAD) == 5 + 15 + 3
    # joint, lambda 3, g 2: pairs 3 min(5, 4) = 12 and 3 min(1, 4) = 3
    assert R.energy(cost, lab, 3, 3, 3, 2, 1, False, prior=QUAD) == 5 + 12 + 3
    assert cref.energy(cost, lab, 3, 3, 3, 2, 1, False, prior=QUAD) == 5 + 12 + 3


CHAIN_CASES = [
    # W, qx, qy, lam, g, mode, lo, hi
    (5, 4, 1, 3, 2, 0, -20, 20),
    (6, 5, 1, 2, 3, 0, 0, 30),
    (7, 3, 1, 1, 9, 0, 0, 3),      # untruncated on this label range, heavy ties
    (5, 2, 2, 3, 2, 0, -9, 9),     # 2D label space, per dimension
    (5, 3, 2, 2, 2, 1, -9, 9),     # 2D label space, joint
]


@pytest.mark.parametrize("case", CHAIN_CASES)
def test_squared_prior_dp_matches_exhaustive_enumeration(case):
    """Scanline DP with the squared prior (Sec. 2 eq. base, Sec. 4.1): the optimum over all Q^W
    labellings, and the reverse-lexicographically smallest optimal labelling, for the straightforward
    search (Python and C) and the general RMS (C)."""
    W, qx, qy, lam, g, mode, lo, hi = case
    for seed in range(4):
        p = synth.random_problem(seed, W, 3, qx, qy, lam, g, mode, lo, hi)
        labels, row_e, tot = R.dp_scanline(p.cost, qx, qy, lam, g, mode, prior=QUAD)
        for y in range(3):
            best, canon = R.chain_exhaustive(p.cost[y], qx, qy, lam, g, mode, prior=QUAD)
            assert row_e[y] == best
            assert list(labels[y]) == list(canon)
        for search in ("sfms", "grms"):
            clab, crow, ctot = cref.dp_scanline(p.cost, qx, qy, lam, g, mode, search, prior=QUAD)
            assert ctot == tot and np.array_equal(clab, labels) and np.array_equal(crow, row_e)
        assert R.energy(p.cost, labels, qx, qy, lam, g, mode, False, prior=QUAD) == tot


@pytest.mark.parametrize("qx,qy,mode,j", [(4, 1, 0, 1), (6, 1, 0, 2), (3, 3, 0, 1), (3, 3, 1, 2), (4, 2, 1, 1)])
def test_squared_prior_edp_searches_agree(qx, qy, mode, j):
    """EDP (Algorithm 1) with the squared prior: Python straightforward search, C straightforward
    search and C general RMS give the same marginals and labels."""
    p = synth.random_problem(3, 5, 4, qx, qy, 4, 2, mode, -10, 40)
    ref = R.edp(p.cost, qx, qy, 4, 2, mode, iterations=j, search="sfms", prior=QUAD)
    for search in ("sfms", "grms"):
        got = cref.edp(p.cost, qx, qy, 4, 2, mode, iterations=j, search=search, marginal=True, prior=QUAD)
        assert np.array_equal(got["marginal"], ref["marginal"])
        assert np.array_equal(got["labels"], ref["labels"])
        assert got["energy"] == ref["energy"]


def test_squared_prior_edp_grid_bounds():
    """EDP labels are a labelling of the grid: their 4-connected energy is at least the exhaustive
    minimum (tiny grids), and with lambda = 0 they are the per-pixel winners (Sec. 4.2)."""
    for seed in range(3):
        p = synth.random_problem(seed, 3, 2, 3, 1, 5, 2, 0, 0, 30)
        best = R.grid_exhaustive(p.cost, 3, 1, 5, 2, 0, prior=QUAD)
        got = cref.edp(p.cost, 3, 1, 5, 2, 0, search="grms", prior=QUAD)
        assert got["energy"] >= best
        zero = cref.edp(p.cost, 3, 1, 0, 2, 0, search="grms", prior=QUAD)
        assert np.array_equal(zero["labels"], R.wta(p.cost))


def test_linear_rms_refuses_the_squared_prior():
    with pytest.raises(ValueError):
        R.edp(np.zeros((2, 2, 3), np.int32), 3, 1, 1, 2, 0, search="lrms", prior=QUAD)
    with pytest.raises(RuntimeError):
        cref.min_search(np.zeros((1, 3), np.int64), 3, 1, 1, 2, 0, "lrms", prior=QUAD)


def test_squared_prior_min_marginals():
    """Sec. 4.1 eq. DP_1D_3 with the squared prior: min_v S_Omega(x, v) is the chain optimum at every
    x (exhaustive enumeration), and its argmin is the optimal labelling where that is unique."""
    for seed in range(4):
        p = synth.random_problem(seed, 6, 2, 4, 1, 3, 3, 0, 0, 40)
        for y in range(2):
            best, canon = R.chain_exhaustive(p.cost[y], 4, 1, 3, 3, 0, prior=QUAD)
            marg = R.dp_min_marginals(p.cost[y], 4, 1, 3, 3, 0, prior=QUAD)
            assert (marg.min(axis=1) == best).all()
            srt = np.sort(marg, axis=1)
            if (srt[:, 0] < srt[:, 1]).all():
                assert list(np.argmin(marg, axis=1)) == list(canon)
