"""Pins of the oracle's steps of Algorithm 2 (Section 3.3) against library
brute force, exact invariants and sampling statistics."""
import numpy as np
import pytest
from scipy import stats
from scipy.spatial.distance import cdist

from paper_1203_6402_amd import synth


def _brute_nearest(X, C):
    D = cdist(np.asarray(X, np.float64), np.asarray(C, np.float64), "sqeuclidean")
    arg = np.argmin(D, axis=1)  # first occurrence = lowest index among equals
    srt = np.sort(D, axis=1)
    snd = srt[:, 1] if C.shape[0] > 1 else np.full(X.shape[0], np.inf)
    return arg, D[np.arange(X.shape[0]), arg], snd


@pytest.mark.parametrize("n,d,m", [(1, 1, 1), (37, 3, 5), (500, 15, 64), (300, 42, 129)])
def test_nearest_matches_cdist(orc, n, d, m):
    rng = np.random.default_rng(n + d + m)
    X = rng.normal(size=(n, d)) * np.exp(rng.normal(size=(1, d)))
    C = X[rng.integers(0, n, size=m)] + rng.normal(size=(m, d)) * 0.1
    a, d2, s = orc.nearest(X, C)
    ba, bd, bs = _brute_nearest(X, C)
    assert np.array_equal(a, ba)
    np.testing.assert_allclose(d2, bd, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(s, bs, rtol=1e-12, atol=1e-12)


def test_nearest_ties_take_lowest_index(orc):
    X = np.array([[0.0, 0.0], [2.0, 0.0]])
    C = np.array([[1.0, 0.0], [1.0, 0.0], [-1.0, 0.0], [3.0, 0.0]])
    a, d2, _ = orc.nearest(X, C)
    assert a.tolist() == [0, 0] and d2.tolist() == [1.0, 1.0]


def test_cost_definition(orc):
    rng = np.random.default_rng(3)
    X, C = rng.normal(size=(200, 7)), rng.normal(size=(9, 7))
    assert orc.cost(X, C) == pytest.approx(cdist(X, C, "sqeuclidean").min(axis=1).sum(), rel=1e-13)


def test_select_probabilities_and_clamp(orc):
    D2 = np.array([0.0, 1.0, 2.0, 7.0, 90.0])
    phi = D2.sum()
    sel, p, u = orc.select(D2, phi, 3.0, 11, 1)
    np.testing.assert_array_equal(p, np.minimum(1.0, 3.0 * D2 / phi))
    assert p[0] == 0.0 and not sel[0]          # D^2 = 0: never re-sampled
    assert p[-1] == 1.0 and sel[-1]            # clamped at 1: always kept
    np.testing.assert_array_equal(sel, u < p)
    sel0, p0, _ = orc.select(np.zeros(5), 0.0, 3.0, 11, 1)   # phi = 0: nothing kept
    assert not sel0.any() and not p0.any()


def test_select_inclusion_frequencies(orc):
    # Each point is kept independently with probability p_i (step 4):
    # per-point frequencies over seeds, and the count's mean sum(p) (Section 3.3:
    # Algorithm 2 keeps ell points per round in expectation).
    rng = np.random.default_rng(5)
    D2 = rng.exponential(size=40) ** 2
    phi, ell, S = D2.sum(), 6.0, 4000
    hits = np.zeros(40)
    cnts = []
    for s in range(S):
        sel, p, _ = orc.select(D2, phi, ell, s, 3)
        hits += sel
        cnts.append(sel.sum())
    z = (hits - S * p) / np.sqrt(S * p * (1 - p) + 1e-12)
    assert np.max(np.abs(z[(p > 0) & (p < 1)])) < 4.5
    assert np.all(hits[p == 1.0] == S)
    mean_z = (np.mean(cnts) - p.sum()) / np.sqrt((p * (1 - p)).sum() / S)
    assert abs(mean_z) < 4.5


def test_select_streams_independent_of_round_and_instance(orc):
    D2 = np.ones(1000)
    a, _, ua = orc.select(D2, 1000.0, 500.0, 0, 1, 0)
    b, _, ub = orc.select(D2, 1000.0, 500.0, 0, 2, 0)
    c, _, uc = orc.select(D2, 1000.0, 500.0, 0, 1, 1)
    assert abs(np.corrcoef(ua, ub)[0, 1]) < 0.15 and abs(np.corrcoef(ua, uc)[0, 1]) < 0.15
    assert not np.array_equal(a, b) and not np.array_equal(a, c)


def test_fold_equals_nearest_over_union(orc):
    rng = np.random.default_rng(8)
    X = rng.normal(size=(400, 6))
    D2 = np.full(400, np.inf)
    A = np.zeros(400, np.int64)
    ids = []
    for blk in (rng.choice(400, 1), rng.choice(400, 17), rng.choice(400, 40)):
        orc.fold(X, X[blk], len(ids), D2, A)
        ids.extend(blk.tolist())
    ba, bd, _ = _brute_nearest(X, X[np.asarray(ids)])
    assert np.array_equal(A, ba)
    np.testing.assert_allclose(D2, bd, rtol=1e-12, atol=0)


def test_weights_sum_to_n(orc):
    rng = np.random.default_rng(2)
    A = rng.integers(0, 50, size=1234)
    w = orc.weights(A, 60)
    assert w.sum() == 1234 and np.array_equal(w, np.bincount(A, minlength=60))


@pytest.mark.parametrize("ell,rounds", [(25.0, 5), (100.0, 5), (5.0, 15)])
def test_init_invariants(orc, ell, rounds):
    X = synth.gauss_mixture(3000, 15, 50, 10.0, seed=1)
    r = orc.kmeans_parallel_init(X, 50, ell, rounds, seed=4)
    phi = np.asarray(r.phi)
    assert np.all(np.diff(phi) <= 0)                           # C only grows
    assert len(set(r.cand_point.tolist())) == r.cand_point.size  # no re-sampling
    assert r.weights.sum() == X.shape[0]                       # step 7
    ba, bd, _ = _brute_nearest(X, X[r.cand_point])
    assert np.array_equal(r.assign, ba)
    np.testing.assert_allclose(r.d2, bd, rtol=1e-12)
    assert phi[-1] == pytest.approx(bd.sum(), rel=1e-12)
    assert sum(r.round_count) == r.cand_point.size
    assert len(set(r.picks.tolist())) == r.picks.size == 50
    np.testing.assert_array_equal(r.centers, X[r.cand_point[r.picks]].astype(np.float64))


def test_expected_round_size(orc):
    # Section 3.3 (Algorithm 2): each round keeps ell points in expectation (no
    # clamping here).
    X = synth.gauss_mixture(4000, 15, 50, 1.0, seed=2)
    counts = []
    for s in range(60):
        r = orc.kmeans_parallel_init(X, 10, 20.0, 3, seed=100 + s)
        counts.extend(r.round_count[1:])
    assert abs(np.mean(counts) - 20.0) < 4 * np.sqrt(20.0 / len(counts)) + 0.5


@pytest.mark.parametrize("shards", [1, 2, 7, 40])
def test_sharded_nearest_is_the_nearest(orc, shards):
    # Section 3.5: per-slice argmins reduced by the minimum give the nearest
    # center over all of them, ties (duplicated centers here) to the lowest id.
    rng = np.random.default_rng(shards)
    X = rng.normal(size=(700, 9))
    C = rng.normal(size=(40, 9))
    C[25] = C[3]
    C[31] = C[30]
    a, d2 = orc.nearest_sharded(X, C, shards)
    ba, bd, _ = _brute_nearest(X, C)
    assert np.array_equal(a, ba)
    np.testing.assert_array_equal(d2, orc.nearest(X, C)[1])
