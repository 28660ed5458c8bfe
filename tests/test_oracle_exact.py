"""Pins of the oracle's exact-ell rounds (Section 5.3: exactly ell points per
round, drawn in proportion to D^2 without replacement), of k-means++ on all
of X (Algorithm 1) and of Lloyd's iteration run until the centers are stable
(Section 1): the laws of the draws against exact enumeration, the k-means++
special case of the exact-ell variant, scikit-learn's Lloyd, and the replay
bands of the new decisions."""
import itertools

import numpy as np
import pytest
from scipy import stats

from paper_1203_6402_amd import synth
from tests.test_oracle_rng import _numpy_block
from tests.test_oracle_theory import _chi2_sequences, _exact_kpp_sequences

EPS = 1e-6


def test_open_uniform_definition(orc):
    # V = ((w >> 11) + 1) 2^-53 in (0, 1], w word 0 of the block keyed
    # (seed, EXACT) at counter (i, t, inst, 0).
    rng = np.random.default_rng(4)
    for _ in range(200):
        seed, a, b, inst = (int(rng.integers(0, 2**63)), int(rng.integers(0, 2**40)),
                            int(rng.integers(0, 64)), int(rng.integers(0, 5000)))
        w = int(_numpy_block((seed, orc.TAG_EXACT), (a, b, inst, 0))[0])
        v = orc.uniform_open(seed, orc.TAG_EXACT, a, b, inst)
        assert v == ((w >> 11) + 1) * 2.0 ** -53 and 0.0 < v <= 1.0


def test_smallest_key_is_a_d2_draw(orc):
    # The argmin of the keys is point i with probability D2_i / sum D2: one
    # step of Algorithm 1.  Zero D^2 is never drawn.
    D2 = np.array([0.0, 1.0, 3.0, 0.5, 2.5, 0.0, 4.0])
    S = 40000
    cnt = np.zeros(D2.size)
    for s in range(S):
        cnt[np.argmin(orc.exact_keys(D2, s, 1))] += 1
    assert cnt[0] == cnt[5] == 0
    pos = D2 > 0
    assert stats.chisquare(cnt[pos], D2[pos] / D2.sum() * S).pvalue > 1e-4


def _successive_law(w, ell):
    """P(set) of ell draws without replacement, each in proportion to w among
    the items not yet drawn, enumerated over the orders."""
    out = {}
    for seq in itertools.permutations(range(len(w)), ell):
        p, rem = 1.0, w.sum()
        for j in seq:
            if w[j] == 0:
                p = 0.0
                break
            p *= w[j] / rem
            rem -= w[j]
        key = tuple(sorted(seq))
        out[key] = out.get(key, 0.0) + p
    return out


@pytest.mark.parametrize("ell", [2, 3])
def test_exact_round_subset_law(orc, ell):
    D2 = np.array([1.0, 0.0, 2.0, 4.0, 0.5, 3.0])
    law = _successive_law(D2, ell)
    S = 30000
    obs = {}
    for s in range(S):
        sel, key, tau = orc.select_exact(D2, ell, s, 2)
        assert sel.sum() == ell and not sel[1]
        assert tau == key[sel].max() and np.all(key[~sel] >= tau)
        q = tuple(np.nonzero(sel)[0].tolist())
        obs[q] = obs.get(q, 0) + 1
    assert all(law.get(q, 0.0) > 0 for q in obs)
    keys = sorted(q for q in law if law[q] > 0)
    o = np.array([obs.get(q, 0) for q in keys])
    e = np.array([law[q] * S for q in keys])
    assert stats.chisquare(o, e * o.sum() / e.sum()).pvalue > 1e-4


def test_exact_round_takes_every_positive_point_when_ell_exceeds_them(orc):
    D2 = np.array([0.0, 2.0, 0.0, 1.0])
    sel, _, _ = orc.select_exact(D2, 10, 3, 1)
    assert sel.tolist() == [False, True, False, True]
    sel, _, tau = orc.select_exact(np.zeros(4), 3, 3, 1)
    assert not sel.any() and tau == np.inf


def test_kmeanspp_pick_sequence_law(orc):
    # Algorithm 1 on all of X: the exact law of the ordered picks.
    X = np.random.default_rng(3).normal(size=(5, 2)) * 2
    exact = _exact_kpp_sequences(X, np.ones(5), 3)
    S = 20000
    obs = {}
    for s in range(S):
        p, phi, _, _ = orc.kmeanspp(X, 3, seed=s)
        obs[tuple(p.tolist())] = obs.get(tuple(p.tolist()), 0) + 1
        assert np.all(np.diff(phi) <= 0)
    assert _chi2_sequences(exact, obs, S) > 1e-4


@pytest.mark.parametrize("seed", [0, 5, 9])
def test_exact_variant_with_one_point_per_round_is_kmeanspp(orc, seed):
    # Section 5.3: with ell = 1 and r = k - 1 rounds the exact-ell variant
    # draws one point from the D^2 distribution per round -- k-means++.  With
    # the same draws the candidates are k-means++'s picks in order, and the
    # recluster of k candidates returns all of them.
    X = synth.gauss_mixture(2000, 6, 10, 10.0, seed=seed)
    k = 12
    r = orc.kmeans_parallel_init(X, k, 1, k - 1, seed, sampling="exact")
    p, phi, _, _ = orc.kmeanspp(X, k, seed)
    assert np.array_equal(r.cand_point, p)
    assert r.round_count == [1] * k and r.phi == phi
    assert sorted(r.cand_point[r.picks].tolist()) == sorted(p.tolist())


def test_exact_rounds_invariants(orc):
    X = synth.heavy_tailed(5000, 12, seed=6)
    r = orc.kmeans_parallel_init(X, 20, 40, 5, seed=2, sampling="exact")
    assert r.round_count == [1] + [40] * 5
    assert len(set(r.cand_point.tolist())) == r.cand_point.size
    assert np.all(np.diff(r.phi) <= 0) and r.weights.sum() == X.shape[0]


def test_exact_round_replay_band(orc):
    # A point on the other side of the round's threshold key tau is accepted
    # when its key lies within the band of tau, and only then.
    X = synth.gauss_mixture(3000, 4, 8, 10.0, seed=1)
    own = orc.kmeans_parallel_init(X, 8, 16, 1, seed=3, sampling="exact")
    i0 = orc.first_center(3000, 3)
    _, D2, _ = orc.nearest(X, X[i0:i0 + 1])
    sel, key, tau = orc.select_exact(D2, 16, 3, 1)
    out = np.nonzero(~sel & np.isfinite(key))[0]
    j = int(out[np.argmin(key[out])])          # the first key above the threshold
    delta = key[j] / tau - 1
    last = np.nonzero(sel)[0][np.argmax(key[sel])]    # j replaces the largest selected key
    inside = sorted(set(np.nonzero(sel)[0].tolist()) - {int(last)} | {j})
    r = orc.kmeans_parallel_init(X, 8, 16, 1, seed=3, sampling="exact",
                                 follow={"rounds": [np.array(inside)]}, band=delta * (1 + EPS))
    assert r.flags["draw"] == 2 and r.bad["draw"] == 0
    r = orc.kmeans_parallel_init(X, 8, 16, 1, seed=3, sampling="exact",
                                 follow={"rounds": [np.array(inside)]}, band=delta * (1 - EPS))
    assert r.bad["draw"] >= 1
    assert own.round_count == [1, 16]


def test_kmeanspp_replay_band(orc):
    X = synth.gauss_mixture(2000, 3, 6, 10.0, seed=2)
    p, _, nf, nb = orc.kmeanspp(X, 2, seed=4)
    assert nf == nb == 0
    i0 = p[0]
    _, D2, _ = orc.nearest(X, X[i0:i0 + 1])
    key = orc.exact_keys(D2, 4, 1)
    order = np.argsort(key)
    runner = int(order[1])
    delta = key[runner] / key[order[0]] - 1
    fol = [int(i0), runner]
    q, _, nf, nb = orc.kmeanspp(X, 2, seed=4, follow=fol, band=delta * (1 + EPS))
    assert (nf, nb) == (1, 0) and q[1] == runner
    _, _, nf, nb = orc.kmeanspp(X, 2, seed=4, follow=fol, band=delta * (1 - EPS))
    assert (nf, nb) == (0, 1)


def test_lloyd_until_stable_matches_sklearn(orc):
    # scikit-learn's Lloyd stops at "strict convergence" (labels unchanged)
    # and counts the iteration that found it: one more than the updates made.
    from sklearn.cluster import KMeans
    for seed in (1, 3):
        X = synth.gauss_mixture(3000, 15, 8, 20.0, seed=seed).astype(np.float64)
        C0 = X[np.random.default_rng(seed).choice(3000, 8, replace=False)]
        C, it, phis, _, _ = orc.lloyd_until_stable(X, C0, 300)
        km = KMeans(n_clusters=8, init=C0, n_init=1, max_iter=300, tol=0.0,
                    algorithm="lloyd").fit(X)
        assert it + 1 == km.n_iter_
        np.testing.assert_allclose(C, km.cluster_centers_, rtol=1e-10, atol=1e-10)
        assert all(phis[i + 1] <= phis[i] * (1 + 1e-12) for i in range(len(phis) - 1))
        assert phis[-1] == pytest.approx(orc.cost(X, C), rel=1e-12)


def test_lloyd_until_stable_respects_the_cap(orc):
    X = synth.gauss_mixture(3000, 15, 8, 20.0, seed=1).astype(np.float64)
    C0 = X[np.random.default_rng(1).choice(3000, 8, replace=False)]
    C, it, phis, _, _ = orc.lloyd_until_stable(X, C0, 3)
    C3 = C0
    for _ in range(3):
        C3, _, _ = orc.lloyd_step(X, C3)
    assert it == 3 and len(phis) == 4 and np.array_equal(C, C3)
