"""Pins of the oracle against what the paper and the mathematics fix:
exact pick distributions of (weighted) k-means++ (Algorithm 1), the k-means++
special case of k-means|| (Section 5.3), Theorem 2 by exact enumeration,
Corollary 3 by Monte Carlo, Lloyd's iteration against scikit-learn, and the
GaussMixture medians of Table 1 (ballpark)."""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

from paper_1203_6402_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _exact_kpp_sequences(C, w, k):
    """Probability of every ordered pick sequence of weighted k-means++,
    enumerated from its definition (first pick ~ w, then ~ w * D^2)."""
    m = C.shape[0]
    D = ((C[:, None, :] - C[None, :, :]) ** 2).sum(-1)
    out = {}

    def rec(seq, prob, E):
        if len(seq) == k:
            out[tuple(seq)] = prob
            return
        v = w * E
        T = v.sum()
        for j in range(m):
            if v[j] > 0:
                rec(seq + [j], prob * v[j] / T, D[j] if not seq else np.minimum(E, D[j]))

    rec([], 1.0, np.ones(m))
    return out


def _chi2_sequences(exact, observed, S):
    keys = sorted(exact)
    exp = np.array([exact[q] * S for q in keys])
    obs = np.array([observed.get(q, 0) for q in keys])
    assert sum(observed.values()) == obs.sum()      # no impossible sequence
    keep = exp >= 5
    obs_k = np.append(obs[keep], obs[~keep].sum())
    exp_k = np.append(exp[keep], exp[~keep].sum())
    if exp_k[-1] == 0:
        obs_k, exp_k = obs_k[:-1], exp_k[:-1]
    return stats.chisquare(obs_k, exp_k * obs_k.sum() / exp_k.sum()).pvalue


def test_weighted_kpp_pick_distribution(orc):
    rng = np.random.default_rng(0)
    C = rng.normal(size=(5, 2)) * 3
    w = np.array([3, 1, 0, 2, 5])
    exact = _exact_kpp_sequences(C, w.astype(float), 3)
    S = 30000
    obs = {}
    for s in range(S):
        picks, _, _ = orc.kpp_weighted(C, w, 3, seed=s)
        obs[tuple(picks.tolist())] = obs.get(tuple(picks.tolist()), 0) + 1
    assert all(2 not in q for q in obs)                   # zero weight never picked
    assert _chi2_sequences(exact, obs, S) > 1e-4


def test_weighted_kpp_matches_sklearn_distribution(orc):
    from sklearn.cluster import kmeans_plusplus
    rng = np.random.default_rng(1)
    C = rng.normal(size=(6, 3)) * 2
    w = np.array([1, 4, 2, 1, 3, 2], dtype=float)
    S = 8000
    mine, theirs = {}, {}
    for s in range(S):
        p, _, _ = orc.kpp_weighted(C, w, 2, seed=s)
        mine[tuple(p.tolist())] = mine.get(tuple(p.tolist()), 0) + 1
        _, idx = kmeans_plusplus(C, 2, sample_weight=w, random_state=s, n_local_trials=1)
        theirs[tuple(idx.tolist())] = theirs.get(tuple(idx.tolist()), 0) + 1
    keys = sorted(set(mine) | set(theirs))
    table = np.array([[mine.get(q, 0) for q in keys], [theirs.get(q, 0) for q in keys]])
    table = table[:, table.sum(0) >= 10]
    assert stats.chi2_contingency(table)[1] > 1e-4


def test_kmeans_parallel_reduces_to_kmeanspp(orc):
    # Section 5.3: with every point kept in one round (ell large enough that
    # p = 1 for every point with D^2 > 0), C = X, w = 1 and the recluster is
    # Algorithm 1 on X -- compared with the exact pick-sequence law.
    rng = np.random.default_rng(2)
    X = rng.normal(size=(5, 2)) * 2
    exact = _exact_kpp_sequences(X, np.ones(5), 3)
    S = 20000
    obs = {}
    for s in range(S):
        r = orc.kmeans_parallel_init(X, 3, ell=1e12, rounds=1, seed=s)
        assert sorted(r.cand_point.tolist()) == list(range(5))
        assert np.all(r.weights == 1)
        q = tuple(r.cand_point[r.picks].tolist())
        obs[q] = obs.get(q, 0) + 1
    assert _chi2_sequences(exact, obs, S) > 1e-4


def _optimal_cost(X, k):
    """phi* by enumerating every labelling (optimal centers are centroids)."""
    n = X.shape[0]
    best = np.inf
    for lab in itertools.product(range(k), repeat=n - 1):
        lab = np.array((0,) + lab)
        c = 0.0
        for j in range(k):
            P = X[lab == j]
            if len(P):
                c += ((P - P.mean(0)) ** 2).sum()
        best = min(best, c)
    return best


def _alpha(ell, k):
    return math.exp(-(1.0 - math.exp(-ell / (2.0 * k))))


@pytest.mark.parametrize("seed,ell", [(0, 1.0), (1, 2.0), (2, 4.0)])
def test_theorem2_exact_expectation(orc, seed, ell):
    # Theorem 2: E[phi(C u C')] <= 8 phi* + (1+alpha)/2 phi(C), with the
    # expectation taken exactly over all 2^n outcomes of one round.
    rng = np.random.default_rng(seed)
    k = 2
    X = np.concatenate([rng.normal(size=(4, 2)), rng.normal(size=(5, 2)) + 6.0])
    n = X.shape[0]
    i0 = orc.first_center(n, seed)
    _, D2, _ = orc.nearest(X, X[i0:i0 + 1])
    phi = orc.total(D2)
    _, p, _ = orc.select(D2, phi, ell, seed, 1)
    E = 0.0
    for mask in range(1 << n):
        sel = np.array([(mask >> i) & 1 for i in range(n)], bool)
        pr = np.prod(np.where(sel, p, 1 - p))
        if pr == 0:
            continue
        E += pr * orc.cost(X, X[np.append([i0], np.nonzero(sel)[0])])
    opt = _optimal_cost(X, k)
    a = _alpha(ell, k)
    assert E <= 8 * opt + (1 + a) / 2 * phi + 1e-9


def test_corollary3_monte_carlo(orc):
    # Corollary 3: E[phi^(i)] <= ((1+alpha)/2)^i psi + 16/(1-alpha) phi*.
    # phi* is bounded above by the cost of the generating centers.
    k, ell = 6, 12.0
    rng = np.random.default_rng(4)
    centers = rng.normal(size=(k, 3)) * 30
    lab = rng.integers(0, k, size=600)
    X = centers[lab] + rng.normal(size=(600, 3))
    opt_ub = sum(((X[lab == j] - X[lab == j].mean(0)) ** 2).sum() for j in range(k))
    a = _alpha(ell, k)
    S = 300
    phis = np.array([orc.kmeans_parallel_init(X, k, ell, 4, seed=s).phi for s in range(S)])
    psi_mean = phis[:, 0].mean()
    for i in range(1, 5):
        bound = ((1 + a) / 2) ** i * psi_mean + 16 / (1 - a) * opt_ub
        assert phis[:, i].mean() <= bound


def test_lloyd_matches_sklearn(orc):
    from sklearn.cluster import KMeans
    X = synth.gauss_mixture(2000, 15, 8, 20.0, seed=3).astype(np.float64)
    C0 = X[np.random.default_rng(0).choice(2000, 8, replace=False)]
    C = C0.copy()
    prev = np.inf
    for it in range(1, 6):
        C, a, phi_in = orc.lloyd_step(X, C)
        assert phi_in <= prev * (1 + 1e-12)      # Lloyd never increases the cost
        prev = phi_in
        km = KMeans(n_clusters=8, init=C0, n_init=1, max_iter=it, tol=0.0,
                    algorithm="lloyd").fit(X)
        np.testing.assert_allclose(C, km.cluster_centers_, rtol=1e-10, atol=1e-10)


def test_lloyd_empty_cluster_keeps_center(orc):
    X = np.array([[0.0], [1.0], [10.0]])
    C = np.array([[0.5], [11.0], [100.0]])
    Cn, a, _ = orc.lloyd_step(X, C)
    assert a.tolist() == [0, 0, 1]
    assert Cn.tolist() == [[0.5], [10.0], [100.0]]


def test_table1_gaussmixture_ballpark(orc):
    # Table 1 (R=10, k=50, ell=2k, r=5): medians over 11 runs, in units of
    # 1e4.  Different data draw and RNG: only the scale is compared.
    with open(os.path.join(GOLDEN, "table1_gaussmixture.json")) as f:
        g = json.load(f)["kmeans_par_ell_2k"]["R=10"]
    X = synth.gauss_mixture(10000, 15, 50, 10.0, seed=0)
    seeds, finals = [], []
    for s in range(11):
        r = orc.kmeans_parallel_init(X, 50, 100.0, 5, seed=s)
        seeds.append(orc.cost(X, r.centers) / 1e4)
        C = r.centers
        for _ in range(20):
            C, _, _ = orc.lloyd_step(X, C)
        finals.append(orc.cost(X, C) / 1e4)
    assert 0.5 * g["seed"] <= np.median(seeds) <= 2.0 * g["seed"]
    assert 0.5 * g["final"] <= np.median(finals) <= 2.0 * g["final"]
    assert np.median(finals) <= np.median(seeds)
