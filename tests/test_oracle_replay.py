"""Pins of the oracle's replay ("follow") acceptance and of the FP32 band it
uses.  The replay decides, for every GPU decision that differs from the FP64
oracle's, whether the difference lies inside the error band (flagged) or not
(bad); the GPU parity tests require bad == 0.  Here each kind of decision --
a round draw (Algorithm 2 step 4), a nearest-candidate argmin (step 7) and a
recluster pick (step 8, Algorithm 1 with weights) -- is made to differ just
inside and just outside its band, so that loosening or tightening any of the
comparisons turns a test red.  The band itself is pinned by measuring FP32
direct-form squared distances against exact ones."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

from paper_1203_6402_amd import synth

EPS = 1e-6   # relative step across a band boundary (far above FP64 rounding)


def _zero(d):
    return all(v == 0 for v in d.values())


def _own(orc, X, k, ell, rounds, seed):
    o = orc.kmeans_parallel_init(X, k, ell, rounds, seed)
    rounds_sets, start = [], 1
    for c in o.round_count[1:]:
        rounds_sets.append(o.cand_point[start:start + c])
        start += c
    return o, rounds_sets


def test_follow_own_decisions_flags_nothing(orc):
    X = synth.gauss_mixture(3000, 6, 12, 10.0, seed=11)
    o, rs = _own(orc, X, 12, 24.0, 4, seed=5)
    f = orc.kmeans_parallel_init(X, 12, 24.0, 4, seed=5,
                                 follow={"rounds": rs, "assign": o.assign, "picks": o.picks})
    assert _zero(f.flags) and _zero(f.bad)
    assert np.array_equal(f.cand_point, o.cand_point) and np.array_equal(f.picks, o.picks)


# ------------------------------------------------------------------ draws
def _closest_draw(orc, X, ell, seed):
    """Round-1 point whose draw lies closest to its probability (relative to p),
    among points with 0 < p < 1, and that relative margin."""
    i0 = orc.first_center(X.shape[0], seed)
    _, D2, _ = orc.nearest(X, X[i0:i0 + 1])
    phi = orc.total(D2)
    _, p, u = orc.select(D2, phi, ell, seed, 1)
    live = (p > 0) & (p < 1)
    rel = np.where(live, np.abs(u - p) / np.where(p > 0, p, 1.0), np.inf)
    i = int(np.argmin(rel))
    return i, float(rel[i])


def test_draw_difference_inside_band_is_flagged(orc):
    X = synth.gauss_mixture(4000, 5, 10, 10.0, seed=3)
    ell, seed = 20.0, 9
    o, rs = _own(orc, X, 5, ell, 1, seed)
    i, delta = _closest_draw(orc, X, ell, seed)
    other = set(rs[0].tolist()) ^ {i}          # the other side took the other decision at i
    follow = {"rounds": [np.array(sorted(other))]}
    inside = orc.kmeans_parallel_init(X, 5, ell, 1, seed, follow=follow, band=delta * (1 + EPS))
    assert inside.flags["draw"] == 1 and inside.bad["draw"] == 0
    assert (i in inside.cand_point) == (i not in o.cand_point)   # the followed decision is kept
    outside = orc.kmeans_parallel_init(X, 5, ell, 1, seed, follow=follow, band=delta * (1 - EPS))
    assert outside.flags["draw"] == 0 and outside.bad["draw"] == 1


def test_draw_band_is_relative_to_p(orc):
    # The same absolute margin |u - p| is inside the band for a large p and
    # outside for a small one: the band scales with p, not with 1.
    X = synth.gauss_mixture(4000, 5, 10, 10.0, seed=4)
    ell, seed = 20.0, 2
    _, rs = _own(orc, X, 5, ell, 1, seed)
    i, delta = _closest_draw(orc, X, ell, seed)
    follow = {"rounds": [np.array(sorted(set(rs[0].tolist()) ^ {i}))]}
    i0 = orc.first_center(X.shape[0], seed)
    _, D2, _ = orc.nearest(X, X[i0:i0 + 1])
    _, p, u = orc.select(D2, orc.total(D2), ell, seed, 1)
    absm = abs(u[i] - p[i])
    # a band equal to the absolute margin (not divided by p < 1) is too
    # narrow relative to p only if p < 1; here p < 1, so delta > absm
    assert p[i] < 1 and delta > absm
    r = orc.kmeans_parallel_init(X, 5, ell, 1, seed, follow=follow, band=absm * (1 + EPS))
    assert r.bad["draw"] == 1


# ----------------------------------------------------------------- argmins
def _closest_tie(orc, X, o):
    """Point whose best and second-best candidates are closest (relative to
    the best distance, which must be > 0), the second-best id and the gap."""
    D = cdist(X, X[o.cand_point], "sqeuclidean")
    order = np.argsort(D, axis=1, kind="stable")
    best = D[np.arange(X.shape[0]), order[:, 0]]
    snd = D[np.arange(X.shape[0]), order[:, 1]]
    gap = np.where(best > 0, (snd - best) / np.where(best > 0, best, 1.0), np.inf)
    i = int(np.argmin(gap))
    assert order[i, 0] == o.assign[i]
    return i, int(order[i, 1]), float(gap[i])


def test_argmin_difference_inside_band_is_flagged(orc):
    X = synth.gauss_mixture(3000, 4, 8, 10.0, seed=7)
    o, _ = _own(orc, X, 8, 16.0, 3, seed=1)
    i, j2, gap = _closest_tie(orc, X, o)
    A = o.assign.copy()
    A[i] = j2
    inside = orc.kmeans_parallel_init(X, 8, 16.0, 3, 1, follow={"assign": A}, band=gap * (1 + EPS))
    assert inside.flags["argmin"] == 1 and inside.bad["argmin"] == 0
    assert inside.assign[i] == j2                       # the followed assignment is kept
    assert inside.weights[j2] == o.weights[j2] + 1      # and it moves a unit of weight
    outside = orc.kmeans_parallel_init(X, 8, 16.0, 3, 1, follow={"assign": A}, band=gap * (1 - EPS))
    assert outside.flags["argmin"] == 0 and outside.bad["argmin"] == 1


def test_argmin_to_a_missing_candidate_is_bad(orc):
    X = synth.gauss_mixture(2000, 4, 8, 10.0, seed=8)
    o, _ = _own(orc, X, 8, 16.0, 2, seed=3)
    for wrong in (-1, o.cand_point.size):
        A = o.assign.copy()
        A[17] = wrong
        r = orc.kmeans_parallel_init(X, 8, 16.0, 2, 3, follow={"assign": A}, band=1e30)
        assert r.bad["argmin"] == 1 and r.flags["argmin"] == 0


# ------------------------------------------------------------ recluster picks
def _integer_instance(seed):
    # integer coordinates and weights: every prefix sum of w*E is exact in FP64
    rng = np.random.default_rng(seed)
    C = rng.integers(-20, 21, size=(40, 3)).astype(np.float64)
    w = rng.integers(1, 9, size=40).astype(np.float64)
    return C, w


def _pick_boundaries(orc, C, w, picks, s, seed):
    """Exact threshold u*T of pick s and the prefix sums P of w*E."""
    E = np.ones(C.shape[0])
    for q in range(s):
        e = ((C - C[picks[q]]) ** 2).sum(axis=1)
        E = e if q == 0 else np.minimum(E, e)
    v = w * E
    P = np.cumsum(v)
    T = P[-1]
    u = orc.uniform(seed, orc.TAG_RECL, s, 0, 0)
    return u * T, P, T


@pytest.mark.parametrize("s", [0, 1, 3])
def test_pick_difference_inside_band_is_flagged(orc, s):
    C, w = _integer_instance(s + 2)
    seed = 40 + s
    k = s + 1
    own, nf, nb = orc.kpp_weighted(C, w, k, seed)
    assert nf == nb == 0
    f, nf, nb = orc.kpp_weighted(C, w, k, seed, follow=own, tol=0.0)
    assert nf == nb == 0 and np.array_equal(f, own)
    thr, P, T = _pick_boundaries(orc, C, w, own, s, seed)
    j = int(own[s])
    assert (P[j - 1] if j else 0.0) <= thr < P[j]
    # the next candidate with mass: its interval starts at P[j]
    up = next(g for g in range(j + 1, C.shape[0]) if P[g] > P[g - 1])
    du = (P[j] - thr) / T
    # the previous candidate with mass: its interval ends at P[j - 1]
    dn_g = next((g for g in range(j - 1, -1, -1) if P[g] > (P[g - 1] if g else 0.0)), None)
    for g, delta in ((up, du),) + (((dn_g, (thr - P[j - 1]) / T),) if dn_g is not None else ()):
        fol = own.copy()
        fol[s] = g
        p_in, nf, nb = orc.kpp_weighted(C, w, k, seed, follow=fol, tol=delta * (1 + EPS))
        assert (nf, nb) == (1, 0) and p_in[s] == g
        _, nf, nb = orc.kpp_weighted(C, w, k, seed, follow=fol, tol=delta * (1 - EPS))
        assert (nf, nb) == (0, 1)


def test_pick_of_zero_mass_candidate_is_bad(orc):
    C, w = _integer_instance(9)
    w[5] = 0.0
    own, _, _ = orc.kpp_weighted(C, w, 1, 3)
    fol = own.copy()
    fol[0] = 5
    _, nf, nb = orc.kpp_weighted(C, w, 1, 3, follow=fol, tol=1.0)
    assert (nf, nb) == (0, 1)


def test_pick_two_intervals_away_needs_the_wider_band(orc):
    C, w = _integer_instance(4)
    seed = 12
    own, _, _ = orc.kpp_weighted(C, w, 1, seed)
    thr, P, T = _pick_boundaries(orc, C, w, own, 0, seed)
    j = int(own[0])
    g = j + 2 if j + 2 < C.shape[0] else j - 2
    fol = own.copy()
    fol[0] = g
    lo, hi = (P[g - 1] if g else 0.0), P[g]
    delta = (lo - thr) / T if g > j else (thr - hi) / T
    _, nf, nb = orc.kpp_weighted(C, w, 1, seed, follow=fol, tol=delta * (1 - EPS))
    assert (nf, nb) == (0, 1)
    _, nf, nb = orc.kpp_weighted(C, w, 1, seed, follow=fol, tol=delta * (1 + EPS))
    assert (nf, nb) == (1, 0)


# ------------------------------------------------------------- the FP32 band
def _fp32_direct(x, c):
    """FP32 direct form as the kernels compute it: t = fl(x_j - c_j),
    acc = fl(t * t + acc) (one rounding: the FP64 product t*t is exact and
    the sum is rounded once more only when it needs more than 53 bits),
    coordinates ascending."""
    x32, c32 = x.astype(np.float32), c.astype(np.float32)
    acc = np.zeros(x.shape[0], np.float32)
    for j in range(x.shape[1]):
        t = (x32[:, j] - c32[:, j]).astype(np.float64)
        acc = (t * t + acc.astype(np.float64)).astype(np.float32)
    return acc


def _pairs(rng, X, npairs, near_frac=0.5):
    n = X.shape[0]
    a = rng.integers(0, n, size=npairs)
    b = rng.integers(0, n, size=npairs)
    # half of the pairs: a point against a nearby one (small D^2 relative to
    # the norms, where cancellation in x - c is largest)
    k = int(npairs * near_frac)
    order = np.lexsort(X.T[::-1])
    pos = rng.integers(0, n - 1, size=k)
    a[:k], b[:k] = order[pos], order[pos + 1]
    return X[a], X[b]


@pytest.mark.parametrize("d,kind", [(1, "gauss"), (2, "gauss"), (15, "gauss"), (42, "heavy"),
                                    (64, "gauss"), (128, "gauss"), (170, "heavy"),
                                    (256, "gauss"), (256, "heavy")])
def test_fp32_band_bounds_direct_form_error(orc, d, kind):
    rng = np.random.default_rng(d)
    if kind == "heavy":
        X = synth.heavy_tailed(20000, d, seed=d).astype(np.float64)
    else:
        X = synth.gauss_mixture_sigma(20000, d, 50, seed=d).astype(np.float64)
    x, c = _pairs(rng, X.astype(np.float32).astype(np.float64), 20000)
    exact = ((x - c) ** 2).sum(axis=1)        # FP64: relative error <= d * 2^-53
    got = _fp32_direct(x, c).astype(np.float64)
    pos = exact > 0
    assert np.all(got[~pos] == 0)              # identical rows give exactly 0
    rel = np.abs(got[pos] - exact[pos]) / exact[pos]
    single = orc.fp32_band(d) / 2              # (d + 2) u: one computed value's bound
    assert rel.max() <= single, (rel.max(), single)
    # the band is not vacuous: observed errors reach a visible part of it
    assert rel.max() >= single / (8 * np.sqrt(d + 2))
