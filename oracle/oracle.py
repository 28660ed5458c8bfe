"""FP64 oracle for k-means|| -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may use
this module.  It wraps ``kmpar_oracle.c`` (plain C, FP64) with ctypes and
composes Algorithm 2 of the paper (Section 3.3) from its steps:

1. first center uniformly at random                     -- ``first_center``
2. psi = phi_X(C)                                        -- ``orc_sum`` of D^2
3-6. r rounds: keep each x with p = min(1, ell d^2/phi)  -- ``orc_select``
     and update d^2(x, C) for the new candidates         -- ``orc_fold``
7. weights w_c = |{x : c nearest to x}|                  -- ``orc_weights``
8. recluster the weighted candidates with k-means++      -- ``orc_kpp_weighted``

plus Lloyd's iteration (Section 1, Section 3.1) -- ``lloyd_step``, Lloyd
until the assignment is stable -- ``lloyd_until_stable``, the exact-ell
rounds of Section 5.3 (exactly ell points per round, drawn in proportion to
D^2 without replacement) -- ``select_exact`` / ``sampling="exact"``, and
k-means++ on all of X (Algorithm 1) -- ``kmeanspp``.  Both draw D^2 samples
as an exponential race (``orc_exact_keys``), so with ell = 1 and r = k - 1
the exact-ell variant makes exactly the draws of k-means++.

Replay ("follow").  Another implementation that computes in lower precision
may legitimately take a different discrete decision where the oracle's margin
is within that precision's error band: a draw with |u - p| small, an argmin
whose top-2 gap is small, a recluster pick whose threshold is near a boundary.
``kmeans_parallel_init(..., follow=...)`` takes that implementation's
decisions, accepts each disagreement that lies inside the stated band (counted
as *flagged*), counts every other one as *bad*, and continues from the
followed decision so the rest of the run stays comparable.

The module never imports the library under test and shares no code with it.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libkmpar_oracle.so")
_SRC_PATH = os.path.join(_HERE, "kmpar_oracle.c")

TAG_FIRST, TAG_ROUND, TAG_RECL, TAG_EXACT = 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, no contraction into FMA)."""
    import subprocess

    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-std=c11", _SRC_PATH, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        u64, i64, i32, dbl = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        vp = ctypes.c_void_p
        L.orc_philox4x64_10.argtypes = [vp, vp, vp]
        L.orc_word.argtypes = [u64, u64, u64, u64, u64]
        L.orc_word.restype = u64
        L.orc_uniform.argtypes = [u64, u64, u64, u64, u64]
        L.orc_uniform.restype = dbl
        L.orc_index.argtypes = [u64, u64, u64, u64, u64, i64]
        L.orc_index.restype = i64
        L.orc_sum.argtypes = [vp, i64]
        L.orc_sum.restype = dbl
        L.orc_nearest.argtypes = [vp, i64, i32, vp, i64, vp, vp, vp]
        L.orc_first_center.argtypes = [i64, u64, u64]
        L.orc_first_center.restype = i64
        L.orc_select.argtypes = [vp, i64, dbl, dbl, u64, i64, u64, vp, vp, vp]
        L.orc_select.restype = i64
        L.orc_fold.argtypes = [vp, i64, i32, vp, i64, i64, vp, vp, vp]
        L.orc_weights.argtypes = [vp, i64, i64, vp]
        L.orc_kpp_weighted.argtypes = [vp, i64, i32, vp, i64, u64, u64, vp, dbl, vp, vp, vp]
        L.orc_kpp_weighted.restype = i64
        L.orc_lloyd_update.argtypes = [vp, i64, i32, vp, i64, vp, vp]
        L.orc_uniform_open.argtypes = [u64, u64, u64, u64, u64]
        L.orc_uniform_open.restype = dbl
        L.orc_exact_keys.argtypes = [vp, i64, u64, i64, u64, vp]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(X) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(X, dtype=np.float64))


def num_threads() -> int:
    return int(lib().orc_num_threads())


# --------------------------------------------------------------------------- RNG
def philox_block(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint64))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64))
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def uniform(seed, tag, a, b, inst=0) -> float:
    return float(lib().orc_uniform(seed, tag, a, b, inst))


def index(seed, tag, a, b, inst, n) -> int:
    return int(lib().orc_index(seed, tag, a, b, inst, n))


def uniform_open(seed, tag, a, b, inst=0) -> float:
    return float(lib().orc_uniform_open(seed, tag, a, b, inst))


def first_center(n: int, seed: int, inst: int = 0) -> int:
    return int(lib().orc_first_center(n, seed, inst))


# --------------------------------------------------------------------- distances
def total(v) -> float:
    v = _f64(v)
    return float(lib().orc_sum(_p(v), v.size))


def nearest(X, C):
    """Section 3.1: (argmin, d^2, second smallest d^2) of each point."""
    X, C = _f64(X), _f64(C)
    n, d = X.shape
    m = C.shape[0]
    arg = np.empty(n, np.int64)
    d2 = np.empty(n, np.float64)
    snd = np.empty(n, np.float64)
    lib().orc_nearest(_p(X), n, d, _p(C), m, _p(arg), _p(d2), _p(snd))
    return arg, d2, snd


def nearest_sharded(X, C, shards):
    """Section 3.5, last paragraph: each mapper holds a slice C' of the
    centers and emits, per point, the nearest center of its slice; the
    reducer keeps the nearest of those (ties to the lower index, the slices
    being consecutive).  Returns (argmin, d^2) like ``nearest``."""
    X, C = _f64(X), _f64(C)
    m = C.shape[0]
    best_a = np.full(X.shape[0], -1, np.int64)
    best_d = np.full(X.shape[0], np.inf)
    for sh in range(shards):
        lo, hi = sh * m // shards, (sh + 1) * m // shards
        if lo == hi:
            continue
        a, d2, _ = nearest(X, C[lo:hi])
        better = d2 < best_d            # a later slice wins only when strictly closer
        best_a[better] = a[better] + lo
        best_d[better] = d2[better]
    return best_a, best_d


def cost(X, C) -> float:
    """phi_X(C) (Section 3.1)."""
    return total(nearest(X, C)[1])


def select(D2, phi, ell, seed, t, inst=0):
    D2 = _f64(D2)
    n = D2.size
    sel = np.empty(n, np.uint8)
    p = np.empty(n, np.float64)
    u = np.empty(n, np.float64)
    lib().orc_select(_p(D2), n, float(phi), float(ell), seed, t, inst, _p(sel), _p(p), _p(u))
    return sel.astype(bool), p, u


def exact_keys(D2, seed, t, inst=0) -> np.ndarray:
    """Exponential-race keys -ln(V_i) / D2_i (+inf where D2_i = 0)."""
    D2 = _f64(D2)
    key = np.empty(D2.size, np.float64)
    lib().orc_exact_keys(_p(D2), D2.size, seed, t, inst, _p(key))
    return key


def select_exact(D2, ell, seed, t, inst=0):
    """Exact-ell round (Section 5.3): the min(ell, #{D2 > 0}) points with the
    smallest keys (ties to the lower index).  Returns (selected mask, keys,
    tau = the largest selected key, or +inf when nothing is selected)."""
    key = exact_keys(D2, seed, t, inst)
    take = int(min(int(ell), int(np.count_nonzero(np.isfinite(key)))))
    order = np.argsort(key, kind="stable")[:take]
    sel = np.zeros(key.size, bool)
    sel[order] = True
    tau = float(key[order[-1]]) if take else np.inf
    return sel, key, tau


def fold(X, Cnew, first_id, D2, A, S=None):
    X, Cnew = _f64(X), _f64(Cnew)
    n, d = X.shape
    lib().orc_fold(_p(X), n, d, _p(Cnew), Cnew.shape[0], first_id, _p(D2), _p(A),
                   _p(S) if S is not None else None)


def weights(A, ncand) -> np.ndarray:
    A = np.ascontiguousarray(np.asarray(A, dtype=np.int64))
    w = np.empty(ncand, np.int64)
    lib().orc_weights(_p(A), A.size, ncand, _p(w))
    return w


def kpp_weighted(C, w, k, seed, inst=0, follow=None, tol=0.0):
    """Weighted k-means++ (Algorithm 1 with weights).  Returns
    (picks, n_flagged, n_bad)."""
    C = _f64(C)
    m, d = C.shape
    wf = _f64(w)
    picks = np.full(k, -1, np.int64)
    nf = ctypes.c_int64(0)
    nb = ctypes.c_int64(0)
    fo = None
    if follow is not None:
        fo = np.full(k, -1, np.int64)
        f = np.asarray(follow, dtype=np.int64)
        fo[:f.size] = f[:k]
    made = lib().orc_kpp_weighted(_p(C), m, d, _p(wf), k, seed, inst,
                                  _p(fo) if fo is not None else None, float(tol), _p(picks),
                                  ctypes.byref(nf), ctypes.byref(nb))
    return picks[:made], int(nf.value), int(nb.value)


def lloyd_update(X, a, C):
    X = _f64(X)
    n, d = X.shape
    C = _f64(C).copy()
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int64))
    cnt = np.empty(C.shape[0], np.int64)
    lib().orc_lloyd_update(_p(X), n, d, _p(a), C.shape[0], _p(C), _p(cnt))
    return C, cnt


def lloyd_step(X, C):
    """One Lloyd iteration: assign, then move centers to centroids.
    Returns (new C, assignment, cost of the input centers)."""
    a, d2, _ = nearest(X, C)
    Cn, _ = lloyd_update(X, a, C)
    return Cn, a, total(d2)


def lloyd_until_stable(X, C, max_iters, follow=None, band=None):
    """Lloyd's iteration repeated until the set of centers is stable
    (Section 1): each iteration assigns every point to its nearest center;
    when the assignment equals the previous iteration's, the centers would
    not move and the iteration stops; otherwise the centers move to the
    centroids (an empty cluster keeps its center).  ``follow`` (optional):
    another implementation's assignment per iteration, accepted where it
    differs inside the relative ``band`` (counted as flagged) and then used.
    Returns (centers, number of center updates made, cost of the input
    centers of every assignment, n_flagged, n_bad)."""
    X = _f64(X)
    d = X.shape[1]
    band = fp32_band(d) if band is None else band
    C = _f64(C).copy()
    prev = None
    phis = []
    nf = nb = 0
    it = 0
    for it in range(max_iters + 1):
        a, d2, _ = nearest(X, C)
        phis.append(total(d2))
        if follow is not None and it < len(follow):
            g = np.asarray(follow[it], dtype=np.int64)
            diff = np.nonzero(g != a)[0]
            if diff.size:
                ok = (g[diff] >= 0) & (g[diff] < C.shape[0])
                dg = np.full(diff.size, np.inf)
                dg[ok] = ((X[diff[ok]] - C[g[diff[ok]]]) ** 2).sum(axis=1)
                within = ok & (dg - d2[diff] <= band * d2[diff])
                nf += int(within.sum())
                nb += int((~within).sum())
                a = a.copy()
                a[diff[ok]] = g[diff[ok]]
        if prev is not None and np.array_equal(a, prev):
            return C, it, phis, nf, nb
        if it == max_iters:
            break
        C, _ = lloyd_update(X, a, C)
        prev = a
    return C, max_iters, phis, nf, nb


# ---------------------------------------------------------------- k-means||
def fp32_band(d: int) -> float:
    """Relative error bound of a squared distance computed in FP32 in direct
    form sum_j (x_j - c_j)^2 against its exact value: each difference and
    square rounds once and a d-term nonnegative sum adds at most (d-1)
    roundings, so |err| <= (d + 2) u D^2 with u = 2^-24.  The bands below use
    twice that (both operands of a comparison carry error)."""
    return 2.0 * (d + 2) * 2.0 ** -24


@dataclass
class InitResult:
    cand_point: np.ndarray            # point index of every candidate, id order
    round_count: list                 # |C'_t| per round (entry 0 is the first center)
    phi: list                         # phi after the first center and after each round
    assign: np.ndarray                # nearest candidate id per point after the rounds
    d2: np.ndarray                    # D^2 per point after the rounds
    weights: np.ndarray               # Step 7 weights per candidate
    picks: np.ndarray                 # candidate ids chosen by the recluster
    centers: np.ndarray               # X rows of the picks (FP64)
    flags: dict = field(default_factory=dict)
    bad: dict = field(default_factory=dict)


@dataclass
class RoundState:
    """State of Algorithm 2 after some rounds: enough to resume the rounds
    (the draws of round t depend only on (seed, t, point), not on history)."""
    cand: list                        # candidate point indices, id order
    D2: np.ndarray                    # d^2(x, C) per point
    A: np.ndarray                     # nearest candidate id per point
    phi: list                         # phi after the first center and each round
    counts: list                      # |C'_t| per round (entry 0 is the first center)
    rounds_done: int


def first_round_state(X, seed, inst=0) -> RoundState:
    """Algorithm 2 steps 1-2: the uniform first center, D^2 against it, psi."""
    X = _f64(X)
    n = X.shape[0]
    i0 = first_center(n, seed, inst)
    D2 = np.full(n, np.inf)
    A = np.zeros(n, np.int64)
    fold(X, X[i0:i0 + 1], 0, D2, A)
    return RoundState(cand=[i0], D2=D2, A=A, phi=[total(D2)], counts=[1], rounds_done=0)


def run_rounds(X, state: RoundState, t_end, ell, seed, inst=0, follow=None, band=None,
               flags=None, bad=None, sampling="bernoulli") -> RoundState:
    """Algorithm 2 steps 3-6 for rounds state.rounds_done+1 .. t_end, updating
    ``state`` in place (a checkpoint taken after any round resumes to the
    same result).  ``follow``/``band``/``flags``/``bad`` as in
    ``kmeans_parallel_init``; ``sampling="exact"`` keeps exactly ell points
    per round (Section 5.3) instead of independent draws."""
    X = _f64(X)
    n, d = X.shape
    band = fp32_band(d) if band is None else band
    for t in range(state.rounds_done + 1, t_end + 1):
        if sampling == "exact":
            sel, key, tau = select_exact(state.D2, ell, seed, t, inst)
        else:
            sel, p, u = select(state.D2, state.phi[-1], ell, seed, t, inst)
        if follow is not None and "rounds" in follow:
            other = np.zeros(n, bool)
            other[np.asarray(follow["rounds"][t - 1], dtype=np.int64)] = True
            diff = np.nonzero(other != sel)[0]
            if diff.size:
                if sampling == "exact":
                    # a key within the band of the round's threshold could
                    # have landed on the other side of it (each key carries
                    # the relative error of its D^2)
                    kd = key[diff]
                    within = np.isfinite(kd) & (kd <= tau * (1 + band)) & (kd * (1 + band) >= tau)
                else:
                    within = np.abs(u[diff] - p[diff]) <= band * p[diff] + 1e-300
                flags["draw"] += int(within.sum())
                bad["draw"] += int((~within).sum())
                sel = other
        new = np.nonzero(sel)[0]
        fold(X, X[new], len(state.cand), state.D2, state.A)
        state.cand.extend(new.tolist())
        state.counts.append(int(new.size))
        state.phi.append(total(state.D2))
        state.rounds_done = t
    return state


def kmeans_parallel_init(X, k, ell, rounds, seed, inst=0, follow=None, band=None, state=None,
                         sampling="bernoulli"):
    """Algorithm 2 (Section 3.3) with k-means++ as the Step-8 recluster.

    ``follow`` (optional) is a dict with any of
      ``rounds``: list of arrays, the point indices kept in round t=1..r,
      ``assign``: the other side's nearest-candidate id per point,
      ``picks``:  the other side's recluster picks (candidate ids),
    and ``band`` the relative error band of the other side's distances
    (default: ``fp32_band(d)``).  ``state`` (optional) is a ``RoundState``
    checkpoint to resume from instead of starting at step 1.
    ``sampling="exact"``: every round keeps exactly ell points, drawn in
    proportion to D^2 without replacement (Section 5.3).
    """
    X = _f64(X)
    n, d = X.shape
    band = fp32_band(d) if band is None else band
    flags = {"draw": 0, "argmin": 0, "pick": 0}
    bad = {"draw": 0, "argmin": 0, "pick": 0}

    st = first_round_state(X, seed, inst) if state is None else state
    run_rounds(X, st, rounds, ell, seed, inst, follow, band, flags, bad, sampling)
    D2, A, phi, counts = st.D2, st.A, st.phi, st.counts

    cand = np.asarray(st.cand, dtype=np.int64)
    if follow is not None and "assign" in follow:
        other = np.asarray(follow["assign"], dtype=np.int64)
        diff = np.nonzero(other != A)[0]
        if diff.size:
            ok = (other[diff] >= 0) & (other[diff] < cand.size)
            dg = np.full(diff.size, np.inf)
            idx = np.nonzero(ok)[0]
            if idx.size:
                xs = X[diff[idx]]
                cs = X[cand[other[diff[idx]]]]
                dg[idx] = ((xs - cs) ** 2).sum(axis=1)
            within = ok & (dg - D2[diff] <= band * D2[diff])
            flags["argmin"] += int(within.sum())
            bad["argmin"] += int((~within).sum())
            A = A.copy()
            A[diff[ok]] = other[diff[ok]]
    w = weights(A, cand.size)
    fpk = None if follow is None else follow.get("picks")
    picks, nf, nb = kpp_weighted(X[cand], w, k, seed, inst, follow=fpk, tol=band)
    flags["pick"] += nf
    bad["pick"] += nb
    return InitResult(cand_point=cand, round_count=counts, phi=phi, assign=A, d2=D2,
                      weights=w, picks=picks, centers=X[cand[picks]], flags=flags, bad=bad)


def kmeanspp(X, k, seed, inst=0, follow=None, band=None):
    """k-means++ on all of X (Algorithm 1): the first center uniformly at
    random (the FIRST draw of Algorithm 2), then k - 1 centers each drawn in
    proportion to D^2 by the exponential race of draw s = 1 .. k - 1 (tag
    EXACT, counter (i, s, inst)).  ``follow``: another implementation's
    picks; a differing pick is accepted (flagged) when its key lies within
    the relative ``band`` of the smallest key.  Returns (picks, phi after
    each pick, n_flagged, n_bad); fewer than k picks when every point
    coincides with a center."""
    X = _f64(X)
    n, d = X.shape
    band = fp32_band(d) if band is None else band
    picks = [first_center(n, seed, inst)]
    D2 = np.full(n, np.inf)
    A = np.zeros(n, np.int64)
    fold(X, X[picks[0]:picks[0] + 1], 0, D2, A)
    phi = [total(D2)]
    nf = nb = 0
    for s in range(1, k):
        key = exact_keys(D2, seed, s, inst)
        j = int(np.argmin(key))               # first occurrence: the lower index on ties
        if not np.isfinite(key[j]):
            break
        if follow is not None and s < len(follow) and int(follow[s]) != j:
            g = int(follow[s])
            if 0 <= g < n and np.isfinite(key[g]) and key[g] <= key[j] * (1 + band):
                nf += 1
            else:
                nb += 1
            j = g if 0 <= g < n else j
        picks.append(j)
        fold(X, X[j:j + 1], s, D2, A)
        phi.append(total(D2))
    return np.asarray(picks, np.int64), phi, nf, nb
