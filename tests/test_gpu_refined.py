"""REFINED mode: MFMA screen + FP32 direct-form refinement.

The screen's lower bound includes the FP32 direct-form error, so every
decision it takes is the decision the plain FP32 path takes: the two modes
must agree bit for bit (candidates, D^2, assignment, weights, picks,
centers, phi), and the refined run must pass the same oracle replay."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1203_6402_amd import synth
from tests.gpu_util import compare_init, decoded_fp64, gpu_init, to_bf16_bits, to_e4m3

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_1203_6402_amd import kmpar
    assert torch.cuda.is_available()
    return kmpar


@pytest.fixture(scope="module")
def plain(K):
    return K.Context(0, K.MODE_PLAIN_FP32)


@pytest.fixture(scope="module")
def refined(K):
    return K.Context(0, K.MODE_REFINED)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _same_init(a, b):
    assert torch.equal(a.centers, b.centers)
    for key in a.trace:
        assert torch.equal(a.trace[key], b.trace[key]), key
    sa, sb = dict(a.stats), dict(b.stats)
    sa.pop("n_rescanned")
    sb.pop("n_rescanned")
    assert sa == sb


@pytest.mark.parametrize("n,d,k,ell,rounds,kind", [
    (10000, 15, 50, 100.0, 5, "gauss"),     # GaussMixture, split-3 screen, K = 64
    (20011, 42, 60, 120.0, 5, "heavy"),     # KDD-shaped heavy tails, K = 128
    (6007, 30, 40, 80.0, 4, "heavy"),       # K = 96: chunks shorter than the staging buffer
    (5003, 85, 40, 80.0, 4, "sigma"),       # split-3 row of K = 256, four row tiles
    (4001, 128, 30, 60.0, 3, "sigma"),      # K = 384: two row tiles per wave
    (2503, 170, 20, 50.0, 3, "heavy"),      # widest split-3 row (K = 512)
    (3001, 3, 20, 40.0, 5, "gauss"),        # tiny d
    (20000, 8, 200, 800.0, 3, "gauss"),     # K = 32: 32-tile chunks, two of them a round
])
def test_refined_equals_plain_f32(plain, refined, n, d, k, ell, rounds, kind):
    if kind == "gauss":
        X = synth.gauss_mixture(n, d, k, 10.0, seed=n)
    elif kind == "heavy":
        X = synth.heavy_tailed(n, d, seed=n)
    else:
        X = synth.gauss_mixture_sigma(n, d, 60, seed=n)
    Xd = _dev(X)
    a = plain.init(Xd, k=k, ell=ell, rounds=rounds, seed=5, trace=True)
    b = refined.init(Xd, k=k, ell=ell, rounds=rounds, seed=5, trace=True)
    torch.cuda.synchronize()
    _same_init(a, b)
    tr = {key: v.cpu().numpy() for key, v in b.trace.items()}
    compare_init(X.astype(np.float64), b, tr, k, ell, rounds, 5)
    # Most points are settled by the screen.
    assert b.stats["n_rescanned"] <= 0.05 * n * rounds


@pytest.mark.parametrize("d,n,k,ell", [(16, 6007, 60, 120.0), (64, 6007, 60, 120.0),
                                        (128, 6007, 60, 120.0), (256, 6007, 60, 120.0),
                                        (32, 20000, 200, 800.0)])  # 32-tile chunks
def test_refined_equals_plain_bf16(plain, refined, d, n, k, ell):
    X = synth.gauss_mixture_sigma(n, d, 80, seed=d)
    Xb = to_bf16_bits(X)
    Xd = _dev(Xb).view(torch.bfloat16)
    a = plain.init(Xd, k=k, ell=ell, rounds=5, seed=2, trace=True)
    b = refined.init(Xd, k=k, ell=ell, rounds=5, seed=2, trace=True)
    torch.cuda.synchronize()
    _same_init(a, b)
    tr = {key: v.cpu().numpy() for key, v in b.trace.items()}
    compare_init(decoded_fp64(Xb, "bf16"), b, tr, k, ell, 5, 2)


@pytest.mark.parametrize("d,n,k,ell,kind", [
    (16, 6007, 40, 80.0, "sigma"),     # one k-step, codes read straight from X
    (42, 5003, 40, 80.0, "heavy"),     # d % 8 != 0: operands prepared by the first pass
    (128, 4001, 30, 60.0, "sigma"),    # four k-steps
    (256, 3001, 30, 60.0, "sigma"),    # eight k-steps (the widest row)
    (8, 20000, 200, 800.0, "gauss"),   # 32-tile chunks, two of them a round
])
def test_refined_equals_plain_fp8(plain, refined, d, n, k, ell, kind):
    # e4m3 codes with per-row scales max|x|/448: the screen multiplies the
    # codes exactly and scales each value afterwards.
    if kind == "gauss":
        X = synth.gauss_mixture(n, d, k, 10.0, seed=n)
    elif kind == "heavy":
        X = synth.heavy_tailed(n, d, seed=n)
    else:
        X = synth.gauss_mixture_sigma(n, d, 60, seed=n)
    q, sc = to_e4m3(X)
    Xd, sd = _dev(q), _dev(sc)
    a = plain.init(Xd, k=k, ell=ell, rounds=4, seed=3, row_scale=sd, trace=True)
    b = refined.init(Xd, k=k, ell=ell, rounds=4, seed=3, row_scale=sd, trace=True)
    torch.cuda.synchronize()
    _same_init(a, b)
    tr = {key: v.cpu().numpy() for key, v in b.trace.items()}
    compare_init(decoded_fp64(q, "fp8", sc), b, tr, k, ell, 4, 3)
    assert b.stats["n_rescanned"] <= 0.05 * n * 4


# FP8 rows against FP32 centers had a screen of their own (codes against a
# two-term split of the centers); a run of ten Lloyd steps at n = 50M, d = 256
# stopped with an illegal-address fault whose cause was not found, so it was
# taken out and these cases only check the direct form against itself.
_FP8_ASSIGN_OFF = pytest.mark.skip(reason="the FP8-rows assignment screen was taken out after an "
                                          "unexplained fault; FP8 assignment uses the direct form")


@pytest.mark.parametrize("dt,d,m", [("f32", 42, 500), ("f32", 15, 37), ("bf16", 128, 300),
                                    ("bf16", 64, 33), ("f32", 8, 700), ("bf16", 16, 700),
                                    pytest.param("fp8", 64, 300, marks=_FP8_ASSIGN_OFF),
                                    pytest.param("fp8", 42, 200, marks=_FP8_ASSIGN_OFF),
                                    pytest.param("fp8", 256, 100, marks=_FP8_ASSIGN_OFF),
                                    pytest.param("fp8", 16, 700, marks=_FP8_ASSIGN_OFF)])
def test_refined_assign_cost_lloyd_equal_plain(plain, refined, dt, d, m):
    X = synth.gauss_mixture_sigma(9001, d, 200, seed=m)
    rs = None
    if dt == "bf16":
        Xh = to_bf16_bits(X)
        Xd = _dev(Xh).view(torch.bfloat16)
        X64 = decoded_fp64(Xh, "bf16")
    elif dt == "fp8":
        q, sc = to_e4m3(X)
        Xd, rs = _dev(q), _dev(sc)
        X64 = decoded_fp64(q, "fp8", sc)
    else:
        Xd = _dev(X)
        X64 = X.astype(np.float64)
    rng = np.random.default_rng(m)
    C = (X64[rng.choice(9001, m, replace=False)] + rng.normal(size=(m, d)) * 0.1).astype(np.float32)
    a1, d1 = plain.assign(Xd, _dev(C), row_scale=rs)
    a2, d2 = refined.assign(Xd, _dev(C), row_scale=rs)
    p1, p2 = plain.cost(Xd, _dev(C), row_scale=rs), refined.cost(Xd, _dev(C), row_scale=rs)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2) and torch.equal(d1, d2) and torch.equal(p1, p2)
    oa, od2, _ = O.nearest(X64, C.astype(np.float64))
    np.testing.assert_allclose(d2.cpu().numpy(), od2, rtol=1e-5)
    C1, C2 = _dev(C), _dev(C)
    for _ in range(3):
        x1, q1 = plain.lloyd_step(Xd, C1, row_scale=rs, want_assign=True)
        x2, q2 = refined.lloyd_step(Xd, C2, row_scale=rs, want_assign=True)
        torch.cuda.synchronize()
        assert torch.equal(x1, x2) and torch.equal(q1, q2) and torch.equal(C1, C2)


def test_refined_heavy_tailed_large_norm_gap(plain, refined):
    # Rows whose norms differ by many orders of magnitude from their nearest
    # candidates: the screen must hand the hard cases to the direct form.
    X = synth.heavy_tailed(30000, 42, seed=99)
    X[::97] *= 1e4
    Xd = _dev(X)
    a = plain.init(Xd, k=100, ell=200.0, rounds=5, seed=7, trace=True)
    b = refined.init(Xd, k=100, ell=200.0, rounds=5, seed=7, trace=True)
    torch.cuda.synchronize()
    _same_init(a, b)


@pytest.mark.parametrize("d", [15, 42])
def test_refined_tile_skip_on_collinear_rows(plain, refined, d):
    # Rows on one ray from the origin: ||x - c|| equals | ||x|| - ||c|| | up
    # to rounding, so the norm bound behind the screen's tile skip is tight
    # for every pair and many points sit right at its margin; a tenth of the
    # rows are repeated (distance 0 once one of them is a center).
    rng = np.random.default_rng(d)
    u = rng.normal(size=d)
    u /= np.linalg.norm(u)
    r = np.exp(rng.uniform(0.0, np.log(1e4), size=12000))
    X = (r[:, None] * u[None, :]).astype(np.float32)
    X[::10] = X[1::10][: X[::10].shape[0]]
    Xd = _dev(X)
    a = plain.init(Xd, k=80, ell=160.0, rounds=5, seed=3, trace=True)
    b = refined.init(Xd, k=80, ell=160.0, rounds=5, seed=3, trace=True)
    torch.cuda.synchronize()
    _same_init(a, b)


@pytest.mark.parametrize("d,kind", [(8, "ray"), (8, "gauss"), (42, "gauss")])
def test_refined_tile_skip_rows_in_norm_order(plain, refined, d, kind):
    # X stored in ascending norm: each row tile of the screen spans a narrow
    # norm interval, so most (row tile, candidate tile) pairs are skipped and
    # many row tiles skip every tile of a round (those points keep D without
    # a rescan).  d = 8 runs one k-step with 24-tile chunks, more tiles than
    # the skip has judges for (tiles 16 on of each chunk are never skipped).
    if kind == "ray":
        rng = np.random.default_rng(d)
        u = rng.normal(size=d)
        u /= np.linalg.norm(u)
        X = (np.exp(rng.uniform(0.0, np.log(1e4), size=20000))[:, None] * u[None, :]).astype(np.float32)
    else:
        X = synth.gauss_mixture(20000, d, 200, 10.0, seed=d)
    X = np.ascontiguousarray(X[np.argsort((X.astype(np.float64) ** 2).sum(1), kind="stable")])
    Xd = _dev(X)
    a = plain.init(Xd, k=200, ell=800.0, rounds=4, seed=2, trace=True)
    b = refined.init(Xd, k=200, ell=800.0, rounds=4, seed=2, trace=True)
    torch.cuda.synchronize()
    _same_init(a, b)
    if kind == "gauss":  # on the ray many points sit at the bound's margin and are listed
        assert b.stats["n_rescanned"] <= 0.05 * 20000 * 4


@pytest.mark.parametrize("d,span", [(4, 6), (20, 3)])
def test_flagged_argmins_on_integer_lattice(plain, refined, d, span):
    # Integer coordinates make every FP32 distance exact, so a runner-up
    # within the band is an exact tie: the count of flagged argmins is the
    # number of points whose two nearest candidates are equally far (a tie
    # at zero included), in both modes.
    X = np.random.default_rng(11).integers(-span, span + 1, size=(6000, d)).astype(np.float32)
    Xd = _dev(X)
    a = plain.init(Xd, k=20, ell=60.0, rounds=4, seed=3, trace=True)
    b = refined.init(Xd, k=20, ell=60.0, rounds=4, seed=3, trace=True)
    torch.cuda.synchronize()
    _same_init(a, b)
    tr = {key: v.cpu().numpy() for key, v in b.trace.items()}
    X64 = X.astype(np.float64)
    o = compare_init(X64, b, tr, 20, 60.0, 4, 3)
    _, d2, snd = O.nearest(X64, X64[o.cand_point])
    ties = int(np.sum(snd == d2))
    assert ties > 0 and b.stats["flagged_argmins"] == ties


@pytest.mark.parametrize("mode", ["plain", "refined"])
def test_lloyd_rows_without_a_finite_distance(plain, refined, mode):
    # Rows holding NaN or Inf have no finite distance to any center: their
    # assignment is -1 and no centroid takes them, while every other row is
    # assigned and averaged as without them.  (Such rows once sent the last
    # cluster's sums into sorted positions the scatter had not written.)
    ctx = refined if mode == "refined" else plain
    X = synth.gauss_mixture(20000, 15, 50, 10.0, seed=5)
    bad = np.arange(3, 20000, 997)
    X[bad[::2], 3] = np.nan
    X[bad[1::2], 7] = np.inf
    X64 = X.astype(np.float64)
    ok = np.isfinite(X64).all(axis=1)
    rng = np.random.default_rng(1)
    C = torch.from_numpy(X[rng.choice(np.nonzero(ok)[0], 50, replace=False)].copy()).to("cuda:0")
    Xd = _dev(X)
    for _ in range(3):
        Cin = C.cpu().numpy().astype(np.float64)
        a, _phi = ctx.lloyd_step(Xd, C, want_assign=True)
        torch.cuda.synchronize()
        a = a.cpu().numpy()
        assert np.all(a[~ok] == -1)
        oa, od2, osnd = O.nearest(X64[ok], Cin)
        diff = a[ok] != oa
        gap = (osnd - od2) / np.maximum(od2, 1e-300)
        assert np.all(gap[diff] <= O.fp32_band(15))
        Co, _ = O.lloyd_update(X64[ok], a[ok], Cin)
        np.testing.assert_allclose(C.cpu().numpy(), Co.astype(np.float32), rtol=1e-6, atol=1e-6)
