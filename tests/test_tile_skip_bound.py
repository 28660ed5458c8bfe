"""The screen's tile skip, replayed in FP32 on the host: whenever its test
rules out a (row tile, candidate tile) pair, every candidate of the tile lies
beyond (1 + 2 band) D of every point of the row tile in the FP32 direct form,
band = 2 (d + 2) 2^-24, so REFINED keeps the decisions of the plain path.

The test is the kernel's, restated: ||x|| from the FP32 ||x||^2 of the first
pass widened by (d + 8) 2^-24, the largest D of the row tile raised by
(8 d + 32) 2^-24, each candidate tile's ||c|| interval from its FP64 ||c||^2
rounded to FP32 and widened by 2^-20, and the squared gap lowered by
(2 d + 16) 2^-24.  It rests on ||x - c||^2 >= (||x|| - ||c||)^2; rows on one
ray from the origin make that bound exact, and each row tile's D is put just
below the skip threshold, so the margins alone must cover every rounding.
A copy of the test without its margins fails on the same inputs."""
import numpy as np
import pytest

U = np.float32(2.0 ** -24)


def _f32_fma_sum(terms):
    """sum_e terms[:, e] in FP32, one fused multiply-add rounding per step
    (terms are exact products held in FP64)."""
    acc = np.zeros(terms.shape[0], np.float32)
    for e in range(terms.shape[1]):
        acc = (acc.astype(np.float64) + terms[:, e]).astype(np.float32)
    return acc


def _direct(x, c):
    """FP32 direct form sum_e (x_e - c_e)^2, e ascending (one row of x per c)."""
    t = (x - c).astype(np.float32).astype(np.float64)
    return _f32_fma_sum(t * t)


def _skip(xt, D, ct, d, margins=True):
    """The kernel's skip test for one row tile xt (16 x d), its D and one
    candidate tile ct (16 x d)."""
    f = (lambda v: np.float32(v)) if margins else (lambda v: np.float32(0.0))
    x64 = xt.astype(np.float64)
    n2 = _f32_fma_sum(x64 * x64)
    x = np.sqrt(n2).astype(np.float32)
    xl = (x * (np.float32(1) - f((d + 8) * U))).min()
    xh = (x * (np.float32(1) + f((d + 8) * U))).max()
    pdl = np.float32(D.max()) * (np.float32(1) + f((8 * d + 32) * U))
    keys = (ct.astype(np.float64) ** 2).sum(1).astype(np.float32)
    w = 2.0 ** -20 if margins else 0.0
    cl = np.float32(np.sqrt(np.float64(keys.min())) * (1 - w))
    ch = np.float32(np.sqrt(np.float64(keys.max())) * (1 + w))
    gap = max(np.float32(cl - xh), np.float32(xl - ch))
    return bool(gap > 0 and np.float32(np.float32(gap * gap) * (np.float32(1) - f((2 * d + 16) * U))) > pdl)


def _cases(d, kind, seed):
    """A row tile of nearby norms and a candidate tile at a relative norm gap
    from 1e-6 to 1, below or above it."""
    rng = np.random.default_rng(seed)
    r0 = np.exp(rng.uniform(-5, np.log(1e4)))
    g = np.exp(rng.uniform(np.log(1e-6), 0.0)) * rng.choice([-0.5, 1.0])
    w = abs(g) * rng.uniform(0.0, 0.5)  # spread of each tile's norms
    rx = r0 * (1 + w * rng.uniform(0, 1, 16))
    rc = r0 * (1 + g + np.sign(g) * w + w * rng.uniform(0, 1, 16))
    u = rng.normal(size=d)
    u /= np.linalg.norm(u)
    if kind == "ray":
        xt = (rx[:, None] * u).astype(np.float32)
        ct = (rc[:, None] * u).astype(np.float32)
    else:  # directions spread around u
        def dirs():
            v = u + 0.3 * rng.normal(size=(16, d)) / np.sqrt(d)
            return v / np.linalg.norm(v, axis=1, keepdims=True)
        xt = (rx[:, None] * dirs()).astype(np.float32)
        ct = (rc[:, None] * dirs()).astype(np.float32)
    return xt, ct


def _threshold_d(xt, ct, d):
    """Each point's D: the largest FP32 value below which the tile is still
    skipped (bisection on the row tile's D_max), then spread below it."""
    lo, hi = 0.0, 1e30
    if not _skip(xt, np.zeros(16, np.float32), ct, d):
        return None
    for _ in range(200):
        mid = (lo + hi) / 2
        if _skip(xt, np.full(16, mid, np.float32), ct, d):
            lo = mid
        else:
            hi = mid
    Dmax = np.float32(lo)
    D = np.full(16, Dmax, np.float32)
    D[::3] = np.float32(Dmax * 0.5)
    return D


@pytest.mark.parametrize("d", [1, 3, 8, 15, 42, 128])
@pytest.mark.parametrize("kind", ["ray", "gauss"])
def test_skipped_candidates_lie_beyond_the_band(d, kind):
    band = 2.0 * (d + 2) * 2.0 ** -24
    checked = 0
    for seed in range(40):
        xt, ct = _cases(d, kind, seed * 97 + d)
        D = _threshold_d(xt, ct, d)
        if D is None:
            continue
        assert _skip(xt, D, ct, d)
        for j in range(16):
            dist = _direct(xt, np.broadcast_to(ct[j], xt.shape))
            assert (dist.astype(np.float64) > (1 + 2 * band) * D.astype(np.float64)).all(), (seed, j)
        checked += 1
    assert checked >= 10


def test_the_margins_are_needed():
    # The same replay without the margins skips pairs whose direct-form
    # distance falls within the band: the checks above have teeth.
    bad = 0
    for d in (8, 42):
        band = 2.0 * (d + 2) * 2.0 ** -24
        for seed in range(40):
            xt, ct = _cases(d, "ray", seed * 97 + d)
            if not _skip(xt, np.zeros(16, np.float32), ct, d, margins=False):
                continue
            lo, hi = 0.0, 1e30
            for _ in range(200):
                mid = (lo + hi) / 2
                if _skip(xt, np.full(16, mid, np.float32), ct, d, margins=False):
                    lo = mid
                else:
                    hi = mid
            D = np.full(16, np.float32(lo), np.float32)
            for j in range(16):
                dist = _direct(xt, np.broadcast_to(ct[j], xt.shape))
                bad += int((dist.astype(np.float64) <= (1 + 2 * band) * D.astype(np.float64)).any())
    assert bad > 0
