"""The candidate-sharded assignment of Section 3.5 (per-slice argmins merged
by a packed (distance, id) minimum): bit for bit kmpar_assign where both
apply, the FP64 oracle beyond kmpar_assign's 16,384 centers."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1203_6402_amd import synth
from tests.gpu_util import D2_RTOL, to_bf16_bits, to_e4m3

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_1203_6402_amd import kmpar
    assert torch.cuda.is_available()
    return kmpar


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("dtype,d,m,shards", [("f32", 42, 3000, 1), ("f32", 42, 3000, 7),
                                               ("f32", 15, 256, 256), ("bf16", 128, 2048, 16),
                                               ("fp8", 256, 700, 5), ("f32", 200, 999, 3)])
def test_sharded_equals_assign(K, dtype, d, m, shards):
    X = synth.gauss_mixture_sigma(20_011, d, 60, seed=d + m)
    rng = np.random.default_rng(m)
    C = X[rng.choice(len(X), m, replace=False)] + 0.1 * rng.normal(size=(m, d)).astype(np.float32)
    C[m // 2] = C[m // 3]                                 # duplicated centers: ties to the lower id
    rs = None
    if dtype == "bf16":
        Xd = _dev(to_bf16_bits(X)).view(torch.bfloat16)
    elif dtype == "fp8":
        q, sc = to_e4m3(X)
        Xd, rs = _dev(q), _dev(sc)
    else:
        Xd = _dev(X)
    for mode in (K.MODE_PLAIN_FP32, K.MODE_REFINED):
        ctx = K.Context(0, mode)
        a0, d0 = ctx.assign(Xd, _dev(C), row_scale=rs)
        a1, d1, phi = ctx.assign_sharded(Xd, _dev(C), shards, row_scale=rs)
        phi0 = ctx.cost(Xd, _dev(C), row_scale=rs)
        torch.cuda.synchronize()
        assert torch.equal(a0, a1) and torch.equal(d0, d1)
        assert phi.item() == phi0.item()


def test_sharded_beyond_the_assign_limit(K):
    # 40,000 centers (kmpar_assign takes at most 16,384) against the oracle.
    X = synth.heavy_tailed(30_000, 42, seed=5)
    C = synth.heavy_tailed(40_000, 42, seed=6)
    ctx = K.Context(0)
    a, d2, phi = ctx.assign_sharded(_dev(X), _dev(C), 64)
    torch.cuda.synchronize()
    a, d2 = a.cpu().numpy(), d2.cpu().numpy()
    oa, od, osnd = O.nearest(X.astype(np.float64), C.astype(np.float64))
    pos = od > 0
    assert np.all(d2[~pos] == 0)
    np.testing.assert_allclose(d2[pos], od[pos], rtol=D2_RTOL)
    diff = a != oa
    gap = (osnd - od) / np.maximum(od, 1e-300)
    assert np.all(gap[diff] <= O.fp32_band(42))
    assert phi.item() == pytest.approx(O.total(od), rel=D2_RTOL)
    with pytest.raises(K.KmparError):
        ctx.assign_sharded(_dev(X), _dev(C), 257)
