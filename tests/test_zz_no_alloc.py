"""kmpar_cost_noalloc (the cost without a workspace, for callers that cannot
allocate) against kmpar_cost through the C ABI: the same launches on the
library's fixed scratch, so the result must be bit-identical; checked on two
calls in a row, the second on a smaller input (the scratch keeps the first
call's contents), in both modes and for BF16 rows, plus the FP64 oracle and
the rejection of a call larger than the scratch."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1203_6402_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_1203_6402_amd import kmpar
    return kmpar


def _abi_noalloc(K, ctx, X, C, dt, row_scale=None):
    phi = torch.full((1,), float("nan"), dtype=torch.float64, device=X.device)
    rc = K._lib.kmpar_cost_noalloc(ctx._h, X.data_ptr(), None if row_scale is None else
                                   row_scale.data_ptr(), dt, X.shape[0], X.shape[1],
                                   C.data_ptr(), C.shape[0], phi.data_ptr(),
                                   torch.cuda.current_stream().cuda_stream)
    assert rc == 0, K._lib.kmpar_last_error(ctx._h).decode()
    return phi


@pytest.mark.parametrize("mode_name", ["plain", "refined"])
def test_noalloc_cost_equals_cost_two_calls(K, mode_name):
    mode = K.MODE_PLAIN_FP32 if mode_name == "plain" else K.MODE_REFINED
    ctx = K.Context(0, mode)
    # the second call is smaller: n, d and m all shrink
    for n, d, m, seed in [(180_000, 42, 300, 1), (37_001, 15, 64, 2)]:
        print(f"noalloc {mode_name}: n={n} d={d} m={m}", flush=True)
        X = synth.heavy_tailed(n, d, seed=seed) if d == 42 else synth.gauss_mixture(n, d, 20, 10.0, seed)
        rng = np.random.default_rng(seed)
        C = X[rng.choice(n, m, replace=False)] + rng.normal(size=(m, d)).astype(np.float32)
        Xd = torch.from_numpy(X).cuda()
        Cd = torch.from_numpy(np.ascontiguousarray(C, np.float32)).cuda()
        ref = ctx.cost(Xd, Cd)
        got = _abi_noalloc(K, ctx, Xd, Cd, K.F32)
        torch.cuda.synchronize()
        assert got.item() == ref.item()                       # same kernels, same order
        want = O.cost(X.astype(np.float64), C.astype(np.float32).astype(np.float64))
        assert abs(got.item() - want) <= 1e-5 * want


def test_noalloc_cost_bf16_rows(K):
    ctx = K.Context(0, K.MODE_REFINED)
    X = synth.gauss_mixture_sigma(50_000, 128, 40, seed=3)
    Xb = torch.from_numpy(X).cuda().to(torch.bfloat16)
    C = Xb[torch.arange(0, 50_000, 500, device="cuda")].float().contiguous()
    ref = ctx.cost(Xb, C)
    got = _abi_noalloc(K, ctx, Xb, C, K.BF16)
    torch.cuda.synchronize()
    assert got.item() == ref.item()


def test_noalloc_rejects_more_than_its_scratch(K):
    ctx = K.Context(0, K.MODE_PLAIN_FP32)
    n, d = 9_000_000, 4                   # 8 n bytes > 64 MiB
    X = torch.zeros(n, d, device="cuda")
    C = torch.zeros(2, d, device="cuda")
    phi = torch.zeros(1, dtype=torch.float64, device="cuda")
    rc = K._lib.kmpar_cost_noalloc(ctx._h, X.data_ptr(), None, K.F32, n, d, C.data_ptr(), 2,
                                   phi.data_ptr(), None)
    assert rc == K.E_WORKSPACE
    assert "fixed" in K._lib.kmpar_last_error(ctx._h).decode()
    assert K.NOALLOC_SCRATCH_BYTES == 64 << 20
