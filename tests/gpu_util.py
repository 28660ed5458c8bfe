"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare it with the FP64 oracle on the same seeded inputs."""
from __future__ import annotations

import numpy as np
import torch

from oracle import oracle as O

# FP32 squared distances (direct form) agree with FP64 to (d+2) u relative
# per value; the tolerance the kernels are held to is 1e-5 relative.
D2_RTOL = 1e-5


def decoded_fp64(X: np.ndarray, dtype: str, row_scale=None, exact=False) -> np.ndarray:
    """FP64 values of stored inputs (FP32 / BF16 bits / e4m3 codes).  FP32 and
    BF16 are exact.  An FP8 element is taken as the library decodes it,
    fl32(q * s) (what every kernel computes with), unless exact: then q * s
    itself (exact in FP64: at most 4 + 24 significant bits)."""
    if dtype == "f32":
        return X.astype(np.float64)
    if dtype == "bf16":
        return (X.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    if dtype == "fp8":
        q = X.astype(np.uint32)
        s = np.where(q & 0x80, -1.0, 1.0)
        e = (q >> 3) & 0xF
        m = (q & 0x7).astype(np.float64)
        v = np.where(e == 0, m * 2.0 ** -9, (1.0 + m / 8.0) * np.exp2(e.astype(np.float64) - 7.0))
        qs = s * v * row_scale[:, None].astype(np.float64)
        return qs if exact else qs.astype(np.float32).astype(np.float64)
    raise ValueError(dtype)


def to_bf16_bits(X: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even FP32 -> BF16, returned as uint16 bits."""
    u = X.astype(np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def to_e4m3(X: np.ndarray):
    """Per-row scale max|x|/448 and RNE e4m3 codes via torch's float8 type."""
    Xt = torch.from_numpy(X.astype(np.float32))
    amax = Xt.abs().amax(dim=1).clamp_min(1e-30)
    scale = amax / 448.0
    q = (Xt / scale[:, None]).to(torch.float8_e4m3fn)
    return q.view(torch.uint8).numpy(), scale.numpy().astype(np.float32)


def split_rounds(cand_point: np.ndarray, round_count) -> list:
    out, start = [], 1
    for c in round_count[1:]:
        out.append(cand_point[start:start + c])
        start += c
    return out


def gpu_init(ctx, Xdev, k, ell, rounds, seed, row_scale=None):
    r = ctx.init(Xdev, k=k, ell=ell, rounds=rounds, seed=seed, row_scale=row_scale, trace=True,
                 allow_toofew=True)
    torch.cuda.synchronize()
    tr = {key: v.cpu().numpy() for key, v in r.trace.items()}
    return r, tr


def compare_init(X64, r, tr, k, ell, rounds, seed, inst=0, band=None, d2_rtol=D2_RTOL,
                 rows_out=None, sampling="bernoulli", argmins=True):
    """Oracle replay of the GPU run; returns the oracle result after checking
    every part of the run against it.  band: the replay's relative error band
    (default: the FP32 direct-form band of the oracle); rows_out: the values
    the library returns as center rows when they differ from the oracle's
    input X64 (FP8 rows fed to the oracle as exact products); argmins: the
    run counts its near-tied argmins (single-instance calls)."""
    d = X64.shape[1]
    st = r.stats
    follow = {"rounds": split_rounds(tr["cand_point"], st["round_count"]),
              "assign": tr["assign"], "picks": tr["center_cand"]}
    o = O.kmeans_parallel_init(X64, k, ell, rounds, seed, inst=inst, follow=follow, band=band,
                               sampling=sampling)
    assert sum(o.bad.values()) == 0, (o.bad, o.flags)
    # A decision that differs from the oracle's lies inside the band, where
    # the GPU counts its own near-ties: it cannot report fewer.
    if "flagged_draws" in st and sampling == "bernoulli":
        assert st["flagged_draws"] >= o.flags["draw"], (st["flagged_draws"], o.flags)
        assert st["flagged_picks"] >= o.flags["pick"], (st["flagged_picks"], o.flags)
    if argmins:
        assert st["flagged_argmins"] >= o.flags["argmin"], (st["flagged_argmins"], o.flags)
        n, m = X64.shape[0], o.cand_point.size
        if n * m * d <= 2e9:
            # A runner-up more than twice the band away is never flagged: the
            # FP32 direct form moves each distance by less than band / 2
            # (2.01: the second-order terms).
            _, d2, snd = O.nearest(X64, X64[o.cand_point])
            assert st["flagged_argmins"] <= int(np.sum(snd - d2 <= 2.01 * O.fp32_band(d) * d2))
    assert o.round_count == st["round_count"]
    assert np.array_equal(o.cand_point, tr["cand_point"])
    assert np.array_equal(o.weights, tr["cand_weight"])
    assert np.array_equal(o.picks, tr["center_cand"])
    pos = o.d2 > 0
    assert np.all(tr["d2"][~pos] == 0)
    np.testing.assert_allclose(tr["d2"][pos], o.d2[pos], rtol=d2_rtol)
    np.testing.assert_allclose(st["phi"], o.phi, rtol=d2_rtol)
    assert np.all(np.diff(st["phi"]) <= 0)
    C = r.centers.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(C, (X64 if rows_out is None else rows_out)[o.cand_point[o.picks]])
    return o
